"""Seeded input generators: reproducibility and the structural facts the
workloads rely on (kinship centring, positive definiteness, genotype law)."""
import numpy as np

from synth import allele_thresholds, make_workload, snp_genotypes


def test_genotypes_counter_based_and_block_invariant():
    a = snp_genotypes(99, 300, 0, 500)
    b = np.concatenate([snp_genotypes(99, 300, s, 100) for s in range(0, 500, 100)])
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a[123], snp_genotypes(99, 300, 123, 1)[0])
    assert set(np.unique(a)) <= {0, 1, 2}
    assert not np.array_equal(a, snp_genotypes(100, 300, 0, 500))


def test_genotypes_padded_rows_are_zero():
    g = snp_genotypes(5, 100, 10, 7, ld=128)
    assert g.shape == (7, 128) and (g[:, 100:] == 0).all()
    np.testing.assert_array_equal(g[:, :100], snp_genotypes(5, 100, 10, 7))


def test_genotype_law_matches_thresholds():
    """Mean genotype 2f per SNP with f = F / 2^24 in [0.05, 0.5)."""
    n = 20000
    g = snp_genotypes(3, n, 0, 40).astype(float)
    f = allele_thresholds(3, 0, 40) / 2.0**24
    assert (f >= 0.05).all() and (f < 0.5).all()
    sd = np.sqrt(2 * f * (1 - f) / n)
    assert (np.abs(g.mean(1) - 2 * f) < 5 * sd).all()


def test_kinship_structure_and_reproducibility():
    w = make_workload(0, n=120, m=10, kin_cols=300)
    Phi = w.Phi
    np.testing.assert_allclose(Phi, Phi.T, atol=0)
    # standardised kinship columns: Phi 1 = 0.01 * 1 exactly up to rounding
    np.testing.assert_allclose(Phi @ np.ones(w.n), 0.01 * np.ones(w.n), atol=1e-12)
    assert np.linalg.eigvalsh(Phi).min() > 0.0099
    np.testing.assert_allclose(np.diag(Phi).mean(), 1.01, rtol=1e-12)
    w2 = make_workload(0, n=120, m=10, kin_cols=300)
    np.testing.assert_array_equal(w.Phi, w2.Phi)
    np.testing.assert_array_equal(w.Y, w2.Y)
    assert w.snp_seed == w2.snp_seed


def test_workload_shapes_and_ranges():
    w = make_workload(2, n=200, m=50, t=40, kin_cols=400)
    assert w.XL.shape == (200, 3) and w.Y.shape == (200, 40)
    assert (w.XL[:, 0] == 1).all() and set(np.unique(w.XL[:, 1])) <= {0.0, 1.0}
    assert ((w.h2 >= 0.05) & (w.h2 <= 0.95)).all() and ((w.s2 >= 0.5) & (w.s2 <= 2)).all()
    assert w.genotypes(0, 5).shape == (5, 200)
    w0 = make_workload(0)
    assert (w0.s2 == 1).all() and w0.n == 256 and w0.m == 2000
