"""Writes tests/golden/c4_sample.npz: oracle values for a sample of cells of
the large multi-trait workload (n = 10^4 individuals, p_L = 8 covariates:
intercept, sex, age and five principal components of Phi; one block of
2 10^4 SNPs; t = 1000 traits), the configuration whose full evaluation by the
oracle is too slow for a test (each trait's Cholesky factor of the
10^4 x 10^4 covariance takes minutes).

Only the seeded input generators (synth) and the oracle are called.  The
sample is 20 random traits x 500 random SNPs of the block (10^4 cells, every
trait of the sample paired with every SNP of the sample).  Stored beside the
values: fingerprints of the inputs (Phi's trace, a few entries of Phi, the
sampled traits' phenotype sums and their h2, s2), so that a test that
regenerates the inputs on another machine first checks they agree (numpy's
BLAS may round differently there; the fingerprints must match to 1e-9
relative, which moves b by far less than the 1e-6 SE bar).

Run:  python tests/golden/make_c4_sample.py   (about half an hour on 8 cores)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import make_workload  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_sample.npz")
M_BLOCK = 20_000
N_TRAITS, N_SNPS = 20, 500
SAMPLE_SEED = 4_0413


def fingerprints(w, traits):
    """Input fingerprints compared before the stored values are used."""
    idx = np.array([0, 1, 17, 4321, w.n - 1])
    return {
        "phi_trace": np.trace(w.Phi),
        "phi_entries": w.Phi[idx, idx[::-1]],
        "xl_colsum": w.XL.sum(0),
        "y_colsum": w.Y[:, traits].sum(0),
        "h2": w.h2[traits],
        "s2": w.s2[traits],
    }


def sample_cells(w):
    rng = np.random.default_rng(SAMPLE_SEED)
    traits = np.sort(rng.choice(w.t, N_TRAITS, replace=False))
    snps = np.sort(rng.choice(M_BLOCK, N_SNPS, replace=False))
    return traits, snps


def main():
    t0 = time.perf_counter()
    w = make_workload(4, m=M_BLOCK)
    print(f"workload n={w.n} p_L={w.pL} m={w.m} t={w.t}: {time.perf_counter() - t0:.0f} s", flush=True)
    traits, snps = sample_cells(w)
    G = np.concatenate([w.genotypes(int(s), 1) for s in snps]).T.astype(np.float64)
    ii, jj = np.meshgrid(np.arange(snps.size), traits, indexing="ij")
    t1 = time.perf_counter()
    b, var, flag = oracle.gls_cells(w.Phi, w.XL, G, w.Y, w.h2, w.s2, ii.ravel(), jj.ravel())
    print(f"oracle {ii.size} cells on {oracle.threads()} threads: {time.perf_counter() - t1:.0f} s", flush=True)
    fp = fingerprints(w, traits)
    np.savez_compressed(OUT, snp=snps[ii.ravel()], trait=jj.ravel(), b=b[:, -1], se=np.sqrt(var[:, -1, -1]),
                        flag=flag, traits=traits, snps=snps, **{"fp_" + k: v for k, v in fp.items()})
    print(f"wrote {OUT}: {int((flag == 0).sum())} of {flag.size} cells unflagged", flush=True)


if __name__ == "__main__":
    main()
