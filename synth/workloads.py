"""Seeded synthetic GWAS workloads.

The paper's experiments use artificial data sets with prescribed n, m, t and
two covariates (supplementary notes, simulated data; scenario C fixes n=1000,
m=10^6 and varies t).  No public data set is involved; these generators stand
in for that simulated data.  Recipe (one seed per role, derived from the
configuration seed):

* kinship: Phi = Gs Gs^T / c + 0.01 I, Gs an n x c matrix of Binomial(2, f)
  genotypes, f ~ U(0.05, 0.5) per column, monomorphic columns redrawn, every
  column standardised with its empirical mean and standard deviation;
* covariates X_L = [1, sex ~ Bernoulli(0.5), age ~ N(50, 10)] (+ principal
  components of Phi scaled to unit variance for the large configuration);
* traits: beta_j ~ N(0, 1)^{p_L}; h2_j, sigma2_j uniform per configuration;
  y_j ~ N(X_L beta_j, sigma2_j (h2_j Phi + (1 - h2_j) I)), drawn either through
  the Cholesky factor of that covariance (small single-trait case) or as
  X_L beta_j + sigma_j (h_j L_Phi e1 + sqrt(1 - h2_j) e2) with one Cholesky
  factor L_Phi of Phi (same law, one factorisation for all traits);
* SNPs: the counter-based generator of ``synth.genotypes``.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .genotypes import snp_genotypes

MASTER_SEED = 12072169

# role ids for independent random streams
_R_KIN, _R_COV, _R_BETA, _R_H2, _R_S2, _R_NOISE, _R_SNP, _R_COHORT = range(8)

CONFIGS = {
    0: dict(name="single-trait n=256 m=2000 t=1 (FP64 plain)", n=256, m=2000, t=1, kin_cols=2000,
            pL=3, block=2000, h2=(0.1, 0.9), s2=None, y_draw="chol_M", pcs=0),
    1: dict(name="single-trait n=1000 m=1e6 t=1, blocks of 1e4", n=1000, m=1_000_000, t=1,
            kin_cols=5000, pL=3, block=10_000, h2=(0.1, 0.9), s2=None, y_draw="chol_Phi", pcs=0),
    2: dict(name="multi-trait n=1000 m=1e5 t=1000", n=1000, m=100_000, t=1000, kin_cols=5000,
            pL=3, block=10_000, h2=(0.05, 0.95), s2=(0.5, 2.0), y_draw="chol_Phi", pcs=0),
    4: dict(name="large multi-trait n=1e4 m=2e6 t=1000 p_L=8, blocks of 2e4", n=10_000,
            m=2_000_000, t=1000, kin_cols=20_000, pL=8, block=20_000, h2=(0.05, 0.95),
            s2=(0.5, 2.0), y_draw="chol_Phi", pcs=5),
}
COHORT_SIZES = (500, 750, 1000, 1500, 2000, 2500, 3000, 4000)


def _rng(cseed: int, role: int) -> np.random.Generator:
    return np.random.default_rng([cseed, role])


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    m: int
    t: int
    pL: int
    block: int
    seed: int          # configuration seed
    snp_seed: int      # seed of the counter-based SNP generator
    Phi: np.ndarray    # (n, n) float64, symmetric
    XL: np.ndarray     # (n, pL) float64, Fortran order
    Y: np.ndarray      # (n, t) float64, Fortran order
    h2: np.ndarray     # (t,) float64
    s2: np.ndarray     # (t,) float64

    def genotypes(self, start: int, count: int, ld: Optional[int] = None) -> np.ndarray:
        """uint8 (count, ld): row s = SNP start+s over the n individuals."""
        return snp_genotypes(self.snp_seed, self.n, start, count, ld=ld)


def kinship(rng: np.random.Generator, n: int, cols: int, chunk: int = 2048) -> np.ndarray:
    """Phi = Gs Gs^T / cols + 0.01 I with column-standardised Binomial(2, f) genotypes."""
    Phi = np.zeros((n, n))
    done = 0
    while done < cols:
        c = min(chunk, cols - done)
        f = rng.uniform(0.05, 0.5, c)
        G = rng.binomial(2, f, (n, c)).astype(np.float64)
        sd = G.std(0)
        while (bad := np.flatnonzero(sd == 0)).size:
            G[:, bad] = rng.binomial(2, f[bad], (n, bad.size))
            sd = G.std(0)
        G = (G - G.mean(0)) / sd
        Phi += G @ G.T
        done += c
    Phi /= cols
    Phi = 0.5 * (Phi + Phi.T)
    Phi[np.diag_indices(n)] += 0.01
    return Phi


def make_workload(config: int = 0, *, n: Optional[int] = None, m: Optional[int] = None,
                  t: Optional[int] = None, kin_cols: Optional[int] = None,
                  seed: Optional[int] = None, name: Optional[str] = None) -> Workload:
    """Inputs of configuration ``config``; keyword overrides shrink it for tests."""
    cfg = dict(CONFIGS[config])
    n = cfg["n"] if n is None else n
    m = cfg["m"] if m is None else m
    t = cfg["t"] if t is None else t
    kc = cfg["kin_cols"] if kin_cols is None else kin_cols
    pL = cfg["pL"]
    cseed = MASTER_SEED + 1000 * config if seed is None else seed
    Phi = kinship(_rng(cseed, _R_KIN), n, kc)
    rc = _rng(cseed, _R_COV)
    cols = [np.ones(n), rc.binomial(1, 0.5, n).astype(np.float64), rc.normal(50.0, 10.0, n)]
    if cfg["pcs"]:
        import scipy.linalg
        w, V = scipy.linalg.eigh(Phi, subset_by_index=[n - cfg["pcs"], n - 1])
        for k in range(cfg["pcs"] - 1, -1, -1):
            cols.append(V[:, k] * np.sqrt(n))
    XL = np.asfortranarray(np.stack(cols, 1)[:, :pL])
    pL = XL.shape[1]
    h2 = _rng(cseed, _R_H2).uniform(*cfg["h2"], t)
    s2 = np.ones(t) if cfg["s2"] is None else _rng(cseed, _R_S2).uniform(*cfg["s2"], t)
    beta = _rng(cseed, _R_BETA).normal(size=(pL, t))
    rn = _rng(cseed, _R_NOISE)
    mean = XL @ beta
    if cfg["y_draw"] == "chol_M":
        Y = np.empty((n, t))
        for j in range(t):
            Lm = np.linalg.cholesky(s2[j] * (h2[j] * Phi + (1 - h2[j]) * np.eye(n)))
            Y[:, j] = mean[:, j] + Lm @ rn.normal(size=n)
    else:
        LP = np.linalg.cholesky(Phi)
        e1 = LP @ rn.normal(size=(n, t))
        e2 = rn.normal(size=(n, t))
        Y = mean + np.sqrt(s2)[None, :] * (np.sqrt(h2)[None, :] * e1 + np.sqrt(1 - h2)[None, :] * e2)
    snp_seed = int(_rng(cseed, _R_SNP).integers(0, 2**63 - 1))
    return Workload(name or cfg["name"], n, m, t, pL, cfg["block"], cseed, snp_seed,
                    np.asfortranarray(Phi), XL, np.asfortranarray(Y), h2, s2)


def cohort_workloads(m: int = 50_000, sizes=COHORT_SIZES, t_range=(10, 2000),
                     t_override: Optional[list] = None) -> list:
    """Eight independent cohorts with uneven n and log-uniform t (batched configuration)."""
    cseed = MASTER_SEED + 3000
    rt = _rng(cseed, _R_COHORT)
    ts = np.rint(np.exp(rt.uniform(np.log(t_range[0]), np.log(t_range[1]), len(sizes)))).astype(int)
    if t_override is not None:
        ts = np.asarray(t_override, int)
    out = []
    for c, (nc, tc) in enumerate(zip(sizes, ts)):
        base = dict(CONFIGS[0])
        base.update(name=f"cohort {c} n={nc} t={tc}", n=nc, m=m, t=int(tc), kin_cols=2 * nc,
                    block=m, h2=(0.05, 0.95), s2=(0.5, 2.0), y_draw="chol_Phi")
        CONFIGS[100 + c] = base
        out.append(make_workload(100 + c, seed=cseed + 17 * (c + 1)))
    return out
