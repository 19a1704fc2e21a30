"""Shared helpers of the GPU tests: run the HIP path through the C ABI on a
workload, run the oracle on chosen cells, and compare."""
from __future__ import annotations

import numpy as np

import oracle


def gpu_run(w, precision, flags=0, block=None, g_dtype="u8", out_dtype="f64", ldg_pad=0, ldo_pad=0,
            snp_range=None, eigen=None, want_flags=True, want_pval=False):
    """b, se, cell flags of every cell in SNPs [start, stop) of workload w.

    Returns b (m, t) or (m, t, p) with CLAK_OUT_FULL, se (m, t), flags (m, t),
    and with want_pval the p-values (m, t) as a fourth item."""
    import torch

    from paper_1207_2169_amd import clak

    dev = torch.device("cuda")
    start, stop = snp_range or (0, w.m)
    m = stop - start
    block = block or min(m, w.block)
    p = w.pL + 1
    odt = torch.float64 if out_dtype == "f64" else torch.float32
    with clak.Plan(w.n, w.pL, w.t, block, precision, flags) as plan:
        if eigen is None:
            clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Phi)).to(dev))
        else:
            Z, ev = eigen
            clak.clak_set_eigen(plan.handle, torch.from_numpy(np.asfortranarray(Z)).to(dev).t().contiguous().t(),
                                torch.from_numpy(ev).to(dev))
        XL = torch.from_numpy(np.ascontiguousarray(w.XL.T)).to(dev).t()
        clak.clak_set_covariates(plan.handle, XL)
        Y = torch.from_numpy(np.ascontiguousarray(w.Y.T)).to(dev).t()
        clak.clak_set_traits(plan.handle, Y, torch.from_numpy(w.h2).to(dev), torch.from_numpy(w.s2).to(dev))
        full = bool(flags & clak.CLAK_OUT_FULL)
        bs, ses, fls, pvs = [], [], [], []
        for s0 in range(start, stop, block):
            mb = min(block, stop - s0)
            g = w.genotypes(s0, mb, ld=w.n + ldg_pad)
            G = torch.from_numpy(g).to(dev)
            if g_dtype == "f16":
                G = G.to(torch.float16)
            ldo = mb + ldo_pad
            b = torch.full((w.t, ldo, p) if full else (w.t, ldo), float("inf"), dtype=odt, device=dev)
            se = torch.full((w.t, ldo), float("inf"), dtype=odt, device=dev)
            fl = torch.full((w.t, ldo), 255, dtype=torch.uint8, device=dev) if want_flags else None
            pv = torch.full((w.t, ldo), float("inf"), dtype=odt, device=dev) if want_pval else None
            clak.clak_run_block(plan.handle, G, b, se, fl, pv)
            torch.cuda.synchronize()
            if ldo_pad:
                assert torch.isinf(se[:, mb:]).all(), "output padding overwritten"
            bs.append(b[:, :mb].cpu().numpy().astype(np.float64))
            ses.append(se[:, :mb].cpu().numpy().astype(np.float64))
            if want_flags:
                fls.append(fl[:, :mb].cpu().numpy())
            if want_pval:
                if ldo_pad:
                    assert torch.isinf(pv[:, mb:]).all(), "p-value padding overwritten"
                pvs.append(pv[:, :mb].cpu().numpy().astype(np.float64))
        b = np.concatenate(bs, axis=1)
        se = np.concatenate(ses, axis=1)
        fl = np.concatenate(fls, axis=1) if want_flags else None
    b = np.moveaxis(b, 0, 1)  # (m, t[, p])
    if want_pval:
        return b, se.T, (fl.T if fl is not None else None), np.concatenate(pvs, axis=1).T
    return b, se.T, (fl.T if fl is not None else None)


def oracle_cells(w, snp, trait, var_paper=False):
    """Oracle b (cells, p) and SE of the SNP effect for cells (snp[c], trait[c])."""
    snp = np.asarray(snp)
    uniq, inv = np.unique(snp, return_inverse=True)
    G = np.concatenate([w.genotypes(int(s), 1) for s in uniq]).T.astype(np.float64)
    b, var, flag = oracle.gls_cells(w.Phi, w.XL, G, w.Y, w.h2, w.s2, inv, trait, var_paper=var_paper)
    return b, np.sqrt(var[:, -1, -1]), flag


def errors(b, se, b_ref, se_ref):
    """(eps_b, eps_se): max |b - b_ref| / SE_ref and max |SE - SE_ref| / SE_ref."""
    eb = np.abs(b - b_ref) / se_ref
    es = np.abs(se - se_ref) / se_ref
    return float(np.max(eb)), float(np.max(es))
