"""Status codes and the call-order state machine of the C ABI, forced from
the host (every kernel still runs to completion)."""
import numpy as np
import pytest

from synth import make_workload

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _col(a):
    return _t(np.ascontiguousarray(np.asarray(a).T)).t()


@pytest.fixture(scope="module")
def w():
    return make_workload(0, n=96, m=20, kin_cols=200)


def test_status_codes(w):
    import torch

    from paper_1207_2169_amd import clak
    from paper_1207_2169_amd.clak import ClakError
    print("ABI status codes", flush=True)
    with pytest.raises(ClakError) as e:
        clak.clak_plan_create(10, 0, 1, 10)
    assert e.value.status == clak.CLAK_E_ARG
    with pytest.raises(ClakError) as e:
        clak.clak_plan_create(40000, 3, 1, 10, clak.CLAK_PREC_MIXED)
    assert e.value.status == clak.CLAK_E_UNSUPPORTED
    h = clak.clak_plan_create(w.n, w.pL, 2, 16)
    try:
        # no workspace yet
        with pytest.raises(ClakError) as e:
            clak.clak_set_kinship(h, _t(w.Phi))
        assert e.value.status == clak.CLAK_E_STATE
        nbytes = clak.clak_plan_workspace_size(h)
        assert nbytes % 256 == 0
        small = torch.empty(nbytes - 256, dtype=torch.uint8, device="cuda")
        with pytest.raises(ClakError) as e:
            clak.clak_plan_set_workspace(h, small)
        assert e.value.status == clak.CLAK_E_WORKSPACE
        ws = torch.empty(nbytes + 512, dtype=torch.uint8, device="cuda")
        with pytest.raises(ClakError) as e:
            clak.clak_plan_set_workspace(h, ws[1:])
        assert e.value.status == clak.CLAK_E_WORKSPACE
        clak.clak_plan_set_workspace(h, ws)
        clak.clak_plan_set_stream(h)
        # covariates before kinship
        with pytest.raises(ClakError) as e:
            clak.clak_set_covariates(h, _col(w.XL))
        assert e.value.status == clak.CLAK_E_STATE
        clak.clak_set_kinship(h, _t(w.Phi))
        # rank-deficient covariates
        XLbad = np.c_[w.XL[:, :2], w.XL[:, 1] * 2.0]
        with pytest.raises(ClakError) as e:
            clak.clak_set_covariates(h, _col(XLbad))
        assert e.value.status == clak.CLAK_E_COV_SINGULAR
        XLnan = w.XL.copy()
        XLnan[3, 2] = np.nan
        with pytest.raises(ClakError) as e:
            clak.clak_set_covariates(h, _col(XLnan))
        assert e.value.status == clak.CLAK_E_ARG
        clak.clak_set_covariates(h, _col(w.XL))
        G = _t(w.genotypes(0, 16))
        b = torch.empty((2, 16), dtype=torch.float64, device="cuda")
        se = torch.empty_like(b)
        with pytest.raises(ClakError) as e:
            clak.clak_run_block(h, G, b, se)
        assert e.value.status == clak.CLAK_E_STATE
        Y = _col(np.c_[w.Y, w.Y])
        for h2, s2 in [([0.5, 1.2], [1.0, 1.0]), ([0.5, -0.1], [1.0, 1.0]), ([0.5, 0.5], [1.0, 0.0]),
                       ([0.5, np.nan], [1.0, 1.0])]:
            with pytest.raises(ClakError) as e:
                clak.clak_set_traits(h, Y, _t(np.array(h2)), _t(np.array(s2)))
            assert e.value.status == clak.CLAK_E_ARG
        clak.clak_set_traits(h, Y, _t(np.array([0.5, 1.0])), _t(np.array([1.0, 2.0])))
        # block larger than max_block, bad leading dimension
        G17 = _t(w.genotypes(0, 17))
        b17 = torch.empty((2, 17), dtype=torch.float64, device="cuda")
        se17 = torch.empty_like(b17)
        with pytest.raises(ValueError):  # the binding checks against the plan's max_block first
            clak.clak_run_block(h, G17, b17, se17)
        # the library refuses the same call on its own
        assert clak.lib().clak_run_block(h, 17, G17.data_ptr(), clak.CLAK_G_U8, w.n, b17.data_ptr(),
                                         se17.data_ptr(), clak.CLAK_OUT_F64, 17, None, None) == clak.CLAK_E_ARG
        assert clak.lib().clak_run_block(h, 16, G.data_ptr(), clak.CLAK_G_U8, w.n - 1, b.data_ptr(),
                                         se.data_ptr(), clak.CLAK_OUT_F64, 16, None, None) == clak.CLAK_E_ARG
        assert clak.lib().clak_run_block(h, 16, G.data_ptr(), clak.CLAK_G_U8, w.n, b.data_ptr(),
                                         se.data_ptr(), clak.CLAK_OUT_F64, 15, None, None) == clak.CLAK_E_ARG
        clak.clak_run_block(h, G, b, se)
        torch.cuda.synchronize()
        assert torch.isfinite(b).all() and (se > 0).all()
        # indefinite kinship with h2 = 1: not positive definite
        ev, V = np.linalg.eigh(w.Phi)
        ev[0] = -0.2
        clak.clak_set_kinship(h, _t((V * ev) @ V.T))
        clak.clak_set_covariates(h, _col(w.XL))
        with pytest.raises(ClakError) as e:
            clak.clak_set_traits(h, Y, _t(np.array([0.5, 1.0])), _t(np.array([1.0, 1.0])))
        assert e.value.status == clak.CLAK_E_NOT_SPD
        # traits invalidated: run_block refuses
        with pytest.raises(ClakError) as e:
            clak.clak_run_block(h, G, b, se)
        assert e.value.status == clak.CLAK_E_STATE
    finally:
        clak.clak_plan_destroy(h)


@pytest.mark.parametrize("prec", [0, 1])
def test_degenerate_and_bad_genotypes(w, prec):
    """Monomorphic, all-zero and covariate-equal SNPs give NaN and flag 1;
    a genotype outside {0, 1, 2} gives NaN and flag 2; the rest match the
    oracle."""
    import torch

    import oracle
    from paper_1207_2169_amd import clak
    print(f"degenerate SNPs precision={prec}", flush=True)
    n = w.n
    XL = w.XL.copy()
    g = w.genotypes(0, 8).astype(np.uint8)
    g[0] = 2
    g[1] = 0
    g[2] = XL[:, 1].astype(np.uint8)
    g[3, 5] = 3
    with clak.Plan(n, w.pL, 1, 8, prec) as plan:
        clak.clak_set_kinship(plan.handle, _t(w.Phi))
        clak.clak_set_covariates(plan.handle, _col(XL))
        clak.clak_set_traits(plan.handle, _col(w.Y), _t(w.h2), _t(w.s2))
        b = torch.empty((1, 8), dtype=torch.float64, device="cuda")
        se = torch.empty_like(b)
        fl = torch.empty((1, 8), dtype=torch.uint8, device="cuda")
        clak.clak_run_block(plan.handle, _t(g), b, se, fl)
        torch.cuda.synchronize()
        b, se, fl = b.cpu().numpy()[0], se.cpu().numpy()[0], fl.cpu().numpy()[0]
    assert list(fl[:4]) == [1, 1, 1, 2] and (fl[4:] == 0).all()
    assert np.isnan(b[:4]).all() and np.isnan(se[:4]).all()
    rb, rv, rf = oracle.gls_cells(w.Phi, XL, g[4:].T.astype(float), w.Y, w.h2, w.s2, np.arange(4),
                                  np.zeros(4, int))
    tol = 1e-9 if prec == 0 else 1e-6
    rse = np.sqrt(rv[:, -1, -1])
    assert np.max(np.abs(b[4:] - rb[:, -1]) / rse) < tol
    assert np.max(np.abs(se[4:] - rse) / rse) < tol


def test_pinned_host_genotypes_and_pageable_refusal():
    """A genotype block in pinned host memory (read over PCIe by the ingest
    kernel) gives bitwise the same cells as one in device memory; pageable host
    memory is refused with CLAK_E_ARG before anything is launched."""
    import ctypes

    import torch

    from paper_1207_2169_amd import clak
    w = make_workload(2, n=300, m=500, t=7, kin_cols=600)
    print("pinned host genotypes", flush=True)
    g = torch.from_numpy(w.genotypes(0, w.m))
    with clak.Plan(w.n, w.pL, w.t, w.m, clak.CLAK_PREC_MIXED) as plan:
        clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Phi)).cuda())
        clak.clak_set_covariates(plan.handle, torch.from_numpy(np.ascontiguousarray(w.XL.T)).cuda().t())
        clak.clak_set_traits(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Y.T)).cuda().t(),
                             torch.from_numpy(w.h2).cuda(), torch.from_numpy(w.s2).cuda())
        outs = []
        for G in (g.cuda(), g.pin_memory()):
            b = torch.full((w.t, w.m), float("nan"), dtype=torch.float64, device="cuda")
            se = torch.full_like(b, float("nan"))
            clak.clak_run_block(plan.handle, G, b, se)
            torch.cuda.synchronize()
            outs.append((b, se))
        assert torch.isfinite(outs[0][0]).all()
        assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
        b, se = outs[0]
        st = clak.lib().clak_run_block(plan.handle, w.m, ctypes.c_void_p(g.data_ptr()), clak.CLAK_G_U8, w.n,
                                       ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(se.data_ptr()),
                                       clak.CLAK_OUT_F64, w.m, None, None)
        assert st == clak.CLAK_E_ARG
        assert b"device-accessible" in clak.lib().clak_last_error()
    # with CLAK_STAGE_GENOTYPES every block goes through the copy engine into a staging buffer
    with clak.Plan(w.n, w.pL, w.t, w.m, clak.CLAK_PREC_MIXED, clak.CLAK_STAGE_GENOTYPES) as plan:
        clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Phi)).cuda())
        clak.clak_set_covariates(plan.handle, torch.from_numpy(np.ascontiguousarray(w.XL.T)).cuda().t())
        clak.clak_set_traits(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Y.T)).cuda().t(),
                             torch.from_numpy(w.h2).cuda(), torch.from_numpy(w.s2).cuda())
        for G in (g.pin_memory(), g.half().pin_memory(), g.cuda(), g.half().cuda()):
            b = torch.full((w.t, w.m), float("nan"), dtype=torch.float64, device="cuda")
            se = torch.full_like(b, float("nan"))
            clak.clak_run_block(plan.handle, G, b, se)
            torch.cuda.synchronize()
            assert torch.equal(b, outs[0][0]) and torch.equal(se, outs[0][1])
