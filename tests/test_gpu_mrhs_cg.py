"""Multi-source CG (lqcd_cg_params.nrhs > 1) against the oracle: every
source's FP64 residual recomputed on the host, every solution against the
single-source solve of the same system, zero sources, and argument checks.
Source counts 3, 4 and 6 cover the three multi-source layouts (blocks of 1,
4 and 2 sources)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import ctx, np_of  # noqa: F401

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1109_2935_amd.lqcd")
from paper_1109_2935_amd import ops  # noqa: E402


@pytest.mark.parametrize("nrhs,sloppy", [(4, None), (3, 1), (6, 2), (4, 3)])
def test_cgne_multi_source(ctx, nrhs, sloppy):
    """CGNE on the Wilson-clover Schur system for nrhs Gaussian sources at once
    (FP64, or FP32/FP16/BF16 sloppy iterations with FP64 reliable updates)."""
    dims, kappa, csw, tile = (8, 8, 4, 8), 0.124, 1.0, (8, 4, 4, 4)
    U = synth.gauge_field(dims, 0.25, 701)
    Ud = torch.from_numpy(U).cuda()
    hi = ops.wilson_clover(ctx, U, dims, kappa, csw, 0, 18, tile=tile, U_device=Ud)
    lo = None if sloppy is None else ops.wilson_clover(ctx, U, dims, kappa, csw, sloppy, 12, tile=tile, U_device=Ud)
    bs = np.stack([synth.gaussian_spinor(dims, 710 + j) for j in range(nrhs)])
    bp = hi.import_spinor(bs, -1, nrhs=nrhs)
    x = hi.spinor(full=True, nrhs=nrhs)
    prm = ops.cg_params(1e-10, 5000, 0.1, nrhs=nrhs)
    st, info = L.lqcd_cg_solve(ctx, hi.op, lo.op if lo else None, prm, x, bp)
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    res_gpu = ops.rhs_residuals(prm)
    assert max(res_gpu) <= 1e-10 and info.true_residual == max(res_gpu)
    xs = np_of(hi.export_spinor(x, -1, nrhs=nrhs))
    M = oracle.WilsonClover(dims, U, kappa, csw, bc_t=-1)
    for j in range(nrhs):
        res = np.linalg.norm(bs[j] - M.M(xs[j])) / np.linalg.norm(bs[j])
        assert res <= 1.05e-10, (j, res)
        assert abs(res - res_gpu[j]) <= 1e-3 * res + 1e-15
    # each source against its own single-source solve (same solution to the
    # accuracy the stopping rule allows)
    for j in (0, nrhs - 1):
        b1 = hi.import_spinor(bs[j], -1)
        x1 = hi.spinor(full=True)
        st, i1 = L.lqcd_cg_solve(ctx, hi.op, lo.op if lo else None, ops.cg_params(1e-10, 5000, 0.1), x1, b1)
        assert st == L.LQCD_OK
        a = np_of(hi.export_spinor(x1, -1))
        assert np.linalg.norm(xs[j] - a) / np.linalg.norm(a) < 1e-8
        if sloppy is None:
            assert abs(i1.iters - info.iters) <= max(3, 0.05 * i1.iters) or i1.iters < info.iters


def test_cgne_multi_source_zero_source(ctx):
    """A zero source among others has the solution zero; the rest converge."""
    dims, kappa, csw = (4, 4, 4, 8), 0.12, 1.0
    U = synth.gauge_field(dims, 0.25, 721)
    hi = ops.wilson_clover(ctx, U, dims, kappa, csw, 0, 18)
    lo = ops.wilson_clover(ctx, U, dims, kappa, csw, 1, 12)
    bs = np.stack([synth.gaussian_spinor(dims, 722), np.zeros(oracle.shape4(dims) + (4, 3), complex),
                   synth.gaussian_spinor(dims, 723), synth.gaussian_spinor(dims, 724)])
    bp = hi.import_spinor(bs, -1, nrhs=4)
    x = hi.spinor(full=True, nrhs=4)
    x.fill_(0)
    prm = ops.cg_params(1e-10, 5000, 0.1, nrhs=4)
    st, info = L.lqcd_cg_solve(ctx, hi.op, lo.op, prm, x, bp)
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    xs = np_of(hi.export_spinor(x, -1, nrhs=4))
    assert np.abs(xs[1]).max() == 0
    M = oracle.WilsonClover(dims, U, kappa, csw, bc_t=-1)
    for j in (0, 2, 3):
        assert np.linalg.norm(bs[j] - M.M(xs[j])) / np.linalg.norm(bs[j]) <= 1.05e-10


@pytest.mark.parametrize("sloppy", [None, 1])
def test_staggered_cg_multi_source(ctx, sloppy):
    """CG on N_e = m^2 - D_eo D_oe / 4 for 4 even-site sources at once."""
    dims, mass = (8, 8, 8, 8), 0.05
    U = synth.gauge_field(dims, 0.2, 731)
    fat = synth.fat_links(dims, U, seed=732)
    hi = ops.staggered(ctx, fat, U, dims, mass, 0, 18)
    lo = None if sloppy is None else ops.staggered(ctx, fat, U, dims, mass, sloppy, 12)
    even = oracle.parity_mask(dims, 0)
    bs = np.stack([np.where(even[..., None], synth.gaussian_spinor(dims, 740 + j, inner=(3,)), 0) for j in range(4)])
    bp = hi.import_spinor(bs, 0, nrhs=4)
    x = hi.spinor(nrhs=4)
    prm = ops.cg_params(1e-10, 5000, 0.1, L.LQCD_CG_STAG_NORMAL, nrhs=4)
    st, info = L.lqcd_cg_solve(ctx, hi.op, lo.op if lo else None, prm, x, bp)
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    xs = np_of(hi.export_spinor(x, 0, nrhs=4))
    op = oracle.Staggered(dims, fat, oracle.long_links(dims, U), mass)
    for j in range(4):
        res = np.linalg.norm(bs[j] - op.normal_even(xs[j])) / np.linalg.norm(bs[j])
        assert res <= 1.05e-10, (j, res)


def test_multi_source_argument_checks(ctx):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.25, 751)
    hi = ops.wilson_clover(ctx, U, dims, 0.12, 1.0, 0, 18)
    b = hi.spinor(full=True, nrhs=2)
    x = hi.spinor(full=True, nrhs=2)
    for bad in (ops.cg_params(nrhs=L.LQCD_MAX_CG_RHS + 1), ops.cg_params(nrhs=2, history=4)):
        with pytest.raises(L.LqcdError) as ei:
            L.lqcd_cg_solve(ctx, hi.op, None, bad, x, b)
        assert ei.value.status == L.LQCD_ERR_INVALID_ARG
