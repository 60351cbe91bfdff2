"""Mixed-precision BiCGstab for Wilson-clover (Section III-A; the baseline of
the GCR-DD comparison in Section IX) against the FP64 oracle: the final
residual is recomputed by the oracle over the full lattice, and the FP64 solve
follows the oracle's BiCGstab on the even-odd system step for step."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import ctx, np_of, rel  # noqa: F401
from oracle import solvers

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1109_2935_amd.lqcd")
from paper_1109_2935_amd import ops  # noqa: E402


def wilson_system(ctx, dims, kappa, csw, eps, seed_u, seed_b, precs, tile=None):
    U = synth.gauge_field(dims, eps, seed_u)
    b = synth.gaussian_spinor(dims, seed_b)
    Ud = torch.from_numpy(U).cuda()
    opsd = {p: ops.wilson_clover(ctx, U, dims, kappa, csw, p, 18 if p in (0, 1) else 12, tile=tile, U_device=Ud)
            for p in precs}
    return U, b, opsd


def oracle_residual(dims, U, kappa, csw, x, b):
    op = oracle.WilsonClover(dims, U, kappa, csw, bc_t=-1)
    return np.linalg.norm(b - op.M(x)) / np.linalg.norm(b), op


def test_bicgstab_fp64_follows_oracle(ctx):
    """All-FP64 BiCGstab, 8^4, kappa 0.124: the oracle's residual <= 1e-10, the
    oracle's BiCGstab solution, and the same number of steps."""
    dims, kappa, csw = (8, 8, 8, 8), 0.124, 1.0
    U, b, o = wilson_system(ctx, dims, kappa, csw, 0.25, 1101, 1102, [0])
    hi = o[0]
    x = hi.spinor(full=True)
    st, info = L.lqcd_bicgstab_solve(ctx, hi.op, None, ops.bicgstab_params(1e-10), x, hi.import_spinor(b, -1))
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    assert info.true_residual <= 1e-10
    assert info.matvecs <= 2 * info.iters
    xs = np_of(hi.export_spinor(x, -1))
    res, op = oracle_residual(dims, U, kappa, csw, xs, b)
    assert res <= 1.05e-10
    bhat = op.schur_source(b)
    xe, _, _ = solvers.bicgstab(op.schur, bhat, tol=1e-13)
    assert rel(xs, op.reconstruct(xe, b)) < 1e-8
    # the library stops on ||bhat - Mhat x_e|| <= tol ||b|| (full source)
    tol_hat = 1e-10 * np.linalg.norm(b) / np.linalg.norm(bhat)
    _, it, _ = solvers.bicgstab(op.schur, bhat, tol=tol_hat)
    assert abs(info.iters - it) <= max(2, 0.05 * it), (info.iters, it)


@pytest.mark.parametrize("sprec", [1, 2, 3])
def test_bicgstab_mixed_precision(ctx, sprec):
    """FP32, FP16 and BF16 sloppy iterations with FP64 reliable updates reach an
    FP64 residual of 1e-10 on a 16x8x8x16 lattice."""
    dims, kappa, csw = (16, 8, 8, 16), 0.124, 1.0
    U, b, o = wilson_system(ctx, dims, kappa, csw, 0.25, 1201, 1202, [0, sprec])
    x = o[0].spinor(full=True)
    st, info = L.lqcd_bicgstab_solve(ctx, o[0].op, o[sprec].op, ops.bicgstab_params(1e-10, 5000, 0.1), x,
                                     o[0].import_spinor(b, -1))
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    assert info.restarts >= 2
    assert info.true_residual <= 1e-10
    res, _ = oracle_residual(dims, U, kappa, csw, np_of(o[0].export_spinor(x, -1)), b)
    assert res <= 1.05e-10


def test_bicgstab_fewer_matvecs_than_cgne(ctx):
    """On the same system, BiCGstab needs fewer applications of Mhat than CG on
    the normal equations (the reason it is the usual Wilson-clover solver)."""
    dims, kappa, csw = (8, 8, 8, 8), 0.124, 1.0
    U, b, o = wilson_system(ctx, dims, kappa, csw, 0.25, 1301, 1302, [0, 1])
    bp = o[0].import_spinor(b, -1)
    x1, x2 = o[0].spinor(full=True), o[0].spinor(full=True)
    st1, bi = L.lqcd_bicgstab_solve(ctx, o[0].op, o[1].op, ops.bicgstab_params(1e-10), x1, bp)
    st2, cg = L.lqcd_cg_solve(ctx, o[0].op, o[1].op, ops.cg_params(1e-10), x2, bp)
    assert st1 == st2 == L.LQCD_OK
    assert bi.matvecs < cg.matvecs
    assert rel(np_of(o[0].export_spinor(x1, -1)), np_of(o[0].export_spinor(x2, -1))) < 1e-8


def test_bicgstab_resume_from_initial_guess(ctx):
    """x_full is the initial guess: stopped after 5 steps and resumed, the solve
    still ends at 1e-10."""
    dims, kappa, csw = (8, 8, 8, 8), 0.124, 1.0
    U, b, o = wilson_system(ctx, dims, kappa, csw, 0.25, 1401, 1402, [0, 1])
    bp = o[0].import_spinor(b, -1)
    x = o[0].spinor(full=True)
    st, i1 = L.lqcd_bicgstab_solve(ctx, o[0].op, o[1].op, ops.bicgstab_params(1e-10, 5), x, bp)
    assert st == L.LQCD_ERR_NOT_CONVERGED
    assert i1.iters == 5 and 1e-10 < i1.true_residual < 1
    st, i2 = L.lqcd_bicgstab_solve(ctx, o[0].op, o[1].op, ops.bicgstab_params(1e-10), x, bp)
    assert st == L.LQCD_OK and i2.true_residual <= 1e-10
    res, _ = oracle_residual(dims, U, kappa, csw, np_of(o[0].export_spinor(x, -1)), b)
    assert res <= 1.05e-10


def test_bicgstab_arguments(ctx):
    dims = (4, 4, 4, 4)
    U, b, o = wilson_system(ctx, dims, 0.12, 1.0, 0.25, 1501, 1502, [0, 1])
    hi = o[0]
    zero = hi.spinor(full=True)
    x = hi.spinor(full=True)
    x.fill_(3)
    st, info = L.lqcd_bicgstab_solve(ctx, hi.op, o[1].op, ops.bicgstab_params(), x, zero)
    assert st == L.LQCD_OK and info.iters == 0
    torch.cuda.synchronize()
    assert bool((x == 0).all())
    nanb = hi.import_spinor(np.full(oracle.shape4(dims) + (4, 3), np.nan + 0j), -1)
    with pytest.raises(L.LqcdError) as ei:
        L.lqcd_bicgstab_solve(ctx, hi.op, None, ops.bicgstab_params(), x, nanb)
    assert ei.value.status == L.LQCD_ERR_INVALID_ARG
    bp = hi.import_spinor(b, -1)
    for prm in (ops.bicgstab_params(0.0), ops.bicgstab_params(1e-10, 0), ops.bicgstab_params(1e-10, 10, 1.0)):
        with pytest.raises(L.LqcdError) as ei:
            L.lqcd_bicgstab_solve(ctx, hi.op, None, prm, x, bp)
        assert ei.value.status == L.LQCD_ERR_INVALID_ARG
    # op_hi must be FP64
    with pytest.raises(L.LqcdError) as ei:
        L.lqcd_bicgstab_solve(ctx, o[1].op, None, ops.bicgstab_params(), x, bp)
    assert ei.value.status == L.LQCD_ERR_UNSUPPORTED
    # a sloppy operator of another system
    other = ops.wilson_clover(ctx, U, dims, 0.121, 1.0, 1, 18)
    with pytest.raises(L.LqcdError) as ei:
        L.lqcd_bicgstab_solve(ctx, hi.op, other.op, ops.bicgstab_params(), x, bp)
    assert ei.value.status == L.LQCD_ERR_INVALID_ARG
