"""GPU solvers against the FP64 oracle: CGNE, GCR (Algorithm 1) with and
without the Schwarz preconditioner, mixed precision, and CG on the staggered
normal operator. Every final residual is recomputed by the oracle on the CPU."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import ctx, np_of, on_parity, rel  # noqa: F401
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


def test_cgne_fp64_8x4(ctx):
    """8^4 Wilson-clover, kappa 0.12, c_sw 1, eps 0.25: FP64 even-odd CGNE to 1e-10."""
    dims, kappa, csw = (8, 8, 8, 8), 0.12, 1.0
    U, b, o = wilson_system(ctx, dims, kappa, csw, 0.25, 1001, 1002, [0])
    hi = o[0]
    bp = hi.import_spinor(b, -1)
    x = hi.spinor(full=True)
    prm = ops.cg_params(1e-10, history=400)
    st, info = L.lqcd_cg_solve(ctx, hi.op, None, prm, x, bp)
    assert st == L.LQCD_OK
    assert info.true_residual <= 1e-10
    hist = ops.residual_history(prm, info)
    assert len(hist) == info.iters
    xs = np_of(hi.export_spinor(x, -1))
    res, op = oracle_residual(dims, U, kappa, csw, xs, b)
    assert res <= 1.05e-10
    # against the oracle's own CGNE solve (same stopping rule, tighter tolerance)
    bhat = op.schur_source(b)
    xe, it, _ = solvers.cgne(op.schur, lambda v: op.schur(v, dagger=True), bhat, tol=1e-12)
    xo = op.reconstruct(xe, b)
    assert rel(xs, xo) < 1e-8
    _, it10, h10 = solvers.cgne(op.schur, lambda v: op.schur(v, dagger=True), bhat, tol=1e-10)
    assert abs(info.iters - it10) <= max(2, 0.02 * it10)
    # the first 10 iterated residuals ||bhat - Mhat x_k|| match the oracle's
    for k in range(10):
        assert abs(hist[k] - h10[k + 1]) <= 1e-10 * h10[k + 1], (k, hist[k], h10[k + 1])


@pytest.mark.parametrize("orth", [1, 2])
@pytest.mark.parametrize("precond", ["none", "schwarz"])
def test_gcr_fp64_matches_oracle(ctx, precond, orth):
    """All-FP64 GCR (FP64 Krylov and K), with one classical Gram-Schmidt pass
    or with CGS2: same solution as the oracle's Algorithm 1 (modified
    Gram-Schmidt), and its first 10 iterated residuals."""
    dims, kappa, csw, block = (8, 8, 8, 8), 0.124, 1.0, (4, 4, 4, 4)
    U, b, o = wilson_system(ctx, dims, kappa, csw, 0.25, 201, 202, [0], tile=block)
    hi = o[0]
    bp = hi.import_spinor(b, -1)
    x = hi.spinor(full=True)
    pk = L.LQCD_PRECOND_SCHWARZ if precond == "schwarz" else L.LQCD_PRECOND_NONE
    prm = ops.gcr_params(1e-10, k_max=8, delta=1e-2, precond=pk, block=block, mr_steps=4, history=200,
                         orth_passes=orth)
    st, info = L.lqcd_gcr_solve(ctx, hi.op, hi.op, hi.op, prm, x, bp)
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    hist = ops.residual_history(prm, info)
    assert len(hist) == info.iters
    xs = np_of(hi.export_spinor(x, -1))
    res, op = oracle_residual(dims, U, kappa, csw, xs, b)
    assert res <= 1.05e-10
    bhat = op.schur_source(b)
    K = (lambda r: solvers.schwarz(op, r, block, 4)) if precond == "schwarz" else None
    rec = {}
    xe, steps, restarts, _ = solvers.gcr(op.schur, K, bhat, tol=1e-10, kmax=8, delta=1e-2, record=rec)
    assert rel(xs, op.reconstruct(xe, b)) < 1e-8
    assert abs(info.iters - steps) <= max(2, 0.05 * steps)  # classical vs modified Gram-Schmidt
    # the first 10 iterated residuals ||rhat_k|| of Algorithm 1 match the oracle's
    for k in range(10):
        ref = rec["rhat"][k]
        assert abs(hist[k] - ref) <= 1e-10 * ref, (k, hist[k], ref)


@pytest.mark.parametrize("kprec,krecon", [(2, 12), (3, 12), (2, 18)])
def test_gcr_dd_mixed_precision(ctx, kprec, krecon):
    """FP64 restarts, FP32 Krylov, FP16/BF16 Schwarz K (12 or 18 link reals):
    FP64 residual 1e-10."""
    dims, kappa, csw, block = (16, 8, 8, 16), 0.124, 1.0, (8, 8, 8, 8)
    U, b, o = wilson_system(ctx, dims, kappa, csw, 0.25, 301, 302, [0, 1], tile=block)
    kop = ops.wilson_clover(ctx, U, dims, kappa, csw, kprec, krecon, tile=block)
    bp = o[0].import_spinor(b, -1)
    x = o[0].spinor(full=True)
    prm = ops.gcr_params(1e-10, k_max=16, delta=1e-3, precond=L.LQCD_PRECOND_SCHWARZ, block=block, mr_steps=8)
    st, info = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, kop.op, prm, x, bp)
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    assert info.true_residual <= 1e-10
    res, _ = oracle_residual(dims, U, kappa, csw, np_of(o[0].export_spinor(x, -1)), b)
    assert res <= 1.05e-10
    # the preconditioner pays: fewer Krylov steps than unpreconditioned GCR
    x2 = o[0].spinor(full=True)
    st2, info2 = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, None, ops.gcr_params(1e-10, 16, 1e-3), x2, bp)
    assert st2 == L.LQCD_OK
    assert info.iters < info2.iters


def test_gcr_restart_every_step_same_solution(ctx):
    dims, kappa, csw, block = (8, 8, 8, 8), 0.124, 1.0, (4, 4, 4, 4)
    U, b, o = wilson_system(ctx, dims, kappa, csw, 0.25, 401, 402, [0, 1], tile=block)
    bp = o[0].import_spinor(b, -1)
    xa, xb = o[0].spinor(full=True), o[0].spinor(full=True)
    st, ia = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, None, ops.gcr_params(1e-10, 16, 1e-3), xa, bp)
    st2, ib = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, None, ops.gcr_params(1e-10, 1, 1e-3), xb, bp)
    assert st == st2 == L.LQCD_OK
    assert ib.restarts == ib.iters
    a, bb = np_of(o[0].export_spinor(xa, -1)), np_of(o[0].export_spinor(xb, -1))
    assert rel(a, bb) < 1e-8


def test_gcr_resume_from_initial_guess(ctx):
    """x is the initial guess: a solve split in two equals an unsplit one."""
    dims, kappa, csw = (8, 8, 8, 8), 0.124, 1.0
    U, b, o = wilson_system(ctx, dims, kappa, csw, 0.25, 501, 502, [0, 1])
    bp = o[0].import_spinor(b, -1)
    x = o[0].spinor(full=True)
    st, i1 = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, None, ops.gcr_params(1e-10, 16, 1e-3, max_iter=5), x, bp)
    assert st == L.LQCD_ERR_NOT_CONVERGED
    assert i1.iters == 5 and i1.true_residual > 1e-10
    st, i2 = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, None, ops.gcr_params(1e-10, 16, 1e-3), x, bp)
    assert st == L.LQCD_OK and i2.true_residual <= 1e-10


def test_solver_zero_and_bad_sources(ctx):
    dims = (4, 4, 4, 4)
    U, b, o = wilson_system(ctx, dims, 0.12, 1.0, 0.25, 601, 602, [0])
    hi = o[0]
    zero = hi.spinor(full=True)
    x = hi.spinor(full=True)
    x.fill_(3)
    st, info = L.lqcd_cg_solve(ctx, hi.op, None, ops.cg_params(), x, zero)
    assert st == L.LQCD_OK
    torch.cuda.synchronize()
    assert bool((x == 0).all())
    nanb = hi.import_spinor(np.full(oracle.shape4(dims) + (4, 3), np.nan + 0j), -1)
    with pytest.raises(L.LqcdError) as ei:
        L.lqcd_cg_solve(ctx, hi.op, None, ops.cg_params(), x, nanb)
    assert ei.value.status == L.LQCD_ERR_INVALID_ARG
    bp = hi.import_spinor(b, -1)
    for bad in (-1, 3):
        with pytest.raises(L.LqcdError) as ei:
            L.lqcd_gcr_solve(ctx, hi.op, hi.op, hi.op, ops.gcr_params(orth_passes=bad), x, bp)
        assert ei.value.status == L.LQCD_ERR_INVALID_ARG


def test_cgne_mixed_precision_reliable_updates(ctx):
    dims, kappa, csw = (8, 8, 8, 8), 0.12, 1.0
    U, b, o = wilson_system(ctx, dims, kappa, csw, 0.25, 1001, 1002, [0, 1])
    bp = o[0].import_spinor(b, -1)
    x = o[0].spinor(full=True)
    st, info = L.lqcd_cg_solve(ctx, o[0].op, o[1].op, ops.cg_params(1e-10, delta_reliable=0.1), x, bp)
    assert st == L.LQCD_OK
    assert info.restarts >= 2
    res, _ = oracle_residual(dims, U, kappa, csw, np_of(o[0].export_spinor(x, -1)), b)
    assert res <= 1.05e-10


def test_gcr_dd_preconditioner_in_its_own_tile(ctx):
    """FP64/FP32 operators tiled for the fastest stencil, the FP16 Schwarz
    operator tiled by its Dirichlet blocks: the solver re-lays out K's input and
    output; same FP64 residual and (up to reduction order) the same steps as
    with one tiling throughout."""
    dims, kappa, csw, block = (8, 8, 8, 8), 0.124, 1.0, (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.25, 301)
    b = synth.gaussian_spinor(dims, 302)
    Ud = torch.from_numpy(U).cuda()
    fast = (8, 4, 4, 4)
    hi = ops.wilson_clover(ctx, U, dims, kappa, csw, 0, 18, tile=fast, U_device=Ud)
    kr = ops.wilson_clover(ctx, U, dims, kappa, csw, 1, 12, tile=fast, U_device=Ud)
    pc = ops.wilson_clover(ctx, U, dims, kappa, csw, 2, 12, tile=block, U_device=Ud)
    same = {p: ops.wilson_clover(ctx, U, dims, kappa, csw, p, 18 if p < 2 else 12, tile=block, U_device=Ud)
            for p in (0, 1)}
    prm = ops.gcr_params(1e-10, 16, 1e-3, precond=L.LQCD_PRECOND_SCHWARZ, block=block, mr_steps=8)
    x = hi.spinor(full=True)
    st, info = L.lqcd_gcr_solve(ctx, hi.op, kr.op, pc.op, prm, x, hi.import_spinor(b, -1))
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    x2 = same[0].spinor(full=True)
    st2, info2 = L.lqcd_gcr_solve(ctx, same[0].op, same[1].op, pc.op, prm, x2, same[0].import_spinor(b, -1))
    assert st2 == L.LQCD_OK
    xs = np_of(hi.export_spinor(x, -1))
    res, _ = oracle_residual(dims, U, kappa, csw, xs, b)
    assert res <= 1.05e-10
    assert abs(info.iters - info2.iters) <= 2


@pytest.mark.parametrize("prec_out", [0, 1, 2])
def test_spinor_convert_between_tiles(ctx, prec_out):
    dims = (8, 8, 4, 8)
    U = synth.gauge_field(dims, 0.25, 311)
    psi = synth.gaussian_spinor(dims, 312)
    a = ops.wilson_clover(ctx, U, dims, 0.124, 1.0, 0, 18, tile=(4, 4, 2, 2))
    bop = ops.wilson_clover(ctx, U, dims, 0.124, 1.0, prec_out, 18 if prec_out < 2 else 12, tile=(8, 2, 4, 4))
    for parity in (-1, 0, 1):
        src = psi if parity < 0 else on_parity(psi, oracle.parity_mask(dims, parity))
        pa = a.import_spinor(src, parity)
        pb = bop.spinor(full=parity < 0)
        L.lqcd_spinor_convert(ctx, bop.op, pb, a.op, pa, parity, scale=2.0)
        got = np_of(bop.export_spinor(pb, parity))
        if prec_out == 0:
            assert np.array_equal(got, 2.0 * src)
        else:
            assert rel(got, 2.0 * src) < {1: 1e-7, 2: 1e-3}[prec_out]
