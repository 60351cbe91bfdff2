"""Multiplicative Schwarz (two block colours) against the oracle: the
preconditioner output for every precision and one or two cycles, its argument
checks, and GCR with it as K (mixed precision and all-FP64, the latter step
for step against the oracle's Algorithm 1 with the oracle's SAP)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import check, ctx, np_of, on_parity, rel  # noqa: F401
from oracle import solvers

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1109_2935_amd.lqcd")
from paper_1109_2935_amd import ops  # noqa: E402

_F = {}


def fields(dims, seed=21):
    if (dims, seed) not in _F:
        U = synth.gauge_field(dims, 0.25, seed)
        _F[(dims, seed)] = (U, synth.gaussian_spinor(dims, seed + 1), torch.from_numpy(U).cuda())
    return _F[(dims, seed)]


def make_op(ctx, dims, prec, tile, kappa=0.124):
    U, _, Ud = fields(dims)
    return ops.wilson_clover(ctx, U, dims, kappa, 1.0, prec, 18 if prec in (0, 1) else 12, tile=tile, U_device=Ud)


@pytest.mark.parametrize("dims,block", [((8, 8, 8, 8), (4, 4, 4, 4)), ((4, 4, 8, 8), (2, 2, 2, 2)),
                                        ((16, 8, 8, 8), (8, 8, 8, 8)), ((8, 4, 4, 12), (4, 4, 4, 4))])
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("cycles", [1, 2])
def test_sap_parity(ctx, dims, block, prec, cycles):
    """K r = the oracle's multiplicative Schwarz with 6 MR steps per visit
    (FP64: 1e-12). (8,4,4,12) in 4^4 blocks has an odd number of blocks along t."""
    U, psi, _ = fields(dims)
    o = make_op(ctx, dims, prec, block)
    ref_op = oracle.WilsonClover(dims, U, 0.124, 1.0, bc_t=-1)
    src = on_parity(psi, ref_op.even)
    ref = solvers.sap(ref_op, src, block, 6, cycles)
    out = o.spinor()
    out.fill_(7)  # overwritten, not accumulated
    L.lqcd_schwarz_precond(ctx, o.op, ops.schwarz_params(block, 6, cycles), out, o.import_spinor(src, 0))
    # the additive K's model (tests/test_gpu_wilson.py, SCHWARZ_TOL) with the
    # roundings of 6 MR steps per visit, `cycles` visits per block and the
    # residual recomputed between visits: at most 2 x 28 + 8 roundings per block
    # instead of 32, sqrt(64 / 32) = 1.4 times the additive bound
    tol = {0: 1e-12, 1: 1e-5, 2: 7e-3, 3: 5.6e-2}[prec]
    check(np_of(o.export_spinor(out, 0)), ref, tol)


def test_sap_differs_from_additive_and_keeps_input(ctx):
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U, psi, _ = fields(dims)
    o = make_op(ctx, dims, 0, block)
    ref_op = oracle.WilsonClover(dims, U, 0.124, 1.0, bc_t=-1)
    src = on_parity(psi, ref_op.even)
    inp = o.import_spinor(src, 0)
    before = inp.clone()
    a, m = o.spinor(), o.spinor()
    L.lqcd_schwarz_precond(ctx, o.op, ops.schwarz_params(block, 6, 0), a, inp)
    L.lqcd_schwarz_precond(ctx, o.op, ops.schwarz_params(block, 6, 1), m, inp)
    torch.cuda.synchronize()
    assert torch.equal(inp, before)
    xa, xm = np_of(o.export_spinor(a, 0)), np_of(o.export_spinor(m, 0))
    assert rel(xa, solvers.schwarz(ref_op, src, block, 6)) < 1e-12
    assert rel(xm, xa) > 1e-3
    # SAP leaves a smaller residual than block Jacobi with the same MR steps
    ra = np.linalg.norm(src - ref_op.schur(xa))
    rm = np.linalg.norm(src - ref_op.schur(xm))
    assert rm < ra


def test_sap_arguments(ctx):
    dims = (8, 8, 8, 8)
    o = make_op(ctx, dims, 1, (8, 4, 4, 4))  # one block along x
    inp, out = o.spinor(), o.spinor()
    with pytest.raises(L.LqcdError) as ei:
        L.lqcd_schwarz_precond(ctx, o.op, ops.schwarz_params((8, 4, 4, 4), 4, 1), out, inp)
    assert ei.value.status == L.LQCD_ERR_UNSUPPORTED
    # the additive form still runs on that tiling
    L.lqcd_schwarz_precond(ctx, o.op, ops.schwarz_params((8, 4, 4, 4), 4, 0), out, inp)
    o2 = make_op(ctx, dims, 1, (4, 4, 4, 4))
    for bad in (-1, 65):
        with pytest.raises(L.LqcdError) as ei:
            L.lqcd_schwarz_precond(ctx, o2.op, ops.schwarz_params((4, 4, 4, 4), 4, bad), out, inp)
        assert ei.value.status == L.LQCD_ERR_INVALID_ARG


def test_gcr_with_sap_fp64_follows_oracle(ctx):
    """All-FP64 GCR with SAP (4 MR steps, one cycle) as K: the oracle's
    solution and step count (oracle Algorithm 1 with the oracle's SAP)."""
    dims, kappa, block = (8, 8, 8, 8), 0.124, (4, 4, 4, 4)
    U, _, Ud = fields(dims)
    b = synth.gaussian_spinor(dims, 2202)
    hi = ops.wilson_clover(ctx, U, dims, kappa, 1.0, 0, 18, tile=block, U_device=Ud)
    x = hi.spinor(full=True)
    prm = ops.gcr_params(1e-10, k_max=8, delta=1e-2, precond=L.LQCD_PRECOND_SCHWARZ, block=block, mr_steps=4, cycles=1)
    st, info = L.lqcd_gcr_solve(ctx, hi.op, hi.op, hi.op, prm, x, hi.import_spinor(b, -1))
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    op = oracle.WilsonClover(dims, U, kappa, 1.0, bc_t=-1)
    xs = np_of(hi.export_spinor(x, -1))
    assert np.linalg.norm(b - op.M(xs)) / np.linalg.norm(b) <= 1.05e-10
    bhat = op.schur_source(b)
    xe, steps, _, _ = solvers.gcr(op.schur, lambda r: solvers.sap(op, r, block, 4, 1), bhat, tol=1e-10, kmax=8,
                                  delta=1e-2)
    assert rel(xs, op.reconstruct(xe, b)) < 1e-8
    assert abs(info.iters - steps) <= max(2, 0.05 * steps)


@pytest.mark.parametrize("kprec", [2, 3])
def test_gcr_dd_sap_mixed_precision(ctx, kprec):
    """FP64 restarts, FP32 Krylov, FP16/BF16 SAP K: FP64 residual 1e-10, and
    fewer outer steps than the additive K with the same MR steps per block."""
    dims, kappa, block = (16, 8, 8, 16), 0.124, (8, 8, 8, 8)
    U = synth.gauge_field(dims, 0.25, 301)
    b = synth.gaussian_spinor(dims, 302)
    Ud = torch.from_numpy(U).cuda()
    o = {p: ops.wilson_clover(ctx, U, dims, kappa, 1.0, p, 18 if p in (0, 1) else 12, tile=block, U_device=Ud)
         for p in (0, 1, kprec)}
    bp = o[0].import_spinor(b, -1)
    res = {}
    for cyc in (0, 1):
        x = o[0].spinor(full=True)
        prm = ops.gcr_params(1e-10, k_max=16, delta=1e-3, precond=L.LQCD_PRECOND_SCHWARZ, block=block, mr_steps=4,
                             cycles=cyc)
        st, info = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, o[kprec].op, prm, x, bp)
        assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
        assert info.true_residual <= 1e-10
        op = oracle.WilsonClover(dims, U, kappa, 1.0, bc_t=-1)
        xs = np_of(o[0].export_spinor(x, -1))
        assert np.linalg.norm(b - op.M(xs)) / np.linalg.norm(b) <= 1.05e-10
        res[cyc] = info.iters
    assert res[1] < res[0], res
