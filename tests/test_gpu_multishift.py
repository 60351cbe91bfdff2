"""GPU parity of the multi-shift CG for eq. (4) (Section III-A) with the
refinement strategy of Section VIII-B, against the FP64 oracle: every shifted
system's residual recomputed by the oracle, the solutions against the oracle's
multi-shift CG, and the argument checks."""
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

_cache = {}


def fields(dims):
    if dims not in _cache:
        U = synth.gauge_field(dims, 0.2, 6001)
        fat = synth.fat_links(dims, U, seed=6003)
        lng = oracle.long_links(dims, U)
        chi = synth.gaussian_spinor(dims, 6002, inner=(3,))
        _cache[dims] = (U, fat, lng, chi, torch.from_numpy(U).cuda(), torch.from_numpy(fat).cuda())
    return _cache[dims]


def make(ctx, dims, prec, recon, mass):
    U, fat, lng, chi, Ud, Fd = fields(dims)
    return ops.staggered(ctx, fat, U, dims, mass, prec, recon, U_device=Ud, fat_device=Fd)


@pytest.mark.parametrize("sloppy", [1, None], ids=["fp32", "fp64"])
@pytest.mark.parametrize("dims,shifts", [((8, 8, 8, 12), (0.0, 0.01, 0.1, 1.0)),
                                         ((4, 4, 6, 8), (0.5, -0.002, 0.03))],
                         ids=["8x8x8x12", "4x4x6x8"])
def test_multishift_parity(ctx, sloppy, dims, shifts):
    """Every x_i solves its own shifted system to 1e-10 (oracle residual in
    FP64) and agrees with the oracle's multi-shift CG; shifts unsorted and one
    negative (m^2 + sigma > 0)."""
    mass = 0.05
    U, fat, lng, chi, _, _ = fields(dims)
    hi = make(ctx, dims, 0, 18, mass)
    lo = make(ctx, dims, sloppy, 12, mass) if sloppy is not None else None
    ref = oracle.Staggered(dims, fat, lng, mass)
    b = on_parity(chi, ref.even)
    bp = hi.import_spinor(b, 0)
    xs = [hi.spinor() for _ in shifts]
    prm = ops.multishift_params(shifts, tol=1e-10, tol_sloppy=1e-8 if sloppy else 1e-10)
    st, info = L.lqcd_multishift_cg_solve(ctx, hi.op, lo.op if lo else None, prm, xs, bp)
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    assert info.ms_iters > 0 and info.ms_matvecs == info.ms_iters
    xr, _, _ = solvers.multishift_cg(ref.normal_even, b, shifts, tol=1e-12)
    bn = np.linalg.norm(b)
    for i, s in enumerate(shifts):
        x = np_of(hi.export_spinor(xs[i], 0))
        res = np.linalg.norm(b - ref.normal_even(x) - s * np.where(ref.even[..., None], x, 0)) / bn
        assert res <= 1.05e-10, (s, res)
        assert info.shift[i].true_residual <= 1e-10
        assert rel(x, xr[i]) < 1e-7, s
        if sloppy is None:
            # the FP64 multi-shift stage already meets the tolerance: nothing left to refine
            assert info.shift[i].iters <= 5


def test_multishift_single_shift_and_zero_source(ctx):
    dims, mass = (4, 4, 6, 8), 0.05
    U, fat, lng, chi, _, _ = fields(dims)
    hi = make(ctx, dims, 0, 18, mass)
    lo = make(ctx, dims, 1, 18, mass)
    ref = oracle.Staggered(dims, fat, lng, mass)
    b = on_parity(chi, ref.even)
    x = [hi.spinor()]
    st, info = L.lqcd_multishift_cg_solve(ctx, hi.op, lo.op, ops.multishift_params([0.0]), x, hi.import_spinor(b, 0))
    assert st == L.LQCD_OK
    xo = np_of(hi.export_spinor(x[0], 0))
    assert np.linalg.norm(b - ref.normal_even(xo)) / np.linalg.norm(b) <= 1.05e-10
    # zero source: zero solutions, no iterations
    z = [hi.spinor(), hi.spinor()]
    z[0].fill_(7)
    st, info = L.lqcd_multishift_cg_solve(ctx, hi.op, lo.op, ops.multishift_params([0.0, 0.1]), z, hi.spinor())
    assert st == L.LQCD_OK and info.ms_iters == 0
    assert all(int(torch.count_nonzero(t)) == 0 for t in z)


def test_multishift_argument_checks(ctx):
    dims, mass = (4, 4, 6, 8), 0.05
    hi = make(ctx, dims, 0, 18, mass)
    lo16 = make(ctx, dims, 2, 12, mass)
    lo32 = make(ctx, dims, 1, 12, mass)
    b = hi.spinor()
    x = [hi.spinor(), hi.spinor()]
    bad = [
        (hi, lo16, ops.multishift_params([0.0, 0.1]), x, L.LQCD_ERR_UNSUPPORTED),       # 16-bit multi-shift stage
        (hi, lo32, ops.multishift_params([0.0, -mass * mass]), x, L.LQCD_ERR_INVALID_ARG),  # m^2 + sigma = 0
        (hi, lo32, ops.multishift_params([0.0, 0.1]), [x[0], x[0]], L.LQCD_ERR_INVALID_ARG),  # aliased solutions
        (lo32, None, ops.multishift_params([0.0]), x[:1], L.LQCD_ERR_UNSUPPORTED),     # op_hi not FP64
    ]
    for op_hi, op_lo, prm, xs, want in bad:
        with pytest.raises(L.LqcdError) as e:
            L.lqcd_multishift_cg_solve(ctx, op_hi.op, op_lo.op if op_lo else None, prm, xs, b)
        assert e.value.status == want, L.lqcd_last_error(ctx)
    prm = ops.multishift_params([0.0])
    prm.nshift = 17
    with pytest.raises(L.LqcdError):
        L.lqcd_multishift_cg_solve(ctx, hi.op, lo32.op, prm, x, b)
