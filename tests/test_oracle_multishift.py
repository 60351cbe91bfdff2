"""Pins of the oracle's multi-shift CG for eq. (4) (CPU only): every shifted
solution against a dense solve of its own system, the one-shift case against
plain CG, and the collinear-residual estimate against the true residual."""
import numpy as np

import oracle
import synth
from oracle import solvers
from util_fields import dense_matrix

DIMS = (2, 2, 4, 4)


def staggered_normal(seed, m=0.05):
    U = synth.gauge_field(DIMS, 0.2, seed)
    fat = synth.fat_links(DIMS, U, seed=seed + 1)
    lng = oracle.long_links(DIMS, U)
    return oracle.Staggered(DIMS, fat, lng, m, bc_t=-1)


def even_source(op, seed):
    chi = synth.gaussian_spinor(DIMS, seed, inner=(3,))
    return np.where(op.even[..., None], chi, 0)


def test_multishift_matches_dense_solves():
    op = staggered_normal(101)
    b = even_source(op, 103)
    shifts = [0.0, 0.01, 0.1, 1.0]
    xs, it, res = solvers.multishift_cg(op.normal_even, b, shifts, tol=1e-13, maxiter=2000)
    shape = oracle.shape4(DIMS) + (3,)
    N, idx = dense_matrix(op.normal_even, shape, mask=op.even)
    bv = b.reshape(-1)[idx]
    for s_, x in zip(shifts, xs):
        ref = np.linalg.solve(N + s_ * np.eye(N.shape[0]), bv)
        got = x.reshape(-1)[idx]
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-10, s_
        # nothing is written on odd sites
        assert np.abs(np.where(op.even[..., None], 0, x)).max() == 0
    # the smallest shift is the slowest: the iteration count is that of plain CG on it
    _, it_cg, _ = solvers.cg(op.normal_even, b, tol=1e-13, maxiter=2000)
    assert abs(it - it_cg) <= 1


def test_multishift_one_shift_is_cg():
    """With the single shift 0 the recurrences reduce to CG: z = 1, a^s = a, b^s = b."""
    op = staggered_normal(111)
    b = even_source(op, 113)
    xs, it, _ = solvers.multishift_cg(op.normal_even, b, [0.0], tol=1e-11)
    x_cg, it_cg, _ = solvers.cg(op.normal_even, b, tol=1e-11)
    assert it == it_cg
    assert np.abs(xs[0] - x_cg).max() <= 1e-13 * np.abs(x_cg).max()


def test_multishift_residual_estimates_and_base_shift():
    """A base operator with its own shift (A = N_e + 0.02) and relative shifts:
    each reported |z_i| ||r|| / ||b|| is the true residual of its system, and
    every system meets the tolerance."""
    op = staggered_normal(121, m=0.03)
    b = even_source(op, 123)
    base = 0.02

    def A(v):
        return op.normal_even(v) + base * np.where(op.even[..., None], v, 0)

    shifts = [0.0, 0.05, 0.5]
    tol = 1e-9
    xs, it, res = solvers.multishift_cg(A, b, shifts, tol=tol)
    bn = np.linalg.norm(b)
    for s_, x, r_est in zip(shifts, xs, res):
        true = np.linalg.norm(b - A(x) - s_ * x) / bn
        assert true <= 1.01 * tol
        assert abs(true - r_est) <= 1e-6 * max(true, r_est) + 1e-14
