"""Pins of the oracle's solvers: dense linear algebra, closed forms and the
algebraic identities of MR, additive Schwarz and Algorithm 1 (CPU only)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import solvers
from util_fields import dense_matrix, momenta, plane_wave

DIMS = (2, 2, 4, 4)


@pytest.fixture(scope="module")
def small_op():
    U = synth.gauge_field(DIMS, 0.25, 101)
    op = oracle.WilsonClover(DIMS, U, 0.124, 1.0, bc_t=-1)
    shape = oracle.shape4(DIMS) + (4, 3)
    Mhat, idx = dense_matrix(op.schur, shape, mask=op.even)
    return op, shape, Mhat, idx


def embed(v, idx, shape):
    out = np.zeros(int(np.prod(shape)), dtype=np.complex128)
    out[idx] = v
    return out.reshape(shape)


def test_cgne_matches_dense_solve(small_op):
    op, shape, Mhat, idx = small_op
    b = synth.gaussian_spinor(DIMS, 102)
    bhat = op.schur_source(b)
    x, it, hist = solvers.cgne(op.schur, lambda v: op.schur(v, dagger=True), bhat, tol=1e-12)
    ref = np.linalg.solve(Mhat, bhat.reshape(-1)[idx])
    assert np.abs(x.reshape(-1)[idx] - ref).max() < 1e-10 * np.abs(ref).max()
    assert it <= len(idx)
    assert np.linalg.norm(op.schur(x) - bhat) <= 1.01e-12 * np.linalg.norm(bhat)


def test_full_system_2x2x2x2_dense_lu():
    """The whole chain (Schur source, CGNE, reconstruction) against an LU solve
    of the full 192 x 192 Wilson-clover matrix on a 2^4 lattice, where the
    forward and backward neighbour along every axis is the same site."""
    dims = (2, 2, 2, 2)
    U = synth.gauge_field(dims, 0.25, 111)
    op = oracle.WilsonClover(dims, U, 0.124, 1.0, bc_t=-1)
    shape = oracle.shape4(dims) + (4, 3)
    M, _ = dense_matrix(op.M, shape)
    b = synth.gaussian_spinor(dims, 112)
    ref = np.linalg.solve(M, b.reshape(-1))  # LU with partial pivoting
    bhat = op.schur_source(b)
    xe, _, _ = solvers.cgne(op.schur, lambda v: op.schur(v, dagger=True), bhat, tol=1e-13)
    x = op.reconstruct(xe, b)
    assert np.abs(x.reshape(-1) - ref).max() < 1e-11 * np.abs(ref).max()


def test_cgne_free_field_closed_form_any_size():
    """Full chain (Schur source, CGNE, reconstruction) against the closed-form
    free-field inverse M^-1 = (a - i b.gamma)/(a^2 + b.b)."""
    dims = (8, 8, 8, 8)
    kappa = 0.12
    op = oracle.WilsonClover(dims, synth.unit_gauge(dims), kappa, 1.0, bc_t=-1)
    p = momenta(dims, (1, 2, 0, 3), -1)
    u = np.linspace(0.5, 2.0, 12).reshape(4, 3) * (1 + 0.5j)
    b = plane_wave(dims, p, u)
    a = 1 - 2 * kappa * sum(np.cos(pm) for pm in p)
    bvec = [2 * kappa * np.sin(pm) for pm in p]
    Minv = (a * np.eye(4) - 1j * sum(bvec[m] * oracle.gamma(m) for m in range(4))) / (a * a + sum(x * x for x in bvec))
    bhat = op.schur_source(b)
    xe, it, _ = solvers.cgne(op.schur, lambda v: op.schur(v, dagger=True), bhat, tol=1e-12)
    x = op.reconstruct(xe, b)
    expect = plane_wave(dims, p, Minv @ u)
    assert np.abs(x - expect).max() < 1e-10


def test_cg_matches_dense_on_staggered_normal():
    dims = DIMS
    U = synth.gauge_field(dims, 0.2, 111)
    fat = synth.fat_links(dims, U, seed=112)
    lng = oracle.long_links(dims, U)
    op = oracle.Staggered(dims, fat, lng, 0.05)
    shape = oracle.shape4(dims) + (3,)
    N, idx = dense_matrix(op.normal_even, shape, mask=op.even)
    b = np.where(op.even[..., None], synth.gaussian_spinor(dims, 113, inner=(3,)), 0)
    x, it, hist = solvers.cg(op.normal_even, b, tol=1e-12)
    ref = np.linalg.solve(N, b.reshape(-1)[idx])
    assert np.abs(x.reshape(-1)[idx] - ref).max() < 1e-9 * np.abs(ref).max()
    assert it <= len(idx)


def test_mr_many_steps_is_block_inverse(small_op):
    """MR run to convergence on each Dirichlet block converges to the dense block inverse,
    so K = block Jacobi of the cut matrix (non-overlapping additive Schwarz)."""
    op, shape, _, idx = small_op
    block = (2, 2, 2, 2)
    Mcut, _ = dense_matrix(lambda v: op.schur(v, block=block), shape, mask=op.even)
    # the cut matrix is block diagonal: no entry couples two blocks
    lab = oracle.block_labels(DIMS, block).reshape(-1)
    lab_e = np.repeat(lab[np.flatnonzero(op.even.reshape(-1))], 12)
    assert np.abs(Mcut[lab_e[:, None] != lab_e[None, :]]).max() == 0
    r = np.where(op.even[..., None, None], synth.gaussian_spinor(DIMS, 121), 0)
    K = solvers.schwarz(op, r, block, nsteps=60)
    ref = np.linalg.solve(Mcut, r.reshape(-1)[idx])
    assert np.abs(K.reshape(-1)[idx] - ref).max() < 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("omega", [0.6, 1.0, 1.5])
def test_mr_relaxation_closed_form(omega):
    """On A = lambda * 1 every MR step has <q,r>/<q,q> = 1/lambda, so with
    over-relaxation omega the residual shrinks by (1 - omega) per step and
    x_n = (1 - (1 - omega)^n) b / lambda exactly."""
    b = synth.gaussian_spinor(DIMS, 151)
    lam = 1.3 - 0.4j
    for n in (1, 2, 5):
        x = solvers.mr_blocks(lambda v: lam * v, b, n, omega=omega)
        ref = (1 - (1 - omega) ** n) * b / lam
        assert np.abs(x - ref).max() < 1e-14 * np.abs(ref).max() + 1e-300


def test_mr_over_relaxed_converges_to_block_inverse(small_op):
    """Over-relaxed block MR (omega = 1.3) still converges to the dense inverse
    of each Dirichlet block."""
    op, shape, _, idx = small_op
    block = (2, 2, 2, 2)
    Mcut, _ = dense_matrix(lambda v: op.schur(v, block=block), shape, mask=op.even)
    r = np.where(op.even[..., None, None], synth.gaussian_spinor(DIMS, 122), 0)
    K = solvers.schwarz(op, r, block, nsteps=80, omega=1.3)
    ref = np.linalg.solve(Mcut, r.reshape(-1)[idx])
    assert np.abs(K.reshape(-1)[idx] - ref).max() < 1e-10 * np.abs(ref).max()


def test_schwarz_homogeneous_and_single_block(small_op):
    op, shape, Mhat, idx = small_op
    r = np.where(op.even[..., None, None], synth.gaussian_spinor(DIMS, 131), 0)
    block = (2, 2, 2, 2)
    K1 = solvers.schwarz(op, r, block, 8)
    c = 0.3 - 1.7j
    Kc = solvers.schwarz(op, c * r, block, 8)
    assert np.abs(Kc - c * K1).max() < 1e-13 * np.abs(K1).max()
    # one block covering the lattice: MR on Mhat with global reductions
    Kfull = solvers.schwarz(op, r, DIMS, 8)
    Kmr = solvers.mr_blocks(op.schur, r, 8)
    assert np.abs(Kfull - Kmr).max() < 1e-13 * np.abs(Kmr).max()
    # block-diagonal: each block's output depends only on that block's input
    lab = oracle.block_labels(DIMS, block)
    r0 = np.where((lab == 0)[..., None, None], r, 0)
    K0 = solvers.schwarz(op, r0, block, 8)
    assert np.abs(K0[lab != 0]).max() == 0
    assert np.abs(K0[lab == 0] - K1[lab == 0]).max() < 1e-13


def test_gcr_exact_preconditioner_one_step(small_op):
    op, shape, Mhat, idx = small_op
    Minv = np.linalg.inv(Mhat)
    b = np.where(op.even[..., None, None], synth.gaussian_spinor(DIMS, 141), 0)
    K = lambda v: embed(Minv @ v.reshape(-1)[idx], idx, shape)
    x, steps, restarts, hist = solvers.gcr(op.schur, K, b, tol=1e-10)
    assert steps == 1
    assert hist[-1] <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("kmax,delta", [(4, 1e-3), (16, 1e-2), (1, 0.5)])
def test_gcr_algorithm1_identities(small_op, kmax, delta):
    op, shape, Mhat, idx = small_op
    b = np.where(op.even[..., None, None], synth.gaussian_spinor(DIMS, 151), 0)
    rec = {}
    x, steps, restarts, hist = solvers.gcr(op.schur, None, b, tol=1e-10, kmax=kmax, delta=delta,
                                           record=rec)
    assert hist[-1] <= 1e-10 * np.linalg.norm(b)
    ref = np.linalg.solve(Mhat, b.reshape(-1)[idx])
    assert np.abs(x.reshape(-1)[idx] - ref).max() < 1e-8 * np.abs(ref).max()
    # minimal residual: |rhat| non-increasing within a cycle; z's orthonormal;
    # residual orthogonal to the z's; implicit update M xhat = r0 - rhat_k
    zs = rec["z"]
    G = np.array([[np.vdot(a, c) for c in zs[:min(kmax, 4)]] for a in zs[:min(kmax, 4)]])
    if len(G) and kmax >= 4:
        assert np.abs(G - np.eye(len(G))).max() < 1e-12
    assert np.abs(np.vdot(zs[0], rec["rvec"][0])) < 1e-12 * np.linalg.norm(b)
    for Mx, d in rec["restart_check"]:
        assert np.linalg.norm(Mx - d) < 1e-11 * np.linalg.norm(b)
    rh = rec["rhat"]
    if kmax > 1:
        assert rh[1] <= rh[0] * (1 + 1e-12)


def test_gcr_with_schwarz_converges(small_op):
    op, shape, Mhat, idx = small_op
    b = np.where(op.even[..., None, None], synth.gaussian_spinor(DIMS, 161), 0)
    K = lambda r: solvers.schwarz(op, r, (2, 2, 2, 2), 4)
    x, steps, restarts, hist = solvers.gcr(op.schur, K, b, tol=1e-10, kmax=8, delta=1e-2)
    ref = np.linalg.solve(Mhat, b.reshape(-1)[idx])
    assert np.abs(x.reshape(-1)[idx] - ref).max() < 1e-8 * np.abs(ref).max()
    x1, steps1, _, _ = solvers.gcr(op.schur, None, b, tol=1e-10, kmax=8, delta=1e-2)
    assert steps < steps1


def test_bicgstab_full_system_2x2x2x2_dense_lu():
    """BiCGstab on the even-odd Schur system, then reconstruction, against an
    LU solve of the full Wilson-clover matrix on 2^4."""
    dims = (2, 2, 2, 2)
    U = synth.gauge_field(dims, 0.25, 131)
    op = oracle.WilsonClover(dims, U, 0.124, 1.0, bc_t=-1)
    shape = oracle.shape4(dims) + (4, 3)
    M, _ = dense_matrix(op.M, shape)
    b = synth.gaussian_spinor(dims, 132)
    ref = np.linalg.solve(M, b.reshape(-1))
    xe, it, hist = solvers.bicgstab(op.schur, op.schur_source(b), tol=1e-13)
    x = op.reconstruct(xe, b)
    assert np.abs(x.reshape(-1) - ref).max() < 1e-11 * np.abs(ref).max()
    assert it > 1


def test_bicgstab_nonhermitian_dense_and_recursive_residual():
    """A random well-conditioned non-Hermitian matrix (no structure BiCGstab
    could lean on): the solution against numpy's solve, and the recursively
    updated residual against the true one at the end."""
    rng = np.random.default_rng(141)
    n = 60
    A = np.eye(n) * 4 + (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) / np.sqrt(n)
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    x, it, hist = solvers.bicgstab(lambda v: A @ v, b, tol=1e-12)
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-10
    true = np.linalg.norm(b - A @ x)
    assert abs(true - hist[-1]) <= 1e-9 * np.linalg.norm(b)


def _dense_sap(M, even, labels, colour, r, ncycles):
    """Multiplicative Schwarz with exact block solves, from the dense full
    matrix M alone: the even-odd Schur complement of M, and of M restricted
    to each block's sites (Dirichlet blocks), inverted densely."""
    dof = lambda sites: (sites[:, None] * 12 + np.arange(12)[None, :]).reshape(-1)
    E, O = dof(np.flatnonzero(even)), dof(np.flatnonzero(~even))
    schur = lambda e, o: M[np.ix_(e, e)] - M[np.ix_(e, o)] @ np.linalg.solve(M[np.ix_(o, o)], M[np.ix_(o, e)])
    Mhat = schur(E, O)
    pos = {int(d): i for i, d in enumerate(E)}
    blocks = []
    for b in np.unique(labels):
        sel = labels == b
        eb, ob = dof(np.flatnonzero(sel & even)), dof(np.flatnonzero(sel & ~even))
        blocks.append((int(colour[sel][0]), np.array([pos[int(d)] for d in eb]), schur(eb, ob)))
    rv = r.reshape(-1)[E]
    x = np.zeros_like(rv)
    for _ in range(ncycles):
        for c in (0, 1):
            res = rv - Mhat @ x
            for cb, ix, Mb in blocks:
                if cb == c:
                    x[ix] += np.linalg.solve(Mb, res[ix])
    return x, E, Mhat


def test_sap_exact_blocks_is_dense_block_gauss_seidel(small_op):
    """SAP with MR run to convergence on each block equals block Gauss-Seidel
    over the two colours built from the dense full matrix (Schur complements
    of its block restrictions), for one and two cycles."""
    op, shape, _, idx = small_op
    block = (2, 2, 2, 2)
    M, _ = dense_matrix(op.M, shape)
    even = op.even.reshape(-1)
    labels = oracle.block_labels(DIMS, block).reshape(-1)
    colour = solvers.block_colour(DIMS, block).reshape(-1)
    assert set(colour.tolist()) == {0, 1}
    r = np.where(op.even[..., None, None], synth.gaussian_spinor(DIMS, 171), 0)
    for ncyc in (1, 2):
        x = solvers.sap(op, r, block, nsteps=80, ncycles=ncyc)
        ref, E, Mhat = _dense_sap(M, even, labels, colour, r, ncyc)
        assert np.abs(x.reshape(-1)[E] - ref).max() < 1e-10 * np.abs(ref).max()
        assert np.abs(x[~op.even]).max() == 0
    # multiplicative, not additive: the second colour sees the first one's update
    xa = solvers.schwarz(op, r, block, 80)
    assert np.abs(xa.reshape(-1)[E] - _dense_sap(M, even, labels, colour, r, 1)[0]).max() > 1e-3 * np.abs(ref).max()


def test_sap_converges_to_the_inverse_and_is_homogeneous(small_op):
    """Many cycles converge to Mhat^-1 r (Gauss-Seidel on this system
    converges); K(c r) = c K(r); one block covering the lattice is plain MR."""
    op, shape, Mhat, idx = small_op
    block = (2, 2, 2, 2)
    r = np.where(op.even[..., None, None], synth.gaussian_spinor(DIMS, 181), 0)
    x = solvers.sap(op, r, block, nsteps=40, ncycles=40)
    ref = np.linalg.solve(Mhat, r.reshape(-1)[idx])
    assert np.abs(x.reshape(-1)[idx] - ref).max() < 1e-10 * np.abs(ref).max()
    c = -0.4 + 2.1j
    K1 = solvers.sap(op, r, block, 6, 2)
    assert np.abs(solvers.sap(op, c * r, block, 6, 2) - c * K1).max() < 1e-13 * np.abs(K1).max()
    assert np.abs(solvers.sap(op, r, DIMS, 8, 1) - solvers.mr_blocks(op.schur, r, 8)).max() < 1e-13 * np.abs(K1).max()


def test_sap_beats_additive_in_gcr(small_op):
    """As a GCR preconditioner, one SAP cycle (MR on each colour in turn)
    needs fewer outer steps than the additive form with the same MR steps."""
    op, shape, Mhat, idx = small_op
    b = np.where(op.even[..., None, None], synth.gaussian_spinor(DIMS, 191), 0)
    block = (2, 2, 2, 2)
    xs, steps_s, _, _ = solvers.gcr(op.schur, lambda r: solvers.sap(op, r, block, 4, 1), b, tol=1e-10, kmax=8,
                                    delta=1e-2)
    xa, steps_a, _, _ = solvers.gcr(op.schur, lambda r: solvers.schwarz(op, r, block, 4), b, tol=1e-10, kmax=8,
                                    delta=1e-2)
    ref = np.linalg.solve(Mhat, b.reshape(-1)[idx])
    assert np.abs(xs.reshape(-1)[idx] - ref).max() < 1e-8 * np.abs(ref).max()
    assert steps_s < steps_a
