"""Pins of the oracle's Wilson-clover operators (CPU only).

Each check is against something the oracle does not compute itself: the
Clifford algebra, the free-field plane-wave closed form of eq. (2), the
adjoint relation, gauge covariance, a constant abelian field with a closed-form
clover term, and dense linear algebra (numpy) for the even-odd Schur identity.
"""
import numpy as np
import pytest

import oracle
import synth
from util_fields import coords, dense_matrix, gauge_transform_links, momenta, plane_wave

ASYM = (2, 4, 6, 8)


def test_gamma_clifford_algebra():
    g = [oracle.gamma(m) for m in range(4)]
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T)
        for n in range(4):
            assert np.allclose(g[m] @ g[n] + g[n] @ g[m], 2.0 * (m == n) * np.eye(4), atol=1e-15)
    g5 = oracle.gamma(4)
    assert np.allclose(g5, g[0] @ g[1] @ g[2] @ g[3])
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("bc_t", [1, -1])
@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 1, 2, 3), (0, 3, 1, 5)])
@pytest.mark.parametrize("dagger", [False, True])
def test_wilson_free_field_plane_wave(bc_t, n, dagger):
    """U = 1: D e^{ipx} u = sum_mu (2 cos p_mu -/+ 2 i gamma_mu sin p_mu) e^{ipx} u."""
    dims = ASYM
    p = momenta(dims, n, bc_t)
    u = np.random.default_rng(7).normal(size=(4, 3)) + 1j * np.random.default_rng(8).normal(size=(4, 3))
    psi = plane_wave(dims, p, u)
    out = oracle.wilson_dslash(dims, synth.unit_gauge(dims), psi, bc_t=bc_t, dagger=dagger)
    s = 1.0 if not dagger else -1.0
    K = sum(2 * np.cos(p[m]) * np.eye(4) - s * 2j * np.sin(p[m]) * oracle.gamma(m) for m in range(4))
    expect = plane_wave(dims, p, K @ u)
    assert np.abs(out - expect).max() < 1e-12


@pytest.mark.parametrize("block", [None, (2, 2, 2, 4)])
def test_wilson_adjoint_and_gamma5_hermiticity(block):
    dims = (4, 4, 4, 8)
    U = synth.gauge_field(dims, 0.25, 11)
    x = synth.gaussian_spinor(dims, 12)
    y = synth.gaussian_spinor(dims, 13)
    Dy = oracle.wilson_dslash(dims, U, y, block=block)
    Ddx = oracle.wilson_dslash(dims, U, x, dagger=True, block=block)
    lhs = np.vdot(x, Dy)
    rhs = np.vdot(Ddx, y)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    g5 = oracle.gamma(4)
    g5Dg5 = np.einsum("ab,...bc->...ac", g5,
                      oracle.wilson_dslash(dims, U, np.einsum("ab,...bc->...ac", g5, x), block=block))
    assert np.abs(g5Dg5 - Ddx).max() < 1e-13


def test_wilson_parity_structure():
    """D only connects sites of opposite parity."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.25, 21)
    psi = synth.gaussian_spinor(dims, 22)
    even = oracle.parity_mask(dims, 0)
    pe = np.where(even[..., None, None], psi, 0)
    out = oracle.wilson_dslash(dims, U, pe)
    assert np.abs(out[even]).max() == 0
    assert np.abs(out - oracle.wilson_dslash(dims, U, pe, out_parity=1)).max() == 0


@pytest.mark.parametrize("block", [None, (2, 4, 2, 4)])
def test_wilson_gauge_covariance(block):
    dims = ASYM
    U = synth.gauge_field(dims, 0.25, 31)
    psi = synth.gaussian_spinor(dims, 32)
    g = synth.su3_site_field(dims, 33)
    Ug = gauge_transform_links(U, g)
    psig = np.einsum("...ab,...sb->...sa", g, psi)
    lhs = oracle.wilson_dslash(dims, Ug, psig, bc_t=-1, block=block)
    rhs = np.einsum("...ab,...sb->...sa", g, oracle.wilson_dslash(dims, U, psi, bc_t=-1, block=block))
    assert np.abs(lhs - rhs).max() < 1e-13


def test_block_cut_decouples_blocks():
    """With a Dirichlet cut, a source inside one block gives output inside that
    block only, and away from the block faces the cut operator equals D."""
    dims = (4, 4, 8, 8)
    block = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.25, 41)
    psi = synth.gaussian_spinor(dims, 42)
    lab = oracle.block_labels(dims, block)
    src = np.where((lab == 3)[..., None, None], psi, 0)
    out = oracle.wilson_dslash(dims, U, src, block=block)
    assert np.abs(out[lab != 3]).max() == 0
    full = oracle.wilson_dslash(dims, U, psi)
    cut = oracle.wilson_dslash(dims, U, psi, block=block)
    x, y, z, t = coords(dims)
    interior = (z % 4 != 0) & (z % 4 != 3) & (t % 4 != 0) & (t % 4 != 3)
    assert np.abs(cut[interior] - full[interior]).max() < 1e-14
    assert np.abs(cut[~interior] - full[~interior]).max() > 1e-3


# ---------------------------------------------------------------- clover

def abelian_field(dims, n):
    """U_x = 1, U_y(x) = diag(exp(i theta_c x)), theta_c = 2 pi n_c / L_x with sum n_c = 0."""
    U = synth.unit_gauge(dims)
    x, y, z, t = coords(dims)
    thetas = [2 * np.pi * nc / dims[0] for nc in n]
    for c, th in enumerate(thetas):
        U[..., 1, c, c] = np.exp(1j * th * x)
    return U, thetas


def test_clover_constant_abelian_field_closed_form():
    """Constant abelian F_xy: the four leaves are exp(i theta) each, F_xy = i sin(theta),
    so A = 1 - kappa c_sw sin(theta_c) sigma_xy in colour c, exactly."""
    dims = (8, 4, 4, 4)
    kappa, csw = 0.124, 1.7
    U, thetas = abelian_field(dims, (1, 2, -3))
    A = oracle.clover_build(dims, U, kappa, csw)
    g = [oracle.gamma(m) for m in range(4)]
    sxy = 0.5j * (g[0] @ g[1] - g[1] @ g[0])
    expect = np.eye(12, dtype=np.complex128)
    for c, th in enumerate(thetas):
        for s in range(4):
            for s2 in range(4):
                expect[3 * s + c, 3 * s2 + c] -= kappa * csw * np.sin(th) * sxy[s, s2]
    assert np.abs(A - expect).max() < 1e-14


def test_clover_properties():
    dims = (4, 4, 4, 8)
    kappa, csw = 0.124, 1.0
    U = synth.gauge_field(dims, 0.25, 51)
    A = oracle.clover_build(dims, U, kappa, csw)
    # free field: A = 1
    A0 = oracle.clover_build(dims, synth.unit_gauge(dims), kappa, csw)
    assert np.abs(A0 - np.eye(12)).max() < 1e-15
    # Hermitian
    assert np.abs(A - np.conj(np.swapaxes(A, -1, -2))).max() < 1e-15
    # commutes with gamma5 (block diagonal in chirality: 2 x 36 = 72 reals)
    G5 = np.kron(oracle.gamma(4), np.eye(3))
    assert np.abs(A @ G5 - G5 @ A).max() < 1e-15
    # the correction is traceless in spin
    Ar = (A - np.eye(12)).reshape(A.shape[:-2] + (4, 3, 4, 3))
    assert np.abs(np.einsum("...sasb->...ab", Ar)).max() < 1e-15
    # inverse
    Ainv = oracle.clover_invert(dims, A)
    assert np.abs(A @ Ainv - np.eye(12)).max() < 1e-14
    # gauge covariance A[U^g](x) = g(x) A[U](x) g(x)^+
    g = synth.su3_site_field(dims, 52)
    Ag = oracle.clover_build(dims, gauge_transform_links(U, g), kappa, csw)
    G = np.einsum("st,...ab->...satb", np.eye(4), g).reshape(g.shape[:-2] + (12, 12))
    assert np.abs(Ag - G @ A @ np.conj(np.swapaxes(G, -1, -2))).max() < 1e-14


# ---------------------------------------------------------------- even-odd

def test_wilson_clover_free_field_inverse_closed_form():
    """U = 1, A = 1: M e^{ipx}u = [a + i b.gamma] e^{ipx}u with a = 1 - 2 kappa sum_mu cos p_mu
    and b_mu = 2 kappa sin p_mu (from the plane-wave form of D)."""
    dims = (4, 4, 6, 8)
    kappa = 0.11
    op = oracle.WilsonClover(dims, synth.unit_gauge(dims), kappa, 1.0, bc_t=-1)
    p = momenta(dims, (1, 0, 2, 1), -1)
    u = np.arange(12).reshape(4, 3) + 1j
    psi = plane_wave(dims, p, u)
    a = 1 - 2 * kappa * sum(np.cos(pm) for pm in p)
    bslash = sum(2 * kappa * np.sin(p[m]) * oracle.gamma(m) for m in range(4))
    expect = plane_wave(dims, p, (a * np.eye(4) + 1j * bslash) @ u)
    assert np.abs(op.M(psi) - expect).max() < 1e-13


def test_schur_complement_matches_dense_inverse():
    dims = (2, 2, 4, 4)
    U = synth.gauge_field(dims, 0.25, 61)
    op = oracle.WilsonClover(dims, U, 0.124, 1.0, bc_t=-1)
    shape = oracle.shape4(dims) + (4, 3)
    M, _ = dense_matrix(op.M, shape)
    Mhat, idx_e = dense_matrix(op.schur, shape, mask=op.even)
    Minv = np.linalg.inv(M)
    assert np.abs(Minv[np.ix_(idx_e, idx_e)] - np.linalg.inv(Mhat)).max() < 1e-12
    # dagger: Mhat^+ is the conjugate transpose
    Mhd, _ = dense_matrix(lambda v: op.schur(v, dagger=True), shape, mask=op.even)
    assert np.abs(Mhd - Mhat.conj().T).max() < 1e-14
    # source / reconstruction identity: x = reconstruct(Mhat^-1 bhat) solves M x = b
    b = synth.gaussian_spinor(dims, 62)
    bhat = op.schur_source(b).reshape(-1)[idx_e]
    xe = np.zeros(int(np.prod(shape)), dtype=np.complex128)
    xe[idx_e] = np.linalg.solve(Mhat, bhat)
    x = op.reconstruct(xe.reshape(shape), b)
    assert np.abs(op.M(x) - b).max() < 1e-12
