"""Pins of the oracle's parallel-transport convolution network (CPU only)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import ptc
from util_fields import gauge_transform_links

DIMS = (4, 4, 2, 4)


def test_transport_is_a_shift_in_the_free_field():
    """U = 1: forward path along mu is psi(x + mu), i.e. np.roll by -1 on that axis."""
    dims = (4, 6, 2, 8)
    psi = synth.gaussian_spinor(dims, 1)[None]
    for mu in range(4):
        axis = 1 + (3 - mu)
        fwd = oracle.transport(dims, synth.unit_gauge(dims), psi, 1 + 2 * mu, bc_t=1)
        assert np.abs(fwd - np.roll(psi, -1, axis=axis)).max() == 0
        bwd = oracle.transport(dims, synth.unit_gauge(dims), psi, 2 + 2 * mu, bc_t=1)
        assert np.abs(bwd - np.roll(psi, 1, axis=axis)).max() == 0


def test_transport_adjoint():
    U = synth.gauge_field(DIMS, 0.25, 2)
    a = synth.gaussian_spinor(DIMS, 3)[None]
    b = synth.gaussian_spinor(DIMS, 4)[None]
    for p in range(ptc.NPATH):
        lhs = np.vdot(oracle.transport(DIMS, U, a, p), b)
        rhs = np.vdot(a, oracle.transport(DIMS, U, b, p, adjoint=True))
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_identity_path_weights_multiply():
    """W[o,i,p] = a_oi delta_p0 * 1: the network multiplies the input by prod of the a's."""
    U = synth.gauge_field(DIMS, 0.25, 5)
    r = synth.gaussian_spinor(DIMS, 6)
    even = oracle.parity_mask(DIMS, 0)
    Ws = []
    rng = np.random.default_rng(7)
    for cin, cout in zip(ptc.CHANNELS[:-1], ptc.CHANNELS[1:]):
        a = rng.normal(size=(cout, cin)) + 1j * rng.normal(size=(cout, cin))
        W = np.zeros((cout, cin, ptc.NPATH, 4, 4), dtype=np.complex128)
        W[:, :, 0] = a[:, :, None, None] * np.eye(4)
        Ws.append(W)
    chain = np.linalg.multi_dot([W[:, :, 0, 0, 0] for W in Ws[::-1]])[0, 0]
    y, _ = ptc.forward(DIMS, U, r, Ws, even)
    assert np.abs(y - chain * np.where(even[..., None, None], r, 0)).max() < 1e-12 * abs(chain) * np.abs(r).max()


def test_gauge_equivariance():
    U = synth.gauge_field(DIMS, 0.25, 8)
    r = synth.gaussian_spinor(DIMS, 9)
    even = oracle.parity_mask(DIMS, 0)
    Ws = ptc.init_weights(10)
    g = synth.su3_site_field(DIMS, 11)
    y, _ = ptc.forward(DIMS, U, r, Ws, even)
    yg, _ = ptc.forward(DIMS, gauge_transform_links(U, g), np.einsum("...ab,...sb->...sa", g, r), Ws, even)
    assert np.abs(yg - np.einsum("...ab,...sb->...sa", g, y)).max() < 1e-12 * np.abs(y).max()


def test_gradients_match_finite_differences():
    U = synth.gauge_field(DIMS, 0.25, 12)
    r = synth.gaussian_spinor(DIMS, 13)
    e = synth.gaussian_spinor(DIMS, 14)
    even = oracle.parity_mask(DIMS, 0)
    Ws = ptc.init_weights(15, channels=(1, 3, 2, 1))
    L0, grads = ptc.loss_and_grads(DIMS, U, r, e, Ws, even)
    rng = np.random.default_rng(16)
    h = 1e-6
    for k in range(len(Ws)):
        for _ in range(3):
            d = rng.normal(size=Ws[k].shape) + 1j * rng.normal(size=Ws[k].shape)
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[k] += h * d
            Wm[k] -= h * d
            fd = (ptc.loss_and_grads(DIMS, U, r, e, Wp, even)[0] - ptc.loss_and_grads(DIMS, U, r, e, Wm, even)[0]) / (2 * h)
            an = 2 * np.vdot(grads[k], d).real
            assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-3), (k, fd, an)


def _fd_check(f, grads, Ws, seed, h=1e-6, rtol=1e-7):
    """Central differences of the real function f(Ws) along random complex
    directions d against 2 Re <G, d> (G = df/d conj W)."""
    rng = np.random.default_rng(seed)
    for k in range(len(Ws)):
        for _ in range(2):
            d = rng.normal(size=Ws[k].shape) + 1j * rng.normal(size=Ws[k].shape)
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[k] += h * d
            Wm[k] -= h * d
            fd = (f(Wp) - f(Wm)) / (2 * h)
            an = 2 * np.vdot(grads[k], d).real
            assert abs(fd - an) <= rtol * max(abs(an), 1e-3), (k, fd, an)


def test_residual_loss_gradients_match_finite_differences():
    """The residual loss goes through the Schur operator and its adjoint; a
    wrong adjoint (Mhat instead of Mhat^+) or a dropped 1/|r|^2 fails here."""
    U = synth.gauge_field(DIMS, 0.25, 22)
    r = synth.gaussian_spinor(DIMS, 23)
    even = oracle.parity_mask(DIMS, 0)
    M = oracle.WilsonClover(DIMS, U, 0.124, 1.0)
    Ws = ptc.init_weights(25, channels=(1, 2, 1))
    L0, grads = ptc.residual_loss_and_grads(DIMS, U, r, Ws, even, M.schur)
    re = np.where(even[..., None, None], r, 0)
    # zero weights: N = 0, so L = |r|^2 / |r|^2 = 1
    Lz, _ = ptc.residual_loss_and_grads(DIMS, U, r, [0 * w for w in Ws], even, M.schur)
    assert abs(Lz - 1) < 1e-14
    # one layer, identity path only, W = c 1: N(r) = c r, L = |c Mhat r - r|^2 / |r|^2,
    # smallest at c = <Mhat r, r> / |Mhat r|^2 with L = 1 - |<Mhat r, r>|^2 / (|Mhat r|^2 |r|^2)
    Mr = np.where(even[..., None, None], M.schur(re), 0)
    c = np.vdot(Mr, re) / np.vdot(Mr, Mr).real
    W1 = np.zeros((1, 1, 9, 4, 4), dtype=complex)
    W1[0, 0, 0] = c * np.eye(4)
    L1, g1 = ptc.residual_loss_and_grads(DIMS, U, r, [W1], even, M.schur)
    rn2 = np.vdot(re, re).real
    assert abs(L1 - (1 - abs(np.vdot(Mr, re)) ** 2 / (np.vdot(Mr, Mr).real * rn2))) < 1e-12
    # at the minimum over c the derivative along W = 1 (identity path) vanishes
    assert abs(np.trace(g1[0][0, 0, 0])) < 1e-12
    _fd_check(lambda W: ptc.residual_loss_and_grads(DIMS, U, r, W, even, M.schur)[0], grads, Ws, 26)


def test_vjp_matches_finite_differences():
    U = synth.gauge_field(DIMS, 0.25, 32)
    r = synth.gaussian_spinor(DIMS, 33)
    dy = synth.gaussian_spinor(DIMS, 34)
    even = oracle.parity_mask(DIMS, 0)
    Ws = ptc.init_weights(35, channels=(1, 3, 1))
    grads = ptc.vjp(DIMS, U, r, dy, Ws, even)
    dye = np.where(even[..., None, None], dy, 0)
    # phi(W) = 2 Re <dy, N_W(r)> has cotangent dy at the output
    _fd_check(lambda W: 2 * np.vdot(dye, ptc.forward(DIMS, U, r, W, even)[0]).real, grads, Ws, 36)
