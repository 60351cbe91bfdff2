"""Pins of the oracle's improved-staggered operator, eq. (3) (CPU only)."""
import numpy as np
import pytest

import oracle
import synth
from util_fields import coords, dense_matrix, gauge_transform_links, momenta, plane_wave


@pytest.mark.parametrize("bc_t", [1, -1])
@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 2, 0, 3)])
def test_staggered_free_field_plane_wave(bc_t, n):
    """Fat = c_F * 1, long = 1: D e^{ipx} chi0 = sum_mu eta_mu(x) 2i (c_F sin p + c_L sin 3p) e^{ipx} chi0."""
    dims = (4, 6, 8, 8)
    w = 0.1
    U = synth.unit_gauge(dims)
    fat = synth.fat_links(dims, U, seed=5, w=w, sigma=0.0)
    cF = 1 + 3 * w
    assert np.abs(fat - cF * U).max() < 1e-15
    lng = oracle.long_links(dims, U)
    p = momenta(dims, n, bc_t)
    chi0 = np.array([1.0 + 2j, -0.5j, 0.25])
    chi = plane_wave(dims, p, chi0)
    out = oracle.stag_dslash(dims, fat, lng, chi, bc_t=bc_t, c_long=0.7)
    x, y, z, t = coords(dims)
    eta = [np.ones_like(x), (-1.0) ** x, (-1.0) ** (x + y), (-1.0) ** (x + y + z)]
    fac = sum(eta[m] * 2j * (cF * np.sin(p[m]) + 0.7 * np.sin(3 * p[m])) for m in range(4))
    assert np.abs(out - fac[..., None] * chi).max() < 1e-12


def test_long_link_of_pure_gauge():
    """U_mu(x) = g(x) g(x+mu)^+  =>  long_mu(x) = g(x) g(x+3mu)^+."""
    dims = (4, 4, 6, 8)
    g = synth.su3_site_field(dims, 71)
    U = gauge_transform_links(synth.unit_gauge(dims), g)
    lng = oracle.long_links(dims, U)
    expect = gauge_transform_links(synth.unit_gauge(dims), g, hop=3)
    assert np.abs(lng - expect).max() < 1e-14


def test_staggered_antihermitian_and_covariant():
    dims = (4, 4, 6, 8)
    U = synth.gauge_field(dims, 0.2, 81)
    fat = synth.fat_links(dims, U, seed=82)
    lng = oracle.long_links(dims, U)
    x = synth.gaussian_spinor(dims, 83, inner=(3,))
    y = synth.gaussian_spinor(dims, 84, inner=(3,))
    Dy = oracle.stag_dslash(dims, fat, lng, y)
    Dx = oracle.stag_dslash(dims, fat, lng, x)
    assert abs(np.vdot(x, Dy) + np.vdot(Dx, y)) < 1e-12 * abs(np.vdot(x, Dy))
    g = synth.su3_site_field(dims, 85)
    fg = gauge_transform_links(fat, g, hop=1)
    lg = gauge_transform_links(lng, g, hop=3)
    xg = np.einsum("...ab,...b->...a", g, x)
    lhs = oracle.stag_dslash(dims, fg, lg, xg)
    rhs = np.einsum("...ab,...b->...a", g, Dx)
    assert np.abs(lhs - rhs).max() < 1e-13


def test_staggered_normal_operator_even_hpd():
    dims = (2, 2, 4, 4)
    U = synth.gauge_field(dims, 0.2, 91)
    fat = synth.fat_links(dims, U, seed=92)
    lng = oracle.long_links(dims, U)
    m = 0.05
    op = oracle.Staggered(dims, fat, lng, m, bc_t=-1)
    shape = oracle.shape4(dims) + (3,)
    N, _ = dense_matrix(op.normal_even, shape, mask=op.even)
    assert np.abs(N - N.conj().T).max() < 1e-13
    ev = np.linalg.eigvalsh(N)
    assert ev.min() >= m * m * (1 - 1e-10)
    # M^+ M restricted to even sites equals N_e (decoupling of the parities)
    Mfull, _ = dense_matrix(op.M, shape)
    MdM = Mfull.conj().T @ Mfull
    ev_idx = np.flatnonzero(op.even.reshape(-1))
    ev_idx = (ev_idx[:, None] * 3 + np.arange(3)).reshape(-1)
    od_idx = np.setdiff1d(np.arange(MdM.shape[0]), ev_idx)
    assert np.abs(MdM[np.ix_(ev_idx, ev_idx)] - N).max() < 1e-12
    assert np.abs(MdM[np.ix_(ev_idx, od_idx)]).max() < 1e-12
