"""Small test helpers: plane waves, dense assembly, gauge transforms."""
import numpy as np

import synth


def coords(dims):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return x, y, z, t


def momenta(dims, n, bc_t):
    """p_mu = 2 pi n_mu / L_mu, plus pi/L_t for an antiperiodic time direction."""
    p = [2 * np.pi * n[m] / dims[m] for m in range(4)]
    if bc_t == -1:
        p[3] += np.pi / dims[3]
    return p


def plane_wave(dims, p, inner):
    x, y, z, t = coords(dims)
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return ph.reshape(ph.shape + (1,) * inner.ndim) * inner


def gauge_transform_links(U, g, hop=1):
    """U_mu(x) -> g(x) U_mu(x) g(x + hop*mu)^+  (natural layout)."""
    out = np.empty_like(U)
    for mu in range(4):
        axis = 3 - mu
        gs = np.roll(g, -hop, axis=axis)
        out[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(gs, -1, -2))
    return out


def dense_matrix(apply, shape, mask=None):
    """Assemble the matrix of a linear map on fields of `shape` (columns = unit vectors).
    mask (bool over sites) restricts rows and columns to those sites."""
    size = int(np.prod(shape))
    nsite_inner = int(np.prod(shape[4:]))
    if mask is None:
        idx = np.arange(size)
    else:
        sidx = np.flatnonzero(mask.reshape(-1))
        idx = (sidx[:, None] * nsite_inner + np.arange(nsite_inner)[None, :]).reshape(-1)
    cols = []
    for j in idx:
        e = np.zeros(size, dtype=np.complex128)
        e[j] = 1.0
        cols.append(apply(e.reshape(shape)).reshape(-1)[idx])
    return np.array(cols).T, idx


def random_fields(dims, seed, eps=0.25):
    U = synth.gauge_field(dims, eps, seed)
    psi = synth.gaussian_spinor(dims, seed + 1)
    return U, psi
