"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

Input preparation only: random SU(3) links U = exp(i eps H) with H a Gaussian
traceless Hermitian matrix, synthetic fat links for the improved-staggered
workload, Gaussian and point sources, and random SU(3) gauge transformations
for covariance tests. Nothing here applies a Dirac operator, builds a clover
term or a long link, or solves anything.

Layout ("natural"): arrays are indexed [t, z, y, x, ...] so that the flat
site index is x + Lx*(y + Ly*(z + Lz*t)); dims are always given as
(Lx, Ly, Lz, Lt). Gauge fields are [t,z,y,x,mu,3,3] complex128 with
mu = 0..3 for x, y, z, t; Wilson spinors are [t,z,y,x,spin(4),colour(3)];
staggered spinors are [t,z,y,x,colour(3)].

Random numbers come from numpy's PCG64 generator, drawn in natural order.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_synth.so")
_lib = None


def build_helper(force=False):
    """Compile the C helper (gcc, OpenMP)."""
    src = os.path.join(_HERE, "_synth.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               src, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _helper():
    global _lib
    if _lib is None:
        build_helper()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        lib.synth_su3_exp.argtypes = [ctypes.c_int64, P, ctypes.c_double, P]
        lib.synth_fat_links.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64, P,
                                        ctypes.c_double, ctypes.c_double, P]
        _lib = lib
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def volume(dims):
    return int(dims[0]) * int(dims[1]) * int(dims[2]) * int(dims[3])


def shape4(dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx)


def gauge_field(dims, eps, seed):
    """U_mu(x) = exp(i eps H), H = sum_a h_a lambda_a/2, h_a ~ N(0,1) iid.

    Draws 8 normals per link in natural (site, mu) order, one t-slice at a time
    from a single PCG64 stream, so the result does not depend on chunking.
    """
    lib = _helper()
    sh = shape4(dims)
    U = np.empty(sh + (4, 3, 3), dtype=np.complex128)
    rng = np.random.Generator(np.random.PCG64(seed))
    per_slice = sh[1] * sh[2] * sh[3] * 4
    Uf = U.reshape(sh[0], per_slice, 9)
    for t in range(sh[0]):
        h = rng.standard_normal(size=(per_slice, 8))
        out = np.empty((per_slice, 9), dtype=np.complex128)
        lib.synth_su3_exp(per_slice, _ptr(h), float(eps), _ptr(out))
        Uf[t] = out
    return U


def unit_gauge(dims):
    sh = shape4(dims)
    U = np.zeros(sh + (4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def fat_links(dims, U, seed, w=0.1, sigma=0.05):
    """Synthetic general-complex 1-hop link for the improved-staggered workload.

    fat_mu(x) = U_mu(x) + w * sum_{nu != mu} [U_nu(x) U_mu(x+nu) U_nu(x+mu)^+ + sigma G_munu(x)],
    G a complex Gaussian 3x3 (real and imaginary parts N(0,1)), drawn in
    natural (site, mu, nu) order, one t-slice at a time.
    """
    lib = _helper()
    sh = shape4(dims)
    L = np.array([int(d) for d in dims], dtype=np.int32)
    Uc = np.ascontiguousarray(U)
    fat = np.empty_like(Uc)
    rng = np.random.Generator(np.random.PCG64(seed))
    per_slice = sh[1] * sh[2] * sh[3]
    ff = fat.reshape(sh[0], per_slice, 4, 3, 3)
    for t in range(sh[0]):
        g = rng.standard_normal(size=(per_slice, 4, 3, 3, 3, 2))
        G = np.ascontiguousarray(g[..., 0] + 1j * g[..., 1])
        out = np.empty((per_slice, 4, 3, 3), dtype=np.complex128)
        lib.synth_fat_links(_ptr(L), _ptr(Uc), t * per_slice, (t + 1) * per_slice, _ptr(G),
                            float(w), float(sigma), _ptr(out))
        ff[t] = out
    return fat


def gaussian_spinor(dims, seed, inner=(4, 3)):
    """Complex Gaussian field: real and imaginary parts N(0,1) iid per component."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sh = shape4(dims) + tuple(inner)
    g = rng.standard_normal(size=sh + (2,))
    return np.ascontiguousarray(g[..., 0] + 1j * g[..., 1])


def point_source(dims, spin, colour):
    """delta at the origin (an even site) in one spin-colour component."""
    b = np.zeros(shape4(dims) + (4, 3), dtype=np.complex128)
    b[0, 0, 0, 0, spin, colour] = 1.0
    return b


def su3_site_field(dims, seed, eps=1.0):
    """One random SU(3) matrix per site, [t,z,y,x,3,3] (gauge transformations)."""
    lib = _helper()
    sh = shape4(dims)
    n = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal(size=(n, 8))
    out = np.empty((n, 9), dtype=np.complex128)
    lib.synth_su3_exp(n, _ptr(h), float(eps), _ptr(out))
    return out.reshape(sh + (3, 3))


def parity_of_sites(dims):
    """(x+y+z+t) mod 2 on the natural grid (0 = even)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    return (x + y + z + t) % 2
