"""CPU oracle (FP64) for the lattice Dirac operators and solvers.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark. The GPU library never imports, links or
calls anything here, and nothing here calls the GPU library.

The stencil operators are plain C (``lqcd_oracle.c``, OpenMP over sites); the
compositions (clover-improved Wilson matrix, even-odd Schur complement,
staggered normal operator) and the solvers (``solvers.py``) are numpy on top
of them, in the order and notation of the paper (Babich et al., SC11):
eq. (1) Mx = b, eq. (2) Wilson-clover, eq. (3) improved staggered, Section III
(Krylov solvers, even-odd preconditioning, additive Schwarz), Algorithm 1
(GCR-DD). Readings of points the paper leaves open are stated where used.

Fields are natural-layout numpy arrays (see ``synth``); even-odd quantities
are full-lattice arrays that are zero on the sites of the other parity.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "lqcd_oracle.c")
_lib = None


def build(force=False):
    """Compile the C part of the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        P, I, D, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
        L.ora_gamma.argtypes = [I, P]
        L.ora_wilson_dslash.argtypes = [P, I, P, P, P, I, I, P, P, I64]
        L.ora_clover_build.argtypes = [P, P, D, D, P]
        L.ora_clover_apply.argtypes = [P, P, P, P, I]
        L.ora_clover_invert.argtypes = [P, P, P]
        L.ora_clover_invert.restype = I64
        L.ora_long_links.argtypes = [P, P, P]
        L.ora_stag_dslash.argtypes = [P, I, P, P, D, P, P, I, P, I64]
        L.ora_transport.argtypes = [P, I, P, I, I, I64, P, P]
        _lib = L
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _dims(dims):
    return np.array([int(d) for d in dims], dtype=np.int32)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def gamma(mu):
    """gamma_mu of the chiral basis (mu = 0..3 for x,y,z,t; 4 = gamma_5)."""
    g = np.empty((4, 4), dtype=np.complex128)
    lib().ora_gamma(mu, _p(g))
    return g


def shape4(dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx)


def parity_mask(dims, parity):
    lx, ly, lz, lt = (int(d) for d in dims)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    return ((x + y + z + t) % 2) == parity


def block_labels(dims, block):
    """Dirichlet block id of every site (blocks tile from the origin)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    bx, by, bz, bt = (int(b) for b in block)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    nbx, nby, nbz = lx // bx, ly // by, lz // bz
    return (x // bx) + nbx * ((y // by) + nby * ((z // bz) + nbz * (t // bt)))


# --------------------------------------------------------------------------
# Wilson-clover, eq. (2), kappa normalisation M = A - kappa D


def wilson_dslash(dims, U, psi, bc_t=-1, out_parity=-1, dagger=False, block=None, sites=None):
    """D psi (D^+ psi if dagger) from eq. (2); block = Dirichlet cut sizes or None."""
    U, psi = _c(U), _c(psi)
    L = _dims(dims)
    blk = np.array(block, dtype=np.int32) if block is not None else None
    if sites is not None:
        sites = np.ascontiguousarray(sites, dtype=np.int64)
        out = np.empty((len(sites), 4, 3), dtype=np.complex128)
        lib().ora_wilson_dslash(_p(L), int(bc_t), _p(U), _p(psi), _p(out), -1, int(bool(dagger)),
                                _p(blk), _p(sites), len(sites))
        return out
    out = np.empty_like(psi)
    lib().ora_wilson_dslash(_p(L), int(bc_t), _p(U), _p(psi), _p(out), int(out_parity),
                            int(bool(dagger)), _p(blk), None, 0)
    return out


def clover_build(dims, U, kappa, csw):
    """A_x (12x12 per site) = 1 + i kappa c_sw sum_{mu<nu} sigma_munu F_munu(x)."""
    U = _c(U)
    A = np.empty(shape4(dims) + (12, 12), dtype=np.complex128)
    lib().ora_clover_build(_p(_dims(dims)), _p(U), float(kappa), float(csw), _p(A))
    return A


def clover_apply(dims, A, psi, parity=-1):
    A, psi = _c(A), _c(psi)
    out = np.empty_like(psi)
    lib().ora_clover_apply(_p(_dims(dims)), _p(A), _p(psi), _p(out), int(parity))
    return out


def clover_invert(dims, A):
    A = _c(A)
    Ainv = np.empty_like(A)
    bad = lib().ora_clover_invert(_p(_dims(dims)), _p(A), _p(Ainv))
    if bad:
        raise ArithmeticError("singular clover matrix at %d sites" % bad)
    return Ainv


class WilsonClover:
    """M = A - kappa D on the full lattice, and its even-odd Schur complement.

    Asymmetric even-site Schur form (Section III-A: even-odd preconditioning
    solves the Schur complement system; the form is not printed, this reading
    is used):
        Mhat     = A_ee - kappa^2 D_eo A_oo^-1 D_oe
        bhat_e   = b_e + kappa D_eo A_oo^-1 b_o
        x_o      = A_oo^-1 (b_o + kappa D_oe x_e)
    """

    def __init__(self, dims, U, kappa, csw, bc_t=-1):
        self.dims = tuple(int(d) for d in dims)
        self.U = _c(U)
        self.kappa = float(kappa)
        self.csw = float(csw)
        self.bc_t = int(bc_t)
        self.A = clover_build(dims, self.U, kappa, csw)
        self.Ainv = clover_invert(dims, self.A)
        self.even = parity_mask(dims, 0)
        self.odd = ~self.even

    def D(self, psi, out_parity=-1, dagger=False, block=None):
        return wilson_dslash(self.dims, self.U, psi, self.bc_t, out_parity, dagger, block)

    def M(self, psi):
        return clover_apply(self.dims, self.A, psi) - self.kappa * self.D(psi)

    def Mdag(self, psi):
        return clover_apply(self.dims, self.A, psi) - self.kappa * self.D(psi, dagger=True)

    def schur(self, x, dagger=False, block=None):
        """Mhat x on even sites (x is read on even sites only)."""
        xe = np.where(self.even[..., None, None], x, 0)
        t = self.D(xe, out_parity=1, dagger=dagger, block=block)
        t = clover_apply(self.dims, self.Ainv, t, parity=1)
        y = self.D(t, out_parity=0, dagger=dagger, block=block)
        return clover_apply(self.dims, self.A, xe, parity=0) - self.kappa ** 2 * y

    def schur_source(self, b):
        bo = np.where(self.odd[..., None, None], b, 0)
        t = clover_apply(self.dims, self.Ainv, bo, parity=1)
        be = np.where(self.even[..., None, None], b, 0)
        return be + self.kappa * self.D(t, out_parity=0)

    def reconstruct(self, xe, b):
        """Full solution from the even part: x_o = A_oo^-1 (b_o + kappa D_oe x_e)."""
        xe = np.where(self.even[..., None, None], xe, 0)
        bo = np.where(self.odd[..., None, None], b, 0)
        xo = clover_apply(self.dims, self.Ainv, bo + self.kappa * self.D(xe, out_parity=1), parity=1)
        return xe + xo


# --------------------------------------------------------------------------
# improved staggered, eq. (3): M = m - D/2


def long_links(dims, U):
    """Long link U_mu(x) U_mu(x+mu) U_mu(x+2mu) (eq. (3) and the text after it)."""
    U = _c(U)
    out = np.empty_like(U)
    lib().ora_long_links(_p(_dims(dims)), _p(U), _p(out))
    return out


def stag_dslash(dims, fat, lng, chi, bc_t=-1, out_parity=-1, c_long=1.0, sites=None):
    fat, lng, chi = _c(fat), _c(lng), _c(chi)
    L = _dims(dims)
    if sites is not None:
        sites = np.ascontiguousarray(sites, dtype=np.int64)
        out = np.empty((len(sites), 3), dtype=np.complex128)
        lib().ora_stag_dslash(_p(L), int(bc_t), _p(fat), _p(lng), float(c_long), _p(chi), _p(out),
                              -1, _p(sites), len(sites))
        return out
    out = np.empty_like(chi)
    lib().ora_stag_dslash(_p(L), int(bc_t), _p(fat), _p(lng), float(c_long), _p(chi), _p(out),
                          int(out_parity), None, 0)
    return out


class Staggered:
    """M = m - D/2; even-site normal operator N_e = m^2 - (1/4) D_eo D_oe.

    M^+ M = m^2 - D^2/4 because D^+ = -D; D^2 connects only sites of equal
    parity, so the even and odd systems decouple (Section III-A).
    """

    def __init__(self, dims, fat, lng, mass, bc_t=-1, c_long=1.0):
        self.dims = tuple(int(d) for d in dims)
        self.fat, self.lng = _c(fat), _c(lng)
        self.mass = float(mass)
        self.bc_t = int(bc_t)
        self.c_long = float(c_long)
        self.even = parity_mask(dims, 0)

    def D(self, chi, out_parity=-1):
        return stag_dslash(self.dims, self.fat, self.lng, chi, self.bc_t, out_parity, self.c_long)

    def M(self, chi):
        return self.mass * chi - 0.5 * self.D(chi)

    def normal_even(self, x):
        xe = np.where(self.even[..., None], x, 0)
        t = self.D(xe, out_parity=1)
        return self.mass ** 2 * xe - 0.25 * self.D(t, out_parity=0)


def transport(dims, U, psi, path, bc_t=-1, adjoint=False):
    """Parallel transport T_p psi over nfield stacked Wilson fields (leading axis)."""
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    V = int(np.prod(dims))
    nfield = psi.size // (12 * V)
    lib().ora_transport(_p(_dims(dims)), int(bc_t), _p(U), int(path), int(bool(adjoint)), nfield,
                        _p(psi), _p(out))
    return out


# --------------------------------------------------------------------------
# 16-bit fixed-point storage (the "half" format of Section V): integer codes
# q in [-32767, 32767] standing for q / 32767, scaled per site by the site's
# largest magnitude (spinors, clover) or unscaled (link entries, |u| <= 1).
# The format is the library's storage convention; its arithmetic is stated
# here in FP32, the precision the codes are decided in, so that a stored code
# is reproduced exactly: m = fp32(max |v|), w = fp32(v) * fp32(1 / m),
# q = round-half-even(fp32(w * 32767)) clamped to +-32767, and a code reads back
# as fp32(q * fp32(1 / 32767)) * m.

FX_SCALE = np.float32(32767.0)


def fixed16_codes(v, inner_axes):
    """Codes and FP32 norms of a real array v whose last `inner_axes` axes are
    the reals of one site (norms: one per site)."""
    v = np.asarray(v, dtype=np.float64)
    axes = tuple(range(v.ndim - inner_axes, v.ndim))
    m = np.max(np.abs(v), axis=axes, keepdims=True).astype(np.float32)
    with np.errstate(divide="ignore"):
        inv = np.where(m > 0, np.float32(1.0) / np.where(m > 0, m, np.float32(1.0)), np.float32(0.0))
    w = v.astype(np.float32) * inv.astype(np.float32)
    q = np.clip(np.rint(w * FX_SCALE), -FX_SCALE, FX_SCALE).astype(np.int16)
    return q, m


def fixed16_decode(q, m):
    """Values of codes q with per-site FP32 norms m (FP64 result)."""
    unit = q.astype(np.float32) * np.float32(np.float32(1.0) / FX_SCALE)
    return unit.astype(np.float64) * m.astype(np.float64)


def fixed16_site_round(psi):
    """A complex spinor field (natural layout, ..., spin, colour) as it reads
    back from fixed-point storage: every site's 24 reals rounded to codes of
    its own norm."""
    psi = np.asarray(psi, dtype=np.complex128)
    r = np.stack([psi.real, psi.imag], axis=-1)  # ..., 4, 3, 2: the 24 reals of a site
    q, m = fixed16_codes(r, 3)
    out = fixed16_decode(q, m)
    return out[..., 0] + 1j * out[..., 1]
