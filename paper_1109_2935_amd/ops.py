"""Operator instances on the GPU: packed links, clover and spinor buffers.

Convenience layer over the C ABI for Python callers: it allocates the packed
fields as torch uint8 device tensors, imports natural FP64 links (device or
host arrays) and builds the derived fields (clover and its inverse, long
links) with the library's own kernels. All arithmetic stays in liblqcd.so.
"""
import ctypes
import numpy as np
import torch

from . import lqcd as L


def _device_complex(a, device="cuda"):
    """Natural complex128 field as a contiguous device tensor."""
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.complex128).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(device)


class Operator:
    """One operator instance (action, geometry, precision, compression)."""

    def __init__(self, ctx, action, dims, prec, recon=18, tile=None, bc_t=-1, kappa=0.0, csw=0.0, mass=0.0,
                 c_long=1.0, device="cuda"):
        self.ctx = ctx
        self.device = device
        self.dims = tuple(int(d) for d in dims)
        tile = self.dims if tile is None else tuple(int(t) for t in tile)
        op = L.lqcd_operator()
        op.action = action
        op.dims[:] = self.dims
        op.tile[:] = tile
        op.bc_t = bc_t
        op.prec = prec
        op.recon = recon
        op.kappa, op.csw, op.mass, op.c_long = kappa, csw, mass, c_long
        self.op = op
        self._keep = {}

    # -- allocation ---------------------------------------------------------
    def bytes(self, kind, nrhs=1):
        return L.lqcd_field_bytes(self.op, kind, nrhs)

    def empty(self, kind, nrhs=1):
        return torch.empty(self.bytes(kind, nrhs), dtype=torch.uint8, device=self.device)

    def spinor(self, full=False, nrhs=1, zero=True):
        kind = L.LQCD_FIELD_SPINOR_FULL if full else L.LQCD_FIELD_SPINOR
        t = self.empty(kind, nrhs)
        if zero:
            t.zero_()
        return t

    def replica(self):
        """The same operator with its own copies of the packed links and clover
        fields (equal values at other addresses)."""
        r = Operator.__new__(Operator)
        r.ctx, r.device, r.dims = self.ctx, self.device, self.dims
        r.op = L.lqcd_operator.from_buffer_copy(self.op)
        r._keep = {}
        for name, field in (("gauge", "gauge"), ("long", "long_links"), ("clover", "clover"),
                            ("clover_inv", "clover_inv")):
            if name in self._keep:
                t = self._keep[name].clone()
                r._keep[name] = t
                setattr(r.op, field, t.data_ptr())
        return r

    @property
    def spinor_bytes(self):
        return self.bytes(L.LQCD_FIELD_SPINOR)

    # -- spinor exchange ----------------------------------------------------
    def import_spinor(self, natural, parity, out=None, nrhs=1):
        """Pack natural field(s); nrhs > 1: natural is [nrhs, t, z, y, x, ...] and the
        right-hand sides are stored one after another (source-major) in the packed field."""
        nat = _device_complex(natural, self.device)
        if out is None:
            out = self.spinor(full=(parity < 0), zero=False, nrhs=nrhs)
        L.lqcd_spinor_import(self.ctx, self.op, out, nat, parity, nrhs)
        return out

    def export_spinor(self, packed, parity, natural=None, nrhs=1):
        """Unpack to a natural complex128 device tensor (zeros on sites not covered)."""
        lx, ly, lz, lt = self.dims
        inner = (4, 3) if self.op.action == L.LQCD_WILSON_CLOVER else (3,)
        lead = (nrhs,) if nrhs > 1 else ()
        if natural is None:
            natural = torch.zeros(lead + (lt, lz, ly, lx) + inner, dtype=torch.complex128, device=self.device)
        L.lqcd_spinor_export(self.ctx, self.op, natural, packed, parity, nrhs)
        return natural


def wilson_clover(ctx, U, dims, kappa, csw, prec, recon=18, tile=None, bc_t=-1, device="cuda", U_device=None):
    """Wilson-clover instance: packs U and builds A, A^-1 from it on the GPU."""
    o = Operator(ctx, L.LQCD_WILSON_CLOVER, dims, prec, recon, tile, bc_t, kappa=kappa, csw=csw, device=device)
    Ud = U_device if U_device is not None else _device_complex(U, device)
    g = o.empty(L.LQCD_FIELD_GAUGE)
    L.lqcd_gauge_import(ctx, o.op, g, Ud, L.LQCD_FIELD_GAUGE)
    c = o.empty(L.LQCD_FIELD_CLOVER)
    ci = o.empty(L.LQCD_FIELD_CLOVER)
    o.op.gauge = g.data_ptr()
    o.op.clover = c.data_ptr()
    o.op.clover_inv = ci.data_ptr()
    L.lqcd_clover_build(ctx, o.op, c, ci, Ud)
    o._keep.update(gauge=g, clover=c, clover_inv=ci)
    return o


def tile_candidates(dims):
    """Layout tiles to try for a lattice: the full x extent with 8, 6, 4 or 2
    sites along y, z and t (each dividing its extent, the same along the
    three), and the hypercubes 8^4 and 4^4 where they divide."""
    out = []
    for e in (8, 6, 4, 2):
        t = (dims[0], e, e, e)
        if all(d % b == 0 for d, b in zip(dims[1:], t[1:])):
            out.append(t)
    for e in (8, 4):
        t = (e, e, e, e)
        if all(d % e == 0 for d in dims) and t not in out:
            out.append(t)
    return out


def tune_tile(ctx, U, dims, kappa, csw, prec, recon, nrhs=1, candidates=None, launches=12, U_device=None):
    """The layout tile under which the hopping term with `nrhs` sources runs
    fastest on this GPU: each candidate operator is built and timed (HIP
    events, after one warm-up launch; the median of `launches` launches).
    Returns (best tile, {tile: microseconds}). The fields of a chosen layout
    are then imported with it; the kernels' own launch parameters are tuned
    separately by the library."""
    cands = [tuple(t) for t in (candidates or tile_candidates(dims))]
    Ud = U_device if U_device is not None else _device_complex(U)
    times = {}
    for t in cands:
        o = wilson_clover(ctx, U, dims, kappa, csw, prec, recon, tile=t, U_device=Ud)
        inp, out = o.spinor(nrhs=nrhs), o.spinor(nrhs=nrhs)
        inp.zero_()
        L.lqcd_dslash(ctx, o.op, out, inp, 0, nrhs=nrhs)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(launches + 1)]
        ev[0].record()
        for k in range(launches):
            L.lqcd_dslash(ctx, o.op, out, inp, 0, nrhs=nrhs)
            ev[k + 1].record()
        ev[-1].synchronize()
        times[t] = float(np.median([ev[k].elapsed_time(ev[k + 1]) * 1e3 for k in range(launches)]))
        del o, inp, out
    best = min(times, key=times.get)
    return best, times


def staggered(ctx, fat, U, dims, mass, prec, recon=18, tile=None, bc_t=-1, c_long=1.0, device="cuda",
              fat_device=None, U_device=None):
    """Improved-staggered instance: packs the fat links and forms the long
    links U_mu(x) U_mu(x+mu) U_mu(x+2mu) from the thin links on the GPU."""
    o = Operator(ctx, L.LQCD_STAGGERED, dims, prec, recon, tile, bc_t, mass=mass, c_long=c_long, device=device)
    Fd = fat_device if fat_device is not None else _device_complex(fat, device)
    Ud = U_device if U_device is not None else _device_complex(U, device)
    g = o.empty(L.LQCD_FIELD_GAUGE)
    L.lqcd_gauge_import(ctx, o.op, g, Fd, L.LQCD_FIELD_GAUGE)
    lg = o.empty(L.LQCD_FIELD_LONG)
    L.lqcd_long_link_build(ctx, o.op, lg, Ud)
    o.op.gauge = g.data_ptr()
    o.op.long_links = lg.data_ptr()
    o._keep.update(gauge=g, long=lg)
    return o


def _history(p, history):
    """Point the params' residual history at a host array of `history` doubles
    (kept alive on the params object; read it back with residual_history)."""
    if history:
        buf = (ctypes.c_double * int(history))()
        p._history_buf = buf
        p.res_history = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
        p.res_history_max = int(history)


def residual_history(p, info):
    """The residual history a solve wrote (a list of info.history_len floats)."""
    buf = getattr(p, "_history_buf", None)
    return [] if buf is None else [buf[i] for i in range(info.history_len)]


def gcr_params(tol=1e-10, k_max=16, delta=1e-3, max_iter=10000, precond=L.LQCD_PRECOND_NONE, block=(8, 8, 8, 8),
               mr_steps=8, cycles=0, omega=1.0, history=0, orth_passes=1):
    p = L.lqcd_gcr_params()
    p.tol, p.k_max, p.delta, p.max_iter, p.precond = tol, k_max, delta, max_iter, precond
    p.orth_passes = orth_passes
    p.schwarz.block[:] = [int(b) for b in block]
    p.schwarz.mr_steps = mr_steps
    p.schwarz.cycles = cycles
    p.schwarz.omega = omega
    p.learned = None
    _history(p, history)
    return p


def cg_params(tol=1e-10, max_iter=10000, delta_reliable=0.1, kind=L.LQCD_CG_CGNE_SCHUR, nrhs=1, history=0):
    p = L.lqcd_cg_params()
    p.tol, p.max_iter, p.delta_reliable, p.kind, p.nrhs = tol, max_iter, delta_reliable, kind, nrhs
    if nrhs > 1:
        buf = (ctypes.c_double * nrhs)()
        p._rhs_buf = buf
        p.rhs_residuals = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
    _history(p, history)
    return p


def rhs_residuals(p):
    """Per-source FP64 true residuals of a multi-source CG solve."""
    buf = getattr(p, "_rhs_buf", None)
    return [] if buf is None else list(buf)


def multishift_params(shifts, tol=1e-10, tol_sloppy=1e-8, max_iter=20000, delta_reliable=0.1):
    p = L.lqcd_multishift_params()
    p.nshift = len(shifts)
    for i, s in enumerate(shifts):
        p.shifts[i] = float(s)
    p.tol, p.tol_sloppy, p.max_iter, p.delta_reliable = tol, tol_sloppy, max_iter, delta_reliable
    return p


def bicgstab_params(tol=1e-10, max_iter=20000, delta_reliable=0.1):
    p = L.lqcd_bicgstab_params()
    p.tol, p.max_iter, p.delta_reliable = tol, max_iter, delta_reliable
    return p


def schwarz_params(block, mr_steps=8, cycles=0, omega=1.0):
    """cycles = 0: additive Schwarz; n >= 1: multiplicative, n sweeps over the two block colours.
    omega: MR over-relaxation (1: plain MR)."""
    p = L.lqcd_schwarz_params()
    p.block[:] = [int(b) for b in block]
    p.mr_steps = mr_steps
    p.cycles = cycles
    p.omega = omega
    return p
