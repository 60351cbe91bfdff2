"""Thin ctypes binding of the C ABI in include/lqcd.h (same names).

Argument marshalling only: every computation runs in the HIP library
liblqcd.so. Pointers may be given as torch tensors (their data_ptr is
passed) or integers; streams as torch.cuda.Stream objects, raw handles or
None (the current torch stream). Every entry point raises LqcdError on a
non-zero status, except the solvers, which return (status, info) so that a
caller can inspect a LQCD_ERR_NOT_CONVERGED result.
"""
import ctypes
import os

import torch  # loaded first so that one HIP runtime serves torch and the library

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblqcd.so")

LQCD_OK = 0
LQCD_ERR_INVALID_ARG = 1
LQCD_ERR_UNSUPPORTED = 2
LQCD_ERR_OUT_OF_MEMORY = 3
LQCD_ERR_DEVICE = 4
LQCD_ERR_NOT_CONVERGED = 5
LQCD_ERR_BREAKDOWN = 6

LQCD_F64, LQCD_F32, LQCD_F16, LQCD_BF16, LQCD_HALF = 0, 1, 2, 3, 4
LQCD_WILSON_CLOVER, LQCD_STAGGERED = 0, 1
LQCD_FIELD_SPINOR, LQCD_FIELD_SPINOR_FULL, LQCD_FIELD_GAUGE, LQCD_FIELD_LONG, LQCD_FIELD_CLOVER = 0, 1, 2, 3, 4
LQCD_PRECOND_NONE, LQCD_PRECOND_SCHWARZ, LQCD_PRECOND_LEARNED = 0, 1, 2
LQCD_CG_CGNE_SCHUR, LQCD_CG_STAG_NORMAL = 0, 1

PREC_BYTES = {LQCD_F64: 8, LQCD_F32: 4, LQCD_F16: 2, LQCD_BF16: 2, LQCD_HALF: 2}


class LqcdError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("lqcd status %d: %s" % (status, message))
        self.status = status


class lqcd_operator(ctypes.Structure):
    _fields_ = [("action", ctypes.c_int32), ("dims", ctypes.c_int32 * 4), ("tile", ctypes.c_int32 * 4),
                ("bc_t", ctypes.c_int32), ("prec", ctypes.c_int32), ("recon", ctypes.c_int32),
                ("kappa", ctypes.c_double), ("csw", ctypes.c_double), ("mass", ctypes.c_double),
                ("c_long", ctypes.c_double), ("gauge", ctypes.c_void_p), ("long_links", ctypes.c_void_p),
                ("clover", ctypes.c_void_p), ("clover_inv", ctypes.c_void_p)]


class lqcd_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("matvecs", ctypes.c_int32),
                ("precond_applies", ctypes.c_int32), ("fallback_applies", ctypes.c_int32),
                ("history_len", ctypes.c_int32), ("true_residual", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class lqcd_schwarz_params(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32 * 4), ("mr_steps", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("omega", ctypes.c_double)]


class lqcd_ptc_shape(ctypes.Structure):
    _fields_ = [("nlayers", ctypes.c_int32), ("channels", ctypes.c_int32 * 9)]


class lqcd_ptc_net(ctypes.Structure):
    _fields_ = [("shape", lqcd_ptc_shape), ("packed", ctypes.c_void_p)]


class lqcd_gcr_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("k_max", ctypes.c_int32), ("delta", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("schwarz", lqcd_schwarz_params), ("learned", ctypes.POINTER(lqcd_ptc_net)),
                ("res_history", ctypes.POINTER(ctypes.c_double)), ("res_history_max", ctypes.c_int32),
                ("orth_passes", ctypes.c_int32)]


class lqcd_dslash_job(ctypes.Structure):
    _fields_ = [("op", ctypes.c_void_p), ("out", ctypes.c_void_p), ("in_", ctypes.c_void_p),
                ("out_parity", ctypes.c_int32), ("nrhs", ctypes.c_int32)]


class lqcd_cg_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("delta_reliable", ctypes.c_double),
                ("kind", ctypes.c_int32), ("record_r", ctypes.c_void_p), ("record_e", ctypes.c_void_p),
                ("record_xstar", ctypes.c_void_p), ("record_every", ctypes.c_int32), ("record_max", ctypes.c_int32),
                ("record_count", ctypes.POINTER(ctypes.c_int32)), ("nrhs", ctypes.c_int32),
                ("rhs_residuals", ctypes.POINTER(ctypes.c_double)), ("res_history", ctypes.POINTER(ctypes.c_double)),
                ("res_history_max", ctypes.c_int32)]


LQCD_MAX_SHIFTS = 16
LQCD_MAX_CG_RHS = 32


class lqcd_multishift_params(ctypes.Structure):
    _fields_ = [("nshift", ctypes.c_int32), ("shifts", ctypes.c_double * LQCD_MAX_SHIFTS), ("tol", ctypes.c_double),
                ("tol_sloppy", ctypes.c_double), ("max_iter", ctypes.c_int32), ("delta_reliable", ctypes.c_double)]


class lqcd_bicgstab_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("delta_reliable", ctypes.c_double)]


class lqcd_multishift_info(ctypes.Structure):
    _fields_ = [("ms_iters", ctypes.c_int32), ("ms_matvecs", ctypes.c_int32), ("ms_seconds", ctypes.c_double),
                ("shift", lqcd_solve_info * LQCD_MAX_SHIFTS), ("seconds", ctypes.c_double)]


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int32
_OPP = ctypes.POINTER(lqcd_operator)
_SIGNATURES = {
    "lqcd_context_create": [ctypes.POINTER(ctypes.c_void_p)],
    "lqcd_context_destroy": [_P],
    "lqcd_last_error": [_P],
    "lqcd_field_bytes": [_OPP, _I, _I, ctypes.POINTER(ctypes.c_size_t)],
    "lqcd_stream_copy": [_P, _P, _P, ctypes.c_size_t, _P],
    "lqcd_tuned_choices": [_P, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
    "lqcd_gauge_import": [_P, _OPP, _P, _P, _I, _P],
    "lqcd_long_link_build": [_P, _OPP, _P, _P, _P],
    "lqcd_clover_build": [_P, _OPP, _P, _P, _P, _P],
    "lqcd_spinor_import": [_P, _OPP, _P, _P, _I, _I, _P],
    "lqcd_spinor_export": [_P, _OPP, _P, _P, _I, _I, _P],
    "lqcd_dslash_batch": [_P, ctypes.POINTER(lqcd_dslash_job), _I, _I, _P],
    "lqcd_spinor_convert": [_P, _OPP, _P, _OPP, _P, _I, _I, ctypes.c_double, _P],
    "lqcd_dslash": [_P, _OPP, _P, _P, _I, _I, ctypes.POINTER(ctypes.c_int32), _I, _P],
    "lqcd_clover_apply": [_P, _OPP, _P, _P, _I, _I, _I, _P],
    "lqcd_schur_apply": [_P, _OPP, _P, _P, _I, ctypes.POINTER(ctypes.c_int32), _I, _P],
    "lqcd_schur_apply_noalloc": [_P, _OPP, _P, _P, _I, ctypes.POINTER(ctypes.c_int32), _I, _P],
    "lqcd_schwarz_precond": [_P, _OPP, ctypes.POINTER(lqcd_schwarz_params), _P, _P, _P],
    "lqcd_gcr_solve": [_P, _OPP, _OPP, _OPP, ctypes.POINTER(lqcd_gcr_params), _P, _P,
                       ctypes.POINTER(lqcd_solve_info), _P],
    "lqcd_cg_solve": [_P, _OPP, _OPP, ctypes.POINTER(lqcd_cg_params), _P, _P, ctypes.POINTER(lqcd_solve_info), _P],
    "lqcd_multishift_cg_solve": [_P, _OPP, _OPP, ctypes.POINTER(lqcd_multishift_params), ctypes.POINTER(_P), _P,
                                 ctypes.POINTER(lqcd_multishift_info), _P],
    "lqcd_bicgstab_solve": [_P, _OPP, _OPP, ctypes.POINTER(lqcd_bicgstab_params), _P, _P,
                            ctypes.POINTER(lqcd_solve_info), _P],
    "lqcd_ptc_sizes": [ctypes.POINTER(lqcd_ptc_shape), ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
    "lqcd_ptc_pack": [_P, ctypes.POINTER(lqcd_ptc_shape), _P, _P, _P],
    "lqcd_ptc_apply": [_P, _OPP, ctypes.POINTER(lqcd_ptc_net), _P, _P, _P],
    "lqcd_ptc_gradient": [_P, _OPP, ctypes.POINTER(lqcd_ptc_net), _P, _P, _P, ctypes.POINTER(ctypes.c_double), _P],
    "lqcd_ptc_residual_gradient": [_P, _OPP, ctypes.POINTER(lqcd_ptc_net), _P, _P, ctypes.POINTER(ctypes.c_double), _P],
    "lqcd_ptc_vjp": [_P, _OPP, ctypes.POINTER(lqcd_ptc_net), _P, _P, _P, _P],
    "lqcd_ptc_adam": [_P, ctypes.POINTER(lqcd_ptc_shape), _P, _P, _P, _P, _I, ctypes.c_double, _P],
}
EXPORTED = tuple(_SIGNATURES)


def lib():
    """The loaded library. Fails loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblqcd.so is not built (%s); run python paper_1109_2935_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name == "lqcd_last_error" else ctypes.c_int
        _lib = L
    return _lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return ctypes.c_void_p(x.data_ptr())
    return ctypes.c_void_p(int(x))


def _stream(s):
    if s is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(s, torch.cuda.Stream):
        return ctypes.c_void_p(s.cuda_stream)
    return ctypes.c_void_p(int(s))


def _block(b):
    if b is None:
        return None
    return (ctypes.c_int32 * 4)(*[int(v) for v in b])


def lqcd_last_error(ctx=None):
    return lib().lqcd_last_error(ctx).decode()


def _check(st, ctx):
    if st != LQCD_OK:
        raise LqcdError(st, lqcd_last_error(ctx))


def lqcd_context_create():
    h = ctypes.c_void_p()
    _check(lib().lqcd_context_create(ctypes.byref(h)), None)
    return h


def lqcd_context_destroy(ctx):
    _check(lib().lqcd_context_destroy(ctx), None)


def lqcd_field_bytes(op, kind, nrhs=1):
    n = ctypes.c_size_t()
    _check(lib().lqcd_field_bytes(ctypes.byref(op), kind, nrhs, ctypes.byref(n)), None)
    return n.value


def lqcd_stream_copy(ctx, dst, src, nbytes, stream=None):
    _check(lib().lqcd_stream_copy(ctx, _ptr(dst), _ptr(src), int(nbytes), _stream(stream)), ctx)


def lqcd_tuned_choices(ctx):
    """The autotuner's choices as a dict {key: value}."""
    n = ctypes.c_size_t()
    _check(lib().lqcd_tuned_choices(ctx, None, 0, ctypes.byref(n)), ctx)
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().lqcd_tuned_choices(ctx, buf, n.value, ctypes.byref(n)), ctx)
    out = {}
    for line in buf.value.decode().splitlines():
        k, _, v = line.rpartition("\t")
        out[k] = int(v)
    return out


def lqcd_gauge_import(ctx, op, packed, natural, which=LQCD_FIELD_GAUGE, stream=None):
    _check(lib().lqcd_gauge_import(ctx, ctypes.byref(op), _ptr(packed), _ptr(natural), which, _stream(stream)), ctx)


def lqcd_long_link_build(ctx, op, packed_long, natural_thin, stream=None):
    _check(lib().lqcd_long_link_build(ctx, ctypes.byref(op), _ptr(packed_long), _ptr(natural_thin),
                                      _stream(stream)), ctx)


def lqcd_clover_build(ctx, op, clover, clover_inv, natural_gauge, stream=None):
    _check(lib().lqcd_clover_build(ctx, ctypes.byref(op), _ptr(clover), _ptr(clover_inv), _ptr(natural_gauge),
                                   _stream(stream)), ctx)


def lqcd_spinor_import(ctx, op, packed, natural, parity, nrhs=1, stream=None):
    _check(lib().lqcd_spinor_import(ctx, ctypes.byref(op), _ptr(packed), _ptr(natural), parity, nrhs,
                                    _stream(stream)), ctx)


def lqcd_spinor_export(ctx, op, natural, packed, parity, nrhs=1, stream=None):
    _check(lib().lqcd_spinor_export(ctx, ctypes.byref(op), _ptr(natural), _ptr(packed), parity, nrhs,
                                    _stream(stream)), ctx)


def lqcd_spinor_convert(ctx, op_out, out, op_in, inp, parity, nrhs=1, scale=1.0, stream=None):
    _check(lib().lqcd_spinor_convert(ctx, ctypes.byref(op_out), _ptr(out), ctypes.byref(op_in), _ptr(inp), parity,
                                     nrhs, float(scale), _stream(stream)), ctx)


def lqcd_dslash_batch(ctx, jobs, dagger=0, stream=None):
    """jobs: sequence of (op, out, in, out_parity, nrhs)."""
    arr = (lqcd_dslash_job * len(jobs))()
    keep = []
    for j, (op, out, inp, parity, nrhs) in enumerate(jobs):
        keep.append(op)
        arr[j].op = ctypes.addressof(op)
        arr[j].out = _ptr(out).value
        arr[j].in_ = _ptr(inp).value
        arr[j].out_parity = parity
        arr[j].nrhs = nrhs
    _check(lib().lqcd_dslash_batch(ctx, arr, len(jobs), int(dagger), _stream(stream)), ctx)


def lqcd_dslash(ctx, op, out, inp, out_parity, dagger=0, block=None, nrhs=1, stream=None):
    _check(lib().lqcd_dslash(ctx, ctypes.byref(op), _ptr(out), _ptr(inp), out_parity, int(dagger), _block(block),
                             nrhs, _stream(stream)), ctx)


def lqcd_clover_apply(ctx, op, out, inp, parity, inverse=0, nrhs=1, stream=None):
    _check(lib().lqcd_clover_apply(ctx, ctypes.byref(op), _ptr(out), _ptr(inp), parity, int(inverse), nrhs,
                                   _stream(stream)), ctx)


def lqcd_schur_apply(ctx, op, out, inp, dagger=0, block=None, nrhs=1, stream=None):
    _check(lib().lqcd_schur_apply(ctx, ctypes.byref(op), _ptr(out), _ptr(inp), int(dagger), _block(block), nrhs,
                                  _stream(stream)), ctx)


def lqcd_schur_apply_noalloc(ctx, op, out, inp, dagger=0, block=None, nrhs=1, stream=None):
    _check(lib().lqcd_schur_apply_noalloc(ctx, ctypes.byref(op), _ptr(out), _ptr(inp), int(dagger), _block(block), nrhs,
                                          _stream(stream)), ctx)


def lqcd_schwarz_precond(ctx, op_precond, params, out_even, in_even, stream=None):
    _check(lib().lqcd_schwarz_precond(ctx, ctypes.byref(op_precond), ctypes.byref(params), _ptr(out_even),
                                      _ptr(in_even), _stream(stream)), ctx)


def lqcd_gcr_solve(ctx, op_hi, op_krylov, op_precond, params, x_full, b_full, stream=None):
    info = lqcd_solve_info()
    st = lib().lqcd_gcr_solve(ctx, ctypes.byref(op_hi), ctypes.byref(op_krylov),
                              ctypes.byref(op_precond) if op_precond is not None else None,
                              ctypes.byref(params), _ptr(x_full), _ptr(b_full), ctypes.byref(info), _stream(stream))
    if st not in (LQCD_OK, LQCD_ERR_NOT_CONVERGED):
        _check(st, ctx)
    return st, info


def lqcd_cg_solve(ctx, op_hi, op_sloppy, params, x, b, stream=None):
    info = lqcd_solve_info()
    st = lib().lqcd_cg_solve(ctx, ctypes.byref(op_hi), ctypes.byref(op_sloppy) if op_sloppy is not None else None,
                             ctypes.byref(params), _ptr(x), _ptr(b), ctypes.byref(info), _stream(stream))
    if st not in (LQCD_OK, LQCD_ERR_NOT_CONVERGED):
        _check(st, ctx)
    return st, info


def lqcd_multishift_cg_solve(ctx, op_hi, op_sloppy, params, xs, b, stream=None):
    """xs: sequence of params.nshift packed even fields of op_hi (outputs)."""
    info = lqcd_multishift_info()
    ptrs = (_P * max(1, len(xs)))(*[_ptr(x) for x in xs])
    st = lib().lqcd_multishift_cg_solve(ctx, ctypes.byref(op_hi),
                                        ctypes.byref(op_sloppy) if op_sloppy is not None else None,
                                        ctypes.byref(params), ptrs, _ptr(b), ctypes.byref(info), _stream(stream))
    if st not in (LQCD_OK, LQCD_ERR_NOT_CONVERGED):
        _check(st, ctx)
    return st, info


def lqcd_bicgstab_solve(ctx, op_hi, op_sloppy, params, x_full, b_full, stream=None):
    info = lqcd_solve_info()
    st = lib().lqcd_bicgstab_solve(ctx, ctypes.byref(op_hi),
                                   ctypes.byref(op_sloppy) if op_sloppy is not None else None,
                                   ctypes.byref(params), _ptr(x_full), _ptr(b_full), ctypes.byref(info),
                                   _stream(stream))
    if st not in (LQCD_OK, LQCD_ERR_NOT_CONVERGED):
        _check(st, ctx)
    return st, info


def lqcd_ptc_sizes(shape):
    nw, nb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().lqcd_ptc_sizes(ctypes.byref(shape), ctypes.byref(nw), ctypes.byref(nb)), None)
    return nw.value, nb.value


def lqcd_ptc_pack(ctx, shape, weights, packed, stream=None):
    _check(lib().lqcd_ptc_pack(ctx, ctypes.byref(shape), _ptr(weights), _ptr(packed), _stream(stream)), ctx)


def lqcd_ptc_apply(ctx, op, net, out_even, in_even, stream=None):
    _check(lib().lqcd_ptc_apply(ctx, ctypes.byref(op), ctypes.byref(net), _ptr(out_even), _ptr(in_even),
                                _stream(stream)), ctx)


def lqcd_ptc_gradient(ctx, op, net, r_even, e_even, grad, stream=None):
    loss = ctypes.c_double()
    _check(lib().lqcd_ptc_gradient(ctx, ctypes.byref(op), ctypes.byref(net), _ptr(r_even), _ptr(e_even), _ptr(grad),
                                   ctypes.byref(loss), _stream(stream)), ctx)
    return loss.value


def lqcd_ptc_residual_gradient(ctx, op, net, r_even, grad, stream=None):
    loss = ctypes.c_double()
    _check(lib().lqcd_ptc_residual_gradient(ctx, ctypes.byref(op), ctypes.byref(net), _ptr(r_even), _ptr(grad),
                                            ctypes.byref(loss), _stream(stream)), ctx)
    return loss.value


def lqcd_ptc_vjp(ctx, op, net, r_even, dy_even, grad, stream=None):
    _check(lib().lqcd_ptc_vjp(ctx, ctypes.byref(op), ctypes.byref(net), _ptr(r_even), _ptr(dy_even), _ptr(grad),
                              _stream(stream)), ctx)


def lqcd_ptc_adam(ctx, shape, weights, m, v, grad, step, lr, stream=None):
    _check(lib().lqcd_ptc_adam(ctx, ctypes.byref(shape), _ptr(weights), _ptr(m), _ptr(v), _ptr(grad), int(step),
                               float(lr), _stream(stream)), ctx)

