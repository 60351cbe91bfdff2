"""The C ABI library builds, loads and exports every symbol of include/lqcd.h (CPU only)."""
import os
import re

from paper_1109_2935_amd import lqcd as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lqcd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lqcd_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = L.lib()
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(L.EXPORTED)


def test_struct_layouts_match_header():
    import ctypes
    # 4 + 16 + 16 + 4*3 ints, padding to 8, 4 doubles, 4 pointers
    assert ctypes.sizeof(L.lqcd_operator) == 48 + 32 + 32
    assert ctypes.sizeof(L.lqcd_solve_info) == 40
    assert ctypes.sizeof(L.lqcd_schwarz_params) == 24
    assert ctypes.sizeof(L.lqcd_gcr_params) == 8 + 4 + 4 + 8 + 4 + 4 + 24 + 8
    assert ctypes.sizeof(L.lqcd_ptc_net) == 40 + 8
    assert ctypes.sizeof(L.lqcd_cg_params) == 8 + 4 + 4 + 8 + 4 + 4 + 3 * 8 + 4 + 4 + 8
    assert ctypes.sizeof(L.lqcd_bicgstab_params) == 8 + 8 + 8
    # int + padding, 16 doubles, 2 doubles, int + padding, double
    assert ctypes.sizeof(L.lqcd_multishift_params) == 8 + 16 * 8 + 2 * 8 + 8 + 8
    # 2 ints, double, 16 solve infos, double
    assert ctypes.sizeof(L.lqcd_multishift_info) == 8 + 8 + 16 * 40 + 8


def test_validation_without_gpu():
    """Argument checks run before any device work, so they answer on a CPU host."""
    op = L.lqcd_operator()
    op.action = L.LQCD_WILSON_CLOVER
    op.dims[:] = (8, 8, 8, 8)
    op.tile[:] = (8, 8, 8, 8)
    op.bc_t, op.prec, op.recon = -1, L.LQCD_F32, 12
    assert L.lqcd_field_bytes(op, L.LQCD_FIELD_SPINOR) == 2048 * 24 * 4
    assert L.lqcd_field_bytes(op, L.LQCD_FIELD_GAUGE) == 8 * 2048 * 12 * 4
    assert L.lqcd_field_bytes(op, L.LQCD_FIELD_CLOVER) == 2 * 2048 * 72 * 4
    for bad in [dict(dims=(7, 8, 8, 8)), dict(tile=(3, 8, 8, 8)), dict(bc_t=0), dict(recon=10),
                dict(prec=L.LQCD_F16, recon=8)]:
        o = L.lqcd_operator.from_buffer_copy(op)
        for k, v in bad.items():
            if isinstance(v, tuple):
                getattr(o, k)[:] = v
            else:
                setattr(o, k, v)
        try:
            L.lqcd_field_bytes(o, L.LQCD_FIELD_SPINOR)
            raise AssertionError("accepted %r" % bad)
        except L.LqcdError as e:
            assert e.status in (L.LQCD_ERR_INVALID_ARG, L.LQCD_ERR_UNSUPPORTED)
            assert L.lqcd_last_error()
