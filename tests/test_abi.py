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


STRUCTS = ("lqcd_operator", "lqcd_solve_info", "lqcd_schwarz_params", "lqcd_ptc_shape", "lqcd_ptc_net",
           "lqcd_gcr_params", "lqcd_cg_params", "lqcd_multishift_params", "lqcd_multishift_info",
           "lqcd_bicgstab_params", "lqcd_dslash_job")


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes struct of the binding has the size and field offsets the C
    compiler gives the header's struct (a small C program prints them)."""
    import ctypes
    import subprocess
    # the binding names the job's `in` field in_ (a Python keyword)
    cname = {("lqcd_dslash_job", "in_"): "in"}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "lqcd.h"', "int main(void) {"]
    for st in STRUCTS:
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (st, st))
        for f, _ in getattr(L, st)._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (st, f, st, cname.get((st, f), f)))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for st in STRUCTS:
        cls = getattr(L, st)
        assert int(got[st]) == ctypes.sizeof(cls), st
        for f, _ in cls._fields_:
            assert int(got["%s.%s" % (st, f)]) == getattr(cls, f).offset, (st, f)


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
