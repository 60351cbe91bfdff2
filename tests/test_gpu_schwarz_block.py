"""The Schwarz preconditioner's block-resident forms (one workgroup per block,
the block's spinor in LDS; x in memory or in registers; 512 threads, or twice
the threads with half the sites each) against the form of separate launches,
and all against the FP64 oracle.

The two forms take the same operations in the same order (the same roundings to
the storage format and the same order of the FP64 block sums of <q,r> and
<q,q>). With BF16 storage, whose conversions are integer operations, the
outputs are bit-identical, and the test requires that. FP16 conversions are
folded by the compiler into its mixed-precision instructions, differently in
the two kernels, and a few percent of the FP16 outputs differ by rounding
steps: there the forms are compared within a tenth of the bound each meets
against the oracle (the derived bound of the 16-bit preconditioner). The same
comparison holds for 16-bit fixed point (codes and a per-site norm), whose
bound is derived beside its own operator tests."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import check, ctx, np_of, on_parity  # noqa: F401

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1109_2935_amd.lqcd")
from paper_1109_2935_amd import ops  # noqa: E402

# derivations beside the Schwarz parity tests of the Wilson kernels (FP16, BF16)
# and of the fixed-point storage (HALF)
SCHWARZ_TOL = {2: 5e-3, 3: 4e-2, 4: 8e-4}

# (dims, block = tile): blocks cut along every axis (128 sites per parity, one
# site per thread); 8^4 blocks spanning y, z and t of the lattice (2048 sites,
# four per thread); one block covering the whole lattice, so that every hop
# wraps inside it with the antiperiodic sign along t (two per thread); and 512
# sites in a block of unequal extents.
CASES = [((8, 8, 8, 8), (4, 4, 4, 4)), ((16, 8, 8, 8), (8, 8, 8, 8)), ((8, 8, 8, 4), (8, 8, 8, 4)),
         ((8, 8, 8, 16), (8, 4, 4, 8))]


class Fields:
    cache = {}

    @classmethod
    def get(cls, dims, seed=31):
        if dims not in cls.cache:
            U = synth.gauge_field(dims, 0.25, seed)
            psi = synth.gaussian_spinor(dims, seed + 1)
            cls.cache[dims] = (U, psi, torch.from_numpy(U).cuda())
        return cls.cache[dims]


def run_form(ctx, monkeypatch, o, prm, inp, form):
    monkeypatch.setenv("LQCD_SCHWARZ_FORM", str(form))
    out = o.spinor()
    out.fill_(255)  # all-ones 16-bit values (a NaN; for fixed point a NaN norm): every element must be written
    L.lqcd_schwarz_precond(ctx, o.op, prm, out, inp)
    torch.cuda.synchronize()
    return out


# the multiplicative form (cycles > 0) needs an even number of blocks along x
FORM_CASES = [(case, cycles) for case in CASES for cycles in (0, 2) if cycles == 0 or (case[0][0] // case[1][0]) % 2 == 0]


@pytest.mark.parametrize("case,cycles", FORM_CASES,
                         ids=lambda v: "x".join(map(str, v[0])) + "_b" + "x".join(map(str, v[1])) if isinstance(v, tuple)
                         else "c%d" % v)
@pytest.mark.parametrize("prec,recon", [(2, 12), (3, 12), (2, 18), (4, 12), (4, 18)])
def test_block_form_matches_launches(ctx, monkeypatch, case, cycles, prec, recon):
    dims, block = case
    U, psi, Ud = Fields.get(dims)
    o = ops.wilson_clover(ctx, U, dims, 0.124, 1.0, prec, recon, tile=block, bc_t=-1, U_device=Ud)
    ref_op = oracle.WilsonClover(dims, U, 0.124, 1.0, bc_t=-1)
    src = on_parity(psi, ref_op.even)
    inp = o.import_spinor(src, 0)
    keep = inp.clone()
    steps = 8 if cycles == 0 else 4
    prm = ops.schwarz_params(block, steps, cycles)
    outs = [run_form(ctx, monkeypatch, o, prm, inp, f) for f in (0, 1, 2, 3, 4)]
    assert torch.equal(inp, keep)  # the input is left as it was
    for f in (1, 2, 3, 4):
        a, b = outs[0], outs[f]
        if prec != 4:  # (a fixed-point code of -1 is a value; an unwritten norm shows as NaN below)
            assert int((b.view(torch.int16) == -1).sum()) == 0, f
        diff = int((a.view(torch.int16) != b.view(torch.int16)).sum())
        n = a.numel() // 2
        va, vb = np_of(o.export_spinor(a, 0)), np_of(o.export_spinor(b, 0))
        check(vb, va, 0.1 * SCHWARZ_TOL[prec], "form %d vs launches (%d of %d values differ)" % (f, diff, n))
        if prec == 3:
            assert diff == 0, ("form %d differs from the launches in %d of %d values" % (f, diff, n))
    from oracle import solvers
    if cycles == 0:
        ref = solvers.schwarz(ref_op, src, block, steps)
    else:
        ref = solvers.sap(ref_op, src, block, steps, cycles)
    check(np_of(o.export_spinor(outs[2], 0)), ref, SCHWARZ_TOL[prec] if cycles == 0 else 1.4 * SCHWARZ_TOL[prec])


def test_block_form_omega_and_repeat(ctx, monkeypatch):
    """Over-relaxed MR in the block form agrees with the launches, also for two
    calls in a row (the second on a new input)."""
    dims, block = (16, 8, 8, 8), (8, 8, 8, 8)
    U, psi, Ud = Fields.get(dims)
    o = ops.wilson_clover(ctx, U, dims, 0.124, 1.0, 2, 12, tile=block, bc_t=-1, U_device=Ud)
    ref_op = oracle.WilsonClover(dims, U, 0.124, 1.0, bc_t=-1)
    src1 = on_parity(psi, ref_op.even)
    src2 = on_parity(synth.gaussian_spinor(dims, 77), ref_op.even)
    prm = ops.schwarz_params(block, 6, 0, omega=1.2)
    in1, in2 = o.import_spinor(src1, 0), o.import_spinor(src2, 0)
    a1 = run_form(ctx, monkeypatch, o, prm, in1, 0)
    a2 = run_form(ctx, monkeypatch, o, prm, in2, 0)
    monkeypatch.setenv("LQCD_SCHWARZ_FORM", "2")
    out = o.spinor()
    L.lqcd_schwarz_precond(ctx, o.op, prm, out, in1)
    b1 = out.clone()
    L.lqcd_schwarz_precond(ctx, o.op, prm, out, in2)
    torch.cuda.synchronize()
    for a, b in ((a1, b1), (a2, out)):
        check(np_of(o.export_spinor(b, 0)), np_of(o.export_spinor(a, 0)), 0.1 * SCHWARZ_TOL[2])


def test_block_form_not_taken_where_it_does_not_fit(ctx, monkeypatch):
    """FP32 storage and blocks too small for the block form (8 sites per parity)
    keep the launches; asking for the block form there is not an error."""
    dims = (8, 8, 8, 8)
    U, psi, Ud = Fields.get(dims)
    ref_op = oracle.WilsonClover(dims, U, 0.124, 1.0, bc_t=-1)
    src = on_parity(psi, ref_op.even)
    from oracle import solvers
    for prec, block, tol in [(1, (4, 4, 4, 4), 1e-5), (2, (2, 2, 2, 2), 5e-3)]:
        o = ops.wilson_clover(ctx, U, dims, 0.124, 1.0, prec, 12, tile=block, bc_t=-1, U_device=Ud)
        out = run_form(ctx, monkeypatch, o, ops.schwarz_params(block, 4, 0), o.import_spinor(src, 0), 2)
        check(np_of(o.export_spinor(out, 0)), solvers.schwarz(ref_op, src, block, 4), tol, "prec %d" % prec)
