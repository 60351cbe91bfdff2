"""The entry point for callers that cannot allocate, lqcd_schur_apply_noalloc,
against lqcd_schur_apply (the same kernels: bit for bit) on two calls in a row,
the second on a smaller input, plus its size limit. Runs through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import ctx, np_of  # noqa: F401

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1109_2935_amd.lqcd")
from paper_1109_2935_amd import ops  # noqa: E402


def schur_pair(ctx, dims, prec, recon, tile, nrhs, dagger, block, seed):
    U = synth.gauge_field(dims, 0.25, seed)
    o = ops.wilson_clover(ctx, U, dims, 0.124, 1.0, prec, recon, tile=tile)
    even = oracle.parity_mask(dims, 0)
    src = np.stack([np.where(even[..., None, None], synth.gaussian_spinor(dims, seed + 1 + r), 0) for r in range(nrhs)])
    inp = o.import_spinor(src if nrhs > 1 else src[0], 0, nrhs=nrhs)
    ref, got = o.spinor(nrhs=nrhs), o.spinor(nrhs=nrhs)
    got.fill_(7)
    L.lqcd_schur_apply(ctx, o.op, ref, inp, dagger, block=block, nrhs=nrhs)
    L.lqcd_schur_apply_noalloc(ctx, o.op, got, inp, dagger, block=block, nrhs=nrhs)
    torch.cuda.synchronize()
    return o, src, ref, got, U


def test_noalloc_schur_equals_schur_two_calls(ctx):
    # first call: 16x8x8x16 FP32 (4.5 MB of intermediate spinor for 2 sources)
    o, src, ref, got, U = schur_pair(ctx, (16, 8, 8, 16), 1, 12, (8, 8, 8, 8), 2, 0, None, 901)
    assert torch.equal(got, ref)
    # and it is the even-odd operator: the oracle on the first source
    M = oracle.WilsonClover((16, 8, 8, 16), U, 0.124, 1.0, bc_t=-1)
    a = np_of(o.export_spinor(got, 0, nrhs=2))[0]
    r = M.schur(src[0])
    assert np.linalg.norm(a - r) / np.linalg.norm(r) < 1e-5
    # second call, smaller: 8^4 FP64, daggered, with a Dirichlet cut
    o2, src2, ref2, got2, _ = schur_pair(ctx, (8, 8, 8, 8), 0, 18, (4, 4, 4, 4), 1, 1, (4, 4, 4, 4), 911)
    assert torch.equal(got2, ref2)


def test_noalloc_schur_rejects_inputs_beyond_its_array(ctx):
    dims = (32, 32, 32, 32)  # FP32: 48 MiB per source, two sources exceed 64 MiB
    U = synth.gauge_field((4, 4, 4, 4), 0.25, 921)
    o = ops.Operator(ctx, L.LQCD_WILSON_CLOVER, dims, L.LQCD_F32, 12, kappa=0.124, csw=1.0)
    small = ops.wilson_clover(ctx, U, (4, 4, 4, 4), 0.124, 1.0, 1, 12)
    # any aligned device pointers: the size check comes before any launch
    o.op.gauge = o.op.clover = o.op.clover_inv = small.op.gauge
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.LqcdError) as ei:
        L.lqcd_schur_apply_noalloc(ctx, o.op, buf, buf[16:], 0, nrhs=2)
    assert ei.value.status == L.LQCD_ERR_UNSUPPORTED
    assert "64" in L.lqcd_last_error(ctx)
    torch.cuda.synchronize()
    assert int(buf.sum()) == 0
