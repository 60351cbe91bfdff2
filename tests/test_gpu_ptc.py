"""GPU parity of the learned (PTC) preconditioner against the FP64 oracle, and
its gain inside flexible GCR."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import check, check_entries, ctx, np_of, on_parity, rel  # noqa: F401
from oracle import ptc as optc

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1109_2935_amd.lqcd")
from paper_1109_2935_amd import ops  # noqa: E402
from paper_1109_2935_amd import ptc  # noqa: E402

DIMS = (4, 4, 4, 8)


def system(ctx, dims, seed, tile=None, precs=(1,)):
    U = synth.gauge_field(dims, 0.25, seed)
    Ud = torch.from_numpy(U).cuda()
    o = {p: ops.wilson_clover(ctx, U, dims, 0.124, 1.0, p, 18 if p == 0 else 12, tile=tile, U_device=Ud)
         for p in precs}
    return U, o


def weights_c64(Ws):
    return [np.asarray(W, dtype=np.complex64).astype(np.complex128) for W in Ws]


# Tolerances of the network (BF16 weights and activations, unit roundoff
# u = 2^-9, FP32 sums). One layer rounds its transported inputs and its
# weights (two roundings of relative RMS u / sqrt(3) each, averaged over the
# 9 x 16 x 4 products of a sum, so of order 2u at most for the output) and
# stores its output in BF16 (another u / sqrt(3)): about 1.5e-3 per layer.
# Four layers in quadrature give 3e-3; a factor 3 for the spread of a
# statistical bound and the worst-conditioned weights: 1e-2 for one layer,
# 1.5e-2 for three, 2e-2 for the four-layer 16-channel network. A weight
# gradient is a sum over sites of products of a forward activation and a
# back-propagated cotangent, both carrying the roundings of the whole
# network (2 x 4 layers): sqrt(2) times the forward bound, 3e-2.
GRAD_TOL = 3e-2

# forward bounds: see the tolerance note above
@pytest.mark.parametrize("channels,tol", [((1, 1), 1e-2), ((1, 4, 4, 1), 1.5e-2), ((1, 16, 16, 16, 1), 2e-2)])
def test_ptc_forward_matches_oracle(ctx, channels, tol):
    U, o = system(ctx, DIMS, 61)
    op32 = o[1]
    net = ptc.Network(ctx, channels)
    Ws = weights_c64(optc.init_weights(62, channels=channels))
    net.set_weights(Ws)
    r = on_parity(synth.gaussian_spinor(DIMS, 63), oracle.parity_mask(DIMS, 0))
    out = op32.spinor()
    net.apply(op32, out, op32.import_spinor(r, 0))
    got = np_of(op32.export_spinor(out, 0))
    ref, _ = optc.forward(DIMS, U, r, Ws, oracle.parity_mask(DIMS, 0))
    check(got, ref, tol)


# every form of the 16-input-channel layers (256 or 512 threads, waves per
# SIMD, colour products on dot2 or on 4x4x4 matrix-core blocks, transport and
# products in the same or in separate waves; both link formats), on a lattice
# whose sites fill whole workgroups and on one that leaves 16 of 32 sites of a
# workgroup empty
PTC_FORMS = (3221, 3231, 3222, 3232, 5031, 5041, 5032, 5042, 5033, 5043, 5034, 5044)


@pytest.mark.parametrize("recon", [12, 18])
@pytest.mark.parametrize("dims", [DIMS, (4, 2, 2, 2)])
@pytest.mark.parametrize("form", PTC_FORMS)
def test_ptc_forward_every_form(ctx, form, dims, recon, monkeypatch):
    channels = (1, 16, 16, 16, 1)
    U = synth.gauge_field(dims, 0.25, 131)
    op32 = ops.wilson_clover(ctx, U, dims, 0.124, 1.0, 1, recon)
    net = ptc.Network(ctx, channels)
    Ws = weights_c64(optc.init_weights(132, channels=channels))
    net.set_weights(Ws)
    r = on_parity(synth.gaussian_spinor(dims, 133), oracle.parity_mask(dims, 0))
    out = op32.spinor()
    monkeypatch.setenv("LQCD_PTC_VARIANT", str(form))
    net.apply(op32, out, op32.import_spinor(r, 0))
    got = np_of(op32.export_spinor(out, 0))
    ref, _ = optc.forward(dims, U, r, Ws, oracle.parity_mask(dims, 0))
    check(got, ref, 2e-2)


def test_ptc_gauge_equivariance_on_gpu(ctx):
    channels = (1, 4, 4, 1)
    U = synth.gauge_field(DIMS, 0.25, 71)
    g = synth.su3_site_field(DIMS, 72)
    from util_fields import gauge_transform_links
    Ug = gauge_transform_links(U, g)
    net = ptc.Network(ctx, channels)
    net.set_weights(weights_c64(optc.init_weights(73, channels=channels)))
    r = on_parity(synth.gaussian_spinor(DIMS, 74), oracle.parity_mask(DIMS, 0))
    outs = []
    for links, src in ((U, r), (Ug, np.einsum("...ab,...sb->...sa", g, r))):
        op32 = ops.wilson_clover(ctx, links, DIMS, 0.124, 1.0, 1, 18)
        out = op32.spinor()
        net.apply(op32, out, op32.import_spinor(src, 0))
        outs.append(np_of(op32.export_spinor(out, 0)))
    assert rel(outs[1], np.einsum("...ab,...sb->...sa", g, outs[0])) < 2e-2


@pytest.mark.parametrize("channels", [(1, 4, 4, 1), (1, 16, 16, 16, 1)])
def test_ptc_gradient_matches_oracle(ctx, channels):
    U, o = system(ctx, DIMS, 81)
    op32 = o[1]
    even = oracle.parity_mask(DIMS, 0)
    net = ptc.Network(ctx, channels)
    Ws = weights_c64(optc.init_weights(82, channels=channels))
    net.set_weights(Ws)
    r = on_parity(synth.gaussian_spinor(DIMS, 83), even)
    e = on_parity(synth.gaussian_spinor(DIMS, 84), even)
    loss = net.gradient(op32, op32.import_spinor(r, 0), op32.import_spinor(e, 0))
    Lref, gref = optc.loss_and_grads(DIMS, U, r, e, Ws, even)
    assert abs(loss - Lref) < 2e-2 * Lref
    flat = net.grad.cpu().numpy().view(np.complex64).astype(np.complex128)
    off = 0
    for k, G in enumerate(gref):
        gk = flat[off:off + G.size].reshape(G.shape)
        off += G.size
        check_entries(gk, G, GRAD_TOL, "layer %d" % k)


def _flat_grads(net, gref):
    flat = net.grad.cpu().numpy().view(np.complex64).astype(np.complex128)
    out, off = [], 0
    for G in gref:
        out.append(flat[off:off + G.size].reshape(G.shape))
        off += G.size
    return out


@pytest.mark.parametrize("channels", [(1, 4, 4, 1), (1, 16, 16, 16, 1)])
def test_ptc_residual_gradient_matches_oracle(ctx, channels):
    """|Mhat N(r) - r|^2 / |r|^2 and its gradient: network, FP32 Schur operator
    and its adjoint on the GPU against the FP64 oracle."""
    U, o = system(ctx, DIMS, 101)
    op32 = o[1]
    even = oracle.parity_mask(DIMS, 0)
    net = ptc.Network(ctx, channels)
    Ws = weights_c64(optc.init_weights(102, channels=channels))
    net.set_weights(Ws)
    r = on_parity(synth.gaussian_spinor(DIMS, 103), even)
    loss = net.residual_gradient(op32, op32.import_spinor(r, 0))
    M = oracle.WilsonClover(DIMS, U, 0.124, 1.0)
    Lref, gref = optc.residual_loss_and_grads(DIMS, U, r, Ws, even, M.schur)
    assert abs(loss - Lref) < 2e-2 * Lref
    for k, (g, G) in enumerate(zip(_flat_grads(net, gref), gref)):
        check_entries(g, G, GRAD_TOL, "layer %d" % k)


def test_ptc_vjp_matches_oracle(ctx):
    channels = (1, 4, 4, 1)
    U, o = system(ctx, DIMS, 111)
    op32 = o[1]
    even = oracle.parity_mask(DIMS, 0)
    net = ptc.Network(ctx, channels)
    Ws = weights_c64(optc.init_weights(112, channels=channels))
    net.set_weights(Ws)
    r = on_parity(synth.gaussian_spinor(DIMS, 113), even)
    dy = on_parity(synth.gaussian_spinor(DIMS, 114), even)
    net.vjp(op32, op32.import_spinor(r, 0), op32.import_spinor(dy, 0))
    gref = optc.vjp(DIMS, U, r, dy, Ws, even)
    for k, (g, G) in enumerate(zip(_flat_grads(net, gref), gref)):
        check_entries(g, G, GRAD_TOL, "layer %d" % k)


def test_ptc_residual_training_reduces_loss(ctx):
    dims = (8, 8, 8, 8)
    U, o = system(ctx, dims, 121, precs=(0, 1))
    net = ptc.Network(ctx, (1, 16, 16, 16, 1), seed=122)
    losses = ptc.train(ctx, net, o[0], o[1], dims, nsources=3, every=1, pairs_per_source=60, lr=3e-3, seed0=9200,
                       objective="residual")
    assert len(losses) >= 100
    assert np.mean(losses[-30:]) < 0.7 * np.mean(losses[:10])


def test_ptc_training_and_fgcr_gain(ctx):
    """Trained on solver pairs, the network preconditions flexible GCR: fewer
    Krylov steps than GCR without it, same FP64 residual (the gain is not
    pinned by the paper, which has no learned preconditioner)."""
    dims = (8, 8, 8, 8)
    U, o = system(ctx, dims, 91, precs=(0, 1))
    net = ptc.Network(ctx, (1, 16, 16, 16, 1), seed=92)
    losses = ptc.train(ctx, net, o[0], o[1], dims, nsources=6, every=1, pairs_per_source=60, lr=3e-3, seed0=9100)
    assert len(losses) >= 200
    assert np.mean(losses[-40:]) < 0.7 * np.mean(losses[:20])
    b = synth.gaussian_spinor(dims, 9999)
    bp = o[0].import_spinor(b, -1)
    x0, x1 = o[0].spinor(full=True), o[0].spinor(full=True)
    st0, i0 = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, None, ops.gcr_params(1e-10, 16, 1e-3), x0, bp)
    prm = ops.gcr_params(1e-10, 16, 1e-3, precond=L.LQCD_PRECOND_LEARNED, mr_steps=0)
    prm.learned = ctypes_pointer(net.net)
    st1, i1 = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, o[1].op, prm, x1, bp)
    assert st0 == L.LQCD_OK and st1 == L.LQCD_OK
    assert i1.true_residual <= 1e-10
    assert i1.iters < i0.iters
    M = oracle.WilsonClover(dims, U, 0.124, 1.0)
    xs = np_of(o[0].export_spinor(x1, -1))
    assert np.linalg.norm(b - M.M(xs)) / np.linalg.norm(b) < 1.05e-10


def ctypes_pointer(s):
    import ctypes
    return ctypes.pointer(s)


@pytest.mark.parametrize("cycles", [0, 1])
@pytest.mark.parametrize("bad", ["zero", "nan"])
def test_learned_fgcr_falls_back_to_schwarz(ctx, bad, cycles):
    """A network whose output is unusable (all zero, or not finite) hands every
    step to the Schwarz fallback (additive, or multiplicative with cycles = 1):
    the solve still reaches an FP64 residual of 1e-10, recomputed by the
    oracle. Without a fallback the same network is a breakdown."""
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U, o = system(ctx, dims, 95, tile=block, precs=(0, 1))
    net = ptc.Network(ctx, (1, 16, 16, 16, 1), seed=96)
    Ws = net.get_weights()
    fill = 0.0 if bad == "zero" else np.nan
    net.set_weights([np.full_like(W, fill) for W in Ws])
    b = synth.gaussian_spinor(dims, 9801)
    bp = o[0].import_spinor(b, -1)
    x = o[0].spinor(full=True)
    prm = ops.gcr_params(1e-10, 16, 1e-3, precond=L.LQCD_PRECOND_LEARNED, block=block, mr_steps=4, cycles=cycles)
    prm.learned = ctypes_pointer(net.net)
    st, info = L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, o[1].op, prm, x, bp)
    assert st == L.LQCD_OK, L.lqcd_last_error(ctx)
    assert info.true_residual <= 1e-10
    assert info.fallback_applies == info.iters
    M = oracle.WilsonClover(dims, U, 0.124, 1.0)
    xs = np_of(o[0].export_spinor(x, -1))
    assert np.linalg.norm(b - M.M(xs)) / np.linalg.norm(b) < 1.05e-10
    # no fallback: the unusable direction is a breakdown
    prm0 = ops.gcr_params(1e-10, 16, 1e-3, precond=L.LQCD_PRECOND_LEARNED, mr_steps=0)
    prm0.learned = ctypes_pointer(net.net)
    x0 = o[0].spinor(full=True)
    with pytest.raises(L.LqcdError) as ei:
        L.lqcd_gcr_solve(ctx, o[0].op, o[1].op, o[1].op, prm0, x0, bp)
    assert ei.value.status == L.LQCD_ERR_BREAKDOWN
