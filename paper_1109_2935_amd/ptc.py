"""Learned preconditioner: a gauge-equivariant parallel-transport convolution
network (channels 1 -> 16 -> 16 -> 16 -> 1, BF16 weights on the matrix cores,
FP32 accumulation) trained on residual -> error pairs produced by the FP64
CGNE solver, and used as the preconditioner of flexible GCR.

This module only orchestrates: weights live on the GPU, and packing,
inference, gradients, Adam and the solver that produces the training pairs
all run in liblqcd.so.
"""
import ctypes
import time

import numpy as np
import torch

from . import lqcd as L
from . import ops

CHANNELS = (1, 16, 16, 16, 1)


def shape_of(channels):
    sh = L.lqcd_ptc_shape()
    sh.nlayers = len(channels) - 1
    for k, c in enumerate(channels):
        sh.channels[k] = int(c)
    return sh


def layer_sizes(channels):
    return [(co, ci) for ci, co in zip(channels[:-1], channels[1:])]


class Network:
    """Master FP32 weights, Adam moments and packed BF16 weights on the GPU."""

    def __init__(self, ctx, channels=CHANNELS, seed=0, noise=0.02, device="cuda"):
        self.ctx = ctx
        self.channels = tuple(int(c) for c in channels)
        self.shape = shape_of(self.channels)
        nw, nb = L.lqcd_ptc_sizes(self.shape)
        self.nweights = nw
        self.weights = torch.zeros(2 * nw, dtype=torch.float32, device=device)
        self.m = torch.zeros_like(self.weights)
        self.v = torch.zeros_like(self.weights)
        self.grad = torch.zeros_like(self.weights)
        self.packed = torch.zeros(nb, dtype=torch.uint8, device=device)
        self.net = L.lqcd_ptc_net()
        self.net.shape = self.shape
        self.net.packed = self.packed.data_ptr()
        self.step = 0
        self.set_weights(self.initial_weights(seed, noise))

    def initial_weights(self, seed, noise):
        """Identity through channel 0 (N(r) = r: the unpreconditioned method)
        plus small complex Gaussian noise on every weight."""
        rng = np.random.Generator(np.random.PCG64(seed))
        Ws = []
        for co, ci in layer_sizes(self.channels):
            g = rng.standard_normal((co, ci, 9, 4, 4, 2)) * noise / np.sqrt(ci * 9 * 4)
            W = g[..., 0] + 1j * g[..., 1]
            W[0, 0, 0] += np.eye(4)
            Ws.append(W)
        return Ws

    def set_weights(self, Ws):
        flat = np.concatenate([np.ascontiguousarray(W, dtype=np.complex64).reshape(-1) for W in Ws])
        assert flat.size == self.nweights
        self.weights.copy_(torch.from_numpy(flat.view(np.float32)))
        self.pack()

    def get_weights(self):
        flat = self.weights.detach().cpu().numpy().view(np.complex64).astype(np.complex128)
        out, off = [], 0
        for co, ci in layer_sizes(self.channels):
            n = co * ci * 9 * 16
            out.append(flat[off:off + n].reshape(co, ci, 9, 4, 4))
            off += n
        return out

    def pack(self):
        L.lqcd_ptc_pack(self.ctx, self.shape, self.weights, self.packed)

    def apply(self, op32, out_even, in_even):
        L.lqcd_ptc_apply(self.ctx, op32.op, self.net, out_even, in_even)

    def gradient(self, op32, r_even, e_even):
        return L.lqcd_ptc_gradient(self.ctx, op32.op, self.net, r_even, e_even, self.grad)

    def residual_gradient(self, op32, r_even):
        """|Mhat N(r) - r|^2 / |r|^2 and its gradient (into self.grad)."""
        return L.lqcd_ptc_residual_gradient(self.ctx, op32.op, self.net, r_even, self.grad)

    def vjp(self, op32, r_even, dy_even):
        L.lqcd_ptc_vjp(self.ctx, op32.op, self.net, r_even, dy_even, self.grad)

    def adam(self, lr):
        self.step += 1
        L.lqcd_ptc_adam(self.ctx, self.shape, self.weights, self.m, self.v, self.grad, self.step, lr)
        self.pack()

    def save(self, path):
        np.savez_compressed(path, channels=np.array(self.channels),
                            **{"w%d" % k: W.astype(np.complex64) for k, W in enumerate(self.get_weights())})

    def load(self, path):
        z = np.load(path, allow_pickle=False)
        assert tuple(int(c) for c in z["channels"]) == self.channels
        self.set_weights([z["w%d" % k] for k in range(len(self.channels) - 1)])


def solver_pairs(ctx, op64, b_even_natural, every, max_pairs, xstar_tol=1e-12, tol=1e-10, max_iter=20000):
    """Residual -> error pairs from the FP64 even-odd CGNE solve of M x = b
    (b on even sites): r_k = bhat - Mhat x_k and e_k = x* - x_k, recorded by
    the solver every `every` iterations (packed even FP64 fields of op64)."""
    b = op64.import_spinor(b_even_natural, -1)
    xs = op64.spinor(full=True)
    st, info = L.lqcd_cg_solve(ctx, op64.op, None, ops.cg_params(xstar_tol, max_iter), xs, b)
    if st != L.LQCD_OK:
        raise RuntimeError("reference solve failed: " + L.lqcd_last_error(ctx))
    sb = op64.spinor_bytes
    rec_r = op64.spinor(nrhs=max_pairs, zero=False)
    rec_e = op64.spinor(nrhs=max_pairs, zero=False)
    count = ctypes.c_int32(0)
    prm = ops.cg_params(tol, max_iter)
    prm.record_r, prm.record_e = rec_r.data_ptr(), rec_e.data_ptr()
    prm.record_xstar = xs.data_ptr()
    prm.record_every, prm.record_max = every, max_pairs
    prm.record_count = ctypes.pointer(count)
    x = op64.spinor(full=True)
    st, _ = L.lqcd_cg_solve(ctx, op64.op, None, prm, x, b)
    n = count.value
    return [(rec_r[k * sb:(k + 1) * sb], rec_e[k * sb:(k + 1) * sb]) for k in range(n)]


def train(ctx, net, op64, op32, dims, nsources, every=2, pairs_per_source=100, lr=2e-3, seed0=5100, log=None,
          lr_end=None, objective="error", max_pairs=None):
    """Online training: for each Gaussian source (seeds seed0 + j) the solver's
    pairs are generated on the GPU, converted to FP32 and used once each.
    nsources sources, or, with max_pairs, as many sources as it takes to reach
    max_pairs pairs (a solve that converges early yields fewer than
    pairs_per_source). With lr_end the step size decays geometrically from lr
    to lr_end, over the sources, or over the pairs when max_pairs is given.
    objective "error": |N(r) - e|^2 / |e|^2; "residual": |Mhat N(r) - r|^2 / |r|^2
    (only the residual of each pair is used)."""
    if objective not in ("error", "residual"):
        raise ValueError("objective must be 'error' or 'residual'")
    import synth
    r32, e32 = op32.spinor(), op32.spinor()
    losses = []
    t0 = time.time()
    even = synth.parity_of_sites(dims) == 0

    def step_size(j):
        if lr_end is None:
            return lr
        if max_pairs:
            return lr * (lr_end / lr) ** (len(losses) / max(1, max_pairs - 1))
        return lr * (lr_end / lr) ** (j / max(1, nsources - 1))

    j = 0
    while (len(losses) < max_pairs) if max_pairs else (j < nsources):
        b = synth.gaussian_spinor(dims, seed0 + j)
        b = np.where(even[..., None, None], b, 0)
        want = pairs_per_source if not max_pairs else min(pairs_per_source, max_pairs - len(losses))
        pairs = solver_pairs(ctx, op64, b, every, want)
        if not pairs:
            raise RuntimeError("the solve for source %d produced no pairs" % j)
        for r64, e64 in pairs:
            L.lqcd_spinor_convert(ctx, op32.op, r32, op64.op, r64, 0)
            if objective == "residual":
                losses.append(net.residual_gradient(op32, r32))
            else:
                L.lqcd_spinor_convert(ctx, op32.op, e32, op64.op, e64, 0)
                losses.append(net.gradient(op32, r32, e32))
            net.adam(step_size(j))
        if log:
            log("source %d: pairs %d, mean loss (last 50) %.4f, %.1fs" % (
                j, len(losses), float(np.mean(losses[-50:])), time.time() - t0))
        j += 1
    return losses
