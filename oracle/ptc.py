"""Gauge-equivariant parallel-transport convolution (PTC) network, FP64
(test infrastructure only).

Layer (one per network stage):
    psi'_o(x) = sum_i sum_p W[o, i, p] (T_p psi_i)(x)
with 9 paths p: 0 = identity, 1 + 2 mu = forward hop along mu,
(T psi)(x) = U_mu(x) psi(x + mu), 2 + 2 mu = backward hop,
(T psi)(x) = U_mu(x - mu)^+ psi(x - mu), boundary phases as for the Dirac
operator. W[o, i, p] is a complex 4x4 matrix acting on spin, so the layer
commutes with gauge transformations. The network is linear (no bias, no
activation) with channels 1 -> 16 -> 16 -> 16 -> 1; its input is a residual on
even sites (zeros on odd sites) and its output is read on even sites.

Gradients use the conjugate (Wirtinger) derivative of the real loss:
G = dL/d(conj W), so that dL = 2 Re <G, dW>. With
L = sum_even |y - e|^2 / |e|^2, delta = dL/d(conj y) = (y - e)/|e|^2 on even sites,
    dL/d(conj W[o,i,p]) = sum_x delta_o(x) (T_p psi_i(x))^+   (spin outer product, traced over colour)
    dL/d(conj psi_i)    = sum_{o,p} T_p^+ (W[o,i,p]^+ delta_o).
With the residual loss L = |Mhat y - r|^2 / |r|^2 (Mhat the even-odd Schur
operator) the output cotangent is delta = Mhat^+ (Mhat y - r) / |r|^2.
"""
import numpy as np

from . import transport

NPATH = 9
CHANNELS = (1, 16, 16, 16, 1)


def layer_forward(dims, U, psi, W, bc_t=-1):
    """psi: (Cin, t, z, y, x, 4, 3); W: (Cout, Cin, 9, 4, 4) -> (Cout, ..., 4, 3)."""
    cout = W.shape[0]
    out = np.zeros((cout,) + psi.shape[1:], dtype=np.complex128)
    for p in range(NPATH):
        Tp = transport(dims, U, psi, p, bc_t=bc_t)
        out += np.einsum("oist,i...tc->o...sc", W[:, :, p], Tp)
    return out


def layer_backward(dims, U, psi, W, delta, bc_t=-1):
    """Conjugate gradients of one layer: returns (dL/d conj W, dL/d conj psi)."""
    gW = np.zeros_like(W)
    gpsi = np.zeros_like(psi)
    for p in range(NPATH):
        Tp = transport(dims, U, psi, p, bc_t=bc_t)
        d2 = delta.reshape(delta.shape[0], -1, 4, 3)
        t2 = Tp.reshape(Tp.shape[0], -1, 4, 3)
        gW[:, :, p] = np.einsum("oxsc,ixtc->oist", d2, np.conj(t2))
        g = np.einsum("oist,o...sc->i...tc", np.conj(W[:, :, p]), delta)
        gpsi += transport(dims, U, g, p, bc_t=bc_t, adjoint=True)
    return gW, gpsi


def init_weights(seed, channels=CHANNELS, scale=None):
    """Random complex weights, scaled so each layer roughly preserves the norm."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ws = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        s = scale if scale is not None else 1.0 / np.sqrt(cin * NPATH * 4)
        w = rng.standard_normal((cout, cin, NPATH, 4, 4, 2)) * s
        Ws.append(w[..., 0] + 1j * w[..., 1])
    return Ws


def forward(dims, U, r, Ws, even_mask, bc_t=-1):
    """Network output on even sites and the list of layer inputs."""
    psi = np.where(even_mask[..., None, None], r, 0)[None]
    acts = [psi]
    for W in Ws:
        psi = layer_forward(dims, U, psi, W, bc_t)
        acts.append(psi)
    y = np.where(even_mask[..., None, None], acts[-1][0], 0)
    return y, acts


def backprop(dims, U, acts, Ws, delta, bc_t=-1):
    """dL/d conj W for every layer from the output cotangent delta = dL/d conj y
    (even sites) and the layer inputs of the forward pass."""
    delta = delta[None]
    grads = [None] * len(Ws)
    for k in range(len(Ws) - 1, -1, -1):
        grads[k], delta = layer_backward(dims, U, acts[k], Ws[k], delta, bc_t)
    return grads


def loss_and_grads(dims, U, r, e, Ws, even_mask, bc_t=-1):
    """L = |y - e|^2 / |e|^2 on even sites and dL/d conj W for every layer."""
    y, acts = forward(dims, U, r, Ws, even_mask, bc_t)
    en2 = np.vdot(e, e).real
    diff = y - np.where(even_mask[..., None, None], e, 0)
    L = np.vdot(diff, diff).real / en2
    return L, backprop(dims, U, acts, Ws, diff / en2, bc_t)


def vjp(dims, U, r, dy, Ws, even_mask, bc_t=-1):
    """dL/d conj W for a loss whose cotangent at the output is dy (even sites)."""
    _, acts = forward(dims, U, r, Ws, even_mask, bc_t)
    return backprop(dims, U, acts, Ws, np.where(even_mask[..., None, None], dy, 0), bc_t)


def residual_loss_and_grads(dims, U, r, Ws, even_mask, schur, bc_t=-1):
    """L = |Mhat y - r|^2 / |r|^2 over even sites, y = N(r), and dL/d conj W.
    schur(x, dagger) applies Mhat (or its adjoint) to a field read on even
    sites; the cotangent is dL/d conj y = Mhat^+ (Mhat y - r) / |r|^2."""
    y, acts = forward(dims, U, r, Ws, even_mask, bc_t)
    re = np.where(even_mask[..., None, None], r, 0)
    rn2 = np.vdot(re, re).real
    z = np.where(even_mask[..., None, None], schur(y, False), 0) - re
    L = np.vdot(z, z).real / rn2
    delta = np.where(even_mask[..., None, None], schur(z, True), 0) / rn2
    return L, backprop(dims, U, acts, Ws, delta, bc_t)
