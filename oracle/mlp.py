"""Warm-start surrogate, plain FP64 numpy (TEST INFRASTRUCTURE ONLY).

The paper has no learned component; this is the oracle of the surrogate that
warm-starts the steady Couette solver.  It restates, with no blocking or fusion:

* a multilayer perceptron 4 -> 128 -> 128 -> 128 -> 4 with SiLU activations,
  silu(z) = z / (1 + e^{-z}) (Elfwing, Uchibe & Doya 2018), and a linear output layer;
* the mean-squared-error loss over all outputs of a mini-batch and its gradient by
  reverse-mode differentiation, written out layer by layer;
* Adam (Kingma & Ba, ICLR 2015, Algorithm 1) with bias-corrected moments;
* a bfloat16 emulation of inference (operands rounded to the nearest bfloat16, ties
  to even; products and sums in FP64) for checking a bfloat16 inference path;
* the features and targets of the surrogate and the warm-start profile, whose
  particle number is rescaled to the cold start's: the steady state of a closed
  Couette cell depends on its total particle number, which the dynamics conserve
  (Sec. III.E, Eq. Ntot_def).

Parameter vector layout (FP64 here, FP32 in the library): for each layer l in
order, W_l as a row-major [fan_in][fan_out] matrix, then b_l[fan_out].
"""
from __future__ import annotations

import math

import numpy as np

D_IN, WIDTH, DEPTH, D_OUT = 4, 128, 3, 4

# feature box of the surrogate: log10 Kn in [-2, 1], u_w in [0.05, 0.5],
# beta = R_in/R_out in [0.3, 0.8], rho = (R - R_in)/(R_out - R_in) in [0, 1]
FEAT_CENTRE = (-0.5, 0.275, 0.55, 0.5)
FEAT_HALF = (1.5, 0.225, 0.25, 0.5)
# targets: ((n - 1) S_N, u^R S_U, u^phi / u_w, (T - 1) S_T)
S_N, S_U, S_T = 10.0, 10.0, 10.0


def layer_dims(width: int = WIDTH, depth: int = DEPTH, d_in: int = D_IN, d_out: int = D_OUT):
    dims = [d_in] + [width] * depth + [d_out]
    return [(dims[l], dims[l + 1]) for l in range(len(dims) - 1)]


def param_count(dims=None) -> int:
    dims = dims or layer_dims()
    return sum(a * b + b for a, b in dims)


def unpack(theta, dims=None):
    """Views (W_l, b_l) into the flat parameter vector."""
    dims = dims or layer_dims()
    out, o = [], 0
    for a, b in dims:
        W = theta[o:o + a * b].reshape(a, b)
        o += a * b
        bias = theta[o:o + b]
        o += b
        out.append((W, bias))
    assert o == len(theta)
    return out


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    """d silu / dz = s + z s (1 - s), s = sigmoid(z)."""
    s = sigmoid(z)
    return s + z * s * (1.0 - s)


def forward(theta, X, dims=None, keep=False):
    """Y = MLP(X) for X[batch][D_IN]; with keep, also the pre-activations z_l and the
    layer inputs h_l needed by the backward pass."""
    layers = unpack(np.asarray(theta, dtype=np.float64), dims)
    h = np.asarray(X, dtype=np.float64)
    hs, zs = [], []
    for l, (W, b) in enumerate(layers):
        hs.append(h)
        z = h @ W + b
        zs.append(z)
        h = silu(z) if l < len(layers) - 1 else z
    return (h, hs, zs) if keep else h


def loss(theta, X, T, dims=None) -> float:
    """Mean of (y - t)^2 over every output of the mini-batch."""
    Y = forward(theta, X, dims)
    return float(np.mean((Y - np.asarray(T, dtype=np.float64)) ** 2))


def loss_and_grad(theta, X, T, dims=None):
    """Loss and its gradient with respect to every parameter (reverse mode):
    g_y = 2 (y - t) / (batch * D_OUT); for each layer from the last, dW = h^T g_z,
    db = sum over the batch of g_z, and g_h = g_z W^T, g_z = g_h * silu'(z) below."""
    theta = np.asarray(theta, dtype=np.float64)
    layers = unpack(theta, dims)
    Y, hs, zs = forward(theta, X, dims, keep=True)
    T = np.asarray(T, dtype=np.float64)
    L = float(np.mean((Y - T) ** 2))
    gz = 2.0 * (Y - T) / Y.size
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (hs[l].T @ gz, gz.sum(axis=0))
        if l:
            gz = (gz @ W.T) * dsilu(zs[l - 1])
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return L, flat


class Adam:
    """Adam with bias correction: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def bf16(x):
    """Round to the nearest bfloat16 (8 significant bits), ties to even; the value is
    first rounded to float32 (the width an FP32 pipeline holds it in)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta, X, dims=None):
    """Inference with every matrix operand (layer input and weight) rounded to
    bfloat16, biases and activations in full precision, sums in FP64."""
    layers = unpack(np.asarray(theta, dtype=np.float64), dims)
    h = np.asarray(X, dtype=np.float64)
    for l, (W, b) in enumerate(layers):
        z = bf16(h) @ bf16(W) + b
        h = silu(z) if l < len(layers) - 1 else z
    return h


def features(Kn, u_w, beta, rho):
    """Surrogate inputs, each mapped affinely from its box to [-1, 1]."""
    raw = (np.log10(Kn), u_w, beta, rho)
    cols = [(np.asarray(v, dtype=np.float64) - c) / h for v, c, h in zip(raw, FEAT_CENTRE, FEAT_HALF)]
    return np.stack(np.broadcast_arrays(*cols), axis=-1)


def targets(n, u_R, u_phi, T, u_w):
    return np.stack([(np.asarray(n) - 1) * S_N, np.asarray(u_R) * S_U, np.asarray(u_phi) / u_w,
                     (np.asarray(T) - 1) * S_T], axis=-1)


def cell_rho(Rc, R_in, R_out):
    return (np.asarray(Rc) - R_in) / (R_out - R_in)


def warm_profile(Y, u_w, dchi, mass_cold):
    """Moments (n, u^R, u^phi, T) of the warm start from surrogate outputs Y[cells][4]:
    n from the first output rescaled so that sum_s dchi_s n_s equals the cold start's
    particle number (sum_k f' = n at every cell), u^R = 0 (the steady Couette flow has
    no radial current), u^phi and T from the other outputs."""
    Y = np.asarray(Y, dtype=np.float64)
    n = 1.0 + Y[:, 0] / S_N
    n = n * (mass_cold / float(np.sum(np.asarray(dchi) * n)))
    return n, np.zeros_like(n), Y[:, 2] * u_w, 1.0 + Y[:, 3] / S_T
