"""Plain numpy oracle of the density surrogate: a 3-128-128-128-1 perceptron
with tanh-form GELU, trained by mean squared error and Adam.

TEST INFRASTRUCTURE: only the tests and the smoke check use this module.

It is the specification the GPU kernels must meet, written out in float64.
Every matrix product takes its two operands rounded to bfloat16 (round to
nearest, ties to even) and accumulates in high precision; biases,
activations, the loss and its gradient stay unrounded. `bf16=False` drops the
rounding, which makes the network an ordinary float64 network that the tests
compare with PyTorch and with finite differences.

Inputs of a row: ((p - 0.16) / 0.07, d, log10(t) / 6), as the p_c search feeds
them; target: log10(rho).

Parameter vector (float32 master copy on the GPU), in this order:
    W1 [128][3], b1 [128], W2 [128][128], b2 [128], W3 [128][128], b3 [128],
    w4 [128], b4 [1]                                    -> 33665 values
Weights are stored output-major (W[o][i]).

Gradient of one step, with z_k the pre-activations, h_k = gelu(z_k) and the
rounding points of the forward pass:
    dy  = 2 (y - target) / M on rows with mask 1 (M = number of such rows), else 0
    dw4 = sum_r dy_r * h3b_r,        db4 = sum_r dy_r,   dh3 = dy * w4b
    dz3 = dh3 * gelu'(z3)
    dW3 = bf(dz3)^T bf(h2),         db3 = sum_r dz3,    dh2 = bf(dz3) W3b
    dz2 = dh2 * gelu'(z2)
    dW2 = bf(dz2)^T bf(h1),         db2 = sum_r dz2,    dh1 = bf(dz2) W2b
    dz1 = dh1 * gelu'(z1)
    dW1 = dz1^T bf(x),              db1 = sum_r dz1
Layer 4 and layer 1 (three inputs) are vector work, not matrix products: there
only the stored bfloat16 activations/weights enter, the upstream gradient
stays unrounded.
"""
from __future__ import annotations

import math

import numpy as np

H = 128
SIZES = [("W1", (H, 3)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)),
         ("b3", (H,)), ("w4", (H,)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)
GELU_C = math.sqrt(2.0 / math.pi)
GELU_A = 0.044715


def bf16(x):
    """Round float64/float32 values to the nearest bfloat16 (ties to even),
    returned as float64. Works on the float32 bit pattern: a value is first
    rounded to float32 (as the GPU holds it), then to 8 mantissa bits."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.float64("nan"), out)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1)
                           for name, _ in SIZES])


def gelu(z):
    """Tanh form of the Gaussian error linear unit (Hendrycks & Gimpel)."""
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + GELU_A * z ** 3)))


def gelu_grad(z):
    u = GELU_C * (z + GELU_A * z ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * z * z)


def forward(theta, x, bf=True):
    """Returns (y [N], cache) for rows x [N, 3]."""
    P = unpack(theta)
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    xb = r(x)
    z1 = xb @ r(P["W1"]).T + P["b1"]
    h1 = gelu(z1)
    z2 = r(h1) @ r(P["W2"]).T + P["b2"]
    h2 = gelu(z2)
    z3 = r(h2) @ r(P["W3"]).T + P["b3"]
    h3 = gelu(z3)
    y = r(h3) @ r(P["w4"]) + P["b4"][0]
    cache = dict(P=P, xb=xb, z1=z1, z2=z2, z3=z3, h1=h1, h2=h2, h3=h3, r=r)
    return y, cache


def loss_and_grad(theta, x, target, mask=None, bf=True):
    """Masked mean squared error of log10 rho and its gradient [N_PARAMS]."""
    y, c = forward(theta, x, bf=bf)
    t = np.asarray(target, dtype=np.float64)
    m = np.ones_like(t) if mask is None else np.asarray(mask, dtype=np.float64)
    M = m.sum()
    if M == 0:
        return 0.0, np.zeros(N_PARAMS)
    loss = float((m * (y - t) ** 2).sum() / M)
    P, r = c["P"], c["r"]
    dy = 2.0 * (y - t) * m / M
    g = {}
    h3b = r(c["h3"])
    g["w4"] = dy @ h3b
    g["b4"] = np.array([dy.sum()])
    dh3 = np.outer(dy, r(P["w4"]))
    dz3 = dh3 * gelu_grad(c["z3"])
    g["W3"] = r(dz3).T @ r(c["h2"])
    g["b3"] = dz3.sum(axis=0)
    dh2 = r(dz3) @ r(P["W3"])
    dz2 = dh2 * gelu_grad(c["z2"])
    g["W2"] = r(dz2).T @ r(c["h1"])
    g["b2"] = dz2.sum(axis=0)
    dh1 = r(dz2) @ r(P["W2"])
    dz1 = dh1 * gelu_grad(c["z1"])
    g["W1"] = dz1.T @ c["xb"]
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def forward_scale(theta, x):
    """Per row, the sum of the magnitudes of the terms the output adds up:
    sum_j |bf(h3_j) bf(w4_j)| + |b4|. Reordering or rounding the accumulation
    moves y by a small multiple of this scale; a changed rounding point of an
    operand moves it by about 2^-9 of it."""
    _, c = forward(theta, x)
    P, r = c["P"], c["r"]
    return np.abs(r(c["h3"])) @ np.abs(r(P["w4"])) + abs(P["b4"][0])


def grad_scale(theta, x, target, mask=None):
    """Per parameter, the magnitude its gradient is computed from: the sum of
    the magnitudes of every term that enters it, carried through the whole
    backward chain. A dot product evaluated in floating point is off by a
    small multiple of the unit roundoff times the sum of the magnitudes of its
    terms, not of its value; when an upstream sum such as dh1 = bf(dz2) W2,
    or the residual y - target, cancels, its absolute error is that of the
    magnitudes, and it reaches every gradient computed from it. So the
    magnitudes are propagated, starting from those of the residual:
        Sy = 2 m / M (sum_j |bf(h3_j) bf(w4_j)| + |b4| + |target|),
        S3 = Sy |bf(w4)| |gelu'(z3)|,  S2 = (S3 |bf(W3)|) |gelu'(z2)|,
        S1 = (S2 |bf(W2)|) |gelu'(z1)|,
    and a weight's scale is S_k^T |bf(h_{k-1})| (|bf(x)| for W1, |bf(h3)|
    with Sy for w4), a bias's sum_r S_k. Element-wise tolerances of the GPU
    gradient are stated relative to this scale."""
    y, c = forward(theta, x)
    t = np.asarray(target, dtype=np.float64)
    m = np.ones_like(t) if mask is None else np.asarray(mask, dtype=np.float64)
    M = m.sum()
    if M == 0:
        return np.zeros(N_PARAMS)
    P, r = c["P"], c["r"]
    a = np.abs
    sy = 2.0 * m / M * (a(r(c["h3"])) @ a(r(P["w4"])) + abs(P["b4"][0]) + a(t))
    g = {}
    g["w4"] = sy @ a(r(c["h3"]))
    g["b4"] = np.array([sy.sum()])
    s3 = np.outer(sy, a(r(P["w4"]))) * a(gelu_grad(c["z3"]))
    g["W3"] = s3.T @ a(r(c["h2"]))
    g["b3"] = s3.sum(axis=0)
    s2 = (s3 @ a(r(P["W3"]))) * a(gelu_grad(c["z2"]))
    g["W2"] = s2.T @ a(r(c["h1"]))
    g["b2"] = s2.sum(axis=0)
    s1 = (s2 @ a(r(P["W2"]))) * a(gelu_grad(c["z1"]))
    g["W1"] = s1.T @ a(c["xb"])
    g["b1"] = s1.sum(axis=0)
    return pack(g)


class Adam:
    """Adam (Kingma & Ba): m, v moments with bias correction."""

    def __init__(self, n, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, theta, grad):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * grad
        self.v = self.b2 * self.v + (1 - self.b2) * grad * grad
        mhat = self.m / (1 - self.b1 ** self.t)
        vhat = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)


def init_params(seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shape in SIZES:
        fan_in = {"W1": 3, "b1": 3, "W2": H, "b2": H, "W3": H, "b3": H, "w4": H, "b4": H}[name]
        bound = 1.0 / math.sqrt(fan_in)
        parts[name] = rng.uniform(-bound, bound, size=shape)
    return pack(parts)


def features(p, d, t):
    """Network inputs of (p, d, t): ((p - 0.16) / 0.07, d, log10(t) / 6)."""
    p, d, t = np.broadcast_arrays(np.asarray(p, float), np.asarray(d, float), np.asarray(t, float))
    return np.stack([(p - 0.16) / 0.07, d, np.log10(t) / 6.0], axis=-1)
