"""Rounding model of the reduced-precision (FP16/BF16) forms, for tests only.

The FP64 oracle defines what the cache computes.  The matrix-core forms round
at fixed points: the weights and every activation and backward delta are
stored in FP16/BF16 (round to nearest even), products accumulate in FP32, the
loss gradient is scaled before rounding and unscaled after the weight-gradient
sum.  This model evaluates the method in float64 with exactly those rounding
points, so the distance between the GPU and this model measures the kernels'
own arithmetic (accumulation order only), while the distance between this
model and the oracle is the precision loss the format itself causes.
"""
import numpy as np
import torch

import synthdata as sd


def quantiser(prec):
    if prec == "fp16":
        return lambda x: np.asarray(x, np.float32).astype(np.float16).astype(np.float64)
    if prec == "bf16":
        return lambda x: torch.from_numpy(np.ascontiguousarray(np.asarray(x, np.float32))).bfloat16().float().numpy().astype(np.float64)
    return lambda x: np.asarray(x, np.float64)


def train_weight_quantiser(prec):
    """Weights as the training kernels see them: the BF16 form takes each weight
    as the pair hi = bf16(w), lo = bf16(w - hi) (two products per weight
    operand), FP16 as one FP16 value."""
    q = quantiser(prec)
    if prec != "bf16":
        return q

    def split(m):
        m32 = np.asarray(m, np.float32)
        hi = q(m32)
        lo = q((m32 - hi.astype(np.float32)).astype(np.float32))
        return hi + lo
    return split


def forward(mats, x, q, qw=None):
    """qw: how the weights are rounded (default: like the activations)."""
    h = q(x)
    hs = [h]
    qm = [(qw or q)(m) for m in mats]
    for l, w in enumerate(qm):
        z = h @ w.T
        if l == len(qm) - 1:
            return z, hs, qm
        h = q(np.maximum(z, 0.0))
        hs.append(h)


def backward(qm, hs, d_out, q):
    grads = [None] * len(qm)
    d = q(d_out)
    for l in range(len(qm) - 1, -1, -1):
        grads[l] = d.T @ hs[l]
        g = d @ qm[l]
        if l == 0:
            return grads, g
        d = q(g * (hs[l] > 0.0))


def factor(x, fcol):
    """Reflectance factor of the encoded rows x (values as stored), in FP32
    arithmetic like the kernels; 1 when fcol is None."""
    if fcol is None:
        return 1.0
    x32 = np.asarray(x, np.float32)
    return (x32[:, fcol:fcol + 3] + x32[:, fcol + 3:fcol + 6]).astype(np.float64)


class TrainModel:
    """FP32 master weights and Adam state, reduced-precision network arithmetic.
    fcol: first albedo column of the reflectance factorisation, or None."""

    def __init__(self, w, prec, width=64, n_hidden=5, loss_scale=128.0, lr=1e-2, b1=0.9, b2=0.99,
                 eps=1e-8, loss_eps=0.01, fcol=None):
        self.fcol = fcol
        self.w = np.asarray(w, np.float32).copy()
        self.m = np.zeros_like(self.w)
        self.v = np.zeros_like(self.w)
        self.t = 0
        self.q = quantiser(prec)
        self.qw = train_weight_quantiser(prec)
        self.width, self.n_hidden = width, n_hidden
        self.scale, self.lr, self.b1, self.b2, self.eps, self.loss_eps = loss_scale, lr, b1, b2, eps, loss_eps

    def mats(self):
        return [m.astype(np.float64) for m in sd.split_weights(self.w, self.width, self.n_hidden)]

    def predict(self, x):
        return forward(self.mats(), x, self.q)[0] * factor(x, self.fcol)

    def step(self, x, y):
        n = x.shape[0]
        z, hs, qm = forward(self.mats(), x, self.q, self.qw)
        r = factor(x, self.fcol)
        z = z * r
        lum = z.mean(axis=1, keepdims=True)
        den = lum * lum + self.loss_eps
        diff = z - y
        loss = float((diff * diff / den).sum() / (3 * n))
        d_out = 2.0 * diff / den * (self.scale / (3 * n)) * r
        grads, _ = backward(qm, hs, d_out, self.q)
        g = (np.concatenate([gg.reshape(-1) for gg in grads]) / self.scale).astype(np.float32)
        self.t += 1
        f = np.float32
        self.m = (f(self.b1) * self.m + f(1 - self.b1) * g).astype(np.float32)
        self.v = (f(self.b2) * self.v + f(1 - self.b2) * g * g).astype(np.float32)
        mh = self.m / f(1 - self.b1 ** self.t)
        vh = self.v / f(1 - self.b2 ** self.t)
        self.w = (self.w - f(self.lr) * mh / (np.sqrt(vh) + f(self.eps))).astype(np.float32)
        return loss


GAMMA_64 = 64 * 2.0 ** -24 / (1 - 64 * 2.0 ** -24)   # gamma_K of a K = 64 FP32 dot product


def relu_undecided_rows(mats, x, rel=GAMMA_64):
    """Records whose ReLU masks FP32 arithmetic does not decide: some hidden
    pre-activation z lies within rel * sum |w h| of zero.  The default is the
    standard bound on the rounding error of an FP32 dot product of K = 64
    terms, |fl(w.h) - w.h| <= gamma_K sum |w h| with gamma_K = K u / (1 - K u),
    u = 2^-24 (Higham, Accuracy and Stability of Numerical Algorithms, 3.1).
    ReLU' is a step at zero, so for such a unit the sign, and with it the
    whole backward contribution through it, depends on summation order; the
    FP64 oracle's choice is no more right than the kernel's.  Returns a
    boolean mask over the records."""
    h = np.asarray(x, np.float64)
    undecided = np.zeros(h.shape[0], bool)
    for w in mats[:-1]:
        z = h @ w.T
        undecided |= np.any(np.abs(z) <= rel * (np.abs(h) @ np.abs(w).T), axis=1)
        h = np.maximum(z, 0.0)
    return undecided
