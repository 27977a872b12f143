"""Plain FP64 NumPy reference of the learned start solution.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this module; the product never
does.

The paper (Sec. 2.3) shows that the choice of start populations decides how
many iterations the accelerated Lambda iteration needs.  The learned start
is a multilayer perceptron from the local thermodynamic stencil of a depth
point to the natural-log departure coefficients ln(n_i / n*_i) of its
levels; the iteration itself is unchanged.  Everything here is written from
the definitions, in float64, without blocking or fusion:

* features: for depth index k of a column, the nine points k + d for d in
  STENCIL (clamped to the column, i.e. the end values repeated) each give
  ln T, ln n_e, ln n_H and v_z / (10 km/s); 36 numbers in that order
  (point-major);
* the network: z-scored features, n_layers hidden layers of SiLU units
  (silu(z) = z / (1 + e^-z)), a linear output layer; each layer is
  y = x W + b with W stored [fan_in][fan_out];
* the loss: mean over samples and outputs of the squared error;
* the gradient: reverse-mode differentiation of that loss (chain rule,
  layer by layer);
* Adam (Kingma & Ba 2015): first and second moment averages with bias
  correction;
* departure coefficients: against the Saha-Boltzmann populations that the
  FP64 MALI oracle computes.
"""
from __future__ import annotations

import numpy as np

STENCIL = (-128, -32, -8, -2, 0, 2, 8, 32, 128)
N_STENCIL = len(STENCIL)
N_FEATURES = 4 * N_STENCIL


def dims_of(n_hidden: int, n_layers: int, n_out: int) -> list[int]:
    return [N_FEATURES] + [n_hidden] * n_layers + [n_out]


def unpack(params: np.ndarray, dims: list[int]):
    """Flat parameter vector -> [(W [fan_in][fan_out], b [fan_out]), ...]."""
    out, o = [], 0
    for fi, fo in zip(dims[:-1], dims[1:]):
        W = params[o:o + fi * fo].reshape(fi, fo)
        o += fi * fo
        b = params[o:o + fo]
        o += fo
        out.append((W, b))
    assert o == params.size, (o, params.size)
    return out


def n_params(dims: list[int]) -> int:
    return sum(fi * fo + fo for fi, fo in zip(dims[:-1], dims[1:]))


def features(offset: np.ndarray, T, n_e, n_H, v_z, samples=None) -> np.ndarray:
    """Stencil features of the points `samples` (global depth indices; all
    points if None) of ragged columns with depth offsets `offset`."""
    offset = np.asarray(offset, dtype=np.int64)
    total = int(offset[-1])
    g = np.arange(total, dtype=np.int64) if samples is None else np.asarray(samples, dtype=np.int64)
    col = np.searchsorted(offset, g, side="right") - 1
    lo, hi = offset[col], offset[col + 1] - 1
    out = np.empty((g.size, N_FEATURES), dtype=np.float64)
    for j, d in enumerate(STENCIL):
        q = np.clip(g + d, lo, hi)
        out[:, 4 * j + 0] = np.log(np.asarray(T, np.float64)[q])
        out[:, 4 * j + 1] = np.log(np.asarray(n_e, np.float64)[q])
        out[:, 4 * j + 2] = np.log(np.asarray(n_H, np.float64)[q])
        out[:, 4 * j + 3] = np.asarray(v_z, np.float64)[q] * 1e-4
    return out


def normalization(x: np.ndarray, floor: float = 1e-6):
    """Per-feature mean and (population) standard deviation."""
    mean = x.mean(axis=0)
    std = np.sqrt(np.maximum(x.var(axis=0), floor * floor))
    return mean, std


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_prime(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, dims, mean, std, x, keep=False):
    """Network output for raw features x [n][36]; with keep=True also the
    per-layer inputs and pre-activations for the backward pass."""
    h = (np.asarray(x, np.float64) - mean) / std
    layers = unpack(np.asarray(params, np.float64), dims)
    ins, zs = [], []
    for li, (W, b) in enumerate(layers):
        ins.append(h)
        z = h @ W + b
        zs.append(z)
        h = z if li == len(layers) - 1 else silu(z)
    return (h, ins, zs) if keep else h


def loss_and_grad(params, dims, mean, std, x, target):
    """Mean squared error and its gradient with respect to the flat
    parameter vector (same layout as the parameters)."""
    y, ins, zs = forward(params, dims, mean, std, x, keep=True)
    n, m = y.shape
    r = y - target
    loss = float(np.mean(r * r))
    d = 2.0 * r / (n * m)            # dL/dy
    layers = unpack(np.asarray(params, np.float64), dims)
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        if li < len(layers) - 1:
            d = d * silu_prime(zs[li])    # through the activation
        grads.append((ins[li].T @ d, d.sum(axis=0)))
        d = d @ W.T                      # to the layer's input
    flat = []
    for gW, gb in reversed(grads):
        flat += [gW.ravel(), gb]
    return loss, np.concatenate(flat)


class Adam:
    """Adam with bias correction (beta1 0.9, beta2 0.999, eps 1e-8)."""

    def __init__(self, n, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.b1, self.b2, self.eps = b1, b2, eps

    def step(self, params, grad, lr):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * grad
        self.v = self.b2 * self.v + (1 - self.b2) * grad * grad
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return params - lr * mh / (np.sqrt(vh) + self.eps)


def departures(atom, T, n_e, n_H, pops) -> np.ndarray:
    """ln(n_i / n*_i) with n* the oracle's Saha-Boltzmann populations for the
    point's total population of the element (abundance x n_H)."""
    out = np.empty_like(np.asarray(pops, np.float64))
    for k in range(out.shape[0]):
        star = atom.lte(float(T[k]), float(n_e[k]), atom.abundance * float(n_H[k]))
        out[k] = np.log(pops[k] / star)
    return out


def pops_from_departures(atom, T, n_e, n_H, log_b, shrink=0.0) -> np.ndarray:
    """n_i proportional to exp(l_i) n*_i, scaled so the levels of the point
    sum to its total population; l_i = log_b_i moved toward 0 by `shrink`
    (soft thresholding: sign(x) max(|x| - shrink, 0))."""
    out = np.empty(np.shape(log_b), dtype=np.float64)
    for k in range(out.shape[0]):
        ntot = atom.abundance * float(n_H[k])
        star = atom.lte(float(T[k]), float(n_e[k]), ntot)
        x = np.asarray(log_b[k], np.float64)
        l = np.sign(x) * np.maximum(np.abs(x) - shrink, 0.0)
        n = np.exp(l) * star
        out[k] = n * (ntot / n.sum())
    return out
