"""Pins of the FP64 reference of the learned start solution (oracle/mlp.py)
against facts that do not come from its own code: finite differences, a
network with a closed-form output, Adam's behaviour under a constant
gradient, brute-force stencils, and invariants of departure coefficients."""
import numpy as np
import pytest

from oracle import mlp as OM
from oracle import oracle as O
from paper_1411_1079_amd import synth

import conftest


def test_gradient_matches_central_differences():
    """Every parameter's derivative of the loss against a central difference
    of the loss (step 1e-6): a dropped term, a wrong sign or a transposed
    factor in the backward pass fails here."""
    dims = OM.dims_of(5, 2, 3)
    p = synth.mlp_params(dims, seed=3, weight_scale=1.5, bias_std=0.3).astype(np.float64)
    x = synth.mlp_features(4, 7).astype(np.float64)
    mean, std = OM.normalization(x)
    t = np.random.default_rng(5).normal(size=(7, 3))
    _, g = OM.loss_and_grad(p, dims, mean, std, x, t)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        lp = np.mean((OM.forward(p + e, dims, mean, std, x) - t) ** 2)
        lm = np.mean((OM.forward(p - e, dims, mean, std, x) - t) ** 2)
        fd[i] = (lp - lm) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9 * np.abs(g).max())


def test_network_with_closed_form_output():
    """silu(x) - silu(-x) = x: one hidden layer of units +x, -x per output
    and output weights +1, -1 reproduce the chosen normalised inputs
    exactly, which pins the weight layout [fan_in][fan_out], the bias
    placement and the normalisation."""
    dims = OM.dims_of(4, 1, 2)
    W1 = np.zeros((36, 4))
    W1[3, 0], W1[3, 1] = 1.0, -1.0      # feature 3 -> units 0, 1
    W1[17, 2], W1[17, 3] = 1.0, -1.0    # feature 17 -> units 2, 3
    b1 = np.zeros(4)
    W2 = np.zeros((4, 2))
    W2[0, 0], W2[1, 0], W2[2, 1], W2[3, 1] = 1.0, -1.0, 1.0, -1.0
    b2 = np.array([0.25, -2.0])
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2])
    x = synth.mlp_features(1, 50).astype(np.float64)
    mean, std = OM.normalization(x)
    y = OM.forward(p, dims, mean, std, x)
    np.testing.assert_allclose(y[:, 0], (x[:, 3] - mean[3]) / std[3] + 0.25, rtol=0, atol=1e-13)
    np.testing.assert_allclose(y[:, 1], (x[:, 17] - mean[17]) / std[17] - 2.0, rtol=0, atol=1e-13)


def test_silu_values():
    assert OM.silu(0.0) == 0.0
    np.testing.assert_allclose(OM.silu(np.log(3.0)), np.log(3.0) * 0.75, rtol=1e-15)   # sigmoid(ln 3) = 3/4
    assert OM.silu_prime(0.0) == 0.5
    z = np.linspace(-8, 8, 33)
    np.testing.assert_allclose(OM.silu_prime(z), (OM.silu(z + 1e-6) - OM.silu(z - 1e-6)) / 2e-6, rtol=1e-8, atol=1e-10)


def test_adam_constant_gradient_steps_are_lr():
    """With a constant gradient the bias-corrected moments equal g and g^2
    at every step, so each step moves a parameter by lr g / (|g| + eps)."""
    n = 6
    g = np.array([3.0, -0.5, 1e-3, -2e2, 1e-6, 0.0])
    a = OM.Adam(n)
    w = np.zeros(n)
    for step in range(1, 40):
        lr = 1e-2 / step
        w2 = a.step(w, g, lr)
        np.testing.assert_allclose(w2 - w, -lr * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-18)
        w = w2


def test_adam_minimises_a_quadratic():
    a = OM.Adam(3)
    w = np.array([5.0, -3.0, 0.1])
    c = np.array([1.0, 2.0, -1.0])
    for s in range(3000):
        w = a.step(w, 2 * (w - c), 0.05 * 0.5 * (1 + np.cos(np.pi * s / 3000)))
    np.testing.assert_allclose(w, c, atol=1e-3)


def test_stencil_features_brute_force():
    """Clamped 9-point stencil (offsets 0, +-2, +-8, +-32, +-128) over ragged
    columns, including a column of one point, against a plain loop."""
    lens = [1, 5, 140, 3, 300]
    off = np.concatenate([[0], np.cumsum(lens)])
    P = off[-1]
    rng = np.random.default_rng(0)
    T = rng.uniform(3e3, 1e4, P)
    ne = rng.uniform(1e9, 1e13, P)
    nH = rng.uniform(1e12, 1e17, P)
    vz = rng.uniform(-1e4, 1e4, P)
    f = OM.features(off, T, ne, nH, vz)
    for c in range(len(lens)):
        for k in range(lens[c]):
            row = []
            for d in (-128, -32, -8, -2, 0, 2, 8, 32, 128):
                q = off[c] + min(max(k + d, 0), lens[c] - 1)
                row += [np.log(T[q]), np.log(ne[q]), np.log(nH[q]), vz[q] / 1e4]
            np.testing.assert_allclose(f[off[c] + k], row, rtol=1e-15, atol=0)
    s = np.array([5, 0, 140, 6, 400, 448])
    np.testing.assert_array_equal(OM.features(off, T, ne, nH, vz, samples=s), f[s])


def test_departure_invariants(atom_dir):
    """LTE populations have zero departures; departures shifted by a
    constant give the same populations (the renormalisation); populations
    -> departures -> populations is the identity."""
    a = O.Atom(atom_dir["h6"])
    col = synth.cfg2_columns(seed=1, n_columns=1).column(0)
    T, ne, nH = col["T"][:10], col["n_e"][:10], col["n_H"][:10]
    lte = np.array([a.lte(T[k], ne[k], a.abundance * nH[k]) for k in range(10)])
    np.testing.assert_allclose(OM.departures(a, T, ne, nH, lte), 0.0, atol=1e-12)
    lb = np.random.default_rng(1).normal(0, 2, (10, a.n_levels))
    p1 = OM.pops_from_departures(a, T, ne, nH, lb)
    np.testing.assert_allclose(p1.sum(axis=1), a.abundance * nH, rtol=1e-13)
    np.testing.assert_allclose(OM.pops_from_departures(a, T, ne, nH, lb + 3.7), p1, rtol=1e-12)
    np.testing.assert_allclose(OM.pops_from_departures(a, T, ne, nH, OM.departures(a, T, ne, nH, p1)), p1,
                               rtol=1e-12)
    # shrinking: a shrink above every |ln b| gives LTE; a shrink s on values
    # all beyond s is the same as subtracting s from the magnitudes
    np.testing.assert_allclose(OM.pops_from_departures(a, T, ne, nH, lb, shrink=100.0), lte, rtol=1e-12)
    big = np.where(lb >= 0, lb + 1.0, lb - 1.0)
    np.testing.assert_allclose(OM.pops_from_departures(a, T, ne, nH, big, shrink=0.75),
                               OM.pops_from_departures(a, T, ne, nH, np.where(lb >= 0, lb + 0.25, lb - 0.25)),
                               rtol=1e-12)
