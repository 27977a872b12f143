"""Pins of the oracle's grid optimisation (Sec. 2.3, "Grid optimisation":
more depth points where temperature, velocity or optical depth change
fast), CPU only."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1411_1079_amd import synth


def _linear_column(z):
    """ln T, v_z and v_turb linear in z, n_e and n_H exponential in z: every
    interval's length is proportional to its height difference."""
    H = z[0] - z[-1]
    s = (z[0] - z) / H
    return dict(z=z, T=np.exp(np.log(4000.0) + 1.2 * s), n_e=1e17 * np.exp(3.0 * s), n_H=1e20 * np.exp(3.0 * s),
                v_z=2e3 - 6e3 * s, v_turb=1e3 + 500.0 * s)


@pytest.mark.parametrize("n_out", [2, 17, 64, 200])
def test_linear_atmosphere_gives_uniform_grid(atom_dir, n_out):
    """Without a background (no optical-depth term) and with every variable
    linear (or log-linear) in z, the length of an interval is proportional
    to its height difference, so the new grid is uniform in z whatever the
    input spacing, and the interpolation reproduces the variables exactly."""
    a = O.Atom(atom_dir["two_level"])
    rng = np.random.default_rng(0)
    z = np.sort(rng.uniform(0.0, 2.0e6, 50))[::-1].copy()
    z[0], z[-1] = 2.0e6, 0.0
    col = _linear_column(z)
    out = O.optimize_grid(a, col, n_out)
    zu = np.linspace(2.0e6, 0.0, n_out)
    np.testing.assert_allclose(out["z"], zu, rtol=0, atol=1e-9 * 2.0e6)
    ref = _linear_column(zu)
    for k in ("T", "n_e", "n_H", "v_z", "v_turb"):
        np.testing.assert_allclose(out[k], ref[k], rtol=1e-11, atol=1e-9, err_msg=k)


def test_points_gather_where_the_temperature_jumps(atom_dir):
    """A transition-region-like jump of T by a factor 10 over 2 % of the
    height draws a large share of the points, in proportion to its share of
    the total length; end points are kept and z stays strictly decreasing."""
    a = O.Atom(atom_dir["two_level"])
    z = np.linspace(2.0e6, 0.0, 400)
    s = (z[0] - z) / 2.0e6
    T = 6000.0 * np.where(s < 0.49, 10.0, np.where(s > 0.51, 1.0, 10.0 ** (1 - (s - 0.49) / 0.02)))
    col = dict(z=z, T=T, n_e=np.full(400, 1e17), n_H=np.full(400, 1e20), v_z=np.zeros(400), v_turb=np.full(400, 1e3))
    w = (1.0, 2.0, 0.0, 0.0)
    out = O.optimize_grid(a, col, 100, weights=w)
    assert out["z"][0] == z[0] and out["z"][-1] == z[-1] and np.all(np.diff(out["z"]) < 0)
    # the jump's length (about 2 ln 10) against about 1 for the height: some
    # 80 % of the points within it (one input interval of margin each side),
    # spaced some 50 times more densely than elsewhere
    h = 2.0e6 / 399
    win = (out["z"] < 2.0e6 * (1 - 0.49) + h) & (out["z"] > 2.0e6 * (1 - 0.51) - h)
    inside = int(np.sum(win))
    assert 0.75 * 99 <= inside <= 0.85 * 99, inside
    dz = -np.diff(out["z"])
    assert np.median(dz[win[1:] & win[:-1]]) * 20 < np.median(dz[~(win[1:] | win[:-1])])


def test_optical_depth_term_and_background(atom_dir):
    """With the background law, points follow log optical depth: on an
    exponential atmosphere without T or v structure (w_T = w_v = 0) the
    increments of ln(tau + 1e-5) between new points are equal where the
    height term is negligible."""
    a = O.Atom(atom_dir["h6"])
    z = np.linspace(2.0e6, 0.0, 300)
    nH = 1e23 * np.exp(-z / 1.5e5)
    col = dict(z=z, T=np.full(300, 6000.0), n_e=1e-4 * nH, n_H=nH, v_z=np.zeros(300), v_turb=np.full(300, 1e3))
    out = O.optimize_grid(a, col, 60, weights=(1e-6, 0.0, 0.0, 1.0))
    # tau of the new grid from the same law (dense trapezoid on the fine input grid)
    cbg = synth.hminus_calibration()
    k = cbg * nH * (1e-4 * nH) * 6000.0 ** -1.5 * np.exp(8750.0 / 6000.0)
    tau = np.concatenate([[0.0], np.cumsum(0.5 * (k[1:] + k[:-1]) * (z[:-1] - z[1:]))])
    lt = np.log(tau + 1e-5)
    lt_new = np.interp(-out["z"], -z, lt)
    steps = np.diff(lt_new)
    assert np.std(steps) < 0.02 * np.mean(steps)


def test_three_point_hand_case(atom_dir):
    """Hand-worked case: three points, heights 2, 1, 0 (in units of 1e6 m),
    T = 5000, 5000 e^(3/2), same, and only w_z = 1, w_T = 2: the two
    intervals have lengths sqrt(1/4 + 9) and 1/2, so a fourth of the way
    along (total length L) lies inside the first interval at the fraction
    L/4 / sqrt(37)/2 of it."""
    a = O.Atom(atom_dir["two_level"])
    z = np.array([2.0e6, 1.0e6, 0.0])
    T = np.array([5000.0, 5000.0 * np.exp(1.5), 5000.0 * np.exp(1.5)])
    col = dict(z=z, T=T, n_e=np.array([1e17, 4e17, 4e17]), n_H=np.full(3, 1e20), v_z=np.array([0.0, 100.0, 300.0]),
               v_turb=np.full(3, 1e3))
    out = O.optimize_grid(a, col, 5, weights=(1.0, 2.0, 0.0, 0.0))
    d1, d2 = np.sqrt(0.25 + 9.0), 0.5
    L = d1 + d2
    for j, frac in enumerate([0.0, 0.25, 0.5, 0.75, 1.0]):
        t = frac * L
        if t <= d1:
            f = t / d1
            ze, lT, lne, ve = 2.0e6 - 1.0e6 * f, np.log(5000.0) + 1.5 * f, np.log(1e17) + np.log(4.0) * f, 100.0 * f
        else:
            f = (t - d1) / d2
            ze, lT, lne, ve = 1.0e6 - 1.0e6 * f, np.log(5000.0) + 1.5, np.log(4e17), 100.0 + 200.0 * f
        assert out["z"][j] == pytest.approx(ze, rel=1e-13, abs=1e-7)
        assert out["T"][j] == pytest.approx(np.exp(lT), rel=1e-13)
        assert out["n_e"][j] == pytest.approx(np.exp(lne), rel=1e-13)
        assert out["v_z"][j] == pytest.approx(ve, rel=1e-13, abs=1e-10)


@pytest.mark.parametrize("case", ["zero_weights", "negative_weight", "z_not_decreasing", "T_zero", "one_point"])
def test_invalid_input_is_an_error(atom_dir, case):
    a = O.Atom(atom_dir["two_level"])
    z = np.linspace(2.0e6, 0.0, 10)
    col = dict(z=z, T=np.full(10, 5000.0), n_e=np.full(10, 1e17), n_H=np.full(10, 1e20), v_z=np.zeros(10),
               v_turb=np.full(10, 1e3))
    w = (1.0, 2.0, 0.0, 0.0)
    n_out = 8
    if case == "zero_weights":
        w = (0.0, 0.0, 0.0, 0.0)
    elif case == "negative_weight":
        w = (1.0, -1.0, 0.0, 0.0)
    elif case == "z_not_decreasing":
        col["z"] = z.copy()
        col["z"][4] = col["z"][3]
    elif case == "T_zero":
        col["T"] = col["T"].copy()
        col["T"][2] = 0.0
    else:
        n_out = 1
    with pytest.raises(ValueError):
        O.optimize_grid(a, col, n_out, weights=w)
