"""Pins of the oracle's collisional-radiative switching (Sec. 2.3; Hummer &
Voels 1988): the switched collisions must not change the answer, only the
path to it.  Checked against what the mathematics fixes: the factor's
schedule, the identity when switching is off, the LTE limit of collision-
dominated statistical equilibrium, the uniqueness of the fixed point, and
no convergence while the collisions are switched."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1411_1079_amd import synth


def test_factor_schedule():
    """f0 / 10^(it-1) while above 1, then 1; off for f0 <= 1."""
    assert [O.crs_factor(1e3, it) for it in range(1, 7)] == [1e3, 1e2, 1e1, 1.0, 1.0, 1.0]
    assert [O.crs_factor(3e4, it) for it in (1, 2, 5, 6)] == [3e4, 3e3, 3.0, 1.0]
    assert O.crs_factor(1.0, 1) == 1.0 and O.crs_factor(0.0, 1) == 1.0 and O.crs_factor(0.5, 4) == 1.0


def test_off_is_bitwise_identity(atom_dir):
    a = O.Atom(atom_dir["h6"])
    col = synth.cfg2_columns(seed=4, n_columns=1).column(0)
    kw = dict(n_mu=3, tol=1e-6, max_iter=60, coll_scale=0.1)
    ref = O.solve_column(a, col, **kw)
    for f0 in (1.0, 0.5):
        r = O.solve_column(a, col, crs_f0=f0, **kw)
        assert r["n_iter"] == ref["n_iter"] and r["status"] == ref["status"]
        np.testing.assert_array_equal(r["pops"], ref["pops"])
        np.testing.assert_array_equal(r["spectrum"], ref["spectrum"])


def test_switched_collisions_reach_lte(atom_dir):
    """With collisions 1e12 times stronger the first iterate's statistical
    equilibrium is collision dominated: the populations are the LTE ones
    (detailed balance of the collisions, to the ratio of radiative to
    switched collisional rates), while without switching the weakly
    collisional upper atmosphere departs from LTE by a factor of e."""
    a = O.Atom(atom_dir["h6"])
    col = synth.cfg2_columns(seed=4, n_columns=1).column(0)
    kw = dict(n_mu=3, tol=0.0, coll_scale=1e-3)
    lte = O.solve_column(a, col, max_iter=0, **kw)["pops"]
    one = O.solve_column(a, col, max_iter=1, crs_f0=1e12, **kw)["pops"]
    free = O.solve_column(a, col, max_iter=1, **kw)["pops"]
    assert np.max(np.abs(one / lte - 1)) < 1e-8
    assert np.max(np.abs(np.log(free / lte))) > 0.5


def test_same_fixed_point_and_no_early_convergence(atom_dir):
    """Converged tightly, the switched and unswitched iterations give the
    same populations and spectrum (the fixed point does not depend on the
    path); the switched one cannot stop before its factor has reached 1."""
    a = O.Atom(atom_dir["h6"])
    for c, col in enumerate(synth.cfg2_columns(seed=9, n_columns=2).column(i) for i in range(2)):
        kw = dict(n_mu=3, tol=1e-11, max_iter=400, coll_scale=0.3)
        ref = O.solve_column(a, col, **kw)
        sw = O.solve_column(a, col, crs_f0=1e4, **kw)
        assert ref["status"] == 0 and sw["status"] == 0
        np.testing.assert_allclose(sw["pops"], ref["pops"], rtol=1e-8)
        np.testing.assert_allclose(sw["spectrum"], ref["spectrum"], rtol=1e-8)
        loose = O.solve_column(a, col, n_mu=3, tol=10.0, max_iter=50, crs_f0=1e4)
        assert loose["status"] == 0 and loose["n_iter"] == 5, loose["n_iter"]
