"""Pins of the oracle's partial frequency redistribution (Sec. 2.1:
angle-averaged PRD after Uitenbroek 2001; Sec. 2.3: PRD switching, Eq. 1)
against what the mathematics fixes (CPU only)."""
import math

import numpy as np
import pytest
from scipy.special import erfc, wofz

from oracle import oracle as O
from paper_1411_1079_amd import synth

import brute
import conftest


# --------------------------------------------------------------------------
# the redistribution function
# --------------------------------------------------------------------------
@pytest.mark.parametrize("a", [1e-3, 1e-2, 0.1])
def test_rII_against_hummer_integral(a):
    """The oracle's quadrature of the Lorentzian-averaged form against
    Hummer's (1962) defining integral (adaptive quadrature), core and wing
    pairs, both signs."""
    pairs = [(0.0, 0.0), (0.3, -0.2), (1.0, 1.4), (-2.0, 2.5), (3.0, 3.3), (0.5, 4.0), (8.0, 8.5), (-20.0, -21.0),
             (50.0, 50.0), (100.0, 104.0), (30.0, -30.0), (5.0, 15.0)]
    for x, x2 in pairs:
        ref = brute.Problem.hummer_rII(a, x, x2)
        got = O.rII(a, x, x2)
        scale = max(brute.Problem.hummer_rII(a, x, x), brute.Problem.hummer_rII(a, x2, x2))
        assert abs(got - ref) <= 1e-4 * scale, (a, x, x2, got, ref)
    # a mistake in the kernel's sign convention (|x| for x) is far outside that
    ref = brute.Problem.hummer_rII(a, 0.3, -0.2)
    assert abs(brute.Problem.hummer_rII(a, 0.3, 0.2) - ref) > 1e-3 * ref


def test_rII_symmetries_and_zero_damping_limit():
    """R(x, x2) = R(x2, x) = R(-x, -x2); for a -> 0 it tends to the
    coherent Doppler kernel (1/2) erfc(max(|x|, |x2|)) (checked at a = 1e-4
    in the Doppler core, to 1e-3 of the row's diagonal)."""
    rng = np.random.default_rng(0)
    for x, x2 in rng.uniform(-6, 6, size=(40, 2)):
        r = O.rII(0.03, x, x2)
        assert O.rII(0.03, x2, x) == pytest.approx(r, rel=1e-13, abs=1e-300)
        assert O.rII(0.03, -x, -x2) == pytest.approx(r, rel=1e-12, abs=1e-300)
    for x, x2 in rng.uniform(-1.5, 1.5, size=(40, 2)):
        row = 0.5 * erfc(min(abs(x), abs(x2)))
        assert abs(O.rII(1e-4, x, x2) - 0.5 * erfc(max(abs(x), abs(x2)))) < 1e-3 * row


@pytest.mark.parametrize("a,x", [(1e-3, 0.0), (1e-3, 2.0), (1e-2, 5.0), (0.05, 1.0), (0.05, 12.0)])
def test_rII_marginal_is_the_voigt_profile(a, x):
    """Integral over x2 of R_II(x, x2) = H(a, x) / sqrt(pi) (Faddeeva
    function): dense trapezoid over the support |x2 - x| < 12."""
    x2 = np.concatenate([np.linspace(x - 12, x - 0.02, 6000), np.linspace(x - 0.02, x + 0.02, 2001),
                         np.linspace(x + 0.02, x + 12, 6000)])
    x2 = np.unique(x2)
    vals = np.array([O.rII(a, x, v) for v in x2])
    integ = np.trapezoid(vals, x2)
    ref = wofz(complex(x, a)).real / math.sqrt(math.pi)
    assert integ == pytest.approx(ref, rel=2e-4)


# --------------------------------------------------------------------------
# the rho update
# --------------------------------------------------------------------------
def test_constant_radiation_field_gives_rho_one(atom_dir):
    """An isotropic, frequency-independent radiation field is redistributed
    into itself: rho = 1 at every depth and frequency, for any populations
    and any switching factor."""
    a = O.Atom(atom_dir["ca2"])
    col = synth.cfg2_columns(seed=0, n_columns=1, n_depth=12).column(0)
    nstar = np.array([a.lte(col["T"][k], col["n_e"][k], a.abundance * col["n_H"][k]) for k in range(12)])
    pops = nstar * np.linspace(0.5, 2.0, a.n_levels)[None, :]
    for eps0, it in ((0.0, 1), (1e-2, 3)):
        rho = O.prd_rho_constant_field(a, col, 3, pops, 1e-9, (0, 1), eps0=eps0, it=it)
        for r in rho:
            np.testing.assert_allclose(r, 1.0, rtol=1e-12)


def test_switching_off_and_full_coherence_loss_give_crd(atom_dir):
    """eps = 0 (PRD switching at its start) and gamma = 0 (elastic
    collisions destroy all coherence) both leave rho = 1: the PRD solve
    equals the CRD solve of the same atom."""
    kw = dict(n_mu=3, tol=1e-9, max_iter=60)
    col = conftest.tiny_column(8)
    cs = dict(coll_scale=1e-2)
    crd = O.solve_column(O.Atom(atom_dir["prd_tiny_crd"]), col, **kw, **cs)
    sw = O.solve_column(O.Atom(atom_dir["prd_tiny"]), col, prd=1, prd_lines=(0,), prd_eps0=1e-300, **kw, **cs)
    # rho = 1 up to the rounding of its normalisation, which the iteration amplifies
    assert sw["n_iter"] == crd["n_iter"]
    np.testing.assert_allclose(sw["pops"], crd["pops"], rtol=1e-9)
    np.testing.assert_allclose(sw["spectrum"], crd["spectrum"], rtol=1e-9)
    crd0 = O.solve_column(O.Atom(atom_dir["prd_tiny_gamma0_crd"]), col, **kw, **cs)
    g0 = O.solve_column(O.Atom(atom_dir["prd_tiny_gamma0"]), col, prd=1, prd_lines=(0,), **kw, **cs)
    np.testing.assert_allclose(g0["pops"], crd0["pops"], rtol=1e-9)
    np.testing.assert_allclose(g0["spectrum"], crd0["spectrum"], rtol=1e-9)
    # and PRD does matter on this atom
    full = O.solve_column(O.Atom(atom_dir["prd_tiny"]), col, prd=1, prd_lines=(0,), **kw, **cs)
    assert np.max(np.abs(full["spectrum"] / crd["spectrum"] - 1)) > 1e-2


def test_fixed_point_does_not_depend_on_switching(atom_dir):
    """PRD switching changes the path, not the answer (both runs converged
    to 1e-11; the PRD iteration contracts by about 0.98 per step here, so
    the remaining distance is about 5e-10)."""
    a = O.Atom(atom_dir["prd_tiny"])
    col = conftest.tiny_column(6)
    kw = dict(n_mu=3, tol=1e-11, max_iter=6000, coll_scale=1e-2, prd=1, prd_lines=(0,))
    r0 = O.solve_column(a, col, **kw)
    r1 = O.solve_column(a, col, prd_eps0=1e-2, **kw)
    assert r0["status"] == 0 and r1["status"] == 0 and r1["n_iter"] != r0["n_iter"]
    np.testing.assert_allclose(r1["pops"], r0["pops"], rtol=1e-8)
    np.testing.assert_allclose(r1["rho"][0], r0["rho"][0], rtol=1e-8)


def test_prd_fixed_point_against_brute_force(atom_dir):
    """The converged PRD solution is a fixed point of the exact problem:
    with the oracle's populations and rho, the exact radiation field
    (explicit Lambda matrices) and Hummer's R_II by adaptive quadrature
    reproduce rho, and the full rate equations (classical Lambda iteration)
    reproduce the populations.  The brute force uses the exact Faddeeva
    profile where the oracle uses Humlicek W4 (about 1e-4), which bounds the
    agreement at a few 1e-6 (the same holds with PRD off)."""
    a, b = O.Atom(atom_dir["prd_tiny"]), brute.BAtom(atom_dir["prd_tiny"])
    col = conftest.tiny_column(6)
    cs = 1e-2
    r = O.solve_column(a, col, n_mu=3, tol=1e-11, max_iter=8000, coll_scale=cs, prd=1, prd_lines=(0,))
    assert r["status"] == 0
    P = brute.Problem(b, col, 3, coll_scale=cs)
    P.rho = {0: r["rho"][0]}
    rho = P.prd_rho(r["pops"])
    assert np.max(np.abs(r["rho"][0] - 1)) > 0.05            # PRD is not CRD here
    np.testing.assert_allclose(rho[0], r["rho"][0], rtol=1e-5)
    n_cl = P.se_solve(P.rate_matrix(r["pops"]), r["pops"])
    np.testing.assert_allclose(n_cl, r["pops"], rtol=1e-5)
    np.testing.assert_allclose(P.emergent(r["pops"]), r["spectrum"], rtol=1e-4)
    # a rho off by a plausible mistake (no normalisation) is far outside that
    P.rho = {0: r["rho"][0] * 1.01}
    assert np.max(np.abs(P.se_solve(P.rate_matrix(r["pops"]), r["pops"]) / r["pops"] - 1)) > 1e-4


def test_two_point_column_stays_finite(atom_dir):
    """A two-point column, where every rho' at the top point can be clamped
    to 0, keeps finite populations (CRD at such a point)."""
    a = O.Atom(atom_dir["prd_tiny"])
    r = O.solve_column(a, conftest.tiny_column(2), n_mu=3, tol=0.0, max_iter=20, coll_scale=1e-2, prd=1,
                       prd_lines=(0,), want_psi=True)
    assert r["status"] == 1 and np.all(np.isfinite(r["pops"])) and np.all(np.isfinite(r["rho"][0]))
    assert np.all(np.isfinite(r["spectrum"])) and np.all(np.isfinite(r["psi_star"]))
