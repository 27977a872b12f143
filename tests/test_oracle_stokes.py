"""Pins of the oracle's polarised emergent spectrum (Sec. 2.1: Zeeman
splitting and the full Stokes vector), CPU only.

* Wigner 3j symbols against sympy; Zeeman patterns against the textbook
  alkali D-line patterns and the effective Lande factor formula.
* The complex Voigt (Faddeeva) function against scipy's wofz.
* The polarised formal solver: exact for a linear source function without
  polarisation, and converging at second order to the Unno-Rachkovsky
  solution of a Milne-Eddington atmosphere (written from the published
  closed form, magneto-optical terms included).
* A column: zero field gives the unpolarised spectrum; symmetries of the
  field's direction; the weak-field law V = gbar nu_L cos(theta) dI/dnu
  (its sign fixes the convention: V > 0 in the blue wing of an absorption
  line for a field toward the observer); Q of a transverse field grows as
  B^2."""
import numpy as np
import pytest

from oracle import oracle as O

import conftest

E_CHARGE = 1.602176634e-19
M_E = 9.1093837015e-31
C_LIGHT = 2.99792458e8


def larmor(B):
    return E_CHARGE * B / (4.0 * np.pi * M_E)


def gbar(Jl, gl, Ju, gu):
    """Effective Lande factor of a line (the first moment of its Zeeman
    pattern), the textbook formula."""
    return 0.5 * (gu + gl) + 0.25 * (gu - gl) * (Ju * (Ju + 1) - Jl * (Jl + 1))


def test_wigner3j_against_sympy():
    from sympy.physics.wigner import wigner_3j
    rng = np.random.default_rng(0)
    checked = 0
    for _ in range(400):
        tj1, tj2 = rng.integers(0, 9, 2)
        tj3 = rng.integers(abs(tj1 - tj2), tj1 + tj2 + 1)
        if (tj1 + tj2 + tj3) % 2:
            continue
        tm1 = rng.integers(-tj1 // 2, tj1 // 2 + 1) * 2 + (tj1 % 2) if tj1 % 2 == 0 else 2 * rng.integers(-(tj1 // 2) - 1, tj1 // 2 + 1) + 1
        tm2 = rng.integers(-tj2 // 2, tj2 // 2 + 1) * 2 if tj2 % 2 == 0 else 2 * rng.integers(-(tj2 // 2) - 1, tj2 // 2 + 1) + 1
        tm3 = -tm1 - tm2
        args = [x / 2 for x in (tj1, tj2, tj3, tm1, tm2, tm3)]
        ref = float(wigner_3j(*[__import__("sympy").Rational(int(2 * a), 2) for a in args]))
        assert O.wigner3j(*args) == pytest.approx(ref, abs=1e-14), args
        checked += 1
    assert checked > 150


@pytest.mark.parametrize("Jl,gl,Ju,gu", [(0.5, 2.0, 0.5, 2 / 3), (0.5, 2.0, 1.5, 4 / 3), (0, 0, 1, 1.0),
                                         (1, 1.5, 2, 7 / 6), (2, 1.0, 1, 0.5), (1.5, 0.8, 2.5, 1.2), (1, 0.5, 1, 2.5)])
def test_zeeman_pattern_normalisation_and_effective_lande(Jl, gl, Ju, gu):
    p = O.zeeman_pattern(Jl, gl, Ju, gu)
    for q in (-1, 0, 1):
        assert p["strength"][p["q"] == q].sum() == pytest.approx(1.0, abs=1e-14)
    m = {q: float(np.sum(p["strength"][p["q"] == q] * p["shift"][p["q"] == q])) for q in (-1, 0, 1)}
    assert m[0] == pytest.approx(0.0, abs=1e-14)
    assert 0.5 * (m[-1] - m[1]) == pytest.approx(gbar(Jl, gl, Ju, gu), abs=1e-13)
    # every component: q = M_l - M_u with the shift g_u M_u - g_l M_l of some
    # projections allowed by J
    Mu = np.arange(-Ju, Ju + 1)
    for q, s in zip(p["q"], p["shift"]):
        assert np.min(np.abs(gu * Mu - gl * (Mu + q) - s)) < 1e-12


def test_alkali_d_line_patterns():
    """D1 (2S1/2 - 2P1/2): pi at +-2/3, sigma at +-4/3, all of equal weight
    within each q; D2 (2S1/2 - 2P3/2): pi at +-1/3, sigma at +-1 (weight
    3/4) and +-5/3 (weight 1/4); the normal triplet: shifts 0, -+g."""
    d1 = O.zeeman_pattern(0.5, 2.0, 0.5, 2 / 3)
    pi = np.sort(d1["shift"][d1["q"] == 0])
    np.testing.assert_allclose(pi, [-2 / 3, 2 / 3], atol=1e-14)
    np.testing.assert_allclose(d1["shift"][d1["q"] == 1], [-4 / 3], atol=1e-14)   # q = +1: the red (lower-frequency) one
    np.testing.assert_allclose(d1["shift"][d1["q"] == -1], [4 / 3], atol=1e-14)
    d2 = O.zeeman_pattern(0.5, 2.0, 1.5, 4 / 3)
    s1 = d2["q"] == 1
    order = np.argsort(d2["shift"][s1])
    np.testing.assert_allclose(d2["shift"][s1][order], [-5 / 3, -1.0], atol=1e-14)
    np.testing.assert_allclose(d2["strength"][s1][order], [0.25, 0.75], atol=1e-14)
    np.testing.assert_allclose(np.sort(d2["shift"][d2["q"] == 0]), [-1 / 3, 1 / 3], atol=1e-14)
    nt = O.zeeman_pattern(0, 0.0, 1, 1.5)
    assert sorted(zip(nt["q"], nt["shift"])) == [(-1, 1.5), (0, 0.0), (1, -1.5)]


def test_faddeeva_against_wofz():
    from scipy.special import wofz
    for a in (1e-4, 1e-3, 0.01, 0.1, 0.5, 2.0):
        for v in np.linspace(-30.0, 30.0, 241):
            w = O.voigt_w(a, v)
            ref = wofz(v + 1j * a)
            assert abs(w - ref) <= 1.5e-4 * abs(ref) + 1e-12, (a, v, w, ref)
            # the dispersion profile is odd in v, positive for v > 0
            if v > 0:
                assert w.imag > 0


def test_delo_exact_for_linear_source_without_polarisation():
    """K6 = 0 and only eps_I: the solver is the linear short-characteristic
    one, exact for S = a + b tau: the emergent intensity is a + b."""
    tau = np.concatenate([[0.0], np.geomspace(1e-3, 30.0, 60)])
    z = -tau                      # chi_I = 1
    a, b = 2.0, 3.0
    S = a + b * tau
    eps = np.zeros((len(z), 4))
    eps[:, 0] = S
    out = O.stokes_formal(z, np.ones(len(z)), np.zeros((len(z), 6)), eps, [S[-1] + b, 0, 0, 0])
    assert out[0] == pytest.approx(a + b, rel=1e-13)
    assert np.all(out[1:] == 0.0)


def unno_rachkovsky(B0, B1, eI, eQ, eU, eV, rQ, rU, rV):
    """Emergent Stokes vector of a Milne-Eddington atmosphere (constant
    absorption matrix in units of the continuum opacity, Planck function
    B0 + B1 tau_c, mu = 1), the published closed form."""
    eI = 1.0 + eI
    P = eQ * rQ + eU * rU + eV * rV
    D = eI ** 2 * (eI ** 2 - eQ ** 2 - eU ** 2 - eV ** 2 + rQ ** 2 + rU ** 2 + rV ** 2) - P ** 2
    I = B0 + B1 * eI * (eI ** 2 + rQ ** 2 + rU ** 2 + rV ** 2) / D
    Q = -B1 * (eI ** 2 * eQ + eI * (eV * rU - eU * rV) + rQ * P) / D
    U = -B1 * (eI ** 2 * eU + eI * (eQ * rV - eV * rQ) + rU * P) / D
    V = -B1 * (eI ** 2 * eV + eI * (eU * rQ - eQ * rU) + rV * P) / D
    return np.array([I, Q, U, V])


ME_CASES = [(2.0, 0.6, 0.3, -0.5, 0.4, -0.2, 0.7), (30.0, 10.0, -4.0, 12.0, 6.0, 3.0, -9.0),
            (0.5, 0.0, 0.0, 0.4, 0.0, 0.0, 0.9)]


def _me_run(case, n, B0, B1, B2):
    eI, eQ, eU, eV, rQ, rU, rV = case
    K = np.array([[1 + eI, eQ, eU, eV], [eQ, 1 + eI, rV, -rU], [eU, -rV, 1 + eI, rQ], [eV, rU, -rQ, 1 + eI]])
    tau = np.concatenate([[0.0], np.geomspace(1e-4, 40.0 / (1 + eI), n)])
    z = -tau
    chi = np.full(len(z), 1.0 + eI)
    K6 = np.tile([eQ, eU, eV, rQ, rU, rV], (len(z), 1))
    Bt = B0 + B1 * tau + B2 * tau ** 2
    eps = Bt[:, None] * K[:, 0][None, :]
    # the exact Stokes vector at the bottom depth t: sum over the derivatives
    # of B(t) times powers of K^-1 applied to e_I
    e0 = np.array([1.0, 0, 0, 0])
    k1 = np.linalg.solve(K, e0)
    k2 = np.linalg.solve(K, k1)
    t = tau[-1]
    Ibot = Bt[-1] * e0 + (B1 + 2 * B2 * t) * k1 + 2 * B2 * k2
    return O.stokes_formal(z, chi, K6, eps, Ibot), K, k1, k2


@pytest.mark.parametrize("case", ME_CASES)
def test_delo_exact_for_milne_eddington(case):
    """Constant (eta_I..rho_V) relative to a unit continuum opacity, LTE
    emission B(tau) K e_I with B linear in tau: the Stokes vector is then
    linear in tau, so is the effective source function, and the solver
    reproduces the Unno-Rachkovsky solution to rounding on any grid."""
    B0, B1 = 1.0, 2.5
    exact = unno_rachkovsky(B0, B1, *case)
    for n in (20, 100):
        out, _, _, _ = _me_run(case, n, B0, B1, 0.0)
        np.testing.assert_allclose(out, exact, rtol=0, atol=1e-13 * exact[0])


@pytest.mark.parametrize("case", ME_CASES)
def test_delo_second_order_for_curved_source(case):
    """B = B0 + B1 tau + B2 tau^2: the exact emergent vector is
    B0 e_I + B1 K^-1 e_I + 2 B2 K^-2 e_I; the error of the solver falls as
    the square of the step."""
    B0, B1, B2 = 1.0, 2.5, 0.8
    errs = []
    for n in (100, 200, 400, 800):
        out, K, k1, k2 = _me_run(case, n, B0, B1, B2)
        exact = B0 * np.array([1.0, 0, 0, 0]) + B1 * k1 + 2 * B2 * k2
        errs.append(np.max(np.abs(out - exact)) / exact[0])
    errs = np.array(errs)
    order = np.log2(errs[:-1] / errs[1:])
    assert errs[-1] < 1e-4 and np.all(order > 1.7), (errs, order)


def zeeman_column(n=40, vz=0.0, T_top=4500.0):
    """Column for the Zeeman test atom: lines thick at the bottom, the two
    deepest points at the same temperature (so the bottom boundary has no
    diffusion term)."""
    z = np.linspace(1.5e6, 0.0, n)
    s = np.linspace(0.0, 1.0, n)
    T = T_top + 2500.0 * s ** 2
    T[-1] = T[-2]
    nH = 1.0e21 * np.exp(-z / 1.5e5)
    return dict(z=z, T=T, n_e=1.0e-3 * nH, n_H=nH, v_z=np.full(n, vz), v_turb=np.full(n, 1.5e3))


@pytest.fixture(scope="module")
def solved(atom_dir):
    a = O.Atom(atom_dir["zeeman_tiny"])
    col = zeeman_column()
    r = O.solve_column(a, col, n_mu=3, tol=1e-10, max_iter=400)
    assert r["status"] == 0
    return a, col, r


def test_zero_field_is_the_unpolarised_spectrum(solved):
    a, col, r = solved
    st = O.stokes_column(a, col, r["pops"], 3, 0.0, 0.7, 0.3)
    np.testing.assert_allclose(st[:, 0], r["spectrum"], rtol=1e-12)
    assert np.max(np.abs(st[:, 1:])) <= 1e-14 * np.max(st[:, 0])


def test_field_direction_symmetries(solved):
    a, col, r = solved
    B = 0.15   # 1.5 kG
    base = O.stokes_column(a, col, r["pops"], 3, B, 0.6, 0.4)
    # line of sight along the field: no linear polarisation
    along = O.stokes_column(a, col, r["pops"], 3, B, 0.0, 0.4)
    assert np.all(along[:, 1] == 0.0) and np.all(along[:, 2] == 0.0)
    # transverse field: no circular polarisation
    trans = O.stokes_column(a, col, r["pops"], 3, B, np.pi / 2, 0.4)
    assert np.max(np.abs(trans[:, 3])) <= 1e-10 * np.max(trans[:, 0])
    # the mirror image theta -> pi - theta, chi -> -chi flips eta_U, eta_V,
    # rho_U and rho_V: the transfer equation is conjugated by
    # diag(1, 1, -1, -1), so I and Q stay and U and V change sign (the plain
    # reversal chi -> chi + pi is no symmetry: Faraday rotation turns the
    # other way)
    rev = O.stokes_column(a, col, r["pops"], 3, B, np.pi - 0.6, -0.4)
    scale = np.max(base[:, 0])
    np.testing.assert_allclose(rev[:, :2], base[:, :2], rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(rev[:, 2:], -base[:, 2:], rtol=0, atol=1e-11 * scale)
    # azimuth turned by d: (Q, U) turns by 2 d, I and V stay
    d = 0.35
    rot = O.stokes_column(a, col, r["pops"], 3, B, 0.6, 0.4 + d)
    c, s = np.cos(2 * d), np.sin(2 * d)
    np.testing.assert_allclose(rot[:, 0], base[:, 0], rtol=1e-11)
    np.testing.assert_allclose(rot[:, 3], base[:, 3], rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(rot[:, 1], c * base[:, 1] - s * base[:, 2], rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(rot[:, 2], s * base[:, 1] + c * base[:, 2], rtol=0, atol=1e-11 * scale)
    # the field splits the lines: real polarisation
    assert np.max(np.abs(base[:, 1:])) > 1e-3 * scale


def test_weak_field_law(atom_dir):
    """Without a background or continuum at the lines, with fixed
    populations: V(nu) = gbar nu_L cos(theta) dI/dnu to first order in B,
    where dI/dnu (the line-profile part) is the central difference of two
    spectra whose atmosphere moves by -+dv (a velocity v shifts every
    profile by nu0 v / c; the Planck function does not move).  The law is
    one of the transfer equation; the discrete solver meets it up to its
    discretisation error, which falls as the square of the depth step.  The
    sign is the one of the standard weak-field relation
    V = -gbar Delta lambda_B cos(theta) dI/dlambda."""
    a = O.Atom(atom_dir["zeeman_tiny_nobg"])
    theta = 0.5
    B = 5.0e-4   # 5 G: about 1e-3 Doppler widths of splitting
    dv = 2.0
    err = {}
    for n in (80, 320):
        col = zeeman_column(n)
        pops = O.solve_column(a, col, n_mu=3, tol=1e-10, max_iter=400)["pops"]
        st = O.stokes_column(a, col, pops, 3, B, theta, 0.2)
        cm, cp = dict(col), dict(col)
        cm["v_z"] = col["v_z"] - dv
        cp["v_z"] = col["v_z"] + dv
        Im = O.stokes_column(a, cm, pops, 3, 0.0, 0.0, 0.0)[:, 0]
        Ip = O.stokes_column(a, cp, pops, 3, 0.0, 0.0, 0.0)[:, 0]
        for t, (Jl, gl, Ju, gu) in ((0, (0.5, 2.0, 0.5, 2 / 3)), (1, (0.5, 2.0, 1.5, 4 / 3))):
            j = a.transition(t)["act"]
            nu0 = C_LIGHT / a.lam[j[len(j) // 2]]
            dI_dnu = (Im - Ip) / (2.0 * nu0 * dv / C_LIGHT)
            pred = gbar(Jl, gl, Ju, gu) * larmor(B) * np.cos(theta) * dI_dnu
            core = j[5:-5]
            scale = np.max(np.abs(pred[core]))
            err[n, t] = np.max(np.abs(st[core, 3] - pred[core])) / scale
            # an absorption line (intensity rising away from the core): the
            # blue wing (higher frequency) has V > 0 for cos(theta) > 0
            blue = j[2:len(j) // 2 - 2]
            blue = blue[np.abs(pred[blue]) > 0.05 * scale]
            assert len(blue) > 0 and np.all(st[blue, 3] > 0)
    for t in (0, 1):
        assert err[320, t] < 1e-4 and err[80, t] > 6.0 * err[320, t], err


def test_transverse_weak_field_linear_polarisation_grows_as_B_squared(atom_dir):
    a = O.Atom(atom_dir["zeeman_tiny_nobg"])
    col = zeeman_column()
    pops = O.solve_column(a, col, n_mu=3, tol=1e-10, max_iter=400)["pops"]
    q1 = O.stokes_column(a, col, pops, 3, 2.0e-3, np.pi / 2, 0.0)
    q2 = O.stokes_column(a, col, pops, 3, 4.0e-3, np.pi / 2, 0.0)
    j = a.transition(1)["act"]
    Q1, Q2 = q1[j, 1], q2[j, 1]
    big = np.abs(Q1) > 0.1 * np.max(np.abs(Q1))
    np.testing.assert_allclose(Q2[big] / Q1[big], 4.0, rtol=2e-3)
    assert np.max(np.abs(q1[:, 2])) <= 1e-10 * np.max(np.abs(Q1))


def test_absorption_matrix_ratios_from_wofz_and_the_d2_pattern(atom_dir):
    """At a point where only the D2-like line absorbs (no background, no
    continuum there), eta_X / eta_I and rho_X / eta_I are ratios of Zeeman
    profile combinations: built here from scipy's wofz (phi + i psi =
    w(v + i a) / sqrt(pi)) and the textbook D2 pattern, with the Doppler
    width and damping of the column preparation.  This fixes the sign of the
    magneto-optical terms and the angle factors."""
    from scipy.special import wofz
    a = O.Atom(atom_dir["zeeman_tiny_nobg"])
    col = zeeman_column(30, vz=1.2e3)
    pops = O.solve_column(a, col, n_mu=3, tol=1e-8, max_iter=400)["pops"]
    dnd, adamp = O.column_damping(a, col)
    B, theta, chi = 0.12, 0.7, 0.45
    pattern = [(+1, -1.0, 0.75), (+1, -5 / 3, 0.25), (0, 1 / 3, 0.5), (0, -1 / 3, 0.5), (-1, 1.0, 0.75),
               (-1, 5 / 3, 0.25)]
    j_all = a.transition(1)["act"]
    nu0 = C_LIGHT / a.lam[j_all[len(j_all) // 2]]
    for k in (3, 17, 28):
        for j in j_all[::4]:
            c = O.stokes_coefficients(a, col, pops, 3, B, theta, chi, int(j), k)
            v = (C_LIGHT / a.lam[j] - nu0 * (1 + col["v_z"][k] / C_LIGHT)) / dnd[1, k]
            vL = larmor(B) / dnd[1, k]
            w = {q: 0j for q in (-1, 0, 1)}
            for q, sh, st in pattern:
                w[q] += st * wofz(v - sh * vL + 1j * adamp[1, k])
            ct, s2 = np.cos(theta), np.sin(theta) ** 2
            I = 0.5 * (w[0] * s2 + 0.5 * (w[1] + w[-1]) * (1 + ct * ct))
            lin = 0.5 * (w[0] - 0.5 * (w[1] + w[-1])) * s2
            circ = 0.5 * (w[1] - w[-1]) * ct
            want = np.array([lin.real * np.cos(2 * chi), lin.real * np.sin(2 * chi), circ.real,
                             lin.imag * np.cos(2 * chi), lin.imag * np.sin(2 * chi), circ.imag]) / I.real
            got = c["K6"] / c["chi"]
            np.testing.assert_allclose(got, want, rtol=0, atol=3e-4 * max(1.0, np.max(np.abs(want))))
            np.testing.assert_allclose(c["eps"][1:] / c["eps"][0], want[:3], rtol=0, atol=3e-4)


def test_zero_field_with_prd_is_the_unpolarised_spectrum(atom_dir):
    """A PRD line: with the final rho of the solve, the zero-field Stokes I
    is the solve's emergent spectrum (emission profile rho phi)."""
    a = O.Atom(atom_dir["zeeman_tiny_prd"])
    col = zeeman_column(24)
    r = O.solve_column(a, col, n_mu=3, tol=1e-9, max_iter=3000, prd=1, prd_lines=(1,))
    assert r["status"] == 0
    assert np.max(np.abs(r["rho"][0] - 1.0)) > 1e-3     # PRD matters here
    st = O.stokes_column(a, col, r["pops"], 3, 0.0, 0.3, 0.1, prd_rho=r["rho"])
    np.testing.assert_allclose(st[:, 0], r["spectrum"], rtol=1e-12)
    st1 = O.stokes_column(a, col, r["pops"], 3, 0.0, 0.3, 0.1)
    assert np.max(np.abs(st1[:, 0] / r["spectrum"] - 1.0)) > 1e-4   # rho = 1 differs
