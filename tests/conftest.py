import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1411_1079_amd import synth  # noqa: E402


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def atom_dir(tmp_path_factory):
    d = tmp_path_factory.mktemp("atoms")
    paths = synth.write_atoms(str(d))
    paths["tiny"] = write_tiny_atom(os.path.join(str(d), "tiny.atom"))
    paths["tiny_nobg"] = write_tiny_atom(os.path.join(str(d), "tiny_nobg.atom"), c_bg=None)
    paths["tiny_voigt"] = write_tiny_atom(os.path.join(str(d), "tiny_voigt.atom"), profile="VOIGT", f_scale=1e6,
                                          n_line=11, x_max=30.0)
    paths["prd_tiny"] = write_prd_tiny_atom(os.path.join(str(d), "prd_tiny.atom"))
    paths["prd_tiny_crd"] = write_prd_tiny_atom(os.path.join(str(d), "prd_tiny_crd.atom"), prd=False)
    paths["prd_tiny_gamma0"] = write_prd_tiny_atom(os.path.join(str(d), "prd_tiny_gamma0.atom"), c_el=1.0e3)
    paths["prd_tiny_gamma0_crd"] = write_prd_tiny_atom(os.path.join(str(d), "prd_tiny_gamma0_crd.atom"), c_el=1.0e3,
                                                       prd=False)
    paths["zeeman_tiny"] = write_zeeman_tiny_atom(os.path.join(str(d), "zeeman_tiny.atom"))
    paths["zeeman_tiny_nobg"] = write_zeeman_tiny_atom(os.path.join(str(d), "zeeman_tiny_nobg.atom"), c_bg=None)
    paths["zeeman_tiny_prd"] = write_zeeman_tiny_atom(os.path.join(str(d), "zeeman_tiny_prd.atom"), prd=True)
    return paths


# levels of the Zeeman test atom: (E [eV], statistical weight, stage), J, Lande g
ZEEMAN_TINY_LEVELS = [((0.0, 2.0, 0), 0.5, 2.0), ((3.0, 2.0, 0), 0.5, 2.0 / 3.0), ((3.05, 4.0, 0), 1.5, 4.0 / 3.0),
                      ((5.0, 2.0, 0), 0.5, 2.0), ((6.5, 1.0, 1), None, None)]


def write_zeeman_tiny_atom(path, c_bg=1.0e-38, prd=False):
    """Five-level atom with three Zeeman-split Voigt lines: two resonance
    lines like the alkali D lines (2S1/2 - 2P1/2, J 1/2 -> 1/2, and
    2S1/2 - 2P3/2, J 1/2 -> 3/2) and a line from 2P3/2 up to a J = 1/2
    level (J 3/2 -> 1/2), on 21-point grids over +-6 Doppler widths, and
    one continuum far away; prd=True makes the D2-like line PRD."""
    levels = [lv for lv, _, _ in ZEEMAN_TINY_LEVELS]
    ev = synth._EV
    hc = synth._H * synth._C

    def lam0(lo, hi):
        return hc / ((levels[hi][0] - levels[lo][0]) * ev) * 1e9

    lines = [dict(l=0, u=1, f=0.3, profile="VOIGT", coll="OMEGA", cval=1.0,
                  lam=synth.line_grid_nm(lam0(0, 1), n=21, x_max=6.0)),
             dict(l=0, u=2, f=0.6, profile="VOIGT", coll="OMEGA", cval=1.0,
                  lam=synth.line_grid_nm(lam0(0, 2), n=21, x_max=6.0)),
             dict(l=2, u=3, f=0.2, profile="VOIGT", coll="OMEGA", cval=1.0,
                  lam=synth.line_grid_nm(lam0(2, 3), n=21, x_max=6.0))]
    conts = [dict(l=0, u=4, alpha=1e-22, coll="OMEGA", cval=0.1, lam=np.sort(synth.continuum_grid_nm(lam0(0, 4), n=4)))]
    zee = [(i, J, g) for i, (_, J, g) in enumerate(ZEEMAN_TINY_LEVELS) if J is not None]
    el = [(1, 1.0e-16, "PRD")] if prd else None
    return synth.write_atom(path, "ZTINY", TINY_MASS, 1.0, levels, lines, conts, c_bg, elastic=el, zeeman=zee)


def write_prd_tiny_atom(path, prd=True, c_el=1.0e-16, n_line=13, x_max=6.0):
    """Four-level atom for partial frequency redistribution on tiny grids:
    a strong Voigt resonance line 0-1 with PRD (elastic collisions c_el
    n_H), a weaker Voigt line 0-2 with complete redistribution, and one
    continuum from level 0."""
    levels = [(0.0, 2.0, 0), (3.0, 6.0, 0), (3.4, 2.0, 0), (6.5, 1.0, 1)]
    ev = synth._EV
    hc = synth._H * synth._C

    def lam0(lo, hi):
        return hc / ((levels[hi][0] - levels[lo][0]) * ev) * 1e9

    lines = [dict(l=0, u=1, f=0.5, profile="VOIGT", coll="OMEGA", cval=1.0,
                  lam=synth.line_grid_nm(lam0(0, 1), n=n_line, x_max=x_max)),
             dict(l=0, u=2, f=0.05, profile="VOIGT", coll="OMEGA", cval=1.0,
                  lam=synth.line_grid_nm(lam0(0, 2), n=7, x_max=3.0))]
    conts = [dict(l=0, u=3, alpha=1e-22, coll="OMEGA", cval=0.1, lam=np.sort(synth.continuum_grid_nm(lam0(0, 3), n=4)))]
    el = [(0, c_el, "PRD" if prd else "CRD")]
    return synth.write_atom(path, "PRDTINY", TINY_MASS, 1.0, levels, lines, conts, 1.0e-38, elastic=el)


TINY_MASS = 1.00794


def write_tiny_atom(path, c_bg=1.0e-38, profile="GAUSS", f_scale=1.0, n_line=9, x_max=4.0):
    """Four-level test atom with Gaussian profiles and every kind of
    overlap: two lines with the same rest wavelength (a full blend), a
    line inside a continuum, and two overlapping continua.  With
    profile="VOIGT", strong lines (f_scale) and wide line grids (x_max
    Doppler units of 10 km/s) the radiative damping shapes the wings."""
    levels = [(0.0, 2.0, 0), (1.5, 2.0, 0), (3.0, 4.0, 0), (5.9, 1.0, 1)]
    ev = synth._EV
    hc = synth._H * synth._C

    def lam0(lo, hi):
        return hc / ((levels[hi][0] - levels[lo][0]) * ev) * 1e9

    lines = [
        dict(l=0, u=1, f=3e-7 * f_scale, profile=profile, coll="OMEGA", cval=1.0,
             lam=synth.line_grid_nm(lam0(0, 1), n=n_line, x_max=x_max)),
        dict(l=1, u=2, f=2e-7 * f_scale, profile=profile, coll="OMEGA", cval=1.0,
             lam=synth.line_grid_nm(lam0(1, 2), n=n_line, x_max=x_max)),
        dict(l=0, u=2, f=1e-7 * f_scale, profile=profile, coll="OMEGA", cval=1.0,
             lam=synth.line_grid_nm(lam0(0, 2), n=n_line, x_max=x_max)),
    ]
    conts = [dict(l=i, u=3, alpha=a, coll="OMEGA", cval=0.1,
                  lam=np.sort(synth.continuum_grid_nm(lam0(i, 3), n=5)))
             for i, a in ((0, 1e-22), (1, 2e-22), (2, 3e-22))]
    return synth.write_atom(path, "TINY", TINY_MASS, 1.0, levels, lines, conts, c_bg)


def tiny_column(n_depth=8, vz=3.0e3):
    """Short column for the tiny atom: lines thin at the top and thick at
    the bottom, a temperature minimum, and a velocity gradient."""
    z = np.linspace(1.2e6, 0.0, n_depth)
    T = 3200.0 + 400.0 * np.cos(np.linspace(0.0, 3.0, n_depth))
    nH = 1.0e20 * np.exp(-z / 1.5e5)
    ne = 1.0e-3 * nH
    v = vz * np.linspace(1.0, -1.0, n_depth)
    return dict(z=z, T=T, n_e=ne, n_H=nH, v_z=v, v_turb=np.full(n_depth, 1.0e3))


def oracle_lockstep_rtol(atom, col, floor=1e-10, **kw):
    """Relative tolerance for element-by-element parity of one column with
    the FP64 oracle: `floor`, or ten times the oracle's own change when its
    input temperatures are perturbed by about one unit in the last place,
    whichever is larger.  Columns whose iteration amplifies rounding (Ng
    steps on nearly parallel iterates, weak collisions) cannot be reproduced
    by any other summation order more closely than that.  The column must
    be stable: the perturbation may not change the oracle's iteration count
    (such a column is no parity case), and the tolerance may not exceed
    1e-8; the value used is printed."""
    from oracle import oracle as O
    r = O.solve_column(atom, col, want_psi=True, **kw)
    c2 = dict(col)
    c2["T"] = col["T"] * (1.0 + 2e-16 * np.cos(np.arange(len(col["T"]))))
    r2 = O.solve_column(atom, c2, want_psi=True, **kw)
    assert r2["n_iter"] == r["n_iter"], "the oracle's iteration count is not stable under a 1-ulp perturbation"
    s = max(float(np.max(np.abs(r2["pops"] / r["pops"] - 1.0))),
            float(np.max(np.abs(r2["spectrum"] / r["spectrum"] - 1.0))))
    rtol = max(floor, 10.0 * s)
    # the per-iteration changes: ten times their own spread under the same
    # perturbation (an Ng extrapolation from nearly parallel iterates
    # amplifies rounding in the next change more than in the populations)
    n = r["n_iter"]
    r["history_spread"] = 10.0 * np.abs(r2["history"][:n] - r["history"][:n])
    print(f"[lockstep] n_iter={r['n_iter']} rtol={rtol:.2e} history spread "
          f"{float(r['history_spread'].max()) if n else 0.0:.2e}", flush=True)
    assert rtol <= 1e-8, rtol
    return r, rtol
