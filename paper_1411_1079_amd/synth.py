"""Seeded synthetic inputs: model atoms and 1D atmosphere columns.

This module is shared by the oracle side and the GPU side and therefore
holds none of the method's arithmetic (no opacities, profiles, rates,
formal solution or level populations).  It only writes

* model-atom files in the project's text format (level energies and
  weights, oscillator strengths, photo-ionisation cross-sections at the
  edge, collision parameters, and each transition's own wavelength
  sampling), and
* atmosphere columns (height, temperature, electron and hydrogen
  densities, vertical and turbulent velocity) as ragged CSR arrays,
  top of the atmosphere first.

The paper computes spectra column by column from 3D MHD snapshots with
model atoms (Sec. 2.2, Sec. 3.3); neither the snapshot nor the atoms are
available, so the workloads below are synthetic stand-ins with the
paper's shapes (a few hundred depth points per column, several hundred
wavelengths, tens of thousands of columns).

Atom text format (whitespace separated, '#' starts a comment)::

    RH15D-ATOM 1
    NAME <str>
    MASS_AMU <float>
    ABUNDANCE <float>                 # n_total = ABUNDANCE * n_H
    LEVELS <L>
      <E [eV]> <g> <stage>            # L rows, level index 0..L-1
    LINES <n>
      <l> <u> <f_lu> <GAUSS|VOIGT> <OMEGA|EPS> <value> <n_lambda>
      <n_lambda wavelengths [nm]>
    CONTINUA <n>
      <l> <u> <alpha_edge [m^2]> <OMEGA|EPS> <value> <n_lambda>
      <n_lambda wavelengths [nm]>
    ELASTIC <n>                       # optional section
      <line index> <c_el [m^3 s^-1]> <PRD|CRD>
    BACKGROUND NONE | HMINUS <C_bg>
    END

ELASTIC lists lines with elastic collisions (rate c_el n_H, which adds to
the line's damping width) and whether their emission follows partial
frequency redistribution; lines not listed have neither.
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

# Physical constants used only to place wavelength grids and to build the
# hydrostatic atmospheres (CODATA 2018, SI).
_H = 6.62607015e-34
_C = 2.99792458e8
_KB = 1.380649e-23
_EV = 1.602176634e-19
_AMU = 1.66053906660e-27
_M_H = 1.00794 * _AMU
_GRAV = 274.0

H_IONISATION_EV = 13.6057


# ----------------------------------------------------------------------------
# atmosphere container
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Columns:
    """Ragged set of atmosphere columns; column c spans rows
    offset[c]:offset[c+1] of every field, ordered top (largest z) first."""

    offset: np.ndarray  # int64 [n_columns + 1]
    z: np.ndarray  # m
    T: np.ndarray  # K
    n_e: np.ndarray  # m^-3
    n_H: np.ndarray  # m^-3
    v_z: np.ndarray  # m/s, positive = upward (towards an observer at mu = 1)
    v_turb: np.ndarray  # m/s

    @property
    def n_columns(self) -> int:
        return len(self.offset) - 1

    def depth(self, c: int) -> int:
        return int(self.offset[c + 1] - self.offset[c])

    def column(self, c: int) -> dict:
        a, b = int(self.offset[c]), int(self.offset[c + 1])
        return {k: getattr(self, k)[a:b] for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}

    def select(self, idx) -> "Columns":
        idx = np.asarray(idx, dtype=np.int64)
        parts = [self.column(int(c)) for c in idx]
        return Columns.from_list(parts)

    @staticmethod
    def from_list(parts: list) -> "Columns":
        nd = np.array([len(p["z"]) for p in parts], dtype=np.int64)
        off = np.zeros(len(parts) + 1, dtype=np.int64)
        off[1:] = np.cumsum(nd)
        cat = {k: np.ascontiguousarray(np.concatenate([p[k] for p in parts] or [np.zeros(0)]).astype(np.float64))
               for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}
        return Columns(offset=off, **cat)


# ----------------------------------------------------------------------------
# model atoms
# ----------------------------------------------------------------------------
def _fmt(x: float) -> str:
    return repr(float(x))


def line_grid_nm(lam0_nm: float, n: int = 41, x_max: float = 30.0, v_ref: float = 1.0e4) -> np.ndarray:
    """Line sampling: x = x_max*sinh(3s)/sinh(3) Doppler units of v_ref,
    s uniform on [-1, 1]; dense in the core, sparse in the wings."""
    s = np.linspace(-1.0, 1.0, n)
    x = x_max * np.sinh(3.0 * s) / np.sinh(3.0)
    return lam0_nm * (1.0 + x * v_ref / _C)


def continuum_grid_nm(edge_nm: float, n: int = 20) -> np.ndarray:
    """Continuum sampling: n points uniform in frequency from the edge
    frequency to twice the edge frequency (edge included)."""
    nu_e = _C / (edge_nm * 1e-9)
    nu = nu_e * (1.0 + np.arange(n) / (n - 1.0))
    return _C / nu * 1e9


def write_atom(path, name, mass_amu, abundance, levels, lines, continua, background, elastic=None, zeeman=None):
    """Write an atom file. levels: [(E_eV, g, stage)]; lines: dicts with
    l, u, f, profile (GAUSS|VOIGT), coll (OMEGA|EPS), cval, lam [nm];
    continua: dicts with l, u, alpha [m^2], coll, cval, lam [nm];
    background: None or the C_bg of the H-minus-like law; elastic: None or
    [(line index, c_el [m^3 s^-1], "PRD" | "CRD")]; zeeman: None or
    [(level index, J, Lande g)] (a line is Zeeman split when both of its
    levels are listed)."""
    out = ["RH15D-ATOM 1", f"NAME {name}", f"MASS_AMU {_fmt(mass_amu)}", f"ABUNDANCE {_fmt(abundance)}",
           f"LEVELS {len(levels)}", "#  E[eV]  g  stage"]
    for E, g, st in levels:
        out.append(f"  {_fmt(E)} {_fmt(g)} {int(st)}")
    out.append(f"LINES {len(lines)}")
    out.append("#  l u f_lu profile coll value n_lambda / wavelengths [nm]")
    for ln in lines:
        out.append(f"  {ln['l']} {ln['u']} {_fmt(ln['f'])} {ln['profile']} {ln['coll']} {_fmt(ln['cval'])} {len(ln['lam'])}")
        out.append("    " + " ".join(_fmt(v) for v in ln["lam"]))
    out.append(f"CONTINUA {len(continua)}")
    out.append("#  l u alpha_edge[m^2] coll value n_lambda / wavelengths [nm]")
    for ct in continua:
        out.append(f"  {ct['l']} {ct['u']} {_fmt(ct['alpha'])} {ct['coll']} {_fmt(ct['cval'])} {len(ct['lam'])}")
        out.append("    " + " ".join(_fmt(v) for v in ct["lam"]))
    if elastic:
        out.append(f"ELASTIC {len(elastic)}")
        for li, c, kind in elastic:
            out.append(f"  {int(li)} {_fmt(c)} {kind}")
    if zeeman:
        out.append(f"ZEEMAN {len(zeeman)}")
        out.append("#  level 2J g_Lande")
        for li, J, gl in zeeman:
            out.append(f"  {int(li)} {int(round(2 * J))} {_fmt(gl)}")
    if background is None:
        out.append("BACKGROUND NONE")
    else:
        out.append(f"BACKGROUND HMINUS {_fmt(background)}")
    out.append("END")
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    return path


# Two-level atom of the isothermal sqrt(eps) test.
TWO_LEVEL_T = 5000.0
TWO_LEVEL_MASS_AMU = 1.00794
TWO_LEVEL_LAMBDA_NM = 100.0
TWO_LEVEL_EPS = 1.0e-4
TWO_LEVEL_F = 0.5


def write_two_level_atom(path: str, n_freq: int = 21, x_max: float = 4.0) -> str:
    """Two bound levels (g = 1, 3) with one line at 100 nm, Gaussian
    (Doppler) profile, destruction probability eps = 1e-4 and
    n_freq frequencies uniform over +-x_max Doppler widths at 5000 K."""
    dE = _H * _C / (TWO_LEVEL_LAMBDA_NM * 1e-9) / _EV
    vth = math.sqrt(2.0 * _KB * TWO_LEVEL_T / (TWO_LEVEL_MASS_AMU * _AMU))
    x = np.linspace(-x_max, x_max, n_freq)
    nu0 = _C / (TWO_LEVEL_LAMBDA_NM * 1e-9)
    nu = nu0 * (1.0 + x * vth / _C)
    lam = np.sort(_C / nu * 1e9)
    levels = [(0.0, 1.0, 0), (dE, 3.0, 0)]
    lines = [dict(l=0, u=1, f=TWO_LEVEL_F, profile="GAUSS", coll="EPS", cval=TWO_LEVEL_EPS, lam=lam)]
    return write_atom(path, "TWO-LEVEL", TWO_LEVEL_MASS_AMU, 1.0, levels, lines, [], None)


def h6_levels():
    lev = [(H_IONISATION_EV * (1.0 - 1.0 / n ** 2), 2.0 * n * n, 0) for n in range(1, 6)]
    lev.append((H_IONISATION_EV, 1.0, 1))
    return lev


def _kramers_f(l: int, u: int) -> float:
    """Kramers (Gaunt factor 1) absorption oscillator strength."""
    return 32.0 / (3.0 * math.sqrt(3.0) * math.pi) / (l ** 5 * u ** 3) / (1.0 / l ** 2 - 1.0 / u ** 2) ** 3


def write_h6_atom(path: str, c_bg: float | None) -> str:
    """Six-level hydrogen-like atom: five bound levels (E_n = 13.6057 eV
    (1 - 1/n^2), g = 2n^2) plus the continuum (g = 1), all ten bound-bound
    lines with Kramers oscillator strengths and Voigt profiles (41
    wavelengths each), five bound-free continua with Kramers edge
    cross-sections 7.91e-22 n m^2 (20 wavelengths each), electron
    collisions with Omega = 1 (lines) and 0.1 (continua)."""
    lev = h6_levels()
    lines, conts = [], []
    for l in range(1, 6):
        for u in range(l + 1, 6):
            dE = (lev[u - 1][0] - lev[l - 1][0]) * _EV
            lam0 = _H * _C / dE * 1e9
            lines.append(dict(l=l - 1, u=u - 1, f=_kramers_f(l, u), profile="VOIGT", coll="OMEGA", cval=1.0,
                              lam=line_grid_nm(lam0)))
    for n in range(1, 6):
        dE = (H_IONISATION_EV - lev[n - 1][0]) * _EV
        edge = _H * _C / dE * 1e9
        conts.append(dict(l=n - 1, u=5, alpha=7.91e-22 * n, coll="OMEGA", cval=0.1,
                          lam=np.sort(continuum_grid_nm(edge))))
    return write_atom(path, "H6", 1.00794, 1.0, lev, lines, conts, c_bg)


# Ca II-like atom: 4s 2S, 3d 2D (one level), 4p 2P1/2, 4p 2P3/2 and the
# Ca III ground state; rounded synthetic data with the right structure, not
# a laboratory atom.
CA_LEVELS = [(0.0, 2.0, 0), (1.697, 10.0, 0), (3.123, 2.0, 0), (3.151, 4.0, 0), (11.871, 1.0, 1)]
CA_LINES = [  # (l, u, f, PRD)
    (0, 3, 0.68, True),     # K-like resonance line
    (0, 2, 0.33, True),     # H-like resonance line
    (1, 3, 0.06, False),    # infrared lines from the metastable level
    (1, 2, 0.03, False),
    (0, 1, 1.0e-8, False),  # weak forbidden-like line
]
# J and L-S Lande factors of the fine-structure levels (the 3d level, a
# merged D3/2 + D5/2 term, carries none: its lines are not split)
CA_ZEEMAN = [(0, 0.5, 2.0), (2, 0.5, 2.0 / 3.0), (3, 1.5, 4.0 / 3.0)]
CA_MASS_AMU = 40.078
CA_ABUNDANCE = 2.2e-6
CA_C_ELASTIC = 1.0e-14      # m^3 s^-1: Q_E = 1e9 s^-1 at n_H = 1e23 m^-3


def write_ca_atom(path: str, c_bg: float | None, n_prd: int = 61, n_crd: int = 41, n_forbidden: int = 21,
                  n_cont: int = 190, prd: bool = True) -> str:
    """Five-level Ca II-like atom: two resonance lines with partial
    frequency redistribution (n_prd wavelengths each, sinh grid over +-300
    km/s), two infrared lines and a weak forbidden line with complete
    redistribution, Voigt profiles, elastic collisions on the four strong
    lines, Zeeman patterns of the two resonance lines (2S1/2 - 2P3/2 and
    2S1/2 - 2P1/2 levels), and four bound-free continua (n_cont wavelengths each): about
    1000 wavelengths with the defaults.  prd=False writes the same atom
    with every line in complete redistribution."""
    lines, conts, el = [], [], []
    for i, (l, u, f, is_prd) in enumerate(CA_LINES):
        dE = (CA_LEVELS[u][0] - CA_LEVELS[l][0]) * _EV
        lam0 = _H * _C / dE * 1e9
        n = n_prd if is_prd else (n_forbidden if f < 1e-6 else n_crd)
        lines.append(dict(l=l, u=u, f=f, profile="VOIGT", coll="OMEGA", cval=1.0, lam=line_grid_nm(lam0, n=n)))
        if f > 1e-6:
            el.append((i, CA_C_ELASTIC, "PRD" if (is_prd and prd) else "CRD"))
    for lo, alpha in ((0, 2.0e-22), (1, 6.0e-22), (2, 2.0e-22), (3, 2.0e-22)):
        dE = (CA_LEVELS[4][0] - CA_LEVELS[lo][0]) * _EV
        edge = _H * _C / dE * 1e9
        conts.append(dict(l=lo, u=4, alpha=alpha, coll="OMEGA", cval=0.1, lam=np.sort(continuum_grid_nm(edge, n=n_cont))))
    return write_atom(path, "CA2", CA_MASS_AMU, CA_ABUNDANCE, CA_LEVELS, lines, conts, c_bg, elastic=el,
                      zeeman=CA_ZEEMAN)


# ----------------------------------------------------------------------------
# atmospheres
# ----------------------------------------------------------------------------
def electron_density(T: np.ndarray, n_H: np.ndarray) -> np.ndarray:
    """Fixed synthetic electron density: 1e-4 n_H from metals plus a
    logistic hydrogen ionisation fraction 1/(1 + exp((9000 K - T)/400 K))."""
    x = np.clip((9000.0 - T) / 400.0, -700.0, 700.0)
    return n_H * (1.0e-4 + 1.0 / (1.0 + np.exp(x)))


def hydrostatic_nH(z_up: np.ndarray, T: np.ndarray, nH0: float = 1.0e23) -> np.ndarray:
    """n_H(z) from dP/dz = -rho g with P = (1.1 n_H + n_e) k T and
    rho = 1.4 m_H n_H, integrated upward from z = 0 (trapezoid in z on
    ln P).  z_up must increase from 0."""
    xe = electron_density(T, np.ones_like(T))
    mu_fac = 1.1 + xe
    dlnP = -1.4 * _M_H * _GRAV / (mu_fac * _KB * T)
    lnP = np.zeros_like(T)
    lnP[1:] = np.cumsum(0.5 * (dlnP[1:] + dlnP[:-1]) * np.diff(z_up))
    P0 = nH0 * mu_fac[0] * _KB * T[0]
    P = P0 * np.exp(lnP)
    return P / (mu_fac * _KB * T)


def cfg1_column(n_depth: int = 64, tau_min: float = 1e-4, tau_max: float = 1e4, n_H: float = 1.0e16) -> Columns:
    """Isothermal (5000 K), static column for the two-level atom.
    The heights are placed so that the line-centre optical depth is
    log-spaced in [tau_min, tau_max]; the estimate uses the ground level
    holding all atoms (stimulated emission and the upper level are ~1e-12
    here) and is only used to place the grid."""
    tau = np.logspace(math.log10(tau_min), math.log10(tau_max), n_depth)
    lam0 = TWO_LEVEL_LAMBDA_NM * 1e-9
    nu0 = _C / lam0
    vth = math.sqrt(2.0 * _KB * TWO_LEVEL_T / (TWO_LEVEL_MASS_AMU * _AMU))
    dnuD = nu0 * vth / _C
    # grid placement only: line-centre opacity of the ground level
    e2 = _EV * _EV
    eps0, m_e = 8.8541878128e-12, 9.1093837015e-31
    A = 2.0 * math.pi * e2 * nu0 ** 2 / (eps0 * m_e * _C ** 3) * (1.0 / 3.0) * TWO_LEVEL_F
    Bul = A * _C ** 2 / (2.0 * _H * nu0 ** 3)
    Blu = 3.0 * Bul
    chi0 = _H * nu0 / (4.0 * math.pi) * n_H * Blu / (math.sqrt(math.pi) * dnuD)
    z = -tau / chi0
    one = np.ones(n_depth)
    return Columns.from_list([dict(z=z, T=TWO_LEVEL_T * one, n_e=n_H * one, n_H=n_H * one, v_z=0.0 * one,
                                   v_turb=0.0 * one)])


# cfg2: T(h) knots (height km, T K)
_CFG2_KNOTS = ((0.0, 6000.0), (500.0, 4200.0), (2000.0, 8000.0), (2200.0, 1.0e5))


def _cfg2_temperature(h_km: np.ndarray, knots) -> np.ndarray:
    (h0, t0), (h1, t1), (h2, t2), (h3, t3) = knots
    T = np.empty_like(h_km)
    a = h_km <= h1
    T[a] = t0 + (t1 - t0) * (h_km[a] - h0) / (h1 - h0)
    b = (h_km > h1) & (h_km <= h2)
    T[b] = t1 + (t2 - t1) * (h_km[b] - h1) / (h2 - h1)
    c = h_km > h2
    T[c] = np.exp(np.log(t2) + (np.log(t3) - np.log(t2)) * (h_km[c] - h2) / (h3 - h2))
    return T


V_TURB = 2.0e3


def cfg2_mean_column(n_depth: int = 82) -> dict:
    h = np.linspace(0.0, 2200.0, n_depth)
    T = _cfg2_temperature(h, _CFG2_KNOTS)
    nH = hydrostatic_nH(h * 1e3, T)
    ne = electron_density(T, nH)
    flip = slice(None, None, -1)
    return dict(z=(h * 1e3)[flip].copy(), T=T[flip].copy(), n_e=ne[flip].copy(), n_H=nH[flip].copy(),
                v_z=np.zeros(n_depth), v_turb=np.full(n_depth, V_TURB))


def hminus_calibration() -> float:
    """C_bg such that the mean cfg2 atmosphere has tau_500nm = 1 at z = 0
    for kappa = C_bg n_H n_e T^-1.5 exp(8750 K / T) (lambda / 500 nm)."""
    col = cfg2_mean_column()
    f = col["n_H"] * col["n_e"] * col["T"] ** -1.5 * np.exp(8750.0 / col["T"])
    z = col["z"]
    integral = float(np.sum(0.5 * (f[1:] + f[:-1]) * (z[:-1] - z[1:])))
    return 1.0 / integral


def cfg2_columns(seed: int = 0, n_columns: int = 64, n_depth: int = 82, noise: float = 0.1) -> Columns:
    """n_columns columns of n_depth heights in 0..2200 km; every knot of
    T(h) scaled by its own factor U(1-noise, 1+noise) per column;
    hydrostatic n_H (n_H(0) = 1e23 m^-3); static; v_turb = 2 km/s."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = np.linspace(0.0, 2200.0, n_depth)
    flip = slice(None, None, -1)
    parts = []
    for _ in range(n_columns):
        fac = rng.uniform(1.0 - noise, 1.0 + noise, size=4)
        knots = tuple((hk, tk * fk) for (hk, tk), fk in zip(_CFG2_KNOTS, fac))
        T = _cfg2_temperature(h, knots)
        nH = hydrostatic_nH(h * 1e3, T)
        ne = electron_density(T, nH)
        parts.append(dict(z=(h * 1e3)[flip].copy(), T=T[flip].copy(), n_e=ne[flip].copy(), n_H=nH[flip].copy(),
                          v_z=np.zeros(n_depth), v_turb=np.full(n_depth, V_TURB)))
    return Columns.from_list(parts)


def _grf(rng, shape, spacing, corr):
    """Unit-variance Gaussian random field: white noise convolved (via FFT,
    periodic) with a Gaussian kernel of standard deviation `corr`."""
    noise = rng.standard_normal(shape)
    k2 = np.zeros(shape)
    for ax, (n, d) in enumerate(zip(shape, spacing)):
        k = 2.0 * np.pi * np.fft.fftfreq(n, d=d)
        sh = [1] * len(shape)
        sh[ax] = n
        k2 = k2 + (k ** 2).reshape(sh)
    filt = np.exp(-0.5 * k2 * corr ** 2)
    f = np.fft.ifftn(np.fft.fftn(noise) * filt).real
    f -= f.mean()
    sd = f.std()
    # a domain much smaller than the kernel keeps only the mean: no variation
    return f / sd if sd > 1e-9 * noise.std() else np.zeros(shape)


CUBE_DZ_KM = 7.5
CUBE_NZ = 400
CUBE_DX_KM = 48.0


def _cube_mean_T(h_km):
    T = np.empty_like(h_km)
    a = h_km <= 500.0
    T[a] = 6000.0 + (4200.0 - 6000.0) * h_km[a] / 500.0
    b = h_km > 500.0
    T[b] = 4200.0 + (8000.0 - 4200.0) * (h_km[b] - 500.0) / 1500.0
    return T


def cube_columns(seed: int, nx: int = 256, ny: int = 256, nz: int = CUBE_NZ, corr_km: float = 1000.0) -> Columns:
    """Synthetic 3D-MHD-like cube, cut into columns (row-major over x, y).

    400 heights at 7.5 km (0..2992.5 km), 48 km horizontal pitch.
    T = T_mean(h) (1 + sigma(h) G), G a unit-variance 3D Gaussian random
    field (1 Mm kernel), sigma = 5% below 500 km rising linearly to 30% at
    1000 km and above; T >= 3000 K.  The transition region lies at
    h_TR = 2250 km + 750 km clip(G2, -1, 1) (G2 a 2D field); above it
    T > 1e5 K and the column is cut there, leaving 200..400 points.
    v_z = 10 km/s (2 Phi(G_v) - 1) (uniform marginal on +-10 km/s).
    n_H hydrostatic per column; fixed electron densities; v_turb 2 km/s."""
    from scipy.special import ndtr

    rng = np.random.Generator(np.random.PCG64(seed))
    h = np.arange(nz) * CUBE_DZ_KM
    G = _grf(rng, (nx, ny, nz), (CUBE_DX_KM, CUBE_DX_KM, CUBE_DZ_KM), corr_km)
    G2 = _grf(rng, (nx, ny), (CUBE_DX_KM, CUBE_DX_KM), corr_km)
    Gv = _grf(rng, (nx, ny, nz), (CUBE_DX_KM, CUBE_DX_KM, CUBE_DZ_KM), corr_km)
    sigma = np.clip(0.05 + 0.25 * (h - 500.0) / 500.0, 0.05, 0.30)
    T = _cube_mean_T(h)[None, None, :] * (1.0 + sigma[None, None, :] * G)
    T = np.maximum(T, 3000.0)
    h_tr = 2250.0 + 750.0 * np.clip(G2, -1.0, 1.0)
    vz = 1.0e4 * (2.0 * ndtr(Gv) - 1.0)
    del G, Gv
    # hydrostatic n_H on the full grid (integration starts at z = 0, so the
    # later cut does not change the kept points)
    xe = electron_density(T, np.ones_like(T))
    mu_fac = 1.1 + xe
    dlnP = -1.4 * _M_H * _GRAV / (mu_fac * _KB * T)
    lnP = np.zeros_like(T)
    lnP[..., 1:] = np.cumsum(0.5 * (dlnP[..., 1:] + dlnP[..., :-1]) * np.diff(h * 1e3), axis=-1)
    P0 = 1.0e23 * mu_fac[..., :1] * _KB * T[..., :1]
    nH = P0 * np.exp(lnP) / (mu_fac * _KB * T)
    ne = electron_density(T, nH)
    nd = np.clip(np.searchsorted(h, h_tr.ravel(), side="left"), 2, nz).astype(np.int64)
    keep = np.arange(nz)[None, :] >= (nz - nd)[:, None]  # on top-first (reversed) rows
    def flat(a):
        return np.ascontiguousarray(a.reshape(nx * ny, nz)[:, ::-1][keep], dtype=np.float64)
    zz = np.broadcast_to((h * 1e3)[None, :], (nx * ny, nz))
    off = np.zeros(nx * ny + 1, dtype=np.int64)
    off[1:] = np.cumsum(nd)
    return Columns(offset=off, z=flat(zz), T=flat(T), n_e=flat(ne), n_H=flat(nH), v_z=flat(vz),
                   v_turb=np.full(int(off[-1]), V_TURB))


def write_atoms(directory: str) -> dict:
    """Write the model atoms and return their paths (ca2_crd: the Ca II-like
    atom with every line in complete redistribution)."""
    os.makedirs(directory, exist_ok=True)
    c_bg = hminus_calibration()
    return {
        "two_level": write_two_level_atom(os.path.join(directory, "two_level.atom")),
        "h6": write_h6_atom(os.path.join(directory, "h6.atom"), c_bg),
        "ca2": write_ca_atom(os.path.join(directory, "ca2.atom"), c_bg),
        "ca2_crd": write_ca_atom(os.path.join(directory, "ca2_crd.atom"), c_bg, prd=False),
    }


def mlp_params(dims, seed: int, weight_scale: float = 1.0, bias_std: float = 0.1) -> np.ndarray:
    """Seeded parameters of a dense network with layer widths `dims`, flat in
    the library's layout (per layer: weights [fan_in][fan_out] row-major,
    then biases): weights uniform within +-sqrt(6 / fan_in) * weight_scale,
    biases normal with standard deviation bias_std.  FP32."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in zip(dims[:-1], dims[1:]):
        parts.append(rng.uniform(-1.0, 1.0, fi * fo) * math.sqrt(6.0 / fi) * weight_scale)
        parts.append(rng.normal(0.0, bias_std, fo))
    return np.concatenate(parts).astype(np.float32)


def mlp_features(seed: int, n: int) -> np.ndarray:
    """Seeded raw feature rows shaped like the stencil features of the cube:
    ln T around 8.8, ln n_e around 28, ln n_H around 37, v_z / 10 km/s in
    [-1, 1], repeated over the 9 stencil points with small offsets.  FP32."""
    rng = np.random.default_rng(seed)
    base = np.stack([rng.normal(8.8, 0.35, n), rng.normal(28.0, 2.0, n), rng.normal(37.0, 3.0, n),
                     rng.uniform(-1.0, 1.0, n)], axis=1)
    rows = [base + rng.normal(0.0, 0.05, (n, 4)) * np.array([1.0, 1.0, 1.0, 0.2]) for _ in range(9)]
    return np.concatenate(rows, axis=1).astype(np.float32)
