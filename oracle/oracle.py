"""ctypes wrapper of the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this module; the product
(the GPU library and its Python binding) never does.
"""
from __future__ import annotations

import concurrent.futures
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

START_LTE, START_ZERO_RADIATION, START_PROVIDED, START_ESCAPE = 0, 1, 2, 3
BAD_INPUT = 4


def build() -> str:
    """Compile the oracle with the host C compiler (plain -O2, no vector
    or fast-math flags: the oracle stays the plain reference)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc_atom_load.argtypes = [C.c_char_p, C.POINTER(C.c_void_p)]
        L.orc_atom_free.argtypes = [C.c_void_p]
        L.orc_atom_info.argtypes = [C.c_void_p, ip, ip, ip, ip]
        L.orc_atom_lambda.argtypes = [C.c_void_p, dp]
        L.orc_atom_transition.argtypes = [C.c_void_p, C.c_int, ip, ip, ip, ip, ip, dp]
        L.orc_atom_einstein_A.argtypes = [C.c_void_p, C.c_int]
        L.orc_atom_einstein_A.restype = C.c_double
        L.orc_atom_abundance.argtypes = [C.c_void_p]
        L.orc_atom_abundance.restype = C.c_double
        L.orc_last_error.restype = C.c_char_p
        L.orc_gauss_legendre.argtypes = [C.c_int, dp, dp]
        L.orc_voigt_H.argtypes = [C.c_double, C.c_double]
        L.orc_voigt_H.restype = C.c_double
        L.orc_sc_coefficients.argtypes = [C.c_double, dp, dp, dp]
        L.orc_formal_ray.argtypes = [C.c_int, dp, dp, C.c_double, dp, dp]
        L.orc_lte_populations.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, dp]
        L.orc_solve_column.argtypes = [C.c_void_p, C.c_int] + [dp] * 7 + [C.c_void_p, dp, dp, ip, ip, dp, dp, dp]
        L.orc_rII.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_rII.restype = C.c_double
        L.orc_column_prd_rho.argtypes = [C.c_void_p, C.c_int] + [dp] * 6 + [C.c_int, dp, C.c_double, C.c_double,
                                                                            C.c_int, dp]
        L.orc_crs_factor.argtypes = [C.c_double, C.c_int]
        L.orc_crs_factor.restype = C.c_double
        L.orc_ng_step.argtypes = [C.c_int, C.c_int, C.POINTER(C.POINTER(C.c_double)), dp]
        L.orc_column_profile_norm.argtypes = [C.c_void_p, C.c_int] + [dp] * 6 + [C.c_int, dp, dp]
        L.orc_column_damping.argtypes = [C.c_void_p, C.c_int] + [dp] * 8
        L.orc_optimize_grid.argtypes = [C.c_void_p, C.c_int] + [dp] * 6 + [C.c_int, dp] + [dp] * 6
        L.orc_wigner3j.argtypes = [C.c_int] * 6
        L.orc_wigner3j.restype = C.c_double
        L.orc_zeeman_pattern.argtypes = [C.c_int, C.c_double, C.c_int, C.c_double, C.c_int, ip, dp, dp]
        L.orc_voigt_w.argtypes = [C.c_double, C.c_double, dp, dp]
        L.orc_voigt_w.restype = None
        L.orc_stokes_formal.argtypes = [C.c_int] + [dp] * 6
        L.orc_stokes_column.argtypes = [C.c_void_p, C.c_int] + [dp] * 6 + [C.c_int] + [dp] * 6
        L.orc_column_psi_ray.argtypes = [C.c_void_p, C.c_int] + [dp] * 6 + [C.c_int, dp, dp, dp]
        L.orc_stokes_coefficients.argtypes = [C.c_void_p, C.c_int] + [dp] * 6 + [C.c_int] + [dp] * 4 + \
            [C.c_int, C.c_int, dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


class _Opts(C.Structure):
    _fields_ = [("n_mu", C.c_int), ("tol", C.c_double), ("max_iter", C.c_int), ("ng_order", C.c_int),
                ("ng_delay", C.c_int), ("ng_period", C.c_int), ("start", C.c_int), ("coll_scale", C.c_double),
                ("crs_f0", C.c_double), ("tol_fp", C.c_double), ("esc_iter", C.c_int), ("prd", C.c_int),
                ("prd_eps0", C.c_double)]


class Atom:
    def __init__(self, path: str):
        h = C.c_void_p()
        if lib().orc_atom_load(path.encode(), C.byref(h)) != 0:
            raise ValueError(lib().orc_last_error().decode())
        self._h = h
        L, nl, nc, NL = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        lib().orc_atom_info(h, C.byref(L), C.byref(nl), C.byref(nc), C.byref(NL))
        self.n_levels, self.n_lines, self.n_cont, self.n_lambda = L.value, nl.value, nc.value, NL.value
        self.n_trans = self.n_lines + self.n_cont
        self.abundance = lib().orc_atom_abundance(h)
        self.lam = np.empty(self.n_lambda)
        lib().orc_atom_lambda(h, _p(self.lam))

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.orc_atom_free(self._h)
            self._h = None

    def transition(self, t: int) -> dict:
        l, u, kind, na = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        lib().orc_atom_transition(self._h, t, C.byref(l), C.byref(u), C.byref(kind), C.byref(na), None, None)
        act = np.empty(na.value, dtype=np.int32)
        w = np.empty(na.value)
        lib().orc_atom_transition(self._h, t, C.byref(l), C.byref(u), C.byref(kind), C.byref(na),
                                  act.ctypes.data_as(C.POINTER(C.c_int)), _p(w))
        return dict(l=l.value, u=u.value, kind=kind.value, act=act, w=w,
                    A=lib().orc_atom_einstein_A(self._h, t) if kind.value == 0 else 0.0)

    def lte(self, T: float, n_e: float, n_tot: float) -> np.ndarray:
        out = np.empty(self.n_levels)
        lib().orc_lte_populations(self._h, T, n_e, n_tot, _p(out))
        return out


def gauss_legendre(n: int):
    x, w = np.empty(n), np.empty(n)
    if lib().orc_gauss_legendre(n, _p(x), _p(w)) != 0:
        raise ValueError("n out of range")
    return x, w


def voigt(a: float, v: float) -> float:
    return lib().orc_voigt_H(float(a), float(v))


def sc_coefficients(x: float):
    e, wa, wb = C.c_double(), C.c_double(), C.c_double()
    lib().orc_sc_coefficients(float(x), C.byref(e), C.byref(wa), C.byref(wb))
    return e.value, wa.value, wb.value


def formal_ray(dtau, S, I0: float):
    dtau = np.ascontiguousarray(dtau, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    n = len(S)
    I, ls = np.empty(n), np.empty(n)
    lib().orc_formal_ray(n, _p(dtau), _p(S), float(I0), _p(I), _p(ls))
    return I, ls


def ng_step(iterates):
    """Order-2 Ng extrapolation from iterates [x0 (newest), x1, x2, x3];
    returns the extrapolated vector or None when the step is skipped."""
    xs = [np.ascontiguousarray(x, dtype=np.float64) for x in iterates]
    arr = (C.POINTER(C.c_double) * len(xs))(*[_p(x) for x in xs])
    out = np.empty_like(xs[0])
    ok = lib().orc_ng_step(2, len(out), arr, _p(out))
    return out if ok else None


def profile_norm(atom: Atom, col: dict, n_mu: int):
    N = len(col["z"])
    cols = {k: np.ascontiguousarray(col[k], dtype=np.float64) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}
    nstar = np.empty((N, atom.n_levels))
    norm = np.empty((max(atom.n_lines, 1), N))
    lib().orc_column_profile_norm(atom._h, N, *(_p(cols[k]) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")),
                                  n_mu, _p(nstar), _p(norm))
    return nstar, norm[: atom.n_lines]


def column_damping(atom: Atom, col: dict):
    """Doppler widths (Hz) and Voigt damping parameters [n_lines][N] of the
    column preparation."""
    N = len(col["z"])
    cols = {k: np.ascontiguousarray(col[k], dtype=np.float64) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}
    dnd = np.empty((max(atom.n_lines, 1), N))
    ad = np.empty((max(atom.n_lines, 1), N))
    lib().orc_column_damping(atom._h, N, *(_p(cols[k]) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")),
                             _p(dnd), _p(ad))
    return dnd[: atom.n_lines], ad[: atom.n_lines]


def rII(a: float, x: float, x2: float) -> float:
    """Angle-averaged R_II(x, x2) in Doppler units (the oracle's quadrature)."""
    return lib().orc_rII(float(a), float(x), float(x2))


def prd_line_sizes(atom: Atom, prd_lines) -> list:
    """(line index, number of active wavelengths) of the given PRD lines."""
    return [(t, len(atom.transition(t)["act"])) for t in prd_lines]


def prd_rho_constant_field(atom: Atom, col: dict, n_mu: int, pops, I_const: float, prd_lines, eps0=0.0, it=1):
    """One rho update with every ray's intensity I_const: rho per PRD line,
    a list of [N][n_act] arrays."""
    N = len(col["z"])
    cols = {k: np.ascontiguousarray(col[k], dtype=np.float64) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}
    sizes = prd_line_sizes(atom, prd_lines)
    out = np.empty(sum(N * n for _, n in sizes))
    pops = np.ascontiguousarray(pops, dtype=np.float64)
    rc = lib().orc_column_prd_rho(atom._h, N, *(_p(cols[k]) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")),
                                  n_mu, _p(pops), float(I_const), float(eps0), int(it), _p(out))
    if rc != 0:
        raise ValueError(lib().orc_last_error().decode())
    res, o = [], 0
    for _, n in sizes:
        res.append(out[o:o + N * n].reshape(N, n))
        o += N * n
    return res


GRID_WEIGHTS = (1.0, 2.0, 2.0e-4, 0.2)     # w_z, w_T, w_v [s/m], w_tau


def optimize_grid(atom: Atom, col: dict, n_out: int, weights=GRID_WEIGHTS) -> dict:
    """Column re-gridded onto n_out points (see orc_optimize_grid)."""
    N = len(col["z"])
    cols = {k: np.ascontiguousarray(col[k], dtype=np.float64) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}
    w = np.ascontiguousarray(weights, dtype=np.float64)
    out = {k: np.empty(n_out) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}
    rc = lib().orc_optimize_grid(atom._h, N, *(_p(cols[k]) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")),
                                 n_out, _p(w), *(_p(out[k]) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")))
    if rc != 0:
        raise ValueError(lib().orc_last_error().decode())
    return out


def crs_factor(f0: float, it: int) -> float:
    """Collision factor of iteration it under collisional-radiative switching."""
    return lib().orc_crs_factor(f0, it)


def solve_column(atom: Atom, col: dict, n_mu: int = 5, tol: float = 1e-4, max_iter: int = 200,
                 ng_order: int = 2, ng_delay: int = 5, ng_period: int = 4, start: int = START_LTE,
                 coll_scale: float = 1.0, init_pops=None, want_spectrum: bool = True,
                 want_psi: bool = False, crs_f0: float = 1.0, tol_fp: float = 0.0, esc_iter: int = 3,
                 prd: int = 0, prd_eps0: float = 0.0, prd_lines=()) -> dict:
    N = len(col["z"])
    cols = {k: np.ascontiguousarray(col[k], dtype=np.float64) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}
    o = _Opts(n_mu, tol, max_iter, ng_order, ng_delay, ng_period, start, coll_scale, crs_f0, tol_fp, esc_iter, prd,
              prd_eps0)
    sizes = prd_line_sizes(atom, prd_lines) if prd else []
    rho = np.empty(max(1, sum(N * n for _, n in sizes)))
    pops = np.empty((N, atom.n_levels))
    hist = np.empty(max(max_iter, 1))
    spec = np.empty(atom.n_lambda) if want_spectrum else None
    psi = np.empty((atom.n_trans, N)) if want_psi else None
    ip = None
    if init_pops is not None:
        ip = np.ascontiguousarray(init_pops, dtype=np.float64).reshape(N, atom.n_levels)
    n_iter, status = C.c_int(), C.c_int()
    rc = lib().orc_solve_column(atom._h, N, *(_p(cols[k]) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")),
                                _p(ip), C.byref(o), _p(pops), _p(hist), C.byref(n_iter), C.byref(status),
                                _p(spec), _p(psi), _p(rho) if sizes else None)
    if rc != 0:
        raise ValueError(lib().orc_last_error().decode())
    out = dict(pops=pops, history=hist[:max_iter], n_iter=n_iter.value, status=status.value, spectrum=spec,
               psi_star=psi)
    if sizes:
        o2, out["rho"] = 0, []
        for _, n in sizes:
            out["rho"].append(rho[o2:o2 + N * n].reshape(N, n))
            o2 += N * n
    return out


def solve_columns(atom: Atom, columns, threads: int | None = None, **kw) -> list:
    """Solve columns independently on a thread pool (ctypes releases the
    GIL during the call), one column per task, dynamic assignment."""
    threads = threads or os.cpu_count() or 1
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        futs = [ex.submit(solve_column, atom, columns.column(c), **kw) for c in range(columns.n_columns)]
        return [f.result() for f in futs]


def wigner3j(j1, j2, j3, m1, m2, m3) -> float:
    """Wigner 3j symbol (half-integers allowed)."""
    return lib().orc_wigner3j(*(int(round(2 * x)) for x in (j1, j2, j3, m1, m2, m3)))


def zeeman_pattern(J_l, g_l, J_u, g_u) -> dict:
    """Zeeman components of a line: q = M_l - M_u, shift (g_u M_u - g_l M_l)
    in Larmor frequencies, strength."""
    mx = int(round((2 * J_l + 1) * (2 * J_u + 1)))
    q = np.zeros(mx, dtype=np.int32)
    sh, st = np.zeros(mx), np.zeros(mx)
    n = lib().orc_zeeman_pattern(int(round(2 * J_l)), g_l, int(round(2 * J_u)), g_u, mx,
                                 q.ctypes.data_as(C.POINTER(C.c_int)), _p(sh), _p(st))
    if n < 0:
        raise ValueError("no pattern")
    return dict(q=q[:n].copy(), shift=sh[:n].copy(), strength=st[:n].copy())


def voigt_w(a: float, v: float) -> complex:
    """Humlicek W4 value of w(v + i a) = H + i L."""
    H, L = C.c_double(), C.c_double()
    lib().orc_voigt_w(a, v, C.byref(H), C.byref(L))
    return complex(H.value, L.value)


def stokes_formal(z, chiI, K6, eps, Ibot) -> np.ndarray:
    """Emergent (top) Stokes vector of the polarised formal solver given
    per-point opacity chi_I, K6 = (eta_Q, eta_U, eta_V, rho_Q, rho_U, rho_V)
    and eps = (eps_I, eps_Q, eps_U, eps_V), top first."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    chiI = np.ascontiguousarray(chiI, dtype=np.float64)
    K6 = np.ascontiguousarray(K6, dtype=np.float64).reshape(-1, 6)
    eps = np.ascontiguousarray(eps, dtype=np.float64).reshape(-1, 4)
    Ib = np.ascontiguousarray(Ibot, dtype=np.float64)
    out = np.empty(4)
    rc = lib().orc_stokes_formal(len(z), _p(z), _p(chiI), _p(K6), _p(eps), _p(Ib), _p(out))
    if rc != 0:
        raise ValueError(lib().orc_last_error().decode())
    return out


def stokes_column(atom: Atom, col: dict, pops, n_mu: int, B, incl, azim, prd_rho=None) -> np.ndarray:
    """Vertical emergent Stokes spectrum [NL][4] of a column from given
    populations (see orc_stokes_column); prd_rho: the list of rho arrays
    solve_column returns, or None."""
    N = len(col["z"])
    cols = {k: np.ascontiguousarray(col[k], dtype=np.float64) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}
    f = [np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64), (N,))) for x in (B, incl, azim)]
    n = np.ascontiguousarray(pops, dtype=np.float64).reshape(N, -1)
    rho = None if prd_rho is None or len(prd_rho) == 0 else np.ascontiguousarray(
        np.concatenate([np.asarray(r, dtype=np.float64).ravel() for r in prd_rho]))
    out = np.empty((atom.n_lambda, 4))
    rc = lib().orc_stokes_column(atom._h, N, *(_p(cols[k]) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")),
                                 n_mu, *(_p(x) for x in f), _p(n), _p(rho), _p(out))
    if rc != 0:
        raise ValueError(lib().orc_last_error().decode())
    return out


def stokes_coefficients(atom: Atom, col: dict, pops, n_mu: int, B, incl, azim, j: int, k: int) -> dict:
    """chi_I, (eta_Q, eta_U, eta_V, rho_Q, rho_U, rho_V) and (eps_I..eps_V)
    of one point and wavelength (rho = 1)."""
    N = len(col["z"])
    cols = {kk: np.ascontiguousarray(col[kk], dtype=np.float64) for kk in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}
    f = [np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64), (N,))) for x in (B, incl, azim)]
    n = np.ascontiguousarray(pops, dtype=np.float64).reshape(N, -1)
    out = np.empty(11)
    rc = lib().orc_stokes_coefficients(atom._h, N, *(_p(cols[kk]) for kk in ("z", "T", "n_e", "n_H", "v_z", "v_turb")),
                                       n_mu, *(_p(x) for x in f), _p(n), j, k, _p(out))
    if rc != 0:
        raise ValueError(lib().orc_last_error().decode())
    return dict(chi=out[0], K6=out[1:7], eps=out[7:11])


def column_psi_ray(atom: Atom, col: dict, pops, n_mu: int, prd_rho=None) -> np.ndarray:
    """Psi* of every ray [N][NL][n_mu][2] from given populations (see
    orc_column_psi_ray)."""
    N = len(col["z"])
    cols = {k: np.ascontiguousarray(col[k], dtype=np.float64) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}
    n = np.ascontiguousarray(pops, dtype=np.float64).reshape(N, -1)
    rho = None if prd_rho is None or len(prd_rho) == 0 else np.ascontiguousarray(
        np.concatenate([np.asarray(r, dtype=np.float64).ravel() for r in prd_rho]))
    out = np.empty((N, atom.n_lambda, n_mu, 2))
    rc = lib().orc_column_psi_ray(atom._h, N, *(_p(cols[k]) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")),
                                  n_mu, _p(n), _p(rho), _p(out))
    if rc != 0:
        raise ValueError(lib().orc_last_error().decode())
    return out
