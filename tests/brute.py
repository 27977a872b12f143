"""Brute-force NLTE reference for tiny problems (tests only).

Independent of the oracle's code: it parses the atom file itself, builds
the wavelength grid and quadratures itself, and obtains the radiation
field from explicit Lambda matrices (the exact formal solution for a
source function that is piecewise linear in optical depth, integrated in
40-digit arithmetic) instead of a depth recurrence.  Line profiles are
Gaussian, or Voigt from the Faddeeva function (scipy.special.wofz) with
the radiative damping width computed here from the Einstein A values.

Used to pin the oracle against what the mathematics fixes:
* the statistical-equilibrium fixed point (classical Lambda iteration,
  no approximate operator);
* one preconditioned step, assembled by evaluating the rate equations on
  basis vectors rather than from accumulated P/Q/X terms;
* the two-level closed form of one preconditioned step.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np

H = 6.62607015e-34
C = 2.99792458e8
KB = 1.380649e-23
ME = 9.1093837015e-31
QE = 1.602176634e-19
EPS0 = 8.8541878128e-12
AMU = 1.66053906660e-27

mpmath.mp.dps = 40


class BAtom:
    def __init__(self, path):
        toks = []
        for line in open(path):
            line = line.split("#", 1)[0]
            toks.extend(line.split())
        it = iter(toks)
        nxt = lambda: next(it)
        assert nxt() == "RH15D-ATOM"
        nxt()
        assert nxt() == "NAME"
        self.name = nxt()
        assert nxt() == "MASS_AMU"
        self.mass = float(nxt()) * AMU
        assert nxt() == "ABUNDANCE"
        self.abund = float(nxt())
        assert nxt() == "LEVELS"
        L = int(nxt())
        self.E = np.zeros(L); self.g = np.zeros(L); self.stage = np.zeros(L, int)
        for i in range(L):
            self.E[i] = float(nxt()) * QE; self.g[i] = float(nxt()); self.stage[i] = int(nxt())
        self.L = L
        self.tr = []
        assert nxt() == "LINES"
        for _ in range(int(nxt())):
            d = dict(kind=0, l=int(nxt()), u=int(nxt()), f=float(nxt()), profile=nxt(), coll=nxt(),
                     cval=float(nxt()))
            n = int(nxt()); d["lam"] = np.array([float(nxt()) for _ in range(n)]) * 1e-9
            self.tr.append(d)
        assert nxt() == "CONTINUA"
        for _ in range(int(nxt())):
            d = dict(kind=1, l=int(nxt()), u=int(nxt()), alpha=float(nxt()), coll=nxt(), cval=float(nxt()))
            n = int(nxt()); d["lam"] = np.array([float(nxt()) for _ in range(n)]) * 1e-9
            self.tr.append(d)
        for d in self.tr:
            d["c_el"], d["prd"] = 0.0, False
        w = nxt()
        if w == "ELASTIC":
            for _ in range(int(nxt())):
                li, c, kind = int(nxt()), float(nxt()), nxt()
                self.tr[li]["c_el"], self.tr[li]["prd"] = c, kind == "PRD"
            w = nxt()
        assert w == "BACKGROUND"
        b = nxt()
        self.c_bg = float(nxt()) if b == "HMINUS" else 0.0
        for d in self.tr:
            d["nu0"] = (self.E[d["u"]] - self.E[d["l"]]) / H
            if d["kind"] == 0:
                # Einstein relations (Rybicki & Lightman eqs. 1.72, 10.64 in SI)
                d["A"] = (QE ** 2 * 2 * math.pi * d["nu0"] ** 2 / (EPS0 * ME * C ** 3)
                          * self.g[d["l"]] / self.g[d["u"]] * d["f"])
                d["Bul"] = d["A"] * C ** 2 / (2 * H * d["nu0"] ** 3)
                d["Blu"] = d["Bul"] * self.g[d["u"]] / self.g[d["l"]]
        # wavelength grid and per-transition trapezoid weights
        self.lam = np.unique(np.concatenate([d["lam"] for d in self.tr]))
        self.nu = C / self.lam
        for d in self.tr:
            act = np.nonzero((self.lam >= d["lam"].min()) & (self.lam <= d["lam"].max()))[0]
            nu = self.nu[act]
            w = np.zeros(len(act))
            w[:-1] += 0.5 * (nu[:-1] - nu[1:])
            w[1:] += 0.5 * (nu[:-1] - nu[1:])
            d["act"], d["w"] = act, w

    def damping(self, ti):
        """Radiative damping width (s^-1) of line ti: the sum of the Einstein
        A values of all lines out of its upper and out of its lower level."""
        d = self.tr[ti]
        return sum(e["A"] for e in self.tr if e["kind"] == 0 and e["u"] in (d["u"], d["l"]))


def _profile_H(kind, a, v):
    """Gaussian exp(-v^2), or the Voigt function H(a, v) = Re w(v + i a)."""
    if kind == "GAUSS":
        return math.exp(-v * v)
    from scipy.special import wofz
    return float(wofz(complex(v, a)).real)


def lte_pops(atom: BAtom, T, ne, ntot):
    """Boltzmann within a stage, Saha between stages (relative to level 0)."""
    kT = KB * T
    lam3 = (H * H / (2 * math.pi * ME * kT)) ** 1.5
    r = np.array([atom.g[i] / atom.g[0] * math.exp(-(atom.E[i] - atom.E[0]) / kT)
                  * (2.0 / (ne * lam3)) ** (atom.stage[i] - atom.stage[0]) for i in range(atom.L)])
    return ntot * r / r.sum()


def planck(nu, T):
    return 2 * H * nu ** 3 / C ** 2 / math.expm1(H * nu / (KB * T))


def lambda_matrix(dtau):
    """Exact Lambda matrix and boundary transmission along a ray with optical
    steps dtau[1..n-1]: I_q = M[q] . S + e_q I_0 for piecewise-linear S."""
    n = len(dtau)
    t = [mpmath.mpf(0)]
    for i in range(1, n):
        t.append(t[-1] + mpmath.mpf(float(dtau[i])))
    M = np.zeros((n, n))
    e = np.zeros(n)
    for q in range(n):
        e[q] = float(mpmath.exp(-t[q]))
        for i in range(1, q + 1):
            D = t[i] - t[i - 1]
            att = mpmath.exp(-(t[q] - t[i]))
            ed = mpmath.exp(-D)
            # integral over [t_{i-1}, t_i] of the two hat functions times exp(-(t_q - t))
            lo = (1 - ed * (1 + D)) / D      # hat of point i-1
            hi = 1 - (1 - ed) / D            # hat of point i
            M[q, i - 1] += float(att * lo)
            M[q, i] += float(att * hi)
    return M, e


class Problem:
    """A column, an atom and n_mu Gauss-Legendre angles: every ray's
    opacity terms as explicit functions of the populations."""

    def __init__(self, atom: BAtom, col: dict, n_mu: int, coll_scale: float = 1.0, damping_scale: float = 1.0):
        self.a, self.col = atom, col
        self.damping_scale = damping_scale
        self.N = len(col["z"])
        x, w = np.polynomial.legendre.leggauss(n_mu)
        self.mu, self.wmu = 0.5 * (x + 1), 0.5 * w
        T, ne, nH = col["T"], col["n_e"], col["n_H"]
        self.ntot = atom.abund * nH
        self.nstar = np.array([lte_pops(atom, T[k], ne[k], self.ntot[k]) for k in range(self.N)])
        self.rays = [(j, m, s) for j in range(len(atom.lam)) for m in range(n_mu) for s in (0, 1)]
        # normalised line profiles phi~[t][k][(j,m,s)]
        self.phi = {}
        self.norm = {ti: np.zeros(self.N) for ti in range(len(atom.tr))}
        for ti, d in enumerate(atom.tr):
            if d["kind"] != 0:
                continue
            ph = np.zeros((self.N, len(self.rays)))
            for k in range(self.N):
                dnd = d["nu0"] / C * math.sqrt(2 * KB * T[k] / atom.mass + col["v_turb"][k] ** 2)
                adamp = damping_scale * (atom.damping(ti) + d["c_el"] * col["n_H"][k]) / (4 * math.pi * dnd)
                tot = 0.0
                for r, (j, m, s) in enumerate(self.rays):
                    if j not in d["act"]:
                        continue
                    mus = self.mu[m] if s else -self.mu[m]
                    v = (atom.nu[j] - d["nu0"] * (1 + mus * col["v_z"][k] / C)) / dnd
                    ph[k, r] = _profile_H(d["profile"], adamp, v) / (math.sqrt(math.pi) * dnd)
                    tot += self.weight(ti, r) * ph[k, r]
                ph[k] /= tot
                self.norm[ti][k] = tot
            self.phi[ti] = ph
        self.C = np.zeros((self.N, atom.L, atom.L))
        for k in range(self.N):
            for d in atom.tr:
                l, u = d["l"], d["u"]
                if d["coll"] == "OMEGA":
                    Cul = ne[k] * 8.629e-12 * d["cval"] / (atom.g[u] * math.sqrt(T[k]))
                else:
                    eps = d["cval"]
                    Cul = eps / (1 - eps) * d["A"] / (-math.expm1(-H * d["nu0"] / (KB * T[k])))
                Cul *= coll_scale
                self.C[k, l, u] += Cul * self.nstar[k, u] / self.nstar[k, l]
                self.C[k, u, l] += Cul

    # ---------------------------------------------------------------- PRD
    rho = None      # {line index: [N][n_act]} emission / absorption profile ratio, None: CRD

    def rho_at(self, ti, k, j):
        if not self.rho or ti not in self.rho:
            return 1.0
        ja = int(np.nonzero(self.a.tr[ti]["act"] == j)[0][0])
        return self.rho[ti][k, ja]

    @staticmethod
    def hummer_rII(a, x, x2):
        """R_II-A of Hummer (1962) from its defining integral,
        pi^-3/2 int_{(xb - xs)/2}^inf exp(-u^2) [atan((xs + u)/a) - atan((xb - u)/a)] du
        (xb, xs the larger and smaller of x, x2), by adaptive quadrature."""
        from scipy.integrate import quad
        xb, xs = max(x, x2), min(x, x2)
        u0 = 0.5 * (xb - xs)
        f = lambda u: math.exp(-u * u) * (math.atan((xs + u) / a) - math.atan((xb - u) / a))
        pts = [p for p in (xb,) if p > u0]
        hi = max(u0, xb) + 9.0
        v1, _ = quad(f, u0, hi, points=pts or None, limit=400, epsabs=0, epsrel=1e-12)
        return v1 / math.pi ** 1.5

    def prd_rho(self, n, eps=1.0):
        """rho of every PRD line for populations n and the exact radiation
        field of the current rho (emission profile of a line whose upper level
        is partly populated by coherent scattering, angle-averaged R_II),
        switched by eps and normalised so that sum W phi rho = 1."""
        a, N, L = self.a, self.N, self.a.L
        T = self.col["T"]
        Ir = {}
        for r in range(len(self.rays)):
            if self.active(r):
                Ir[r] = self.intensity(r, n)
        out = {}
        for ti, d in enumerate(a.tr):
            if d["kind"] != 0 or not d["prd"]:
                continue
            l, u, act = d["l"], d["u"], d["act"]
            na = len(act)
            rho = np.zeros((N, na))
            for k in range(N):
                Pu = sum(self.C[k, u, i] for i in range(L) if i != u)
                for t2, d2 in enumerate(a.tr):
                    if d2["u"] != u and d2["l"] != u:
                        continue
                    for r, I in Ir.items():
                        if self.weight(t2, r) == 0.0:
                            continue
                        Vlu, Vul, U, kap = self.terms(t2, r, k)
                        Pu += kap * (U + Vul * I[k]) if d2["u"] == u else kap * Vlu * I[k]
                dnd = d["nu0"] / C * math.sqrt(2 * KB * T[k] / a.mass + self.col["v_turb"][k] ** 2)
                ad = (a.damping(ti) + d["c_el"] * self.col["n_H"][k]) / (4 * math.pi * dnd)
                x = (a.nu[act] - d["nu0"]) / dnd
                J = np.zeros(na)
                Jbar = 0.0
                for r, I in Ir.items():
                    j, m, s_ = self.rays[r]
                    if j not in act:
                        continue
                    ja = int(np.nonzero(act == j)[0][0])
                    J[ja] += 0.5 * self.wmu[m] * I[k]
                    Jbar += self.weight(ti, r) * self.phi[ti][k, r] * I[k]
                R = np.array([[self.hummer_rII(ad, x[i], x[i2]) for i2 in range(na)] for i in range(na)])
                gam = Pu / (Pu + d["c_el"] * self.col["n_H"][k])
                fac = gam * n[k, l] * d["Blu"] / (n[k, u] * Pu)
                for ja in range(na):
                    g = d["w"] * R[:, ja]
                    rr = 1.0 + fac * (g @ J / g.sum() - Jbar)
                    rho[k, ja] = max(rr * eps + (1.0 - eps), 0.0)
                norm = 0.0
                for r in Ir:
                    j, m, s_ = self.rays[r]
                    if j in act:
                        norm += self.weight(ti, r) * self.phi[ti][k, r] * rho[k, int(np.nonzero(act == j)[0][0])]
                rho[k] /= norm
            out[ti] = rho
        return out

    def weight(self, ti, r):
        j, m, s = self.rays[r]
        d = self.a.tr[ti]
        idx = np.nonzero(d["act"] == j)[0]
        return 0.0 if len(idx) == 0 else d["w"][idx[0]] * 0.5 * self.wmu[m]

    def terms(self, ti, r, k):
        """(V_lu, V_ul, U, kappa) of transition ti at ray r, depth k."""
        a, d = self.a, self.a.tr[ti]
        j = self.rays[r][0]
        nu = a.nu[j]
        W = self.weight(ti, r)
        if d["kind"] == 0:
            p = self.phi[ti][k, r]
            ps = p * self.rho_at(ti, k, j)
            c = H * d["nu0"] / (4 * math.pi)
            return c * d["Blu"] * p, c * d["Bul"] * ps, c * d["A"] * ps, 4 * math.pi * W / (H * d["nu0"])
        T = self.col["T"][k]
        alpha = d["alpha"] * (d["nu0"] / nu) ** 3
        G = self.nstar[k, d["l"]] / self.nstar[k, d["u"]] * math.exp(-H * nu / (KB * T))
        return alpha, G * alpha, 2 * H * nu ** 3 / C ** 2 * G * alpha, 4 * math.pi * W / (H * nu)

    def active(self, r):
        j = self.rays[r][0]
        return [ti for ti, d in enumerate(self.a.tr) if j in d["act"]]

    def background(self, r, k):
        j = self.rays[r][0]
        T = self.col["T"][k]
        kap = (self.a.c_bg * self.col["n_H"][k] * self.col["n_e"][k] * T ** -1.5 * math.exp(8750.0 / T)
               * self.a.lam[j] / 500e-9)
        return kap, kap * planck(self.a.nu[j], T)

    def ray_operator(self, r, chi):
        """Order of points along ray r, its Lambda matrix, boundary intensity
        and boundary transmission, for total opacity chi[k]."""
        j, m, s = self.rays[r]
        mu, z, N = self.mu[m], self.col["z"], self.N
        order = list(range(N)) if s == 0 else list(range(N - 1, -1, -1))
        dtau = np.zeros(N)
        for i in range(1, N):
            ka, kb = order[i - 1], order[i]
            dtau[i] = 0.5 * (chi[ka] + chi[kb]) * abs(z[ka] - z[kb]) / mu
        M, e = lambda_matrix(dtau)
        if s == 0:
            I0 = 0.0
        else:
            T = self.col["T"]
            nu = self.a.nu[j]
            B1, B2 = planck(nu, T[N - 1]), planck(nu, T[N - 2])
            dtv = 0.5 * (chi[N - 1] + chi[N - 2]) * (z[N - 2] - z[N - 1])
            I0 = B1 + mu * (B1 - B2) / dtv
        return order, M, e, I0

    def opacities(self, r, n):
        chi, eta, etabg = np.zeros(self.N), np.zeros(self.N), np.zeros(self.N)
        for k in range(self.N):
            cb, eb = self.background(r, k)
            chi[k], eta[k], etabg[k] = cb, eb, eb
            for ti in self.active(r):
                d = self.a.tr[ti]
                Vlu, Vul, U, _ = self.terms(ti, r, k)
                chi[k] += n[k, d["l"]] * Vlu - n[k, d["u"]] * Vul
                eta[k] += n[k, d["u"]] * U
        return chi, eta, etabg

    def intensity(self, r, n):
        """Exact I[k] of ray r for populations n (piecewise-linear S)."""
        chi, eta, _ = self.opacities(r, n)
        order, M, e, I0 = self.ray_operator(r, chi)
        S = (eta / chi)[order]
        Iord = M @ S + e * I0
        I = np.zeros(self.N)
        I[order] = Iord
        return I

    def rate_matrix(self, n):
        """Full rate matrix with the exact radiation field of populations n
        (classical Lambda iteration: no approximate operator)."""
        L, N = self.a.L, self.N
        G = np.zeros((N, L, L))
        for r in range(len(self.rays)):
            act = self.active(r)
            if not act:
                continue
            I = self.intensity(r, n)
            for k in range(N):
                for ti in act:
                    d = self.a.tr[ti]
                    Vlu, Vul, U, kap = self.terms(ti, r, k)
                    up = kap * Vlu * I[k]
                    down = kap * (U + Vul * I[k])
                    G[k, d["u"], d["l"]] += up; G[k, d["l"], d["l"]] -= up
                    G[k, d["l"], d["u"]] += down; G[k, d["u"], d["u"]] -= down
        for k in range(N):
            for i in range(L):
                for j in range(L):
                    if i != j:
                        G[k, j, i] += self.C[k, i, j]; G[k, i, i] -= self.C[k, i, j]
        return G

    def se_solve(self, G, nref):
        L = self.a.L
        out = np.zeros_like(nref)
        for k in range(self.N):
            A = G[k].copy()
            b = np.zeros(L)
            i = int(np.argmax(nref[k]))
            A[i, :] = 1.0
            b[i] = self.ntot[k]
            out[k] = np.linalg.solve(A, b)
        return out

    def preconditioned_step(self, nold):
        """One MALI step assembled by brute force: the net radiative rates
        with I = I_eff + Psi* eta(n_new), the opacity of the transition
        taken at n_old and the diagonal operator of the exact Lambda
        matrix, are linear in n_new; their matrix is read off by
        evaluating them on the basis vectors."""
        L, N = self.a.L, self.N
        # per ray: I_eff = I - Psi* eta_atom(n_old), Psi* = Lambda*_kk / chi_k
        ray_data = []
        for r in range(len(self.rays)):
            act = self.active(r)
            if not act:
                continue
            chi, eta, etabg = self.opacities(r, nold)
            order, M, e, I0 = self.ray_operator(r, chi)
            S = (eta / chi)[order]
            Iord = M @ S + e * I0
            I = np.zeros(N); lst = np.zeros(N)
            I[order] = Iord
            lst[order] = np.diag(M)
            psi = lst / chi
            Ieff = I - psi * (eta - etabg)
            ray_data.append((r, act, Ieff, psi))

        def net_rates(nnew):
            F = np.zeros((N, L))
            for r, act, Ieff, psi in ray_data:
                for k in range(N):
                    eta_new = 0.0
                    for ti in act:
                        d = self.a.tr[ti]
                        _, _, U, _ = self.terms(ti, r, k)
                        eta_new += nnew[k, d["u"]] * U
                    for ti in act:
                        d = self.a.tr[ti]
                        Vlu, Vul, U, kap = self.terms(ti, r, k)
                        chi_old = nold[k, d["l"]] * Vlu - nold[k, d["u"]] * Vul
                        # net upward rate with the transition's opacity at n_old
                        # multiplying Psi* eta, and at n_new multiplying I_eff
                        net = kap * ((nnew[k, d["l"]] * Vlu - nnew[k, d["u"]] * Vul) * Ieff[k]
                                     + chi_old * psi[k] * eta_new - nnew[k, d["u"]] * U)
                        F[k, d["u"]] += net
                        F[k, d["l"]] -= net
            return F

        G = np.zeros((N, L, L))
        for i in range(L):
            e = np.zeros((N, L)); e[:, i] = 1.0
            F = net_rates(e)
            for k in range(N):
                G[k, :, i] = F[k]
        for k in range(N):
            for i in range(L):
                for j in range(L):
                    if i != j:
                        G[k, j, i] += self.C[k, i, j]; G[k, i, i] -= self.C[k, i, j]
        return self.se_solve(G, nold)

    def emergent(self, n):
        """Exact vertical (mu = 1) emergent intensity at every wavelength."""
        a, N, z, T = self.a, self.N, self.col["z"], self.col["T"]
        out = np.zeros(len(a.lam))
        for j in range(len(a.lam)):
            nu = a.nu[j]
            chi, eta = np.zeros(N), np.zeros(N)
            for k in range(N):
                kap = (a.c_bg * self.col["n_H"][k] * self.col["n_e"][k] * T[k] ** -1.5
                       * math.exp(8750.0 / T[k]) * a.lam[j] / 500e-9)
                chi[k], eta[k] = kap, kap * planck(nu, T[k])
                for ti, d in enumerate(a.tr):
                    if j not in d["act"]:
                        continue
                    if d["kind"] == 0:
                        dnd = d["nu0"] / C * math.sqrt(2 * KB * T[k] / a.mass + self.col["v_turb"][k] ** 2)
                        v = (nu - d["nu0"] * (1 + self.col["v_z"][k] / C)) / dnd
                        adamp = self.damping_scale * (a.damping(ti) + d["c_el"] * self.col["n_H"][k]) / (4 * math.pi * dnd)
                        p = _profile_H(d["profile"], adamp, v) / (math.sqrt(math.pi) * dnd) / self.norm[ti][k]
                        ps = p * self.rho_at(ti, k, j)
                        c = H * d["nu0"] / (4 * math.pi)
                        Vlu, Vul, U = c * d["Blu"] * p, c * d["Bul"] * ps, c * d["A"] * ps
                    else:
                        alpha = d["alpha"] * (d["nu0"] / nu) ** 3
                        G = self.nstar[k, d["l"]] / self.nstar[k, d["u"]] * math.exp(-H * nu / (KB * T[k]))
                        Vlu, Vul, U = alpha, G * alpha, 2 * H * nu ** 3 / C ** 2 * G * alpha
                    chi[k] += n[k, d["l"]] * Vlu - n[k, d["u"]] * Vul
                    eta[k] += n[k, d["u"]] * U
            order = list(range(N - 1, -1, -1))
            dtau = np.zeros(N)
            for i in range(1, N):
                ka, kb = order[i - 1], order[i]
                dtau[i] = 0.5 * (chi[ka] + chi[kb]) * abs(z[ka] - z[kb])
            M, e = lambda_matrix(dtau)
            B1, B2 = planck(nu, T[N - 1]), planck(nu, T[N - 2])
            I0 = B1 + (B1 - B2) / dtau[1]
            out[j] = M[-1] @ (eta / chi)[order] + e[-1] * I0
        return out

    def psi_star(self, n):
        """Per-transition average of Psi* = Lambda*_kk / chi_k over the
        transition's rays, weighted by W phi~ (lines) or W / sum W (continua)."""
        a, N = self.a, self.N
        out = np.zeros((len(a.tr), N))
        wsum = [d["w"].sum() for d in a.tr]
        for r in range(len(self.rays)):
            act = self.active(r)
            if not act:
                continue
            chi, _, _ = self.opacities(r, n)
            order, M, _, _ = self.ray_operator(r, chi)
            lst = np.zeros(N)
            lst[order] = np.diag(M)
            for ti in act:
                d = a.tr[ti]
                for k in range(N):
                    W = self.weight(ti, r)
                    om = W * self.phi[ti][k, r] if d["kind"] == 0 else W / wsum[ti]
                    out[ti, k] += om * lst[k] / chi[k]
        return out


def psi_ray(P: Problem, n):
    """Psi* = Lambda*_kk / chi_k of every ray, [N][NL][n_mu][2] (0 where the
    ray has no active transition)."""
    NL, nmu = len(P.a.lam), len(P.mu)
    out = np.zeros((P.N, NL, nmu, 2))
    for r, (j, m, s) in enumerate(P.rays):
        if not P.active(r):
            continue
        chi, _, _ = P.opacities(r, n)
        order, M, _, _ = P.ray_operator(r, chi)
        lst = np.zeros(P.N)
        lst[order] = np.diag(M)
        out[:, j, m, s] = lst / chi
    return out
