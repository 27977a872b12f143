// Host-side model-atom setup of librh15d: file parser, atomic data, the
// union wavelength grid with each transition's active points and
// frequency weights, the Gauss-Legendre angles, and the ray groups that
// the formal-solution kernel maps onto 64-lane wavefronts.
#include <algorithm>
#include <iterator>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <fstream>
#include <sstream>

#include "rh15d_internal.h"

namespace rh15d {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

const char *last_error() { return g_err; }

namespace {

class Tokens {
  public:
    explicit Tokens(std::istream &in) {
        std::string line;
        while (std::getline(in, line)) {
            auto h = line.find('#');
            if (h != std::string::npos) line.resize(h);
            std::istringstream ls(line);
            std::string t;
            while (ls >> t) toks_.push_back(t);
        }
    }
    bool word(std::string &w) {
        if (pos_ >= toks_.size()) return false;
        w = toks_[pos_++];
        return true;
    }
    bool expect(const char *kw) {
        std::string w;
        return word(w) && w == kw;
    }
    bool num(double &v) {
        std::string w;
        if (!word(w)) return false;
        char *e = nullptr;
        v = std::strtod(w.c_str(), &e);
        return e && *e == 0;
    }
    bool integer(int &v) {
        double d;
        if (!num(d) || d != std::floor(d)) return false;
        v = static_cast<int>(d);
        return true;
    }

  private:
    std::vector<std::string> toks_;
    size_t pos_ = 0;
};

bool read_transition(Tokens &tk, HostTransition &t, int kind, int L) {
    t.kind = kind;
    if (!tk.integer(t.l) || !tk.integer(t.u)) return false;
    if (t.l < 0 || t.u >= L || t.l >= t.u) return false;
    std::string w;
    if (kind == 0) {
        if (!tk.num(t.f) || !tk.word(w)) return false;
        if (w == "VOIGT") t.voigt = 1;
        else if (w == "GAUSS") t.voigt = 0;
        else return false;
    } else if (!tk.num(t.alpha0)) {
        return false;
    }
    if (!tk.word(w)) return false;
    if (w == "OMEGA") t.coll_kind = 0;
    else if (w == "EPS") t.coll_kind = 1;
    else return false;
    int n;
    if (!tk.num(t.coll_val) || !tk.integer(n) || n < 2) return false;
    t.own.resize(n);
    for (auto &x : t.own) {
        if (!tk.num(x)) return false;
        x *= 1e-9;
    }
    return true;
}

}  // namespace

// Zeeman pattern of a dipole line (Sec. 2.1: Zeeman splitting), from the
// Condon & Shortley relative strengths of the components for J_u - J_l =
// +1, 0, -1 (J, M of the lower level; M_u = M, M + 1, M - 1), normalised
// to unit sum per q = M_l - M_u; the component M_u -> M_l is shifted by
// g_u M_u - g_l M_l Larmor frequencies.  Nothing for |J_u - J_l| > 1 or
// J_u = J_l = 0.
void zeeman_components(int twoJl, double gl, int twoJu, double gu, HostTransition &t) {
    t.zq.clear(); t.zshift.clear(); t.zstr.clear();
    const int d2 = twoJu - twoJl;
    if (d2 != 2 && d2 != 0 && d2 != -2) return;
    const double J = 0.5 * twoJl, Ju = 0.5 * twoJu;
    double sum[3] = {0, 0, 0};
    for (int tm = -twoJl; tm <= twoJl; tm += 2) {
        const double M = 0.5 * tm;
        for (int q = -1; q <= 1; q++) {
            const double Mu = M - q;
            if (std::fabs(Mu) > Ju + 1e-9) continue;
            double s;
            if (d2 == 2) s = q == 0 ? (J + 1) * (J + 1) - M * M
                           : q == -1 ? 0.25 * (J + M + 1) * (J + M + 2) : 0.25 * (J - M + 1) * (J - M + 2);
            else if (d2 == 0) s = q == 0 ? M * M : q == -1 ? 0.25 * (J - M) * (J + M + 1) : 0.25 * (J + M) * (J - M + 1);
            else s = q == 0 ? J * J - M * M : q == -1 ? 0.25 * (J - M) * (J - M - 1) : 0.25 * (J + M) * (J + M - 1);
            if (!(s > 0.0)) continue;
            t.zq.push_back(q);
            t.zshift.push_back(gu * Mu - gl * M);
            t.zstr.push_back(s);
            sum[q + 1] += s;
        }
    }
    for (size_t i = 0; i < t.zq.size(); i++) t.zstr[i] /= sum[t.zq[i] + 1];
    // a pattern needs components of every q (J_u = J_l = 0 has none)
    if (!(sum[0] > 0 && sum[1] > 0 && sum[2] > 0)) { t.zq.clear(); t.zshift.clear(); t.zstr.clear(); }
}

int parse_atom_file(const char *path, rh15d_atom *a, std::string &err) {
    std::ifstream in(path);
    if (!in) { err = std::string("cannot open ") + path; return RH15D_EIO; }
    Tokens tk(in);
    std::string w;
    int ver, nl, nc;
    bool ok = tk.expect("RH15D-ATOM") && tk.integer(ver) && tk.expect("NAME") && tk.word(w) &&
              tk.expect("MASS_AMU") && tk.num(a->mass) && tk.expect("ABUNDANCE") && tk.num(a->abund) &&
              tk.expect("LEVELS") && tk.integer(a->L);
    if (!ok || a->L < 2) { err = "malformed header or level count"; return RH15D_EIO; }
    if (a->L > RH15D_MAX_LEVELS) { err = "too many levels"; return RH15D_EINVAL; }
    a->mass *= kAMU;
    a->E.resize(a->L); a->g.resize(a->L); a->stage.resize(a->L);
    for (int i = 0; i < a->L; i++) {
        if (!tk.num(a->E[i]) || !tk.num(a->g[i]) || !tk.integer(a->stage[i])) { err = "malformed level"; return RH15D_EIO; }
        a->E[i] *= kQE;
    }
    if (!tk.expect("LINES") || !tk.integer(nl) || nl < 0) { err = "malformed LINES"; return RH15D_EIO; }
    a->tr.resize(nl);
    for (int i = 0; i < nl; i++)
        if (!read_transition(tk, a->tr[i], 0, a->L)) { err = "malformed line"; return RH15D_EIO; }
    if (!tk.expect("CONTINUA") || !tk.integer(nc) || nc < 0) { err = "malformed CONTINUA"; return RH15D_EIO; }
    a->tr.resize(nl + nc);
    for (int i = 0; i < nc; i++)
        if (!read_transition(tk, a->tr[nl + i], 1, a->L)) { err = "malformed continuum"; return RH15D_EIO; }
    a->n_lines = nl; a->n_cont = nc;
    // optional: elastic collisions and the redistribution of lines
    if (!tk.word(w)) { err = "malformed atom file"; return RH15D_EIO; }
    if (w == "ELASTIC") {
        int ne;
        if (!tk.integer(ne) || ne < 0) { err = "malformed ELASTIC"; return RH15D_EIO; }
        for (int i = 0; i < ne; i++) {
            int li;
            double c;
            std::string kind;
            if (!tk.integer(li) || li < 0 || li >= nl || !tk.num(c) || !(c >= 0.0) || !tk.word(kind) ||
                (kind != "PRD" && kind != "CRD")) {
                err = "malformed ELASTIC row"; return RH15D_EIO;
            }
            a->tr[li].c_el = c;
            a->tr[li].prd = kind == "PRD";
        }
        if (!tk.word(w)) { err = "malformed atom file"; return RH15D_EIO; }
    }
    a->twoJ.assign(a->L, -1);
    a->gL.assign(a->L, 0.0);
    if (w == "ZEEMAN") {
        int nz;
        if (!tk.integer(nz) || nz < 0) { err = "malformed ZEEMAN"; return RH15D_EIO; }
        for (int i = 0; i < nz; i++) {
            int li, tj;
            double gl;
            if (!tk.integer(li) || li < 0 || li >= a->L || !tk.integer(tj) || tj < 0 || tj > 40 || !tk.num(gl)) {
                err = "malformed ZEEMAN row"; return RH15D_EIO;
            }
            a->twoJ[li] = tj;
            a->gL[li] = gl;
        }
        if (!tk.word(w)) { err = "malformed atom file"; return RH15D_EIO; }
    }
    if (w != "BACKGROUND" || !tk.word(w)) { err = "malformed BACKGROUND"; return RH15D_EIO; }
    if (w == "NONE") a->bg_kind = 0;
    else if (w == "HMINUS") { a->bg_kind = 1; if (!tk.num(a->c_bg)) { err = "malformed HMINUS"; return RH15D_EIO; } }
    else { err = "unknown background"; return RH15D_EIO; }
    if (!tk.expect("END")) { err = "missing END"; return RH15D_EIO; }
    if (a->tr.empty()) { err = "atom has no transitions"; return RH15D_EIO; }

    // atomic data
    for (auto &t : a->tr) {
        double dE = a->E[t.u] - a->E[t.l];
        if (!(dE > 0)) { err = "transition without a positive energy gap"; return RH15D_EIO; }
        t.nu0 = dE / kH;
        if (t.kind == 0) {
            // A_ul = (2 pi e^2 nu^2 / (eps0 m_e c^3)) (g_l / g_u) f_lu; B from the Einstein relations
            t.A = 2.0 * kPI * kQE * kQE * t.nu0 * t.nu0 / (kEPS0 * kME * kC * kC * kC) * (a->g[t.l] / a->g[t.u]) * t.f;
            t.Bul = t.A * kC * kC / (2.0 * kH * t.nu0 * t.nu0 * t.nu0);
            t.Blu = t.Bul * a->g[t.u] / a->g[t.l];
        }
        auto mm = std::minmax_element(t.own.begin(), t.own.end());
        t.lam_min = *mm.first;
        t.lam_max = *mm.second;
    }
    // radiative damping width: spontaneous rates out of the upper and lower level
    for (auto &t : a->tr) {
        if (t.kind != 0) continue;
        double gam = 0;
        for (const auto &s : a->tr)
            if (s.kind == 0 && (s.u == t.u || s.u == t.l)) gam += s.A;
        t.gamma = gam;
    }
    // Zeeman patterns of the lines whose two levels carry J and g
    for (auto &t : a->tr) {
        if (t.kind != 0 || a->twoJ[t.l] < 0 || a->twoJ[t.u] < 0) continue;
        zeeman_components(a->twoJ[t.l], a->gL[t.l], a->twoJ[t.u], a->gL[t.u], t);
        if (t.zq.empty()) { err = "a Zeeman-split line whose J values allow no dipole transition"; return RH15D_EIO; }
    }
    // union wavelength grid
    std::vector<double> all;
    for (const auto &t : a->tr) all.insert(all.end(), t.own.begin(), t.own.end());
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    a->lam = all;
    a->nu.resize(all.size());
    for (size_t j = 0; j < all.size(); j++) a->nu[j] = kC / all[j];
    const int NL = static_cast<int>(all.size());
    for (auto &t : a->tr) {
        for (int j = 0; j < NL; j++)
            if (a->lam[j] >= t.lam_min && a->lam[j] <= t.lam_max) t.act.push_back(j);
        const int n = static_cast<int>(t.act.size());
        t.w.assign(n, 0.0);
        for (int i = 0; i + 1 < n; i++) {  // trapezoid in frequency
            double h = 0.5 * (a->nu[t.act[i]] - a->nu[t.act[i + 1]]);
            t.w[i] += h;
            t.w[i + 1] += h;
        }
    }
    // per wavelength: which transitions are active (CSR)
    a->jact_off.assign(NL + 1, 0);
    for (int j = 0; j < NL; j++) {
        for (int ti = 0; ti < static_cast<int>(a->tr.size()); ti++) {
            const auto &t = a->tr[ti];
            if (std::binary_search(t.act.begin(), t.act.end(), j)) a->jact_t.push_back(ti);
        }
        a->jact_off[j + 1] = static_cast<int>(a->jact_t.size());
    }
    return RH15D_OK;
}

void gauss_legendre_01(int n, std::vector<double> &x, std::vector<double> &w) {
    // Newton iteration on the roots of P_n, mapped from (-1,1) to (0,1).
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; i++) {
        double r = std::cos(kPI * (n - i - 0.25) / (n + 0.5));  // ascending roots
        double dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = r;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2 * k - 1) * r * p1 - (k - 1) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (r * p1 - p0) / (r * r - 1.0);
            double step = p1 / dp;
            r -= step;
            if (std::fabs(step) < 1e-16) break;
        }
        double p0 = 1.0, p1 = r;
        for (int k = 2; k <= n; k++) {
            double p2 = ((2 * k - 1) * r * p1 - (k - 1) * p0) / k;
            p0 = p1; p1 = p2;
        }
        dp = n * (r * p1 - p0) / (r * r - 1.0);
        x[i] = 0.5 * (r + 1.0);
        w[i] = 1.0 / ((1.0 - r * r) * dp * dp);
    }
}

// Lanes of one direction are taken in order of wavelength (then angle chunk)
// and cut into groups of at most 64.  With pack = 0 a group shares one set
// of active transitions; with pack = 1 neighbouring wavelengths with
// different sets share a group as long as their union has at most
// kMaxSlots transitions (a lane contributes zero to a slot whose
// transition is not active at its wavelength).
void build_group_tables(const rh15d_atom &a, int n_mu, SweepShape shape, HostGroupTables &out) {
    out = HostGroupTables{};
    gauss_legendre_01(n_mu, out.mu, out.wmu);
    const int T = static_cast<int>(a.tr.size());
    const int NL = static_cast<int>(a.lam.size());
    const int mc = shape.mc;
    const int chunks = n_mu / mc;
    std::vector<int> ray_off(T, -1);
    int cols = 0;
    for (int t = 0; t < a.n_lines; t++) {
        // per line: quadrature rays (2 directions x n_mu angles x wavelengths),
        // then the vertical emergent ray at each wavelength
        ray_off[t] = cols;
        cols += (2 * n_mu + 1) * static_cast<int>(a.tr[t].act.size());
    }
    out.ray_cols = cols;
    // PRD lines: their rays' columns in the emission-profile row (same order
    // as in the profile row); wavelengths whose intensities the rho update
    // reads: those of the PRD lines and of every transition into or out of
    // a PRD line's upper level (its total depopulation rate)
    out.psi_off.assign(T, -1);
    int pcols = 0;
    std::vector<char> upper(a.L, 0), stored(T, 0);
    for (int t = 0; t < a.n_lines; t++)
        if (a.tr[t].prd) {
            out.psi_off[t] = pcols;
            pcols += (2 * n_mu + 1) * static_cast<int>(a.tr[t].act.size());
            upper[a.tr[t].u] = 1;
        }
    out.psi_cols = pcols;
    for (int t = 0; t < T; t++) stored[t] = a.tr[t].prd || upper[a.tr[t].u] || upper[a.tr[t].l];
    out.st_idx.assign(NL, -1);
    int nst = 0;
    if (pcols > 0)
        for (int j = 0; j < NL; j++)
            for (int i = a.jact_off[j]; i < a.jact_off[j + 1]; i++)
                if (stored[a.jact_t[i]]) { out.st_idx[j] = nst++; break; }
    out.ist_cols = nst * n_mu * 2;

    std::vector<std::vector<int>> p_keys(T), q_keys(T);
    std::map<std::pair<int, int>, std::vector<int>> x_keys;
    int key = 0;
    auto active_set = [&](int j) {
        return std::vector<int>(a.jact_t.begin() + a.jact_off[j], a.jact_t.begin() + a.jact_off[j + 1]);
    };
    for (int s = 0; s < 2; s++) {
        std::vector<std::pair<int, int>> lanes;  // (j, chunk)
        std::vector<int> cur;                     // sorted union of the group's transitions
        auto flush = [&]() {
            if (lanes.empty()) return;
            if (static_cast<int>(cur.size()) > kMaxSlots) { out.overflow = true; lanes.clear(); return; }
            DevGroup G{};
            G.s = s;
            G.n_slots = static_cast<int>(cur.size());
            for (int q = 0; q < G.n_slots; q++) G.t[q] = cur[q];
            G.n_pairs = 0;
            for (int q = 0; q < G.n_slots; q++)
                for (int q2 = 0; q2 < G.n_slots; q2++)
                    if (q != q2) G.pair[G.n_pairs++] = q * kMaxSlots + q2;
            G.key_off = key;
            G.n_keys = 2 * G.n_slots + G.n_pairs;
            G.n_lanes = static_cast<int>(lanes.size());
            G.n_line_slots = 0;
            for (int q = 0; q < G.n_slots; q++) G.n_line_slots += a.tr[cur[q]].kind == 0;
            for (int q = 0; q < G.n_slots; q++) {
                p_keys[cur[q]].push_back(key + q);
                q_keys[cur[q]].push_back(key + G.n_slots + q);
            }
            for (int p = 0; p < G.n_pairs; p++) {
                int q = G.pair[p] / kMaxSlots, q2 = G.pair[p] % kMaxSlots;
                x_keys[{cur[q], cur[q2]}].push_back(key + 2 * G.n_slots + p);
            }
            key += G.n_keys;
            out.groups.push_back(G);
            for (int l = 0; l < kWave; l++) {
                const bool real = l < static_cast<int>(lanes.size());
                const int j = real ? lanes[l].first : lanes[0].first;
                const int m0 = (real ? lanes[l].second : lanes[0].second) * mc;
                const double nu = a.nu[j];
                out.lane_j.push_back(j);
                out.lane_m0.push_back(m0);
                out.lane_lamfac.push_back(a.lam[j] / kBgLambdaRef);
                out.lane_hnu_k.push_back(kH * nu / kKB);
                out.lane_2hnu3c2.push_back(2.0 * kH * nu * nu * nu / (kC * kC));
                out.lane_ist.push_back(real && out.st_idx[j] >= 0 ? (out.st_idx[j] * n_mu + m0) * 2 + s : -1);
                for (int q = 0; q < kMaxSlots; q++) {
                    int pb = -1, ps = -1;
                    double wj = 0, kapj = 0, alpha = 0;
                    // padding lanes repeat lane 0's ray with zero weights, so their
                    // opacity stays finite and their contributions vanish
                    if (q < G.n_slots) {
                        const auto &tr = a.tr[cur[q]];
                        auto it = std::lower_bound(tr.act.begin(), tr.act.end(), j);
                        if (it != tr.act.end() && *it == j) {
                            const int ja = static_cast<int>(it - tr.act.begin());
                            const int na = static_cast<int>(tr.act.size());
                            wj = real ? tr.w[ja] : 0.0;
                            if (tr.kind == 0) {
                                pb = ray_off[cur[q]] + (s * na + ja) * n_mu + m0;
                                if (out.psi_off[cur[q]] >= 0) ps = out.psi_off[cur[q]] + (s * na + ja) * n_mu + m0;
                                kapj = 4.0 * kPI * wj * 0.5 / (kH * tr.nu0);
                            } else {
                                kapj = 4.0 * kPI * wj * 0.5 / (kH * nu);
                                alpha = tr.alpha0 * std::pow(tr.nu0 / nu, 3.0);
                            }
                        }
                    }
                    out.pbase.push_back(pb);
                    out.psb.push_back(ps);
                    out.wj.push_back(wj);
                    out.kapj.push_back(kapj);
                    out.alpha.push_back(alpha);
                }
            }
            out.lanes_used += static_cast<int>(lanes.size()) * mc;
            lanes.clear();
            cur.clear();
        };
        for (int j = 0; j < NL; j++) {
            const std::vector<int> set = active_set(j);
            if (set.empty()) continue;
            for (int ch = 0; ch < chunks; ch++) {
                std::vector<int> uni;
                std::set_union(cur.begin(), cur.end(), set.begin(), set.end(), std::back_inserter(uni));
                const bool full = static_cast<int>(lanes.size()) == kWave;
                const bool differs = shape.pack == 0 ? (!lanes.empty() && set != cur)
                                                     : static_cast<int>(uni.size()) > kMaxSlots;
                if (full || differs) {
                    flush();
                    uni = set;
                }
                cur = uni;
                lanes.push_back({j, ch});
            }
        }
        flush();
    }
    out.n_keys = key;
    auto csr = [&](const std::vector<std::vector<int>> &lists, std::vector<int> &off, std::vector<int> &val) {
        off.assign(lists.size() + 1, 0);
        for (size_t i = 0; i < lists.size(); i++) {
            val.insert(val.end(), lists[i].begin(), lists[i].end());
            off[i + 1] = static_cast<int>(val.size());
        }
    };
    csr(p_keys, out.p_off, out.p_key);
    csr(q_keys, out.q_off, out.q_key);
    out.x_off.push_back(0);
    for (const auto &kv : x_keys) {
        out.x_t.push_back(kv.first.first);
        out.x_t2.push_back(kv.first.second);
        out.x_key.insert(out.x_key.end(), kv.second.begin(), kv.second.end());
        out.x_off.push_back(static_cast<int>(out.x_key.size()));
    }
}

}  // namespace rh15d
