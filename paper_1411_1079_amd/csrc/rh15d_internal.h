// Internal data structures of librh15d shared by the host-side setup
// (atom_setup.cpp) and the gfx950 kernels (mali.hip).
#pragma once

#include <cstdint>
#include <string>
#include <vector>
#include <map>
#include <mutex>

#include "rh15d.h"

namespace rh15d {

// CODATA 2018, SI
constexpr double kH = 6.62607015e-34;
constexpr double kC = 2.99792458e8;
constexpr double kKB = 1.380649e-23;
constexpr double kME = 9.1093837015e-31;
constexpr double kQE = 1.602176634e-19;
constexpr double kEPS0 = 8.8541878128e-12;
constexpr double kAMU = 1.66053906660e-27;
constexpr double kPI = 3.14159265358979323846;
// Omega electron-impact model: C_ul = n_e * kCollC0 * Omega / (g_u sqrt(T))
constexpr double kCollC0 = 8.629e-12;
// background law kappa = C_bg n_H n_e T^-3/2 exp(kBgTheta/T) (lambda / kBgLambdaRef)
constexpr double kBgLambdaRef = 500.0e-9;
constexpr double kBgTheta = 8750.0;

// A wavefront of 64 rays ("group") touches at most this many transitions.
constexpr int kMaxSlots = 4;
constexpr int kMaxPairs = kMaxSlots * (kMaxSlots - 1);
constexpr int kMaxKeys = 2 * kMaxSlots + kMaxPairs;
// Groups are classed by (slots n, continuum slots c), c <= n <= kMaxSlots,
// in the order of n, then c; class ids run over 0 .. kGroupClasses - 1
// (n = 0 is not a real group but keeps the formula simple).
constexpr int kGroupClasses = (kMaxSlots + 1) * (kMaxSlots + 2) / 2 + (kMaxSlots + 2);
__host__ __device__ constexpr int group_class(int n, int c) { return n * (n + 1) / 2 + c; }
constexpr int kWave = 64;

struct HostTransition {
    int kind = 0;  // 0 line, 1 continuum
    int l = 0, u = 0;
    double f = 0, alpha0 = 0, coll_val = 0;
    double c_el = 0;          // elastic-collision rate per hydrogen atom, m^3 s^-1
    int voigt = 0, coll_kind = 0;
    int prd = 0;              // line with partial frequency redistribution
    // Zeeman components of a line whose levels carry J and g: q = M_l - M_u,
    // shift g_u M_u - g_l M_l (Larmor frequencies), strength (sums to 1 per q)
    std::vector<int> zq;
    std::vector<double> zshift, zstr;
    std::vector<double> own;  // own sampling, m
    // derived
    double nu0 = 0, A = 0, Bul = 0, Blu = 0, gamma = 0, lam_min = 0, lam_max = 0;
    std::vector<int> act;     // active union indices (increasing wavelength)
    std::vector<double> w;    // trapezoid weights in frequency
};

// Plain-old-data transition record as the kernels read it.
struct DevTransition {
    int kind, l, u, voigt;
    int coll_kind, n_act, act_off, ray_off;  // ray_off: offset of this line's rays in a depth row
    int prd, psi_off;                         // PRD line: offset of its rays in the emission-profile row, else -1
    int g_off, pad0;                          // PRD line: offset of its redistribution weights per depth
    double nu0, A, Bul, Blu;                  // Einstein coefficients (per unit frequency)
    double alpha0, coll_val, gamma, hnu4pi;   // hnu4pi = h nu0 / (4 pi)
    double wsum;                              // sum of the trapezoid weights
    double c_el;                              // elastic-collision rate per hydrogen atom
    int n_zc, zc_off;                         // Zeeman components (0: not split) and their offset
};

// A group: up to 64 rays of one direction sharing one set of transitions.
struct DevGroup {
    int s;            // 0 down (top to bottom), 1 up
    int n_slots;      // transitions touched
    int t[kMaxSlots]; // transition index of each slot
    int n_pairs;      // ordered slot pairs (q, q') accumulated as cross terms
    int pair[kMaxPairs];  // q * kMaxSlots + q'
    int key_off;      // first key of this group
    int n_keys;       // 2 n_slots + n_pairs
    int n_lanes;      // rays carried (the rest of the 64 lanes are padding)
    int n_line_slots; // slots that are lines (read a profile row per ray-step)
};

// Per-lane constants (structure of arrays, index group * 64 + lane).  A lane
// carries one wavelength and `mc` consecutive angles of one direction.
struct DevLanes {
    int *j;           // union wavelength index
    int *m0;          // first angle index of the lane
    double *lamfac;   // lambda / kBgLambdaRef
    double *hnu_k;    // h nu / k_B
    double *two_hnu3c2;
    // per slot q (index (group*64+lane)*kMaxSlots + q); zero/-1 where the
    // slot's transition is not active at this lane's wavelength
    int *pbase;       // line: profile column of the lane's first angle; else -1
    double *wj;       // frequency weight w(t, j)
    double *kapj;     // 4 pi w(t, j) / (2 h nu_t): times w_mu gives the rate weight
    double *alpha;    // continuum cross-section at nu_j
    int *psb;         // per slot: PRD line: emission-profile column of the lane's first angle; else -1
    int *ist;         // stored-intensity column of the lane's first angle (step 2 per angle), or -1
};
// Everything the kernels need about an atom and an angle quadrature.
struct DevAtom {
    int L, n_lines, n_cont, T, NL, n_mu;
    int n_groups, n_keys;       // ray groups and rate keys per depth
    int mc, pack;               // angles per lane, packing of wavelengths into groups
    int g_begin[kGroupClasses + 1]; // groups of class c (group_class) are [g_begin[c], g_begin[c+1])
    int ray_cols;               // line rays per depth row: sum over lines of 2 n_act n_mu
    int pad0;
    double mass, abund, c_bg;
    int bg_kind, pad1;
    double *E, *g; int *stage;  // levels
    DevTransition *tr;
    double *lam, *nu;           // union grid
    int *act_j; double *act_w;  // concatenated active lists and weights
    double *mu, *wmu;           // Gauss-Legendre on (0,1)
    int *jact_off, *jact_t;     // per wavelength: active transitions (CSR)
    int *jact_ja;               // ... and the wavelength's index in each one's active list
    // per line ray, in the order the preparation visits them (CSR over
    // lines): place in the profile table's row, frequency, signed direction
    // cosine, quadrature weight
    int *prof_off, *prof_dst; double *prof_nu, *prof_mus, *prof_w;
    float *prof_dnu, *prof_musf;  // the same rays in FP32: nu - nu0 of the ray's line, mu
                                  // (for the FP32 profile table, without FP64 arithmetic)
    DevGroup *groups;
    DevLanes lanes;
    // rate keys per transition and per ordered transition pair (CSR)
    int *p_off, *p_key;         // [T+1], keys of P_t
    int *q_off, *q_key;         // [T+1], keys of Q'_t
    int n_xpairs;
    int *x_t, *x_t2, *x_off, *x_key;  // [n_xpairs], [n_xpairs+1]
    // rate-matrix entry (i, j), i != j (rate from level j into level i):
    // the transition whose upward (l = j, u = i) or downward (u = j, l = i)
    // rates land there, or -1; and the cross terms landing there (CSR over
    // i * L + j, +xpair+1 adds, -(xpair+1) subtracts)
    int *up_t, *dn_t;           // [L * L]
    int *xe_off, *xe_val;       // [L * L + 1], [...]
    // partial frequency redistribution (PRD lines of the atom)
    int n_prd;                  // PRD lines
    int psi_cols;               // emission-profile (psi = rho phi) values per depth row
    int ist_cols;               // stored intensities per depth row: (stored wavelength, angle, direction)
    int g_cols;                 // redistribution weights per depth row: sum over PRD lines of n_act^2
    int *prd_t;                 // [n_prd] line index of each PRD line
    int *st_idx;                // [NL] stored-wavelength index of each wavelength, or -1
    // Zeeman components of the split lines, concatenated (DevTransition.zc_off)
    int *zq;
    double *zshift, *zstr;
    // algorithmic work of one rate-mode sweep per depth point of a column
    double rays_per_depth;        // rays (wavelength x angle x direction)
    double flops_per_depth;       // see k_raysweep: 27 + 19 n_slots + 4 n_pairs per ray-step
    double reads_per_depth;       // profile values read
    double keys_per_depth;        // reduced rate values written
};

// Shape of the formal-solution work: angles carried per lane and how
// wavelengths with different active transitions are packed into groups.
struct SweepShape {
    int mc = 1;      // angles per lane (divides n_mu)
    int pack = 0;    // 0: one set of active transitions per group; 1: mixed sets up to kMaxSlots
    bool operator<(const SweepShape &o) const { return mc != o.mc ? mc < o.mc : pack < o.pack; }
};

struct HostGroupTables {
    std::vector<DevGroup> groups;
    std::vector<int> lane_j, lane_m0, pbase, psb, lane_ist;
    std::vector<int> psi_off, st_idx;   // per transition; per wavelength
    int psi_cols = 0, ist_cols = 0;
    std::vector<double> lane_lamfac, lane_hnu_k, lane_2hnu3c2, wj, kapj, alpha;
    std::vector<int> p_off, p_key, q_off, q_key, x_t, x_t2, x_off, x_key;
    int n_keys = 0, ray_cols = 0;
    std::vector<double> mu, wmu;
    int lanes_used = 0;
    bool overflow = false;  // a wavelength had more than kMaxSlots active transitions
};

}  // namespace rh15d

struct rh15d_atom {
    double mass = 0, abund = 1, c_bg = 0;
    int bg_kind = 0;
    int L = 0, n_lines = 0, n_cont = 0;
    std::vector<double> E, g;
    std::vector<int> stage;
    std::vector<int> twoJ;                  // 2 J per level, -1 if the atom gives none
    std::vector<double> gL;                 // Lande factor per level
    std::vector<rh15d::HostTransition> tr;  // lines, then continua
    std::vector<double> lam, nu;            // union grid
    std::vector<int> jact_off, jact_t;
    // device copies per (device, n_mu), built on first use
    std::mutex mu_;
    std::map<std::pair<std::pair<int, int>, rh15d::SweepShape>, rh15d::DevAtom> dev;
    std::map<std::pair<std::pair<int, int>, int>, rh15d::SweepShape> tuned;  // (device, n_mu), precision -> shape
    std::vector<void *> dev_allocs;
};

namespace rh15d {
// host setup (atom_setup.cpp)
int parse_atom_file(const char *path, rh15d_atom *a, std::string &err);
void gauss_legendre_01(int n, std::vector<double> &x, std::vector<double> &w);
void zeeman_components(int twoJl, double gl, int twoJu, double gu, HostTransition &t);
void build_group_tables(const rh15d_atom &a, int n_mu, SweepShape shape, HostGroupTables &out);
void set_error(const char *fmt, ...);
const char *last_error();
// the solve (mali.hip); fixed_ws: workspace is a fixed region of
// workspace_bytes and nothing is allocated
int solve_columns_impl(const rh15d_atom *atom, const rh15d_columns *cols, const rh15d_options *o,
                       const rh15d_outputs *out, void *workspace, size_t workspace_bytes, void *hip_stream,
                       bool fixed_ws);
}  // namespace rh15d
