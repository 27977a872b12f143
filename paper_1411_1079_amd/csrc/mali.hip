// librh15d: per-column multi-level accelerated Lambda iteration (MALI) on
// MI355X (gfx950).
//
// Method (paper Sec. 2.1-2.3): Rybicki & Hummer (1992) MALI with a local
// diagonal Psi* operator, fully preconditioned rate equations and
// overlapping transitions, per column (1.5D), Ng acceleration, LTE /
// zero-radiation / provided start solutions, convergence on the maximum
// relative population change; vertical emergent spectra only.
//
// Mapping onto CDNA4:
//  * formal solution (k_sweep): one lane per ray (wavelength, angle,
//    direction) of a column; the 64 rays of a wavefront share one set of
//    active transitions, walk the depth recurrence in lock-step, read the
//    per-depth column data as wave-uniform (scalar) loads and the
//    normalised line profiles as coalesced rows, and sum their rate
//    contributions over the wavefront through LDS in blocks of depth
//    points, in a fixed order, into per-depth rate keys (no atomics:
//    results are bitwise reproducible); one kernel per class of groups
//    (transition slots, continua among them), the classes of a stage
//    running concurrently on side streams;
//  * rate-equation solve: the radiative part of every rate-matrix entry is
//    gathered from the rate keys (k_rad_rates, one lane per depth point and
//    entry), then one lane per depth point adds the collisional rates and
//    solves the L x L FP64 system in registers by Gaussian elimination with
//    partial pivoting (k_se);
//  * convergence test and Ng (k_converge): one workgroup per column;
//  * columns live in "slots" of a fixed depth stride; one iteration is a
//    fixed sequence of kernels (sweep, rate solve, convergence + Ng, output
//    of finished columns, refill of free slots from a column queue on the
//    device), so it can be captured once as a hipGraph and replayed.  The
//    plain scheduler refills only when every slot is free (fixed chunks);
//    the slot scheduler refills a slot as soon as its column is done;
//  * precision form: the sweep and its rate accumulation in FP32, the rate
//    solve, Ng and the convergence test in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rh15d_internal.h"

using namespace rh15d;

namespace {

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));                  \
            return RH15D_EDEVICE;                                                      \
        }                                                                              \
    } while (0)

// ---------------------------------------------------------------------------
// device math
// ---------------------------------------------------------------------------
__device__ __forceinline__ double d_exp(double x) { return exp(x); }
__device__ __forceinline__ float d_exp(float x) { return __expf(x); }
__device__ __forceinline__ double d_expm1(double x) { return expm1(x); }
__device__ __forceinline__ float d_expm1(float x) { return expm1f(x); }

// 1 - exp(-x) for x >= 0, given ex = exp(-x): the difference itself where it
// keeps its relative precision (x > 0.5); below, expm1 in FP64 and in FP32
// the Taylor series through x^7 (truncation below 2e-7 relative at x = 0.5).
__device__ __forceinline__ double one_m_exp(double x, double ex) { return x > 0.5 ? 1.0 - ex : -expm1(-x); }
__device__ __forceinline__ float one_m_exp(float x, float ex) {
    float r = 1.0f - ex;
    // the series only when a lane of the wavefront needs it
    if (__builtin_amdgcn_ballot_w64(!(x > 0.5f)) != 0) {
        const float s = x * (1.0f + x * (-1.0f / 2.0f + x * (1.0f / 6.0f + x * (-1.0f / 24.0f + x * (1.0f / 120.0f +
                        x * (-1.0f / 720.0f + x * (1.0f / 5040.0f)))))));
        r = x > 0.5f ? r : s;
    }
    return r;
}

// Reciprocals: hardware estimate, refined by Newton steps in FP64.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Linear short-characteristic weights (Olson & Kunasz 1987) of an optical
// step x: I_b = I_a e + wa S_a + wb S_b.  Below the threshold the weights
// come from their Taylor series, which avoids the cancellation in
// 1 - (1 - e^-x)/x: through x^6 in FP64 (below 1e-2), in FP32 (below 0.1)
// through x^4 for wb and x^5 for wa, whose truncation (3e-7 and 3e-8
// relative at 0.1) is below the FP32 rounding of the rest of the step.
template <typename R>
__device__ __forceinline__ void sc_weights(R x, R &e, R &wa, R &wb) {
    if constexpr (sizeof(R) == 4) {
        // e from one exponential for both branches (lanes of a wavefront
        // often take both: thin and thick rays side by side)
        e = d_exp(-x);
        if (x < R(0.1)) {
            wb = x * (R(0.5) + x * (R(-1.0 / 6.0) + x * (R(1.0 / 24.0) + x * R(-1.0 / 120.0))));
            wa = x * (R(0.5) + x * (R(-1.0 / 3.0) + x * (R(1.0 / 8.0) + x * (R(-1.0 / 30.0) + x * R(1.0 / 144.0)))));
        } else {
            // x >= 0.1: 1 - e^-x carries at most a few ulp of relative error
            const R q = (R(1) - e) * __builtin_amdgcn_rcpf(x);
            wb = R(1) - q;
            wa = q - e;
        }
    } else if (x < R(1.0e-2)) {
        wb = x * (R(0.5) + x * (R(-1.0 / 6.0) + x * (R(1.0 / 24.0) + x * (R(-1.0 / 120.0) +
             x * (R(1.0 / 720.0) + x * R(-1.0 / 5040.0))))));
        wa = x * (R(0.5) + x * (R(-1.0 / 3.0) + x * (R(1.0 / 8.0) + x * (R(-1.0 / 30.0) +
             x * (R(1.0 / 144.0) + x * R(-1.0 / 840.0))))));
        e = d_exp(-x);
    } else {
        const R one_m_e = -d_expm1(-x);
        const R q = one_m_e * rcp(x);
        e = R(1) - one_m_e;
        wb = R(1) - q;
        wa = q - e;
    }
}

template <typename F>
struct cplx_t { F r, i; };
template <typename F>
__device__ __forceinline__ cplx_t<F> cmul(cplx_t<F> a, cplx_t<F> b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
template <typename F>
__device__ __forceinline__ cplx_t<F> cadd(cplx_t<F> a, F b) { return {a.r + b, a.i}; }
// real part of a / b; in FP32 through the hardware reciprocal (about 1 ulp),
// well inside the approximation's own error
template <typename F>
__device__ __forceinline__ F cdiv_re(cplx_t<F> a, cplx_t<F> b) {
    const F d = b.r * b.r + b.i * b.i;
    const F n = a.r * b.r + a.i * b.i;
    if constexpr (sizeof(F) == 4) return n * __builtin_amdgcn_rcpf(d);
    else return n / d;
}
__device__ __forceinline__ double d_cos(double x) { return cos(x); }
__device__ __forceinline__ float d_cos(float x) { return __cosf(x); }

// Voigt function H(a, v) = Re w(v + i a), Humlicek (1982) W4: a rational
// approximation in four regions of s = |v| + a (relative accuracy ~1e-4),
// evaluated in the precision F.
template <typename F>
__device__ __forceinline__ F voigt_w4_body(F a, F v) {
    using C = cplx_t<F>;
    const C t = {a, -v};          // t = a - i v
    const F s = fabs(v) + a;
    if (s >= F(15.0)) {
        C den = cadd(cmul(t, t), F(0.5));
        return cdiv_re(C{F(0.5641896) * t.r, F(0.5641896) * t.i}, den);
    }
    if (s >= F(5.5)) {
        const C u = cmul(t, t);
        const C num = cmul(t, cadd(C{F(0.5641896) * u.r, F(0.5641896) * u.i}, F(1.410474)));
        const C den = cadd(cmul(u, cadd(u, F(3.0))), F(0.75));
        return cdiv_re(num, den);
    }
    if (a >= F(0.195) * fabs(v) - F(0.176)) {
        C num = {F(0.5642236), F(0)};
        num = cadd(cmul(num, t), F(3.778987));
        num = cadd(cmul(num, t), F(11.96482));
        num = cadd(cmul(num, t), F(20.20933));
        num = cadd(cmul(num, t), F(16.4955));
        C den = {F(1), F(0)};
        den = cadd(cmul(den, t), F(6.699398));
        den = cadd(cmul(den, t), F(21.69274));
        den = cadd(cmul(den, t), F(39.27121));
        den = cadd(cmul(den, t), F(38.82363));
        den = cadd(cmul(den, t), F(16.4955));
        return cdiv_re(num, den);
    }
    const C u = cmul(t, t);
    C p = {F(0.56419), F(0)};
    p = cadd(cmul(p, u), F(-1.320522));
    p = cadd(cmul(p, u), F(35.76683));
    p = cadd(cmul(p, u), F(-219.0313));
    p = cadd(cmul(p, u), F(1540.787));
    p = cadd(cmul(p, u), F(-3321.9905));
    p = cadd(cmul(p, u), F(36183.31));
    C q = {F(-1), F(0)};
    q = cadd(cmul(q, u), F(1.841439));
    q = cadd(cmul(q, u), F(-61.57037));
    q = cadd(cmul(q, u), F(364.2191));
    q = cadd(cmul(q, u), F(-2186.181));
    q = cadd(cmul(q, u), F(9022.228));
    q = cadd(cmul(q, u), F(-24322.84));
    q = cadd(cmul(q, u), F(32066.6));
    const F frac = cdiv_re(cmul(t, p), q);
    return d_exp(u.r) * d_cos(u.i) - frac;
}
// The same as a call (for the FP64 callers, whose registers it would
// otherwise crowd); the FP32 profile preparation inlines the body.
template <typename F>
__device__ __noinline__ F voigt_w4(F a, F v) { return voigt_w4_body<F>(a, v); }

template <typename R>
__device__ __forceinline__ R wave_sum(R v) {
    // butterfly over the 64 lanes: every lane ends with the same total,
    // summed in the same order on every launch
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t rfl_wave(int64_t x) { return (int64_t)__builtin_amdgcn_readfirstlane((int)x); }

// rays (2 directions x angles x wavelengths) of one line at one depth that
// the profile-preparation wavefront holds in registers
constexpr int kMaxLineRays = 1536;
// wavelengths of a line with partial frequency redistribution
constexpr int kMaxPrdFreq = 256;

// ---------------------------------------------------------------------------
// per-launch arguments
// ---------------------------------------------------------------------------
enum SlotState { SLOT_FREE = 0, SLOT_ACTIVE = 1, SLOT_DONE = 2, SLOT_PENDING = 3 };
enum Counter { CTR_NEXT = 0, CTR_EMITTED = 1, CTR_RETIRE = 2, CTR_REFILL = 3, CTR_COUNT = 8 };

struct RunArgs {
    DevAtom A;
    const int64_t *doff;      // [n_columns+1] depth offsets of the columns (device)
    int64_t n_columns;
    int S, ND;                // slots, depth stride of a slot
    int chunked;              // refill only when every slot is free
    int rec_w;
    // inputs (global depth index)
    const double *z, *T, *ne, *nH, *vz, *vt, *init;
    const double *Bf, *Bincl, *Bazim;   // magnetic field (NULL: none), read for the Stokes spectrum
    // outputs (global depth / column index)
    double *pops, *history, *spectrum, *psi;
    double *stokes;           // [n_columns][NL][4] or NULL
    double *psi_ray;          // [total_depth][NL][n_mu][2] or NULL
    int32_t *n_iter, *status;
    // per slot
    int *slot_col, *slot_state, *slot_it, *ng_count, *ng_head;
    int *slot_bad;            // nonzero: the column's data failed the input checks
    double *slot_dprev;       // change of the slot's previous plain iteration, -1 if none
    int *ctr;                 // [CTR_COUNT]
    int *retire_list, *refill_list;
    // workspace, slot-local depth index gc = slot * ND + k
    double *lnr;              // [gc][L] Saha-Boltzmann log ratios to level 0
    double *kbg;              // [gc] background opacity at the reference wavelength
    double *gr;               // [gc][n_cont] n*_l / n*_u of each continuum
    double *norm;             // [gc][n_lines] profile normalisation sums
    void *phi;                // [gc][ray_cols] normalised profiles (sweep precision)
    void *part;               // rate keys: slot block at slot*ND*n_keys, [key][N]
    void *rec;                // [gc][rec_w] per-depth data of the sweep (sweep precision)
    float *popsf;             // [gc][L] FP32 copy of the populations (FP32 form)
    double *rad;              // [L*L][gc] radiative part of the rate-matrix entries (i, j)
    double *nse;              // [gc][L] rate-equation solution
    double *dk;               // [gc] max relative change per depth point
    int *flag;                // [gc] 0 ok, 1 non-finite/non-positive, 2 singular
    double *ring;             // [4][S*ND][L] Ng history
    // partial frequency redistribution (prd = 1), sweep precision
    void *emis;               // [gc][psi_cols] emission profiles psi = rho phi of the PRD lines' rays
    void *ist;                // [gc][ist_cols] intensities of the stored rays (last sweep)
    void *gtab;               // [gc][g_cols] redistribution weights of the PRD lines, per line
                              // [j'][j] = g(j <- j') (input frequency major)
    double *rho;              // [gc][sum of PRD n_act] new rho (between the two update kernels)
    int max_iter, ng_order, ng_delay, ng_period, start, esc_iter, prd;
    double tol, tol_fp, coll_scale, crs_f0, prd_eps0;
};

// Per-depth data of the sweep (slot-local depth gc), in the sweep's precision:
// [0] z(k-1) - z(k) (0 at the top point), [1] 1/T, [2] background opacity at
// the reference wavelength, [3] unused, [4 + c] n*_l / n*_u of continuum c.
constexpr int kRecHead = 4;
__host__ __device__ __forceinline__ int rec_width(int n_cont) { return (kRecHead + n_cont + 1) & ~1; }

struct ColGeom {
    int col, N;
    int64_t g0, gc0;
};
__device__ __forceinline__ ColGeom geom(const RunArgs &a, int slot) {
    ColGeom c;
    c.col = a.slot_col[slot];
    c.g0 = a.doff[c.col];
    c.N = (int)(a.doff[c.col + 1] - c.g0);
    c.gc0 = (int64_t)slot * a.ND;
    return c;
}

// ---------------------------------------------------------------------------
// column preparation (slots being refilled)
// ---------------------------------------------------------------------------
template <typename R>
__device__ void prep_point(const RunArgs &a, int slot, int k) {
    const ColGeom cg = geom(a, slot);
    if (k >= cg.N) return;
    const int64_t g = cg.g0 + k, gc = cg.gc0 + k;
    const DevAtom &A = a.A;
    const int L = A.L;
    const double T = a.T[g], ne = a.ne[g], nH = a.nH[g];
    // column data the method can use; a failing point marks its column
    {
        const bool ok = isfinite(T) && T > 0.0 && isfinite(ne) && ne > 0.0 && isfinite(nH) && nH > 0.0 &&
                        isfinite(a.vz[g]) && isfinite(a.vt[g]) && a.vt[g] >= 0.0 && isfinite(a.z[g]) &&
                        (k == 0 || a.z[g] < a.z[g - 1]);
        if (!ok) atomicOr(&a.slot_bad[slot], 1);
    }
    const double kT = kKB * T;
    const double saha = log(2.0 / ne) + 1.5 * log(2.0 * kPI * kME * kT / (kH * kH));
    double lr[RH15D_MAX_LEVELS];
    double mx = -1e300;
    for (int i = 0; i < L; i++) {
        lr[i] = log(A.g[i] / A.g[0]) - (A.E[i] - A.E[0]) / kT + (A.stage[i] - A.stage[0]) * saha;
        a.lnr[gc * L + i] = lr[i];
        mx = fmax(mx, lr[i]);
    }
    double sum = 0.0;
    for (int i = 0; i < L; i++) sum += exp(lr[i] - mx);
    const double ntot = A.abund * nH;
    for (int i = 0; i < L; i++) {
        double v;
        if (a.start == RH15D_START_PROVIDED) v = a.init[g * L + i];
        else v = ntot * exp(lr[i] - mx) / sum;
        a.pops[g * L + i] = v;
        if (a.popsf) a.popsf[gc * L + i] = static_cast<float>(v);
    }
    const double kbg = A.bg_kind == 1 ? A.c_bg * nH * ne * pow(T, -1.5) * exp(kBgTheta / T) : 0.0;
    a.kbg[gc] = kbg;
    R *rec = reinterpret_cast<R *>(a.rec) + gc * a.rec_w;
    // spacings to the points above (rec[0]) and below (rec[3]): a sweep
    // reads the one towards the previous point along its direction from the
    // point's own record
    rec[0] = static_cast<R>(k == 0 ? 0.0 : a.z[g - 1] - a.z[g]);
    rec[1] = static_cast<R>(1.0 / T);
    rec[2] = static_cast<R>(kbg);
    rec[3] = static_cast<R>(k == cg.N - 1 ? 0.0 : a.z[g] - a.z[g + 1]);
    for (int c = 0; c < A.n_cont; c++) {
        const DevTransition &tr = A.tr[A.n_lines + c];
        const double gr = exp(lr[tr.l] - lr[tr.u]);
        a.gr[gc * A.n_cont + c] = gr;
        rec[kRecHead + c] = static_cast<R>(gr);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_prep_depth(RunArgs a) {
    const int64_t n = (int64_t)a.ctr[CTR_REFILL] * a.ND;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n; w += (int64_t)gridDim.x * blockDim.x)
        prep_point<R>(a, a.refill_list[w / a.ND], (int)(w % a.ND));
}

// One wavefront per (depth point, line): every quadrature ray's profile,
// normalised so that sum over rays of W phi = 1 at this depth.
template <typename R>
__device__ void prep_profile_item(const RunArgs &a, int slot, int k, int t, int lane) {
    const ColGeom cg = geom(a, slot);
    if (k >= cg.N) return;
    const DevAtom &A = a.A;
    const int64_t g = cg.g0 + k, gc = cg.gc0 + k;
    const DevTransition &tr = A.tr[t];
    const double T = a.T[g], vt = a.vt[g], vz = a.vz[g];
    const double dnd = tr.nu0 / kC * sqrt(2.0 * kKB * T / A.mass + vt * vt);
    const R adamp = static_cast<R>((tr.gamma + tr.c_el * a.nH[g]) / (4.0 * kPI * dnd));
    const double rdnd = 1.0 / dnd;
    const double pre = rdnd / sqrt(kPI);
    const double vzc = vz / kC;
    const int r0 = A.prof_off[t], nr = A.prof_off[t + 1] - r0;
    const double *pnu = A.prof_nu + r0, *pmus = A.prof_mus + r0, *pw = A.prof_w + r0;
    const int *pdst = A.prof_dst + r0;
    R *phi = reinterpret_cast<R *>(a.phi) + gc * A.ray_cols + tr.ray_off;
    // PRD line: the emission profile starts as the absorption profile (rho = 1)
    R *psi = (a.prd && tr.prd) ? reinterpret_cast<R *>(a.emis) + gc * A.psi_cols + tr.psi_off : nullptr;
    // The line's rays in order of distance from the line centre, each stored
    // at its place in the row (quadrature rays by direction, wavelength and
    // angle, then the vertical emergent ray of each wavelength: mu = 1,
    // upward, weight 0), scaled by the row's normalisation sum.  Four rays
    // per lane at a time, their table entries loaded together; in FP32 a row
    // of up to kHeld rays per lane stays in registers until the wavefront
    // has the sum, otherwise it is written unnormalised and scaled in a
    // second pass.
    constexpr int U = 4, kHeld = sizeof(R) == 4 ? 8 : 0;
    auto profile = [&](int r, double nu, double mus) -> R {
        const double v = (nu - tr.nu0 * (1.0 + mus * vzc)) * rdnd;
        const R H = tr.voigt ? voigt_w4<R>(adamp, static_cast<R>(v)) : d_exp(static_cast<R>(-v * v));
        return H * static_cast<R>(pre);
    };
    // FP32: v = ((nu - nu0) - nu0 vz/c mu) / dnu_D from the FP32 ray table,
    // the Voigt function inlined
    const float *pdnu = A.prof_dnu + r0, *pmusf = A.prof_musf + r0;
    const float nvz = static_cast<float>(tr.nu0 * vzc), rdndf = static_cast<float>(rdnd);
    const float pref = static_cast<float>(pre), adf = static_cast<float>(adamp);
    const bool voigt = tr.voigt != 0;
    auto profile32 = [&](float dnu, float mus) -> float {
        const float v = (dnu - nvz * mus) * rdndf;
        const float H = voigt ? voigt_w4_body<float>(adf, v) : d_exp(-v * v);
        return H * pref;
    };
    double acc = 0.0, tot;
    if (kHeld > 0 && nr <= kHeld * kWave) {
        R val[kHeld > 0 ? kHeld : 1];
        int dst[kHeld > 0 ? kHeld : 1];
#pragma unroll
        for (int h0 = 0; h0 < kHeld; h0 += U) {
            float dnu[U], musf[U];
            double w[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int r = lane + (h0 + u) * kWave;
                if (r < nr) { dnu[u] = pdnu[r]; musf[u] = pmusf[r]; w[u] = pw[r]; dst[h0 + u] = pdst[r]; }
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int r = lane + (h0 + u) * kWave;
                if (r < nr) {
                    val[h0 + u] = static_cast<R>(profile32(dnu[u], musf[u]));
                    acc += w[u] * static_cast<double>(val[h0 + u]);
                }
            }
        }
        tot = wave_sum(acc);
        const R rtot = static_cast<R>(1.0 / tot);
#pragma unroll
        for (int h = 0; h < kHeld; h++)
            if (lane + h * kWave < nr) {
                const R v = sizeof(R) == 8 ? static_cast<R>(val[h] / tot) : val[h] * rtot;
                phi[dst[h]] = v;
                if (psi) psi[dst[h]] = v;
            }
    } else {
        for (int r0 = lane; r0 < nr; r0 += U * kWave) {
            double nu[U], mus[U], w[U];
            float dnu[U], musf[U];
            int dst[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int r = r0 + u * kWave;
                if (r < nr) {
                    if constexpr (sizeof(R) == 4) { dnu[u] = pdnu[r]; musf[u] = pmusf[r]; }
                    else { nu[u] = pnu[r]; mus[u] = pmus[r]; }
                    w[u] = pw[r];
                    dst[u] = pdst[r];
                }
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int r = r0 + u * kWave;
                if (r < nr) {
                    R ph;
                    if constexpr (sizeof(R) == 4) ph = profile32(dnu[u], musf[u]);
                    else ph = profile(r, nu[u], mus[u]);
                    acc += w[u] * static_cast<double>(ph);
                    phi[dst[u]] = ph;
                }
            }
        }
        tot = wave_sum(acc);
        const R rtot = static_cast<R>(1.0 / tot);
        for (int r0 = lane; r0 < nr; r0 += U * kWave) {
            R x[U];
#pragma unroll
            for (int u = 0; u < U; u++)
                if (r0 + u * kWave < nr) x[u] = phi[r0 + u * kWave];
#pragma unroll
            for (int u = 0; u < U; u++)
                if (r0 + u * kWave < nr) {
                    const R v = sizeof(R) == 8 ? static_cast<R>(x[u] / tot) : x[u] * rtot;
                    phi[r0 + u * kWave] = v;
                    if (psi) psi[r0 + u * kWave] = v;
                }
        }
    }
    if (lane == 0) a.norm[gc * A.n_lines + t] = tot;
}

template <typename R>
__global__ __launch_bounds__(256) void k_prep_profile(RunArgs a) {
    const int lane = threadIdx.x & 63;
    const int nl = a.A.n_lines;
    const int64_t n = (int64_t)a.ctr[CTR_REFILL] * a.ND * nl;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t w = rfl_wave(blockIdx.x * 4 + (threadIdx.x >> 6)); w < n; w += waves) {
        const int t = (int)(w % nl);
        const int64_t sk = w / nl;
        prep_profile_item<R>(a, a.refill_list[sk / a.ND], (int)(sk % a.ND), t, lane);
    }
}

enum { MODE_RATES = 0, MODE_PSI = 1 };

constexpr unsigned kXcds = 8;   // accelerator complex dies of the MI355X, one L2 each

__device__ __forceinline__ int rfl(int x) { return __builtin_amdgcn_readfirstlane(x); }

// One DPP stage of a sum that only lane 63 reads: the value of another lane
// (row shift) or of the last lane of an earlier row (row broadcast), 0 where
// the shift has no source.  Every row is written (full row mask) with
// out-of-range sources zero-filled, so the compiler folds the move into the
// following add; lanes whose broadcast source is undefined end with values
// nobody reads, lane 63 with the total of the fixed summation order.
template <int CTRL>
__device__ __forceinline__ float dpp_src(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_src(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Uniform (per wavefront) description of the transitions a group touches.
template <typename R, int NS>
struct Slots {
    int kind[NS], l[NS], u[NS], c[NS];
    R cblu[NS], cbul[NS], ca[NS], wsum[NS];
};

// Angle-independent terms of a lane's wavelength at one depth point:
// Planck function, background, continua (not Doppler shifted), populations.
template <typename R, int NS>
struct Shared {
    R B, etabg, chi0, eta0;
    R nl[NS], nu[NS];
    R cvlu[NS], cvul[NS], cU[NS], ccht[NS];
};

// Inputs of one depth point: per-depth record fields, populations and the
// lane's profile values.  The sweep loads them one step ahead of their use,
// so their latency overlaps the previous point's arithmetic.  The records
// and populations are read through pointers the kernel receives as
// separate restrict-qualified arguments: the compiler then knows the
// sweep's own stores (rate sums) cannot change them, and the
// wavefront-uniform reads become scalar loads.
template <typename R, int NS, int MC>
struct PointIn {
    R invT, kbg, dz;
    R gfac[NS];        // continuum slots: n_l*/n_u* exp(h nu / k T) of the record
    R nl[NS], nu[NS];
    R ph[NS][MC];      // line slots: profile values of the lane's angles
    R ps[NS][MC];      // PRD line slots: emission-profile values (psi = rho phi)
};

// Where the partial-frequency-redistribution variant of the sweep reads
// the emission profiles (psi) and stores the intensities of the rays the
// rho update needs.
template <typename R>
struct PrdIO {
    const R *psi;      // [gc][psi_cols]
    R *ist;            // [gc][ist_cols]
    int psi_cols, ist_cols;
};

// Where one depth point's inputs start, as byte offsets from the bases the
// sweep kernel receives: its record, its populations, its profile row and
// (PRD) its emission-profile row.  The loads index the restrict-qualified
// bases directly, so the compiler still sees that the sweep's own stores
// cannot change them (and keeps the uniform ones scalar).
struct PointRows {
    int64_t rec, pops, phi, psi;
};

template <typename R>
__device__ __forceinline__ const R *at_bytes(const R *base, int64_t off) {
    return reinterpret_cast<const R *>(reinterpret_cast<const char *>(base) + off);
}

// Records and populations are not written while a sweep kernel runs:
// read through the constant address space, uniform loads of them are
// scalar loads whatever stores the kernel makes elsewhere.
template <typename R>
using const_as = const __attribute__((address_space(4))) R;

template <typename R>
__device__ __forceinline__ const_as<R> *at_bytes_c(const R *base, int64_t off) {
    return (const_as<R> *)(reinterpret_cast<const char *>(base) + off);
}
template <typename R>
__device__ __forceinline__ const_as<R> *at_bytes_c(const_as<R> *base, uint32_t off) {
    return (const_as<R> *)((const __attribute__((address_space(4))) char *)base + off);
}

// The point's wavefront-uniform inputs (record fields and populations).
// dzi: the record field with the spacing to the previous point along the
// sweep (0 going down, 3 going up).
template <typename R, int NS, int MC>
__device__ __forceinline__ void load_uniform(const R *__restrict__ recb, const R *__restrict__ popsb,
                                             const PointRows &rw, int dzi, const Slots<R, NS> &sl,
                                             PointIn<R, NS, MC> &p) {
    const_as<R> *rec = at_bytes_c(recb, rw.rec);
    p.invT = rec[1];
    p.kbg = rec[2];
    // level and continuum fields as 32-bit byte offsets: the loads then
    // take them as the scalar load's register offset
    constexpr uint32_t sz = sizeof(R);
    p.dz = *at_bytes_c<R>(rec, (uint32_t)dzi * sz);
    const_as<R> *n = at_bytes_c(popsb, rw.pops);
#pragma unroll
    for (int q = 0; q < NS; q++) {
        p.nl[q] = *at_bytes_c<R>(n, (uint32_t)sl.l[q] * sz);
        p.nu[q] = *at_bytes_c<R>(n, (uint32_t)sl.u[q] * sz);
        p.gfac[q] = sl.kind[q] == 1 ? *at_bytes_c<R>(rec, (uint32_t)(kRecHead + sl.c[q]) * sz) : R(0);
    }
}

// The lane's profile values at the point (and, PRD, its emission-profile
// values).  A lane without line slot q reads its row's first value (a
// valid address in any group with a line); ray_terms replaces it by 0.
// An unconditional load, selected at its use, instead of a branch around
// the load.
template <typename R, int NS, int MC, bool PRD = false>
__device__ __forceinline__ void load_profiles(const R *__restrict__ phi, const PointRows &rw, const Slots<R, NS> &sl,
                                              const int *pb, PointIn<R, NS, MC> &p, const PrdIO<R> *pio = nullptr,
                                              const int *psb = nullptr) {
    const R *phirow = at_bytes(phi, rw.phi);
#pragma unroll
    for (int q = 0; q < NS; q++) {
#pragma unroll
        for (int r = 0; r < MC; r++)
            p.ph[q][r] = sl.kind[q] == 0 ? phirow[(pb[q] >= 0 ? pb[q] : 0) + r] : R(0);
        if constexpr (PRD) {
            const R *psirow = at_bytes(pio->psi, rw.psi);
#pragma unroll
            for (int r = 0; r < MC; r++) p.ps[q][r] = (sl.kind[q] == 0 && psb[q] >= 0) ? psirow[psb[q] + r] : p.ph[q][r];
        }
    }
}

template <typename R, int NS, int MC, bool PRD = false>
__device__ __forceinline__ void load_rows(const R *__restrict__ recb, const R *__restrict__ popsb,
                                          const R *__restrict__ phi, const PointRows &rw, int dzi,
                                          const Slots<R, NS> &sl, const int *pb, PointIn<R, NS, MC> &p,
                                          const PrdIO<R> *pio = nullptr, const int *psb = nullptr) {
    load_uniform<R, NS, MC>(recb, popsb, rw, dzi, sl, p);
    load_profiles<R, NS, MC, PRD>(phi, rw, sl, pb, p, pio, psb);
}

// The offsets of the point with global depth index g (slot-local gc).
template <typename R, bool PRD = false>
__device__ __forceinline__ PointRows point_rows(int rec_w, int L, int ray_cols, int64_t g, int64_t gc,
                                                const PrdIO<R> *pio = nullptr) {
    PointRows rw;
    rw.rec = gc * rec_w * (int64_t)sizeof(R);
    rw.pops = (sizeof(R) == 8 ? g : gc) * L * (int64_t)sizeof(R);
    rw.phi = gc * ray_cols * (int64_t)sizeof(R);
    rw.psi = PRD ? gc * pio->psi_cols * (int64_t)sizeof(R) : 0;
    return rw;
}

template <typename R, int NS, int MC>
__device__ __forceinline__ void shared_terms(const PointIn<R, NS, MC> &in, const Slots<R, NS> &sl, const R *alpha,
                                             R hnu_k, R two_hnu3, R lamfac, Shared<R, NS> &sh) {
    const R x = hnu_k * in.invT;
    const R ex = d_exp(-x);  // exp(-h nu / k T)
    sh.B = two_hnu3 * ex * rcp(one_m_exp(x, ex));
    const R chibg = in.kbg * lamfac;
    sh.etabg = chibg * sh.B;
    R chi = chibg, eta = sh.etabg;
#pragma unroll
    for (int q = 0; q < NS; q++) {
        sh.nl[q] = in.nl[q];
        sh.nu[q] = in.nu[q];
        if (sl.kind[q] == 1) {
            const R gf = in.gfac[q] * ex;
            sh.cvlu[q] = alpha[q];
            sh.cvul[q] = gf * alpha[q];
            sh.cU[q] = two_hnu3 * sh.cvul[q];
            sh.ccht[q] = sh.nl[q] * sh.cvlu[q] - sh.nu[q] * sh.cvul[q];
            chi += sh.ccht[q];
            eta += sh.nu[q] * sh.cU[q];
        }
    }
    sh.chi0 = chi;
    sh.eta0 = eta;
}

// Terms of one ray (angle r of the lane) at one depth point.
template <typename R, int NS>
struct RayPt {
    R chi, rchi, S;
    R vlu[NS], vul[NS], U[NS], cht[NS], ph[NS];
};

// pon[q]: the lane's wavelength lies in line slot q's active set (its
// loaded profile value counts; otherwise the value is 0)
template <typename R, int NS, int MC, bool PRD = false>
__device__ __forceinline__ void ray_terms(const Slots<R, NS> &sl, const Shared<R, NS> &sh, const PointIn<R, NS, MC> &in,
                                          const bool *pon, int r, RayPt<R, NS> &p) {
    R chi = sh.chi0, eta = sh.eta0;
#pragma unroll
    for (int q = 0; q < NS; q++) {
        if (sl.kind[q] == 0) {
            const R ph = pon[q] ? in.ph[q][r] : R(0);
            // emission (spontaneous and stimulated) with psi for PRD lines
            const R ps = PRD ? (pon[q] ? in.ps[q][r] : R(0)) : ph;
            p.ph[q] = ph;
            p.vlu[q] = sl.cblu[q] * ph;
            p.vul[q] = sl.cbul[q] * ps;
            p.U[q] = sl.ca[q] * ps;
            p.cht[q] = sh.nl[q] * p.vlu[q] - sh.nu[q] * p.vul[q];
            chi += p.cht[q];
            eta += sh.nu[q] * p.U[q];
        } else {
            p.ph[q] = R(1);
            p.vlu[q] = sh.cvlu[q];
            p.vul[q] = sh.cvul[q];
            p.U[q] = sh.cU[q];
            p.cht[q] = sh.ccht[q];
        }
    }
    p.chi = chi;
    p.rchi = rcp(chi);
    p.S = eta * p.rchi;
}

template <int NS, int MODE>
constexpr int n_acc() { return MODE == MODE_PSI ? NS : 2 * NS + NS * (NS - 1); }

// Adds one ray's contributions (angle weight wmu) into the lane's sums.
// FIRST: the point's first ray, whose terms start the sums.
template <typename R, int NS, int MODE, bool FIRST>
__device__ __forceinline__ void contribute(const RayPt<R, NS> &p, const R *wpsi, R wmu, R Ieff, R psi, R *acc) {
    auto add = [&](int i, R t) { acc[i] = FIRST ? t : acc[i] + t; };
    if constexpr (MODE == MODE_PSI) {
#pragma unroll
        for (int q = 0; q < NS; q++) add(q, wpsi[q] * wmu * p.ph[q] * psi);
    } else {
#pragma unroll
        for (int q = 0; q < NS; q++) {
            add(q, wmu * p.vlu[q] * Ieff);
            add(NS + q, wmu * (p.U[q] * (R(1) - p.cht[q] * psi) + p.vul[q] * Ieff));
        }
#pragma unroll
        for (int q = 0; q < NS; q++) {
#pragma unroll
            for (int q2 = 0; q2 < NS; q2++) {
                if (q2 == q) continue;
                const int rank = q * (NS - 1) + (q2 < q ? q2 : q2 - 1);
                add(2 * NS + rank, wmu * p.cht[q] * psi * p.U[q2]);
            }
        }
    }
}

// Sums over the wavefront, through LDS.  Each depth point's per-lane terms
// (one row of 64 values per sum key, weighted by the lane's slot factor)
// go to the wavefront's own LDS area; after B points the block's S = K B
// rows are summed, P lanes per row, each lane reading every P-th 16-byte
// chunk of the row (row pitch padded by P chunks, so the lanes of one read
// cover distinct banks), the P partial sums are combined by DPP, and the
// first lane of each row stores the total.  The data movement of the sums
// runs on the LDS pipe and the vector unit adds each value once, where a
// DPP tree per key and point spends six vector instructions on it.
// `out` is key-major ([key][depth] per column, N depths), which the
// rate-equation kernel reads with consecutive depth points in consecutive
// lanes.
template <typename R, int NS, int MODE>
struct Red {
    static constexpr int K = n_acc<NS, MODE>();            // sums per depth point
    static constexpr int T = sizeof(R) == 4 ? 16 : 8;       // rows per block aimed at
    static constexpr int B = K >= T ? 1 : T / K;            // depth points per block
    static constexpr int S = K * B;                         // rows per block
    static constexpr int P = S <= 16 ? 4 : (S <= 32 ? 2 : 1);
    static constexpr int CE = 16 / static_cast<int>(sizeof(R));
    static constexpr int STRIDE = kWave + CE * P;           // row pitch, elements
    static constexpr int SIZE = S * STRIDE;                 // elements per wavefront
    static_assert(S * P <= kWave, "rows of a block exceed the wavefront");
};

template <typename R, int NS, int MODE>
__device__ __forceinline__ void red_put(const R *acc, const R *kapj, R *lds, int b, int lane) {
    using RS = Red<R, NS, MODE>;
#pragma unroll
    for (int i = 0; i < RS::K; i++) {
        R v = acc[i];
        if constexpr (MODE == MODE_RATES) {
            const int q = i < 2 * NS ? (i % NS) : (i - 2 * NS) / (NS > 1 ? NS - 1 : 1);
            v *= kapj[q];
        }
        lds[(i * RS::B + b) * RS::STRIDE + lane] = v;
    }
}

// Totals of the block's first nb points, stored at depths k_first,
// k_first + step, ...
template <typename R, int NS, int MODE>
__device__ __forceinline__ void red_flush(const R *lds, R *out, int N, int k_first, int step, int nb, int lane) {
    using RS = Red<R, NS, MODE>;
    using V = R __attribute__((ext_vector_type(RS::CE)));
    // the rows were written by other lanes of this wavefront: keep the
    // reads after the writes (LDS executes one wavefront's operations in
    // order)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int s = lane / RS::P, p = lane % RS::P;
    R sum = R(0);
    if (s < RS::S) {
        const V *row = reinterpret_cast<const V *>(lds + s * RS::STRIDE);
#pragma unroll
        for (int j = 0; j < kWave / (RS::CE * RS::P); j++) {
            const V c = row[p + j * RS::P];
#pragma unroll
            for (int e = 0; e < RS::CE; e++) sum = (j == 0 && e == 0) ? c[0] : sum + c[e];
        }
    }
    if constexpr (RS::P >= 2) sum += dpp_src<0xb1>(sum);   // quad_perm [1,0,3,2]
    if constexpr (RS::P >= 4) sum += dpp_src<0x4e>(sum);   // quad_perm [2,3,0,1]
    const int key = s / RS::B, b = s % RS::B;
    if (p == 0 && s < RS::S && b < nb) out[(size_t)key * N + k_first + b * step] = sum;
    // the next block's writes stay after these reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront: 64 lanes, each one wavelength and MC angles of one
// direction, through one column.  Down rays start at the top with no
// incoming radiation; up rays start at the bottom with the diffusion
// approximation I = B + mu dB/dtau.
template <typename R, int MODE, int NS, int NC, int MC, bool PRD = false>
__device__ __forceinline__ void sweep_group(const RunArgs &a, int grp, int slot, int lane, const R *__restrict__ rec,
                                            const R *__restrict__ phi, const R *__restrict__ popsb,
                                            R *__restrict__ part, R *lds) {
    const DevAtom &A = a.A;
    const ColGeom cg = geom(a, slot);
    const int64_t g0 = cg.g0;
    const int N = rfl(cg.N);
    const int64_t gc0 = cg.gc0;
    const DevGroup &G = A.groups[grp];
    const int s_dir = rfl(G.s);
    const int key_off = rfl(G.key_off);
    Slots<R, NS> sl;
#pragma unroll
    for (int q = 0; q < NS; q++) {
        const DevTransition &tr = A.tr[rfl(G.t[q])];
        // a group lists its lines first and its NC continua last
        sl.kind[q] = q >= NS - NC ? 1 : 0;
        sl.l[q] = rfl(tr.l);
        sl.u[q] = rfl(tr.u);
        sl.c[q] = rfl(tr.kind == 1 ? G.t[q] - A.n_lines : 0);
        sl.cblu[q] = static_cast<R>(tr.hnu4pi * tr.Blu);
        sl.cbul[q] = static_cast<R>(tr.hnu4pi * tr.Bul);
        sl.ca[q] = static_cast<R>(tr.hnu4pi * tr.A);
        sl.wsum[q] = static_cast<R>(tr.wsum);
    }
    const int li = grp * kWave + lane;
    const int m0 = A.lanes.m0[li];
    const R lamfac = static_cast<R>(A.lanes.lamfac[li]);
    const R hnu_k = static_cast<R>(A.lanes.hnu_k[li]);
    const R two_hnu3 = static_cast<R>(A.lanes.two_hnu3c2[li]);
    int pb[NS], psb[NS];
    bool pon[NS];
    R kapj[NS], alpha[NS], wpsi[NS];
    PrdIO<R> pio{};
    int ist_base = -1;
    if constexpr (PRD) {
        pio.psi = reinterpret_cast<const R *>(a.emis);
        pio.ist = reinterpret_cast<R *>(a.ist);
        pio.psi_cols = A.psi_cols;
        pio.ist_cols = A.ist_cols;
        ist_base = MODE == MODE_RATES ? A.lanes.ist[li] : -1;
    }
#pragma unroll
    for (int q = 0; q < NS; q++) {
        pb[q] = A.lanes.pbase[li * kMaxSlots + q];
        pon[q] = pb[q] >= 0;
        psb[q] = PRD ? A.lanes.psb[li * kMaxSlots + q] : -1;
        kapj[q] = static_cast<R>(A.lanes.kapj[li * kMaxSlots + q]);
        alpha[q] = static_cast<R>(A.lanes.alpha[li * kMaxSlots + q]);
        const R wj = static_cast<R>(A.lanes.wj[li * kMaxSlots + q]);
        // Psi* weights: W phi~ for lines, W / sum W for continua (W = w_nu w_mu / 2)
        wpsi[q] = sl.kind[q] == 1 ? R(0.5) * wj / sl.wsum[q] : R(0.5) * wj;
    }
    // Psi* of every ray (final stage, when the caller asks for it): the
    // lane's rays are (wavelength j, angles m0.., direction s_dir)
    double *pray = nullptr;
    int64_t pray_base = 0;
    bool pray_nan = false;
    if constexpr (MODE == MODE_PSI) {
        if (a.psi_ray && lane < G.n_lanes) {
            pray = a.psi_ray;
            pray_base = ((int64_t)A.lanes.j[li] * A.n_mu + m0) * 2 + s_dir;
            pray_nan = a.status[cg.col] == RH15D_BAD_INPUT;
        }
    }
    const int64_t pray_row = (int64_t)A.NL * A.n_mu * 2;
    auto store_psi = [&](int kk, int r, R v) {
        if constexpr (MODE == MODE_PSI)
            if (pray) pray[(g0 + kk) * pray_row + pray_base + 2 * r] = pray_nan ? NAN : static_cast<double>(v);
    };
    R mu[MC], hinvmu[MC], wmu[MC];     // hinvmu = 1 / (2 mu)
#pragma unroll
    for (int r = 0; r < MC; r++) {
        mu[r] = static_cast<R>(A.mu[m0 + r]);
        hinvmu[r] = R(0.5) / mu[r];
        wmu[r] = static_cast<R>(A.wmu[m0 + r]);
    }
    if constexpr (MC == 1) {
        // one angle per lane: its weight joins the lane's per-slot factors
        // applied once per depth point, and the rays add unweighted terms
#pragma unroll
        for (int q = 0; q < NS; q++) {
            kapj[q] *= wmu[0];
            wpsi[q] *= wmu[0];
        }
        wmu[0] = R(1);
    }
    R *out = part + gc0 * A.n_keys + (size_t)key_off * N;
    const int rec_w = a.rec_w, L = A.L;
    constexpr int NK = n_acc<NS, MODE>();
    const int step = s_dir == 0 ? 1 : -1;
    int k = s_dir == 0 ? 0 : N - 1;
    R I[MC], chi_p[MC], S_p[MC];
    R acc[NK];
    const int ray_cols = A.ray_cols;
#pragma unroll
    for (int i = 0; i < NK; i++) acc[i] = R(0);   // every point's first ray sets them
    // reduction blocks: the current point's row within its block, the depth
    // of the block's first point and the points still to come
    using RS = Red<R, NS, MODE>;
    int rb = 0, k_first = k, left = N;
    auto emit = [&]() {
        red_put<R, NS, MODE>(acc, kapj, lds, rb, lane);
        left--;
        if (rb == RS::B - 1 || left == 0) {
            red_flush<R, NS, MODE>(lds, out, N, k_first, step, rb + 1, lane);
            rb = 0;
            k_first = k + step;
        } else {
            rb++;
        }
    };
    // PRD: the intensity of every ray that the rho update reads, per point
    auto store_I = [&](int kk, int r, R v) {
        if constexpr (PRD)
            if (ist_base >= 0) pio.ist[(gc0 + kk) * pio.ist_cols + ist_base + 2 * r] = v;
    };
    {
        PointIn<R, NS, MC> in0;
        load_rows<R, NS, MC, PRD>(rec, popsb, phi, point_rows<R, PRD>(rec_w, L, ray_cols, g0 + k, gc0 + k, &pio), 0,
                                  sl, pb, in0, &pio, psb);
        Shared<R, NS> sh;
        shared_terms<R, NS, MC>(in0, sl, alpha, hnu_k, two_hnu3, lamfac, sh);
        PointIn<R, NS, MC> in2;
        Shared<R, NS> sh2;
        R dzb = R(0);
        if (s_dir != 0) {
            load_rows<R, NS, MC, PRD>(rec, popsb, phi, point_rows<R, PRD>(rec_w, L, ray_cols, g0 + N - 2, gc0 + N - 2, &pio),
                                      3, sl, pb, in2, &pio, psb);
            shared_terms<R, NS, MC>(in2, sl, alpha, hnu_k, two_hnu3, lamfac, sh2);
            dzb = in2.dz;
        }
#pragma unroll
        for (int r = 0; r < MC; r++) {
            RayPt<R, NS> p;
            ray_terms<R, NS, MC, PRD>(sl, sh, in0, pon, r, p);
            R I0 = R(0);
            if (s_dir != 0) {
                RayPt<R, NS> p2;
                ray_terms<R, NS, MC, PRD>(sl, sh2, in2, pon, r, p2);
                const R dtv = R(0.5) * (p.chi + p2.chi) * dzb;
                I0 = dtv > R(0) ? sh.B + mu[r] * (sh.B - sh2.B) * rcp(dtv) : sh.B;
            }
            store_I(k, r, I0);
            store_psi(k, r, R(0));
            if (r == 0) contribute<R, NS, MODE, true>(p, wpsi, wmu[r], I0, R(0), acc);
            else contribute<R, NS, MODE, false>(p, wpsi, wmu[r], I0, R(0), acc);
            I[r] = I0;
            chi_p[r] = p.chi;
            S_p[r] = p.S;
        }
        emit();
    }
    // the rows of consecutive points along the sweep are these many bytes apart
    const int64_t st_rec = (int64_t)step * rec_w * (int64_t)sizeof(R);
    const int64_t st_pop = (int64_t)step * L * (int64_t)sizeof(R);
    const int64_t st_phi = (int64_t)step * ray_cols * (int64_t)sizeof(R);
    const int64_t st_psi = PRD ? (int64_t)step * pio.psi_cols * (int64_t)sizeof(R) : 0;
    // One depth step to the new point k.  Its wavefront-uniform inputs are
    // read at the start of the step (scalar loads, whose short latency the
    // other wavefronts cover); its profile values were loaded into `cur`
    // one step earlier.
    PointRows urow = point_rows<R, PRD>(rec_w, L, ray_cols, g0 + k + step, gc0 + k + step, &pio);
    const int dzi = step > 0 ? 0 : 3;   // the record field with the spacing to the previous point
    auto advance = [&](PointIn<R, NS, MC> &cur) {
        k += step;
        load_uniform<R, NS, MC>(rec, popsb, urow, dzi, sl, cur);
        urow.rec += st_rec;
        urow.pops += st_pop;
        Shared<R, NS> sh;
        shared_terms<R, NS, MC>(cur, sl, alpha, hnu_k, two_hnu3, lamfac, sh);
        const R dz = cur.dz;
#pragma unroll
        for (int r = 0; r < MC; r++) {
            RayPt<R, NS> p;
            ray_terms<R, NS, MC, PRD>(sl, sh, cur, pon, r, p);
            const R x = (chi_p[r] + p.chi) * dz * hinvmu[r];
            R e, wa, wb;
            sc_weights<R>(x, e, wa, wb);
            const R up = I[r] * e + wa * S_p[r];
            const R psi = wb * p.rchi;
            const R Ieff = up + psi * sh.etabg;
            I[r] = up + wb * p.S;
            store_I(k, r, I[r]);
            store_psi(k, r, psi);
            if (r == 0) contribute<R, NS, MODE, true>(p, wpsi, wmu[r], Ieff, psi, acc);
            else contribute<R, NS, MODE, false>(p, wpsi, wmu[r], Ieff, psi, acc);
            chi_p[r] = p.chi;
            S_p[r] = p.S;
        }
        emit();
    };
    // The profile values (vector loads) are read one step ahead of their
    // use, in depth order along the sweep: the rows of the next point to
    // load advance by one point per load.  Past the column's last point
    // they stay on it (a repeated load whose values are not used), so the
    // loads are unconditional and neither input buffer has to keep its old
    // contents on some path.
    const int k1 = N > 1 ? k + step : k;   // the first point to load (the only one of a 1-point column)
    PointRows nxt = point_rows<R, PRD>(rec_w, L, ray_cols, g0 + k1, gc0 + k1, &pio);
    int rows_left = N - 1;
    auto load = [&](PointIn<R, NS, MC> &dst) {
        load_profiles<R, NS, MC, PRD>(phi, nxt, sl, pb, dst, &pio, psb);
        const bool more = --rows_left > 0;
        nxt.rec += more ? st_rec : 0;
        nxt.pops += more ? st_pop : 0;
        nxt.phi += more ? st_phi : 0;
        if constexpr (PRD) nxt.psi += more ? st_psi : 0;
    };
    // two profile buffers used alternately (the loop is unrolled by two), so
    // the values of the next point load into the buffer not in use and no
    // registers are copied between steps
    PointIn<R, NS, MC> ba, bb;
    load(ba);
    for (int i = 1; i < N; i += 2) {
        load(bb);
        advance(ba);
        if (i + 1 >= N) break;
        load(ba);
        advance(bb);
    }
}

// Groups are ordered by their number of slots and, within that, by their
// number of continuum slots; one launch per (slots, continua) covers the
// range [g_begin, g_end), so each variant gets its own registers and the
// line / continuum choice of every slot is fixed at compile time.
template <typename R, int MODE, int NS, int NC, int MC, bool PRD = false>
__global__ __launch_bounds__(256) void k_sweep(RunArgs a, int g_begin, int g_end, const R *__restrict__ rec,
                                               const R *__restrict__ phi, const R *__restrict__ popsb,
                                               R *__restrict__ part) {
    __shared__ __align__(16) R red_lds[4 * Red<R, NS, MODE>::SIZE];
    // The hardware deals consecutive workgroups to the eight XCDs in turn.
    // Renumber them so that each XCD gets a contiguous run of (slot, group
    // block) pairs: the groups of one column then share one L2 for the
    // column's records, populations and profile rows.
    const unsigned nb = gridDim.x * gridDim.y, lin = blockIdx.y * gridDim.x + blockIdx.x;
    const unsigned per = nb / kXcds, rem = nb % kXcds, x = lin % kXcds, r = lin / kXcds;
    const unsigned logical = x < rem ? x * (per + 1) + r : rem * (per + 1) + (x - rem) * per + r;
    const int bx = (int)(logical % gridDim.x), by = (int)(logical / gridDim.x);
    const int grp = rfl(g_begin + bx * 4 + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (grp >= g_end) return;
    int slot;
    if (MODE == MODE_RATES) {
        slot = by;
        if (a.slot_state[slot] != SLOT_ACTIVE) return;
    } else {
        if (by >= a.ctr[CTR_RETIRE]) return;
        slot = rfl(a.retire_list[by]);
    }
    sweep_group<R, MODE, NS, NC, MC, PRD>(a, grp, slot, lane, rec, phi, popsb, part,
                                          red_lds + (threadIdx.x >> 6) * Red<R, NS, MODE>::SIZE);
}

// ---------------------------------------------------------------------------
// statistical equilibrium per depth point
// ---------------------------------------------------------------------------
// Collisional rate coefficient u -> l of transition t at this point.
// Collisional-radiative switching (Sec. 2.3; Hummer & Voels 1988): factor
// of the collision rates in iteration it (1, 2, ...), f0 / 10^(it-1) while
// that exceeds 1, formed by repeated division (the same IEEE operations
// wherever it is evaluated); 1 for f0 <= 1.
__device__ __forceinline__ double crs_factor(double f0, int it) {
    double f = f0;
    for (int i = 1; i < it && f > 1.0; i++) f /= 10.0;
    return f > 1.0 ? f : 1.0;
}

__device__ __forceinline__ double coll_down(const RunArgs &a, const DevTransition &tr, double T, double ne) {
    double Cul;
    if (tr.coll_kind == 0) {
        Cul = ne * kCollC0 * tr.coll_val / (a.A.g[tr.u] * sqrt(T));
    } else {
        const double x = kH * tr.nu0 / (kKB * T);
        Cul = tr.coll_val / (1.0 - tr.coll_val) * tr.A / (-expm1(-x));
    }
    return Cul * a.coll_scale;
}

// Sum of the rate sums `keys[b..e)` at depth k of a column whose key-major
// block ([key][depth], N depths) starts at `part`.
// The loads of eight keys are issued before their sum, which adds them in
// key order.
template <typename R>
__device__ __forceinline__ double key_sum(const R *part, const int *keys, int b, int e, int N, int k) {
    double v = 0.0;
    int i = b;
    for (; i + 8 <= e; i += 8) {
        R x[8];
#pragma unroll
        for (int u = 0; u < 8; u++) x[u] = part[(size_t)keys[i + u] * N + k];
#pragma unroll
        for (int u = 0; u < 8; u++) v += static_cast<double>(x[u]);
    }
    for (; i < e; i++) v += static_cast<double>(part[(size_t)keys[i] * N + k]);
    return v;
}

// Radiative part of the rate-matrix entry (i, j) = blockIdx.y / L, % L at
// every depth point of the active slots: the sweep's rate sums of the
// upward or downward transition from j to i, plus the cross terms of
// overlapping transitions, added in key order.  One lane per depth point
// and entry, with nothing else live, so many lanes' loads are in flight
// together; the rate-equation kernel adds the collisional rates and solves.
template <typename R>
__global__ __launch_bounds__(256) void k_rad_rates(RunArgs a) {
    const DevAtom &A = a.A;
    const int L = A.L;
    const int ij = blockIdx.y;
    const int i = ij / L, j = ij % L;
    if (i == j) return;
    const size_t P = (size_t)a.S * a.ND;
    const int64_t gc = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gc >= (int64_t)P) return;
    const int slot = (int)(gc / a.ND);
    if (a.slot_state[slot] != SLOT_ACTIVE) return;
    const ColGeom cg = geom(a, slot);
    const int k = (int)(gc - cg.gc0);
    if (k >= cg.N) return;
    const R *part = reinterpret_cast<const R *>(a.part) + cg.gc0 * A.n_keys;
    const int N = cg.N;
    double v = 0.0;
    const int tu = A.up_t[ij];
    if (tu >= 0) v += key_sum<R>(part, A.p_key, A.p_off[tu], A.p_off[tu + 1], N, k);
    const int td = A.dn_t[ij];
    if (td >= 0) v += key_sum<R>(part, A.q_key, A.q_off[td], A.q_off[td + 1], N, k);
    for (int x = A.xe_off[ij]; x < A.xe_off[ij + 1]; x++) {
        const int e = A.xe_val[x];
        const int xp = (e > 0 ? e : -e) - 1;
        const double X = key_sum<R>(part, A.x_key, A.x_off[xp], A.x_off[xp + 1], N, k);
        v += e > 0 ? X : -X;
    }
    a.rad[(size_t)ij * P + gc] = v;
}

// Rate matrix entry (i, j), i != j: the radiative rates from j into i with
// the cross terms of overlapping transitions (gathered by k_rad_rates; with
// zero radiation the spontaneous rates alone), plus the collisional rates.
// Kinds of rate-equation solve: an iteration (preconditioned radiative
// rates), the zero-radiation start, an escape-probability start iteration.
enum { SE_ITERATION = 0, SE_ZERO_RADIATION = 1, SE_ESCAPE = 2 };

template <int KIND>
__device__ __forceinline__ double rate_entry(const RunArgs &a, int i, int j, int L, int64_t gc, double T, double ne,
                                             double cf) {
    constexpr bool ZERO_RAD = KIND != SE_ITERATION;
    const DevAtom &A = a.A;
    double v = 0.0;
    if (!ZERO_RAD) v = a.rad[(size_t)(i * L + j) * ((size_t)a.S * a.ND) + gc];
    const int tu = A.up_t[i * L + j];
    if (tu >= 0) {  // j = l, i = u: excitation / ionisation
        const DevTransition &tr = A.tr[tu];
        v += coll_down(a, tr, T, ne) * exp(a.lnr[gc * L + tr.u] - a.lnr[gc * L + tr.l]) * cf;
    }
    const int td = A.dn_t[i * L + j];
    if (td >= 0) {  // j = u, i = l: de-excitation / recombination
        const DevTransition &tr = A.tr[td];
        if (ZERO_RAD) {
            // spontaneous rate, times the transition's escape probability
            // (stored in the rate-entry buffer) in an escape iteration
            const double beta = KIND == SE_ESCAPE ? a.rad[(size_t)td * ((size_t)a.S * a.ND) + gc] : 1.0;
            if (tr.kind == 0) {
                v += tr.A * beta;
            } else {
                const double G0 = a.gr[gc * A.n_cont + (td - A.n_lines)];
                double q = 0.0;
                for (int ja = 0; ja < tr.n_act; ja++) {
                    const double nu = A.nu[A.act_j[tr.act_off + ja]];
                    const double G = G0 * exp(-kH * nu / (kKB * T));
                    const double r = tr.nu0 / nu;
                    const double alpha = tr.alpha0 * r * r * r;
                    q += 4.0 * kPI * A.act_w[tr.act_off + ja] / (kH * nu) * 2.0 * kH * nu * nu * nu / (kC * kC) * G * alpha;
                }
                v += q * beta;
            }
        }
        v += coll_down(a, tr, T, ne) * cf;
    }
    return v;
}

template <typename R, int L, int KIND>
__device__ __forceinline__ void se_point(const RunArgs &a, int slot, int k) {
    constexpr bool ZERO_RAD = KIND != SE_ITERATION;
    const ColGeom cg = geom(a, slot);
    if (k >= cg.N) return;
    const int64_t g = cg.g0 + k, gc = cg.gc0 + k;
    const DevAtom &A = a.A;
    const double T = a.T[g], ne = a.ne[g];
    // collision factor of this iteration (the start solutions use 1)
    const double cf = ZERO_RAD ? 1.0 : crs_factor(a.crs_f0, a.slot_it[slot] + 1);
    double M[L][L];
    double nold[L], b[L];
#pragma unroll
    for (int i = 0; i < L; i++) nold[i] = a.pops[g * L + i];
    // off-diagonal entries; every column of the rate matrix sums to zero, so
    // the diagonal is minus the rest of its column
#pragma unroll
    for (int i = 0; i < L; i++)
#pragma unroll
        for (int j = 0; j < L; j++)
            M[i][j] = i == j ? 0.0 : rate_entry<KIND>(a, i, j, L, gc, T, ne, cf);
#pragma unroll
    for (int j = 0; j < L; j++) {
        double c = 0.0;
#pragma unroll
        for (int i = 0; i < L; i++) if (i != j) c += M[i][j];
        M[j][j] = -c;
    }
    // particle conservation replaces the equation of the most populated level
    int istar = 0;
#pragma unroll
    for (int i = 1; i < L; i++) if (nold[i] > nold[istar]) istar = i;
    const double ntot = A.abund * a.nH[g];
#pragma unroll
    for (int i = 0; i < L; i++) {
        b[i] = (i == istar) ? ntot : 0.0;
#pragma unroll
        for (int j = 0; j < L; j++) if (i == istar) M[i][j] = 1.0;
    }
    // Gaussian elimination with partial pivoting (first largest pivot)
    bool singular = false;
#pragma unroll
    for (int col = 0; col < L; col++) {
        int p = col;
        double best = fabs(M[col][col]);
#pragma unroll
        for (int r = col + 1; r < L; r++) if (fabs(M[r][col]) > best) { best = fabs(M[r][col]); p = r; }
        if (best == 0.0) singular = true;
#pragma unroll
        for (int r = col + 1; r < L; r++) {
            if (r == p) {
#pragma unroll
                for (int j = 0; j < L; j++) { double tmp = M[col][j]; M[col][j] = M[r][j]; M[r][j] = tmp; }
                double tmp = b[col]; b[col] = b[r]; b[r] = tmp;
            }
        }
#pragma unroll
        for (int r = col + 1; r < L; r++) {
            const double f = M[r][col] / M[col][col];
#pragma unroll
            for (int j = col; j < L; j++) M[r][j] -= f * M[col][j];
            b[r] -= f * b[col];
        }
    }
#pragma unroll
    for (int r = L - 1; r >= 0; r--) {
        double s = b[r];
#pragma unroll
        for (int j = r + 1; j < L; j++) s -= M[r][j] * b[j];
        b[r] = s / M[r][r];
    }
    if (ZERO_RAD) {
#pragma unroll
        for (int i = 0; i < L; i++) {
            a.pops[g * L + i] = b[i];
            if (a.popsf) a.popsf[gc * L + i] = static_cast<float>(b[i]);
        }
        return;
    }
    double dmax = 0.0;
    int fl = singular ? 2 : 0;
#pragma unroll
    for (int i = 0; i < L; i++) {
        a.nse[gc * L + i] = b[i];
        if (!(b[i] > 0.0) || !isfinite(b[i])) { if (fl == 0) fl = 1; }
        else dmax = fmax(dmax, fabs(b[i] - nold[i]) / b[i]);
    }
    a.dk[gc] = dmax;
    a.flag[gc] = fl;
}

template <typename R, int L>
__global__ __launch_bounds__(256) void k_se(RunArgs a) {
    const int64_t gc = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gc >= (int64_t)a.S * a.ND) return;
    const int slot = (int)(gc / a.ND);
    if (a.slot_state[slot] != SLOT_ACTIVE) return;
    se_point<R, L, SE_ITERATION>(a, slot, (int)(gc % a.ND));
}

// Start solutions of the slots being refilled: the rate equations with zero
// radiation, or one escape-probability iteration (KIND).
template <int L, int KIND>
__global__ __launch_bounds__(256) void k_se_start(RunArgs a) {
    const int64_t n = (int64_t)a.ctr[CTR_REFILL] * a.ND;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n; w += (int64_t)gridDim.x * blockDim.x)
        se_point<double, L, KIND>(a, a.refill_list[w / a.ND], (int)(w % a.ND));
}

// Escape probabilities of one escape-probability start iteration (Sec. 2.3,
// starting solutions), one lane per (slot being refilled, transition): the
// vertical optical depth from the top at the transition's reference
// frequency with the current populations, line centre in the rest frame
// (chi = h nu0 / 4 pi (n_l B_lu - n_u B_ul) H(a, 0) / (sqrt(pi) Delta nu_D))
// or continuum edge (chi = (n_l - n_u G) alpha), negative opacities as 0,
// accumulated by the trapezoid rule in z; beta = (1 - e^-tau) / tau (1 at
// tau = 0) goes to the rate-entry buffer at [t][gc].
__global__ __launch_bounds__(256) void k_escape_beta(RunArgs a) {
    const DevAtom &A = a.A;
    const int L = A.L, T = A.T;
    const size_t P = (size_t)a.S * a.ND;
    const int64_t n = (int64_t)a.ctr[CTR_REFILL] * T;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n; w += (int64_t)gridDim.x * blockDim.x) {
        const int slot = a.refill_list[w / T], t = (int)(w % T);
        const ColGeom cg = geom(a, slot);
        const DevTransition &tr = A.tr[t];
        double tau = 0.0, chi_prev = 0.0;
        for (int k = 0; k < cg.N; k++) {
            const int64_t g = cg.g0 + k, gc = cg.gc0 + k;
            const double Tk = a.T[g];
            const double nl = a.pops[g * L + tr.l], nu = a.pops[g * L + tr.u];
            double c;
            if (tr.kind == 0) {
                const double dnd = tr.nu0 / kC * sqrt(2.0 * kKB * Tk / A.mass + a.vt[g] * a.vt[g]);
                const double H0 = tr.voigt ? voigt_w4<double>(tr.gamma / (4.0 * kPI * dnd), 0.0) : 1.0;
                c = tr.hnu4pi * (nl * tr.Blu - nu * tr.Bul) * H0 / (sqrt(kPI) * dnd);
            } else {
                const double G = exp(a.lnr[gc * L + tr.l] - a.lnr[gc * L + tr.u]) * exp(-kH * tr.nu0 / (kKB * Tk));
                c = (nl - nu * G) * tr.alpha0;
            }
            c = c > 0.0 ? c : 0.0;
            if (k > 0) tau += 0.5 * (chi_prev + c) * (a.z[g - 1] - a.z[g]);
            chi_prev = c;
            a.rad[(size_t)t * P + gc] = tau > 0.0 ? -expm1(-tau) / tau : 1.0;
        }
    }
}

// ---------------------------------------------------------------------------
// partial frequency redistribution (angle-averaged, Uitenbroek 2001)
// ---------------------------------------------------------------------------
// Angle-averaged redistribution function R_II (Hummer 1962) in Doppler units
// as the Lorentzian average, over the scattering's atom-frame frequency xi,
// of the angle-averaged coherent Doppler kernel:
//   R(x, x2) = 1/2 int (a/pi)/(a^2 + xi^2) erfc(|xi - m| + d) dxi,
// m = (x + x2)/2, d = |x - x2|/2; 0 for d >= 6 (erfc(6) = 2e-17).  The
// integral runs over [m - w, m + w], w = 6 - d, cut at xi = m and at
// xi = +-0.5 where inside; pieces within the Lorentzian core |xi| <= 0.5 by
// 4-point Gauss-Legendre on 8 panels uniform in t = asinh(xi / a) (measure
// dt / (pi cosh t)), the others on ceil(length) panels uniform in xi.
constexpr double kRiiCore = 0.5;
constexpr int kRiiCorePanels = 8;
__device__ double rII(double a, double x, double x2) {
    const double gx[4] = {-0.8611363115940526, -0.3399810435848563, 0.3399810435848563, 0.8611363115940526};
    const double gw[4] = {0.3478548451374538, 0.6521451548625461, 0.6521451548625461, 0.3478548451374538};
    const double m = 0.5 * (x + x2), d = 0.5 * fabs(x - x2);
    if (d >= 6.0) return 0.0;
    const double w = 6.0 - d;
    double e[5];
    int ne = 0;
    e[ne++] = m - w;
    if (-kRiiCore > m - w && -kRiiCore < m) e[ne++] = -kRiiCore;
    if (kRiiCore > m - w && kRiiCore < m) e[ne++] = kRiiCore;
    e[ne++] = m;
    if (-kRiiCore > m && -kRiiCore < m + w) e[ne++] = -kRiiCore;
    if (kRiiCore > m && kRiiCore < m + w) e[ne++] = kRiiCore;
    e[ne++] = m + w;
    double sum = 0.0;
    for (int i = 0; i + 1 < ne; i++) {
        const double lo = e[i], hi = e[i + 1];
        if (!(hi > lo)) continue;
        if (lo >= -kRiiCore && hi <= kRiiCore) {
            const double t0 = asinh(lo / a), h = (asinh(hi / a) - t0) / kRiiCorePanels;
            for (int p = 0; p < kRiiCorePanels; p++) {
                const double c = t0 + (p + 0.5) * h;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const double sh = sinh(c + 0.5 * h * gx[q]);
                    sum += 0.5 * h * gw[q] * erfc(fabs(a * sh - m) + d) / (kPI * sqrt(1.0 + sh * sh));
                }
            }
        } else {
            int np = (int)ceil(hi - lo);
            if (np < 1) np = 1;
            const double h = (hi - lo) / np;
            for (int p = 0; p < np; p++) {
                const double c = lo + (p + 0.5) * h;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const double xi = c + 0.5 * h * gx[q];
                    sum += 0.5 * h * gw[q] * (a / kPI) / (a * a + xi * xi) * erfc(fabs(xi - m) + d);
                }
            }
        }
    }
    return 0.5 * sum;
}

// Redistribution weights of the PRD lines at the depth points of the slots
// being refilled, one 64-lane workgroup per (slot, depth, PRD line):
// g(j, j') = w_j' R(x_j', x_j) / sum_j'' w_j'' R(x_j'', x_j) (x in Doppler
// widths of the point, w the trapezoid frequency weights), row j of the
// table holding the weights of the inputs j'.  A constant mean intensity is
// redistributed into itself exactly.
template <typename R>
__global__ __launch_bounds__(64) void k_prd_tables(RunArgs a) {
    const DevAtom &A = a.A;
    const int lane = threadIdx.x;
    const int64_t n = (int64_t)a.ctr[CTR_REFILL] * a.ND * A.n_prd;
    for (int64_t w = blockIdx.x; w < n; w += gridDim.x) {
        const int ip = (int)(w % A.n_prd);
        const int64_t sk = w / A.n_prd;
        const int slot = a.refill_list[sk / a.ND], k = (int)(sk % a.ND);
        const ColGeom cg = geom(a, slot);
        if (k >= cg.N) continue;
        const int64_t g = cg.g0 + k, gc = cg.gc0 + k;
        const DevTransition &tr = A.tr[A.prd_t[ip]];
        const int na = tr.n_act;
        const double dnd = tr.nu0 / kC * sqrt(2.0 * kKB * a.T[g] / A.mass + a.vt[g] * a.vt[g]);
        const double ad = (tr.gamma + tr.c_el * a.nH[g]) / (4.0 * kPI * dnd);
        R *G = reinterpret_cast<R *>(a.gtab) + gc * A.g_cols + tr.g_off;
        // R(x_j, x_j2) for j >= j2, stored at both places
        for (int p = lane; p < na * (na + 1) / 2; p += 64) {
            int j = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
            while (j * (j + 1) / 2 > p) j--;
            while ((j + 1) * (j + 2) / 2 <= p) j++;
            const int j2 = p - j * (j + 1) / 2;
            const double x = (A.nu[A.act_j[tr.act_off + j]] - tr.nu0) / dnd;
            const double x2 = (A.nu[A.act_j[tr.act_off + j2]] - tr.nu0) / dnd;
            const R r = static_cast<R>(rII(ad, x, x2));
            G[j * na + j2] = r;
            G[j2 * na + j] = r;
        }
        __syncthreads();
        // row sums of output frequency j first (every lane reads the whole,
        // still symmetric table), then the weights stored transposed,
        // G[j2 * na + j] = g(j <- j2), so that the rho update's lanes (one
        // output frequency each) read consecutive addresses; each lane
        // rewrites only its own column
        double sums[kMaxPrdFreq / 64];
#pragma unroll
        for (int c = 0; c < kMaxPrdFreq / 64; c++) {
            const int j = lane + 64 * c;
            double sum = 0.0;
            if (j < na)
                for (int j2 = 0; j2 < na; j2++) sum += A.act_w[tr.act_off + j2] * static_cast<double>(G[j * na + j2]);
            sums[c] = sum;
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kMaxPrdFreq / 64; c++) {
            const int j = lane + 64 * c;
            if (j < na)
                for (int j2 = 0; j2 < na; j2++)
                    G[j2 * na + j] =
                        static_cast<R>(A.act_w[tr.act_off + j2] * static_cast<double>(G[j2 * na + j]) / sums[c]);
        }
        __syncthreads();
    }
}

// Actual radiative rate coefficient of transition t at depth point gc from
// the stored intensities of the last sweep: out of its upper level
// (UP = false: spontaneous and stimulated emission with the current
// emission profile) or out of its lower level (UP = true: absorption);
// the lanes of the wavefront share the rays, the sum is over the wavefront.
template <typename R, bool UP>
__device__ double actual_rate(const RunArgs &a, const DevTransition &tr, int t, int64_t gc, double T, int lane) {
    const DevAtom &A = a.A;
    const int na = tr.n_act, nmu = A.n_mu;
    const R *ist = reinterpret_cast<const R *>(a.ist) + gc * A.ist_cols;
    const R *phi = reinterpret_cast<const R *>(a.phi) + gc * A.ray_cols + tr.ray_off;
    const R *psi = (a.prd && tr.prd) ? reinterpret_cast<const R *>(a.emis) + gc * A.psi_cols + tr.psi_off : phi;
    double acc = 0.0;
    // one wavelength per lane, its angles and directions in turn: the
    // wavelength's factors (and a continuum's exponential) once per lane
    for (int ja = lane; ja < na; ja += 64) {
        const int j = A.act_j[tr.act_off + ja];
        const R *Ij = ist + A.st_idx[j] * nmu * 2;
        const double wj = A.act_w[tr.act_off + ja] * 0.5;
        if (tr.kind == 0) {
            for (int s = 0; s < 2; s++)
                for (int m = 0; m < nmu; m++) {
                    const int col = (s * na + ja) * nmu + m;
                    const double W = wj * A.wmu[m], I = static_cast<double>(Ij[m * 2 + s]);
                    if (UP) acc += W * static_cast<double>(phi[col]) * tr.Blu * I;
                    else acc += W * static_cast<double>(psi[col]) * (tr.A + tr.Bul * I);
                }
        } else {
            const double nu = A.nu[j];
            const double rr = tr.nu0 / nu;
            const double alpha = tr.alpha0 * rr * rr * rr;
            const double kap = 4.0 * kPI * wj / (kH * nu);
            double G = 0.0, spont = 0.0;
            if (!UP) {
                G = a.gr[gc * A.n_cont + (t - A.n_lines)] * exp(-kH * nu / (kKB * T));
                spont = 2.0 * kH * nu * nu * nu / (kC * kC) * G * alpha;
            }
            for (int s = 0; s < 2; s++)
                for (int m = 0; m < nmu; m++) {
                    const double I = static_cast<double>(Ij[m * 2 + s]);
                    if (UP) acc += kap * A.wmu[m] * alpha * I;
                    else acc += kap * A.wmu[m] * (spont + G * alpha * I);
                }
        }
    }
    return wave_sum(acc);
}

// rho of the PRD lines after an iteration (angle-averaged PRD, Uitenbroek
// 2001), one wavefront per (slot still iterating, depth point, PRD line):
//   rho(j) = 1 + gamma n_l B_lu / (n_u P_u) [sum_j' g(j, j') J(j') - Jbar]
// with J the angle-averaged and Jbar the profile-weighted mean intensity of
// the iteration's formal solution, P_u the total rate out of the upper level
// (radiative with the same intensities and the current emission profiles,
// plus collisional), gamma = P_u / (P_u + c_el n_H), the new populations;
// then PRD switching (Sec. 2.3, Eq. 1) rho' = rho eps + (1 - eps),
// eps = min(1, eps0 it^2) (1 if eps0 <= 0), negative values as 0, and
// normalisation so that sum over rays of W phi rho' = 1 (rho = 1 where that
// sum is not positive).  The result goes
// to a.rho; k_prd_psi then rewrites the emission profiles (every line's
// rates here read the previous ones).
template <typename R>
__global__ __launch_bounds__(256) void k_prd_rho(RunArgs a) {
    __shared__ double sh[4][kMaxPrdFreq];
    const DevAtom &A = a.A;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t n = (int64_t)a.S * a.ND * A.n_prd;
    const int64_t waves = (int64_t)gridDim.x * 4;
    const int L = A.L, nmu = A.n_mu;
    for (int64_t w = rfl_wave(blockIdx.x * 4 + wv); w < n; w += waves) {
        const int ip = (int)(w % A.n_prd);
        const int64_t sk = w / A.n_prd;
        const int slot = (int)(sk / a.ND), k = (int)(sk % a.ND);
        if (a.slot_state[slot] != SLOT_ACTIVE) continue;
        const ColGeom cg = geom(a, slot);
        if (k >= cg.N) continue;
        const int64_t g = cg.g0 + k, gc = cg.gc0 + k;
        const int t = A.prd_t[ip];
        const DevTransition &tr = A.tr[t];
        const int na = tr.n_act, u = tr.u;
        const double T = a.T[g], ne = a.ne[g];
        const double cf = crs_factor(a.crs_f0, a.slot_it[slot]);
        // total rate out of the upper level
        double Pu = 0.0;
        for (int t2 = 0; t2 < A.T; t2++) {
            const DevTransition &d = A.tr[t2];
            if (d.u == u) {
                Pu += actual_rate<R, false>(a, d, t2, gc, T, lane) + coll_down(a, d, T, ne) * cf;
            } else if (d.l == u) {
                Pu += actual_rate<R, true>(a, d, t2, gc, T, lane) +
                      coll_down(a, d, T, ne) * exp(a.lnr[gc * L + d.u] - a.lnr[gc * L + d.l]) * cf;
            }
        }
        const double gam = Pu / (Pu + tr.c_el * a.nH[g]);
        const double fac = gam * a.pops[g * L + tr.l] * tr.Blu / (a.pops[g * L + u] * Pu);
        // mean intensities
        const R *ist = reinterpret_cast<const R *>(a.ist) + gc * A.ist_cols;
        const R *phi = reinterpret_cast<const R *>(a.phi) + gc * A.ray_cols + tr.ray_off;
        for (int ja = lane; ja < na; ja += 64) {
            const int j = A.act_j[tr.act_off + ja];
            double J = 0.0;
            for (int m = 0; m < nmu; m++)
                for (int s2 = 0; s2 < 2; s2++) J += 0.5 * A.wmu[m] * static_cast<double>(ist[(A.st_idx[j] * nmu + m) * 2 + s2]);
            sh[wv][ja] = J;
        }
        double jb = 0.0;
        for (int r = lane; r < na * nmu * 2; r += 64) {
            const int s2 = r / (na * nmu), rem = r % (na * nmu), ja = rem / nmu, m = rem % nmu;
            const int j = A.act_j[tr.act_off + ja];
            jb += A.act_w[tr.act_off + ja] * 0.5 * A.wmu[m] * static_cast<double>(phi[(s2 * na + ja) * nmu + m]) *
                  static_cast<double>(ist[(A.st_idx[j] * nmu + m) * 2 + s2]);
        }
        const double Jbar = wave_sum(jb);
        double eps = 1.0;
        if (a.prd_eps0 > 0.0) eps = fmin(1.0, a.prd_eps0 * (double)a.slot_it[slot] * (double)a.slot_it[slot]);
        const R *G = reinterpret_cast<const R *>(a.gtab) + gc * A.g_cols + tr.g_off;
        // the wavefront's J values are in LDS; rho per output frequency
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double rloc[kMaxPrdFreq / 64];
#pragma unroll
        for (int c = 0; c < kMaxPrdFreq / 64; c++) {
            const int ja = lane + 64 * c;
            rloc[c] = 1.0;
            if (ja < na) {
                double sJ = 0.0;
                for (int j2 = 0; j2 < na; j2++) sJ += static_cast<double>(G[j2 * na + ja]) * sh[wv][j2];
                double r = isfinite(fac) ? 1.0 + fac * (sJ - Jbar) : 1.0;
                r = r * eps + (1.0 - eps);
                rloc[c] = r > 0.0 ? r : 0.0;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int c = 0; c < kMaxPrdFreq / 64; c++)
            if (lane + 64 * c < na) sh[wv][lane + 64 * c] = rloc[c];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double nrm = 0.0;
        for (int r = lane; r < na * nmu * 2; r += 64) {
            const int s2 = r / (na * nmu), rem = r % (na * nmu), ja = rem / nmu, m = rem % nmu;
            nrm += A.act_w[tr.act_off + ja] * 0.5 * A.wmu[m] * static_cast<double>(phi[(s2 * na + ja) * nmu + m]) *
                   sh[wv][ja];
        }
        const double norm = wave_sum(nrm);
        int off = 0;
        for (int i = 0; i < ip; i++) off += A.tr[A.prd_t[i]].n_act;
        double *rho = a.rho + gc * (A.psi_cols / (2 * nmu + 1)) + off;
        // no positive emission left (every rho' clamped to 0): CRD at this point
        const bool ok = norm > 0.0 && isfinite(norm);
#pragma unroll
        for (int c = 0; c < kMaxPrdFreq / 64; c++)
            if (lane + 64 * c < na) rho[lane + 64 * c] = ok ? rloc[c] / norm : 1.0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Emission profiles of the PRD lines from the new rho: psi = rho(j) phi for
// every ray of the line (quadrature rays and the vertical emergent ray).
template <typename R>
__global__ __launch_bounds__(256) void k_prd_psi(RunArgs a) {
    const DevAtom &A = a.A;
    const int nmu = A.n_mu, rw = A.psi_cols / (2 * nmu + 1);
    const int64_t n = (int64_t)a.S * a.ND * A.psi_cols;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n; w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t gc = w / A.psi_cols;
        const int col = (int)(w % A.psi_cols);
        const int slot = (int)(gc / a.ND), k = (int)(gc % a.ND);
        if (a.slot_state[slot] != SLOT_ACTIVE) continue;
        if (k >= (int)(a.doff[a.slot_col[slot] + 1] - a.doff[a.slot_col[slot]])) continue;
        // the PRD line owning this column and the column's wavelength
        int ip = 0, off = 0;
        while (ip + 1 < A.n_prd && col >= A.tr[A.prd_t[ip + 1]].psi_off) { off += A.tr[A.prd_t[ip]].n_act; ip++; }
        const DevTransition &tr = A.tr[A.prd_t[ip]];
        const int lc = col - tr.psi_off, na = tr.n_act;
        const int ja = lc < 2 * nmu * na ? (lc % (na * nmu)) / nmu : lc - 2 * nmu * na;
        const double r = a.rho[gc * rw + off + ja];
        const R ph = reinterpret_cast<const R *>(a.phi)[gc * A.ray_cols + tr.ray_off + lc];
        reinterpret_cast<R *>(a.emis)[gc * A.psi_cols + col] = static_cast<R>(r * static_cast<double>(ph));
    }
}

// ---------------------------------------------------------------------------
// convergence test and Ng acceleration, one workgroup per slot
// ---------------------------------------------------------------------------
constexpr int kConvThreads = 256;

__device__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = kConvThreads / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}
__device__ double block_max(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = kConvThreads / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Stopping test of iteration k: change d < tol and, with tol_fp > 0, the
// remainder d r / (1 - r) of the contraction r = d / dprev of two plain
// iterations below tol_fp, tested as d^2 < tol_fp (dprev - d); dprev < 0
// (first iteration, or an Ng extrapolation just applied) has no ratio and
// passes only d = 0.
__device__ __forceinline__ bool converged_at(double d, double dprev, double tol, double tol_fp) {
    if (!(d < tol)) return false;
    if (!(tol_fp > 0.0)) return true;
    if (dprev < 0.0) return d == 0.0;
    return d < dprev && d * d < tol_fp * (dprev - d);
}

__global__ __launch_bounds__(kConvThreads) void k_converge(RunArgs a) {
    __shared__ double sh[kConvThreads];
    const int slot = blockIdx.x;
    if (a.slot_state[slot] != SLOT_ACTIVE) return;
    const ColGeom cg = geom(a, slot);
    const int c = cg.col, N = cg.N;
    const int64_t g0 = cg.g0, gc0 = cg.gc0;
    const int L = a.A.L;
    const int NV = N * L;
    const int it = a.slot_it[slot] + 1;
    double dm = 0.0, fl = 0.0;
    for (int k = threadIdx.x; k < N; k += kConvThreads) {
        dm = fmax(dm, a.dk[gc0 + k]);
        fl = fmax(fl, (double)a.flag[gc0 + k]);
    }
    dm = block_max(dm, sh);
    fl = block_max(fl, sh);
    double *pops = a.pops + g0 * L;
    const double *nse = a.nse + gc0 * L;
    int status = -1;
    if (fl == 2.0) status = RH15D_SINGULAR;
    else if (fl == 1.0) status = RH15D_NONFINITE;
    if (a.history && threadIdx.x == 0) a.history[(size_t)c * a.max_iter + it - 1] = fl > 0.0 ? NAN : dm;
    double dprev = dm;    // the next iteration's ratio partner
    if (status < 0) {
        for (int i = threadIdx.x; i < NV; i += kConvThreads) pops[i] = nse[i];
        // while the collisions are switched the iterate solves another
        // problem: it may not end the iteration or enter Ng's history
        const bool switched = crs_factor(a.crs_f0, it) > 1.0;
        if (!switched && converged_at(dm, a.slot_dprev[slot], a.tol, a.tol_fp)) {
            status = RH15D_CONVERGED;
        } else if (a.ng_order == 2 && it >= a.ng_delay && !switched) {
            const size_t stride = (size_t)a.S * a.ND * L;
            const int head = (a.ng_head[slot] + 1) & 3;
            double *newest = a.ring + head * stride + gc0 * L;
            for (int i = threadIdx.x; i < NV; i += kConvThreads) newest[i] = nse[i];
            int cnt = a.ng_count[slot] + 1;
            const int need = a.ng_period > 4 ? a.ng_period : 4;
            if (cnt >= need) {
                const double *x0 = a.ring + head * stride + gc0 * L;
                const double *x1 = a.ring + ((head + 3) & 3) * stride + gc0 * L;
                const double *x2 = a.ring + ((head + 2) & 3) * stride + gc0 * L;
                const double *x3 = a.ring + ((head + 1) & 3) * stride + gc0 * L;
                double s11 = 0, s12 = 0, s22 = 0, r1 = 0, r2 = 0;
                for (int i = threadIdx.x; i < NV; i += kConvThreads) {
                    const double w = 1.0 / (x0[i] * x0[i]);
                    const double d0 = x0[i] - x1[i], d1 = x1[i] - x2[i], d2 = x2[i] - x3[i];
                    const double e1 = d0 - d1, e2 = d0 - d2;
                    s11 += w * e1 * e1; s12 += w * e1 * e2; s22 += w * e2 * e2;
                    r1 += w * d0 * e1; r2 += w * d0 * e2;
                }
                s11 = block_sum(s11, sh); s12 = block_sum(s12, sh); s22 = block_sum(s22, sh);
                r1 = block_sum(r1, sh); r2 = block_sum(r2, sh);
                const double det = s11 * s22 - s12 * s12;
                if (fabs(det) > 1e-14 * s11 * s22) {
                    const double a1 = (r1 * s22 - r2 * s12) / det, a2 = (r2 * s11 - r1 * s12) / det;
                    double bad = 0.0;
                    for (int i = threadIdx.x; i < NV; i += kConvThreads) {
                        const double v = (1.0 - a1 - a2) * x0[i] + a1 * x1[i] + a2 * x2[i];
                        if (!(v > 0.0)) bad = 1.0;
                    }
                    bad = block_max(bad, sh);
                    if (bad == 0.0) {
                        for (int i = threadIdx.x; i < NV; i += kConvThreads)
                            pops[i] = (1.0 - a1 - a2) * x0[i] + a1 * x1[i] + a2 * x2[i];
                        dprev = -1.0;   // no contraction ratio across an extrapolation
                    }
                }
                cnt = 0;
            }
            if (threadIdx.x == 0) { a.ng_head[slot] = head; a.ng_count[slot] = cnt; }
        }
        if (status < 0 && it >= a.max_iter) status = RH15D_MAX_ITER;
    }
    __syncthreads();
    if (a.popsf)
        for (int i = threadIdx.x; i < NV; i += kConvThreads) a.popsf[gc0 * L + i] = static_cast<float>(pops[i]);
    if (threadIdx.x == 0) {
        a.slot_it[slot] = it;
        a.slot_dprev[slot] = dprev;
        if (status >= 0) {
            a.status[c] = status;
            a.n_iter[c] = it;
            a.slot_state[slot] = SLOT_DONE;
            a.retire_list[atomicAdd(&a.ctr[CTR_RETIRE], 1)] = slot;
        }
    }
}

// ---------------------------------------------------------------------------
// output of finished columns: vertical emergent intensity and Psi*
// ---------------------------------------------------------------------------
// Opacity and source function of the vertical (mu = 1, upward) ray at
// wavelength j, depth point k; line profiles come from the prepared table.
// One thread per (column, wavelength); the active transitions of the
// wavelength are unpacked once, and each depth point's inputs are loaded one
// step ahead of their use.  The prepared tables (per-depth records, line
// profiles) are read in the sweep's precision TB and the arithmetic runs in
// AR: FP64 for the plain path; FP32 for the precision form, where the
// emergent intensity spans more decades than FP32 holds (the Planck
// function's Wien tail in the far ultraviolet), so every emissivity, source
// function and intensity of the wavelength carries the factor
// exp(h nu / k T_max) of the column's hottest point, removed in FP64 at the
// end.  Opacities are not scaled.
template <typename AR>
struct EmTrans {
    int na;
    int kind[kMaxSlots], l[kMaxSlots], u[kMaxSlots], col[kMaxSlots];  // col: profile column or continuum index
    int pcol[kMaxSlots];           // PRD line: emission-profile column, else -1
    AR cblu[kMaxSlots], cbul[kMaxSlots], ca[kMaxSlots], alpha[kMaxSlots];
};

template <typename AR>
struct EmIn {
    AR invT, kbg, dz;
    AR f[kMaxSlots];               // profile value (lines) or continuum G factor of the record
    AR fs[kMaxSlots];              // emission-profile value (PRD lines; else f)
    AR nl[kMaxSlots], nu[kMaxSlots];
};

// Populations: FP64 by global depth index g (FP64 path), or the FP32 copy by
// slot-local index gc (FP32 path; the same values rounded to FP32).
template <typename TB, typename AR>
__device__ __forceinline__ void em_load(const TB *__restrict__ rec, const TB *__restrict__ phi,
                                        const TB *__restrict__ pops, int rec_w, int ray_cols, int L,
                                        const EmTrans<AR> &et, int64_t g, int64_t gc, int64_t gc_dz, EmIn<AR> &p,
                                        const TB *psi, int psi_cols) {
    const TB *r = rec + gc * rec_w;
    p.invT = static_cast<AR>(r[1]);
    p.kbg = static_cast<AR>(r[2]);
    p.dz = static_cast<AR>(rec[gc_dz * rec_w]);
    const TB *n = pops + (sizeof(TB) == 8 ? g : gc) * L;
    const TB *pr = phi + gc * ray_cols;
#pragma unroll
    for (int q = 0; q < kMaxSlots; q++) {
        if (q < et.na) {
            p.nl[q] = static_cast<AR>(n[et.l[q]]);
            p.nu[q] = static_cast<AR>(n[et.u[q]]);
            p.f[q] = static_cast<AR>(et.kind[q] == 0 ? pr[et.col[q]] : r[kRecHead + et.col[q]]);
            p.fs[q] = et.pcol[q] >= 0 ? static_cast<AR>(psi[gc * psi_cols + et.pcol[q]]) : p.f[q];
        }
    }
}

// chi, and the source function and Planck function times exp(x0)
template <typename AR>
__device__ __forceinline__ void em_point(const EmIn<AR> &in, const EmTrans<AR> &et, AR hnu_k, AR two_hnu3, AR lamfac,
                                         AR x0, AR scale, AR &chi, AR &S, AR &B) {
    const AR x = hnu_k * in.invT;
    const AR ex = d_exp(-x), omx = one_m_exp(x, ex);
    const AR exs = sizeof(AR) == 8 ? ex : d_exp(x0 - x);
    if constexpr (sizeof(AR) == 8) B = two_hnu3 * exs / omx;
    else B = two_hnu3 * exs * rcp(omx);
    AR c = in.kbg * lamfac;
    AR e = c * B;
#pragma unroll
    for (int q = 0; q < kMaxSlots; q++) {
        if (q < et.na) {
            AR vlu, vul, U;
            if (et.kind[q] == 0) {
                vlu = et.cblu[q] * in.f[q];
                vul = et.cbul[q] * in.fs[q];
                U = et.ca[q] * in.fs[q] * scale;
            } else {
                vlu = et.alpha[q];
                vul = in.f[q] * ex * et.alpha[q];
                U = two_hnu3 * (in.f[q] * exs) * et.alpha[q];
            }
            c += in.nl[q] * vlu - in.nu[q] * vul;
            e += in.nu[q] * U;
        }
    }
    chi = c;
    if constexpr (sizeof(AR) == 8) S = e / c;
    else S = e * rcp(c);
}

template <typename TB, typename AR>
__global__ __launch_bounds__(256) void k_emergent(RunArgs a, const TB *__restrict__ rec, const TB *__restrict__ phi,
                                                  const TB *__restrict__ pops) {
    const TB *psi = reinterpret_cast<const TB *>(a.emis);
    const int psi_cols = a.A.psi_cols;
    const DevAtom &A = a.A;
    const int64_t n = (int64_t)a.ctr[CTR_RETIRE] * A.NL;
    const int rec_w = a.rec_w, ray_cols = A.ray_cols, L = A.L;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n; w += (int64_t)gridDim.x * blockDim.x) {
        const int slot = a.retire_list[w / A.NL];
        const int j = (int)(w % A.NL);
        const double nu = A.nu[j];
        const AR hnu_k = static_cast<AR>(kH * nu / kKB);
        const AR two_hnu3 = static_cast<AR>(2.0 * kH * nu * nu * nu / (kC * kC));
        const AR lamfac = static_cast<AR>(A.lam[j] / kBgLambdaRef);
        EmTrans<AR> et;
        et.na = A.jact_off[j + 1] - A.jact_off[j];
#pragma unroll
        for (int q = 0; q < kMaxSlots; q++) {
            if (q < et.na) {
                const int i = A.jact_off[j] + q;
                const int t = A.jact_t[i];
                const DevTransition &tr = A.tr[t];
                et.kind[q] = tr.kind;
                et.l[q] = tr.l;
                et.u[q] = tr.u;
                et.pcol[q] = -1;
                if (tr.kind == 0) {
                    et.col[q] = tr.ray_off + 2 * A.n_mu * tr.n_act + A.jact_ja[i];
                    if (a.prd && tr.prd) et.pcol[q] = tr.psi_off + 2 * A.n_mu * tr.n_act + A.jact_ja[i];
                    const double c0 = tr.hnu4pi;
                    et.cblu[q] = static_cast<AR>(c0 * tr.Blu);
                    et.cbul[q] = static_cast<AR>(c0 * tr.Bul);
                    et.ca[q] = static_cast<AR>(c0 * tr.A);
                } else {
                    et.col[q] = t - A.n_lines;
                    const double r = tr.nu0 / nu;
                    et.alpha[q] = static_cast<AR>(tr.alpha0 * r * r * r);
                }
            }
        }
        const ColGeom cg = geom(a, slot);
        if (a.status[cg.col] == RH15D_BAD_INPUT) {
            a.spectrum[(size_t)cg.col * A.NL + j] = NAN;
            continue;
        }
        const int N = cg.N;
        const int64_t g0 = cg.g0, gc0 = cg.gc0;
        // scaling exponent: h nu / k T at the column's hottest point (FP32 only)
        AR x0 = AR(0);
        if (sizeof(AR) == 4) {
            AR itmin = static_cast<AR>(rec[gc0 * rec_w + 1]);
            for (int k = 1; k < N; k++) itmin = fmin(itmin, static_cast<AR>(rec[(gc0 + k) * rec_w + 1]));
            x0 = fmin(hnu_k * itmin, AR(60));
        }
        const AR scale = sizeof(AR) == 8 ? AR(1) : d_exp(x0);
        EmIn<AR> in;
        AR chi2, S2, B2, chi, S, B;
        em_load<TB, AR>(rec, phi, pops, rec_w, ray_cols, L, et, g0 + N - 2, gc0 + N - 2, gc0 + N - 2, in, psi, psi_cols);
        em_point<AR>(in, et, hnu_k, two_hnu3, lamfac, x0, scale, chi2, S2, B2);
        em_load<TB, AR>(rec, phi, pops, rec_w, ray_cols, L, et, g0 + N - 1, gc0 + N - 1, gc0 + N - 1, in, psi, psi_cols);
        em_point<AR>(in, et, hnu_k, two_hnu3, lamfac, x0, scale, chi, S, B);
        const AR dtv = AR(0.5) * (chi + chi2) * in.dz;
        AR I = dtv > AR(0) ? B + (B - B2) / dtv : B;
        AR chi_p = chi, S_p = S;
        // upward from k = N - 2 to the top; the step from k + 1 uses the
        // spacing stored with point k + 1
        EmIn<AR> nxt;
        em_load<TB, AR>(rec, phi, pops, rec_w, ray_cols, L, et, g0 + N - 2, gc0 + N - 2, gc0 + N - 1, nxt, psi, psi_cols);
        for (int k = N - 2; k >= 0; k--) {
            const EmIn<AR> cur = nxt;
            // issued on every step (the last one reloads the top point), so
            // the wait for this point's values leaves it in flight
            const int kn = k > 0 ? k - 1 : 0;
            em_load<TB, AR>(rec, phi, pops, rec_w, ray_cols, L, et, g0 + kn, gc0 + kn, gc0 + kn + 1, nxt, psi, psi_cols);
            em_point<AR>(cur, et, hnu_k, two_hnu3, lamfac, x0, scale, chi, S, B);
            const AR x = AR(0.5) * (chi_p + chi) * cur.dz;
            AR e, wa, wb;
            sc_weights<AR>(x, e, wa, wb);
            I = I * e + wa * S_p + wb * S;
            chi_p = chi; S_p = S;
        }
        a.spectrum[(size_t)cg.col * A.NL + j] = static_cast<double>(I) * exp(-static_cast<double>(x0));
    }
}

// ---------------------------------------------------------------------------
// polarised emergent spectrum (Zeeman effect), FP64
// ---------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ cplx_t<F> cdiv(cplx_t<F> a, cplx_t<F> b) {
    const F d = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}

// Faddeeva function w(v + i a) = H + i L by the same four-region W4
// approximation as voigt_w4, keeping the imaginary part (the dispersion
// function L, odd in v), in FP64.
__device__ __noinline__ cplx_t<double> faddeeva_w4(double a, double v) {
    using C = cplx_t<double>;
    const C t = {a, -v};
    const double s = fabs(v) + a;
    if (s >= 15.0) return cdiv(C{0.5641896 * t.r, 0.5641896 * t.i}, cadd(cmul(t, t), 0.5));
    if (s >= 5.5) {
        const C u = cmul(t, t);
        const C num = cmul(t, cadd(C{0.5641896 * u.r, 0.5641896 * u.i}, 1.410474));
        const C den = cadd(cmul(u, cadd(u, 3.0)), 0.75);
        return cdiv(num, den);
    }
    if (a >= 0.195 * fabs(v) - 0.176) {
        C num = {0.5642236, 0.0};
        num = cadd(cmul(num, t), 3.778987);
        num = cadd(cmul(num, t), 11.96482);
        num = cadd(cmul(num, t), 20.20933);
        num = cadd(cmul(num, t), 16.4955);
        C den = {1.0, 0.0};
        den = cadd(cmul(den, t), 6.699398);
        den = cadd(cmul(den, t), 21.69274);
        den = cadd(cmul(den, t), 39.27121);
        den = cadd(cmul(den, t), 38.82363);
        den = cadd(cmul(den, t), 16.4955);
        return cdiv(num, den);
    }
    const C u = cmul(t, t);
    C p = {0.56419, 0.0};
    p = cadd(cmul(p, u), -1.320522);
    p = cadd(cmul(p, u), 35.76683);
    p = cadd(cmul(p, u), -219.0313);
    p = cadd(cmul(p, u), 1540.787);
    p = cadd(cmul(p, u), -3321.9905);
    p = cadd(cmul(p, u), 36183.31);
    C q = {-1.0, 0.0};
    q = cadd(cmul(q, u), 1.841439);
    q = cadd(cmul(q, u), -61.57037);
    q = cadd(cmul(q, u), 364.2191);
    q = cadd(cmul(q, u), -2186.181);
    q = cadd(cmul(q, u), 9022.228);
    q = cadd(cmul(q, u), -24322.84);
    q = cadd(cmul(q, u), 32066.6);
    const C f = cdiv(cmul(t, p), q);
    const double eu = exp(u.r);
    return {eu * cos(u.i) - f.r, eu * sin(u.i) - f.i};
}

// Absorption-matrix entries, emission vector and Planck function of one
// depth point at one wavelength.
struct StkPoint {
    double chi;       // eta_I, total opacity
    double k[6];      // eta_Q, eta_U, eta_V, rho_Q, rho_U, rho_V
    double e[4];      // emission vector
    double B;
};

// The transitions active at a lane's wavelength (up to kMaxSlots).
struct StkTrans {
    int na;
    int t[kMaxSlots];
    int rho_i[kMaxSlots];   // PRD line: index of this wavelength in the depth row of rho, else -1
};

__device__ void stokes_point(const RunArgs &a, const StkTrans &st, int64_t g, int64_t gc, int j, double nu,
                             double lamfac, double hnu_k, double two_hnu3, double Bk, double ik, double ak,
                             StkPoint &p) {
    const DevAtom &A = a.A;
    const int L = A.L;
    const double T = a.T[g];
    const double x = hnu_k / T;
    p.B = two_hnu3 / expm1(x);
    double chi = a.kbg[gc] * lamfac;
    for (int i = 0; i < 6; i++) p.k[i] = 0.0;
    p.e[0] = chi * p.B;
    p.e[1] = p.e[2] = p.e[3] = 0.0;
    const double ct = cos(ik), sn = sin(ik), s2 = sn * sn, c2 = cos(2.0 * ak), sn2 = sin(2.0 * ak);
    const int rw = A.psi_cols / (2 * A.n_mu + 1);
    for (int q = 0; q < st.na; q++) {
        const DevTransition &tr = A.tr[st.t[q]];
        const double nl = a.pops[g * L + tr.l], nup = a.pops[g * L + tr.u];
        if (tr.kind != 0) {
            const double r = tr.nu0 / nu;
            const double alpha = tr.alpha0 * r * r * r;
            const double G = a.gr[gc * A.n_cont + (st.t[q] - A.n_lines)] * exp(-x);
            chi += (nl - nup * G) * alpha;
            p.e[0] += nup * two_hnu3 * G * alpha;
            continue;
        }
        const double rho = st.rho_i[q] >= 0 ? a.rho[gc * rw + st.rho_i[q]] : 1.0;
        const double cc = tr.hnu4pi / a.norm[gc * A.n_lines + st.t[q]];
        const double cabs = cc * (nl * tr.Blu - nup * tr.Bul * rho);
        const double cem = cc * nup * tr.A * rho;
        const double dnd = tr.nu0 / kC * sqrt(2.0 * kKB * T / A.mass + a.vt[g] * a.vt[g]);
        const double ad = (tr.gamma + tr.c_el * a.nH[g]) / (4.0 * kPI * dnd);
        const double v = (nu - tr.nu0 * (1.0 + a.vz[g] / kC)) / dnd;
        const double pre = 1.0 / (sqrt(kPI) * dnd);
        if (tr.n_zc == 0) {
            const double H = tr.voigt ? faddeeva_w4(ad, v).r : exp(-v * v);
            chi += cabs * H * pre;
            p.e[0] += cem * H * pre;
            continue;
        }
        const double vL = kQE * Bk / (4.0 * kPI * kME) / dnd;
        double ph[3] = {0.0, 0.0, 0.0}, ps[3] = {0.0, 0.0, 0.0};
        for (int c = tr.zc_off; c < tr.zc_off + tr.n_zc; c++) {
            const double vc = v - A.zshift[c] * vL;
            const cplx_t<double> w = faddeeva_w4(tr.voigt ? ad : 0.0, vc);
            const double H = tr.voigt ? w.r : exp(-vc * vc);
            const int iq = A.zq[c] + 1;
            ph[iq] += A.zstr[c] * H;
            ps[iq] += A.zstr[c] * w.i;
        }
        for (int i = 0; i < 3; i++) { ph[i] *= pre; ps[i] *= pre; }
        // index 2: q = +1, index 0: q = -1
        const double pI = 0.5 * (ph[1] * s2 + 0.5 * (ph[2] + ph[0]) * (1.0 + ct * ct));
        const double pl = 0.5 * (ph[1] - 0.5 * (ph[2] + ph[0])) * s2;
        const double pV = 0.5 * (ph[2] - ph[0]) * ct;
        const double rl = 0.5 * (ps[1] - 0.5 * (ps[2] + ps[0])) * s2;
        const double rV = 0.5 * (ps[2] - ps[0]) * ct;
        chi += cabs * pI;
        p.k[0] += cabs * pl * c2; p.k[1] += cabs * pl * sn2; p.k[2] += cabs * pV;
        p.k[3] += cabs * rl * c2; p.k[4] += cabs * rl * sn2; p.k[5] += cabs * rV;
        p.e[0] += cem * pI; p.e[1] += cem * pl * c2; p.e[2] += cem * pl * sn2; p.e[3] += cem * pV;
    }
    p.chi = chi;
}

// One DELO step (linear effective source function) from the deeper point d
// to the point c, optical step x: solves
//   (1 + wb K'_c) I_c = (e - wa K'_d) I_d + wa S'_d + wb S'_c,
// K' = K / chi - 1, S' = eps / chi, in closed form: with the Q, U, V parts
// e = wb (eta_Q, eta_U, eta_V) / chi and r = wb (rho_Q, rho_U, rho_V) / chi,
// the system is x0 + e.x = y0, e x0 + x + x * r = y (x * r the cross
// product), and (I + [. * r])^-1 b = (b - b * r + (b.r) r) / (1 + r.r)
// with a Sherman-Morrison correction for the e e^T term.
__device__ __forceinline__ void delo_step(const StkPoint &d, const StkPoint &c, double x, double I[4]) {
    double e, wa, wb;
    sc_weights<double>(x, e, wa, wb);
    const double id = 1.0 / d.chi, ic = 1.0 / c.chi;
    const double dQ = d.k[0] * id, dU = d.k[1] * id, dV = d.k[2] * id;
    const double dq = d.k[3] * id, du = d.k[4] * id, dv = d.k[5] * id;
    // K'_d I
    const double k0 = dQ * I[1] + dU * I[2] + dV * I[3];
    const double k1 = dQ * I[0] + dv * I[2] - du * I[3];
    const double k2 = dU * I[0] - dv * I[1] + dq * I[3];
    const double k3 = dV * I[0] + du * I[1] - dq * I[2];
    const double y0 = e * I[0] - wa * k0 + wa * d.e[0] * id + wb * c.e[0] * ic;
    const double y1 = e * I[1] - wa * k1 + wa * d.e[1] * id + wb * c.e[1] * ic;
    const double y2 = e * I[2] - wa * k2 + wa * d.e[2] * id + wb * c.e[2] * ic;
    const double y3 = e * I[3] - wa * k3 + wa * d.e[3] * id + wb * c.e[3] * ic;
    const double wc = wb * ic;
    const double e1 = c.k[0] * wc, e2 = c.k[1] * wc, e3 = c.k[2] * wc;
    const double r1 = c.k[3] * wc, r2 = c.k[4] * wc, r3 = c.k[5] * wc;
    const double b1 = y1 - e1 * y0, b2 = y2 - e2 * y0, b3 = y3 - e3 * y0;
    const double rr = 1.0 / (1.0 + r1 * r1 + r2 * r2 + r3 * r3);
    // A^-1 v = (v - v * r + (v.r) r) / (1 + r.r)
    const double br = b1 * r1 + b2 * r2 + b3 * r3;
    const double ab1 = (b1 - (b2 * r3 - b3 * r2) + br * r1) * rr;
    const double ab2 = (b2 - (b3 * r1 - b1 * r3) + br * r2) * rr;
    const double ab3 = (b3 - (b1 * r2 - b2 * r1) + br * r3) * rr;
    const double er = e1 * r1 + e2 * r2 + e3 * r3;
    const double ae1 = (e1 - (e2 * r3 - e3 * r2) + er * r1) * rr;
    const double ae2 = (e2 - (e3 * r1 - e1 * r3) + er * r2) * rr;
    const double ae3 = (e3 - (e1 * r2 - e2 * r1) + er * r3) * rr;
    const double f = (e1 * ab1 + e2 * ab2 + e3 * ab3) / (1.0 - (e1 * ae1 + e2 * ae2 + e3 * ae3));
    I[1] = ab1 + ae1 * f;
    I[2] = ab2 + ae2 * f;
    I[3] = ab3 + ae3 * f;
    I[0] = y0 - (e1 * I[1] + e2 * I[2] + e3 * I[3]);
}

// One lane per (retired column, wavelength): the vertical upward Stokes
// vector through the column's depth points.
__global__ __launch_bounds__(256) void k_stokes(RunArgs a) {
    const DevAtom &A = a.A;
    const int64_t n = (int64_t)a.ctr[CTR_RETIRE] * A.NL;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n; w += (int64_t)gridDim.x * blockDim.x) {
        const int slot = a.retire_list[w / A.NL];
        const int j = (int)(w % A.NL);
        const ColGeom cg = geom(a, slot);
        double *out = a.stokes + ((size_t)cg.col * A.NL + j) * 4;
        if (a.status[cg.col] == RH15D_BAD_INPUT) {
            out[0] = out[1] = out[2] = out[3] = NAN;
            continue;
        }
        const double nu = A.nu[j];
        const double lamfac = A.lam[j] / kBgLambdaRef;
        const double hnu_k = kH * nu / kKB;
        const double two_hnu3 = 2.0 * kH * nu * nu * nu / (kC * kC);
        StkTrans st;
        st.na = A.jact_off[j + 1] - A.jact_off[j];
        for (int q = 0; q < kMaxSlots; q++) {
            st.t[q] = 0;
            st.rho_i[q] = -1;
            if (q >= st.na) continue;
            const int i = A.jact_off[j] + q;
            const int t = A.jact_t[i];
            st.t[q] = t;
            if (a.prd && A.tr[t].prd) {
                int off = 0;
                for (int ip = 0; ip < A.n_prd && A.prd_t[ip] != t; ip++) off += A.tr[A.prd_t[ip]].n_act;
                st.rho_i[q] = off + A.jact_ja[i];
            }
        }
        const int N = cg.N;
        const int64_t g0 = cg.g0, gc0 = cg.gc0;
        bool ok = true;
        auto field = [&](int k, double &Bk, double &ik, double &ak) {
            if (a.Bf) {
                Bk = a.Bf[g0 + k]; ik = a.Bincl[g0 + k]; ak = a.Bazim[g0 + k];
                if (!isfinite(Bk + ik + ak)) { ok = false; Bk = ik = ak = 0.0; }
            } else {
                Bk = ik = ak = 0.0;
            }
        };
        StkPoint pd, pc;
        double Bk, ik, ak;
        field(N - 1, Bk, ik, ak);
        stokes_point(a, st, g0 + N - 1, gc0 + N - 1, j, nu, lamfac, hnu_k, two_hnu3, Bk, ik, ak, pd);
        field(N - 2, Bk, ik, ak);
        stokes_point(a, st, g0 + N - 2, gc0 + N - 2, j, nu, lamfac, hnu_k, two_hnu3, Bk, ik, ak, pc);
        const double dtv = 0.5 * (pd.chi + pc.chi) * (a.z[g0 + N - 2] - a.z[g0 + N - 1]);
        double I[4] = {dtv > 0.0 ? pd.B + (pd.B - pc.B) / dtv : pd.B, 0.0, 0.0, 0.0};
        for (int k = N - 2; k >= 0; k--) {
            if (k < N - 2) {
                field(k, Bk, ik, ak);
                stokes_point(a, st, g0 + k, gc0 + k, j, nu, lamfac, hnu_k, two_hnu3, Bk, ik, ak, pc);
            }
            const double x = 0.5 * (pd.chi + pc.chi) * (a.z[g0 + k] - a.z[g0 + k + 1]);
            delo_step(pd, pc, x, I);
            pd = pc;
        }
        for (int i = 0; i < 4; i++) out[i] = ok ? I[i] : NAN;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_psi_gather(RunArgs a) {
    const DevAtom &A = a.A;
    const int64_t n = (int64_t)a.ctr[CTR_RETIRE] * a.ND * A.T;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n; w += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(w % A.T);
        const int64_t sk = w / A.T;
        const int slot = a.retire_list[sk / a.ND], k = (int)(sk % a.ND);
        const ColGeom cg = geom(a, slot);
        if (k >= cg.N) continue;
        const R *part = reinterpret_cast<const R *>(a.part) + cg.gc0 * A.n_keys;
        double s = 0.0;
        for (int i = A.p_off[t]; i < A.p_off[t + 1]; i++) s += static_cast<double>(part[(size_t)A.p_key[i] * cg.N + k]);
        a.psi[(cg.g0 + k) * A.T + t] = a.status[cg.col] == RH15D_BAD_INPUT ? NAN : s;
    }
}

// Finished columns leave their slots; free slots take the next columns of
// the queue (in slot order, so a run is reproducible).  The plain scheduler
// waits until every slot is free.
constexpr int kRefillThreads = 1024;

__global__ __launch_bounds__(kRefillThreads) void k_refill(RunArgs a) {
    __shared__ int sh[kRefillThreads];
    __shared__ int busy;
    const int t = threadIdx.x;
    const int nret = a.ctr[CTR_RETIRE];
    for (int i = t; i < nret; i += kRefillThreads) a.slot_state[a.retire_list[i]] = SLOT_FREE;
    if (t == 0) busy = 0;
    __syncthreads();
    const int per = (a.S + kRefillThreads - 1) / kRefillThreads;
    const int s0 = t * per, s1 = min(a.S, s0 + per);
    int nfree = 0;
    for (int s = s0; s < s1; s++) {
        if (a.slot_state[s] == SLOT_FREE) nfree++;
        else atomicOr(&busy, 1);
    }
    sh[t] = nfree;
    __syncthreads();
    for (int o = 1; o < kRefillThreads; o <<= 1) {  // inclusive scan
        const int v = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    const int next = a.ctr[CTR_NEXT];
    const int total_free = sh[kRefillThreads - 1];
    int avail = (int)min<int64_t>((int64_t)total_free, a.n_columns - next);
    if (a.chunked && busy) avail = 0;
    int rank = sh[t] - nfree;
    for (int s = s0; s < s1; s++) {
        if (a.slot_state[s] != SLOT_FREE) continue;
        if (rank < avail) {
            a.slot_col[s] = next + rank;
            a.slot_state[s] = SLOT_PENDING;
            a.refill_list[rank] = s;
        }
        rank++;
    }
    __syncthreads();
    if (t == 0) {
        a.ctr[CTR_EMITTED] += nret;
        a.ctr[CTR_RETIRE] = 0;
        a.ctr[CTR_REFILL] = avail;
        a.ctr[CTR_NEXT] = next + avail;
    }
}

__global__ void k_init_slots(RunArgs a) {
    const int n = a.ctr[CTR_REFILL];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int slot = a.refill_list[i];
        const int c = a.slot_col[slot];
        a.slot_it[slot] = 0;
        a.ng_count[slot] = 0;
        a.ng_head[slot] = 0;
        a.slot_dprev[slot] = -1.0;
        a.status[c] = RH15D_MAX_ITER;
        a.n_iter[c] = 0;
        if (a.history)
            for (int k = 0; k < a.max_iter; k++) a.history[(size_t)c * a.max_iter + k] = NAN;
        if (a.slot_bad[slot]) {
            // unusable column data: no iteration, NaN populations (the
            // emergent-spectrum and Psi* outputs of the column are NaN too)
            a.slot_bad[slot] = 0;
            a.status[c] = RH15D_BAD_INPUT;
            const int64_t g0 = a.doff[c], g1 = a.doff[c + 1];
            for (int64_t g = g0; g < g1; g++)
                for (int l = 0; l < a.A.L; l++) a.pops[g * a.A.L + l] = NAN;
            a.slot_state[slot] = SLOT_DONE;
            a.retire_list[atomicAdd(&a.ctr[CTR_RETIRE], 1)] = slot;
        } else if (a.max_iter == 0) {
            a.slot_state[slot] = SLOT_DONE;
            a.retire_list[atomicAdd(&a.ctr[CTR_RETIRE], 1)] = slot;
        } else {
            a.slot_state[slot] = SLOT_ACTIVE;
        }
    }
}

__global__ void k_setup(RunArgs a) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < a.S; s += gridDim.x * blockDim.x) {
        a.slot_state[s] = SLOT_FREE;
        a.slot_col[s] = 0;
        a.slot_bad[s] = 0;
        a.slot_dprev[s] = -1.0;
    }
    if (blockIdx.x == 0 && threadIdx.x < CTR_COUNT) a.ctr[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// departure coefficients (learned start solution)
// ---------------------------------------------------------------------------
// ln of the Saha-Boltzmann populations of one point (sum = n_total).
__device__ __forceinline__ void lte_log_pops(const DevAtom &A, double T, double ne, double nH, double *lnstar) {
    const int L = A.L;
    const double kT = kKB * T;
    const double saha = log(2.0 / ne) + 1.5 * log(2.0 * kPI * kME * kT / (kH * kH));
    double mx = -1e300;
    for (int i = 0; i < L; i++) {
        lnstar[i] = log(A.g[i] / A.g[0]) - (A.E[i] - A.E[0]) / kT + (A.stage[i] - A.stage[0]) * saha;
        mx = fmax(mx, lnstar[i]);
    }
    double sum = 0.0;
    for (int i = 0; i < L; i++) sum += exp(lnstar[i] - mx);
    const double lnorm = log(A.abund * nH) - mx - log(sum);
    for (int i = 0; i < L; i++) lnstar[i] += lnorm;
}

// log_b[g][i] = ln(n_i / n*_i)
__global__ void k_departures(DevAtom A, int64_t n, const double *T, const double *ne, const double *nH,
                             const double *pops, float *log_b) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        double ls[RH15D_MAX_LEVELS];
        lte_log_pops(A, T[g], ne[g], nH[g], ls);
        for (int i = 0; i < A.L; i++) log_b[g * A.L + i] = (float)(log(pops[g * A.L + i]) - ls[i]);
    }
}

// n_i = b_i n*_i, renormalised to the total population of the point, with
// ln b_i first shrunk toward 0 (LTE) by `shrink`: predictions smaller than
// the network's error level are better replaced by the LTE value.
constexpr double kMaxLogB = 50.0;
__global__ void k_pops_from_departures(DevAtom A, int64_t n, const double *T, const double *ne, const double *nH,
                                       const float *log_b, double shrink, double *pops) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        double ls[RH15D_MAX_LEVELS];
        lte_log_pops(A, T[g], ne[g], nH[g], ls);
        double mx = -1e300;
        for (int i = 0; i < A.L; i++) {
            // a non-finite prediction falls back to LTE; others are clamped to |ln b| <= 50
            const float lb = log_b[g * A.L + i];
            const double v = isfinite(lb) ? fmin(fmax((double)lb, -kMaxLogB), kMaxLogB) : 0.0;
            ls[i] += copysign(fmax(fabs(v) - shrink, 0.0), v);
            mx = fmax(mx, ls[i]);
        }
        double sum = 0.0;
        for (int i = 0; i < A.L; i++) sum += exp(ls[i] - mx);
        const double ntot = A.abund * nH[g];
        for (int i = 0; i < A.L; i++) pops[g * A.L + i] = ntot * exp(ls[i] - mx) / sum;
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
thread_local rh15d_stats g_stats;

// HIP events bracketing the library's launches on the caller's stream
struct Timer {
    bool on = false;
    hipEvent_t ev[8] = {};
    int init(bool enable) {
        on = enable;
        if (!on) return RH15D_OK;
        for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
        return RH15D_OK;
    }
    void mark(int i, hipStream_t st) { if (on) (void)hipEventRecord(ev[i], st); }
    double ms(int a, int b) {
        float t = 0.f;
        if (on) (void)hipEventElapsedTime(&t, ev[a], ev[b]);
        return t;
    }
    ~Timer() { if (on) for (auto &e : ev) (void)hipEventDestroy(e); }
};

template <typename T>
int upload(rh15d_atom *atom, const std::vector<T> &v, T **out) {
    *out = nullptr;
    if (v.empty()) return RH15D_OK;
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, v.size() * sizeof(T)));
    atom->dev_allocs.push_back(p);
    HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    *out = static_cast<T *>(p);
    return RH15D_OK;
}

// The atom's device tables for (device, n_mu, shape), built and uploaded on
// first use; with build = false an absent entry is an error instead (the
// caller may not allocate).
int get_dev_atom(rh15d_atom *atom, int n_mu, SweepShape shape, DevAtom **out, bool build = true) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (shape.mc != 1 && shape.mc != 3 && shape.mc != 5) { set_error("angles per lane must be 1, 3 or 5"); return RH15D_EINVAL; }
    if (n_mu % shape.mc != 0) { set_error("angles per lane must divide n_mu"); return RH15D_EINVAL; }
    std::lock_guard<std::mutex> lock(atom->mu_);
    auto key = std::make_pair(std::make_pair(dev, n_mu), shape);
    auto it = atom->dev.find(key);
    if (it != atom->dev.end()) { *out = &it->second; return RH15D_OK; }
    if (!build) {
        set_error("the atom has no device tables for this device, n_mu and sweep shape yet (run rh15d_solve_columns "
                  "once with the same options first)");
        return RH15D_EINVAL;
    }
    HostGroupTables H;
    build_group_tables(*atom, n_mu, shape, H);
    if (H.overflow) { set_error("a wavelength has more than %d active transitions", kMaxSlots); return RH15D_EINVAL; }
    // order the groups by slot count (stable), permuting the lane tables alike
    const int NG = static_cast<int>(H.groups.size());
    std::vector<int> order(NG);
    for (int i = 0; i < NG; i++) order[i] = i;
    auto cls = [&](int x) { return group_class(H.groups[x].n_slots, H.groups[x].n_slots - H.groups[x].n_line_slots); };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cls(x) < cls(y); });
    auto permute = [&](auto &v, int per_group) {
        auto w = v;
        for (int i = 0; i < NG; i++)
            std::copy(v.begin() + (size_t)order[i] * per_group, v.begin() + (size_t)(order[i] + 1) * per_group,
                      w.begin() + (size_t)i * per_group);
        v.swap(w);
    };
    permute(H.groups, 1);
    permute(H.lane_j, kWave); permute(H.lane_m0, kWave); permute(H.lane_lamfac, kWave);
    permute(H.lane_hnu_k, kWave); permute(H.lane_2hnu3c2, kWave);
    permute(H.pbase, kWave * kMaxSlots); permute(H.wj, kWave * kMaxSlots); permute(H.psb, kWave * kMaxSlots);
    permute(H.lane_ist, kWave);
    permute(H.kapj, kWave * kMaxSlots); permute(H.alpha, kWave * kMaxSlots);
    DevAtom D{};
    D.L = atom->L; D.n_lines = atom->n_lines; D.n_cont = atom->n_cont;
    D.T = static_cast<int>(atom->tr.size()); D.NL = static_cast<int>(atom->lam.size()); D.n_mu = n_mu;
    D.n_groups = NG; D.n_keys = H.n_keys; D.ray_cols = H.ray_cols;
    D.mc = shape.mc; D.pack = shape.pack;
    for (int id = 0; id <= kGroupClasses; id++) {
        int c = 0;
        while (c < NG && group_class(H.groups[c].n_slots, H.groups[c].n_slots - H.groups[c].n_line_slots) < id) c++;
        D.g_begin[id] = c;
    }
    D.mass = atom->mass; D.abund = atom->abund; D.c_bg = atom->c_bg; D.bg_kind = atom->bg_kind;
    std::vector<DevTransition> tr(D.T);
    std::vector<int> prd_t;
    D.psi_cols = H.psi_cols;
    D.ist_cols = H.ist_cols;
    D.g_cols = 0;
    std::vector<int> act_j;
    std::vector<double> act_w;
    std::vector<int> zq;
    std::vector<double> zshift, zstr;
    int ray_off = 0;
    for (int t = 0; t < D.T; t++) {
        const auto &h = atom->tr[t];
        DevTransition d{};
        d.kind = h.kind; d.l = h.l; d.u = h.u; d.voigt = h.voigt; d.coll_kind = h.coll_kind;
        d.n_act = static_cast<int>(h.act.size()); d.act_off = static_cast<int>(act_j.size());
        d.ray_off = h.kind == 0 ? ray_off : -1;
        // quadrature rays (2 directions x n_mu angles x n_act wavelengths),
        // then the vertical emergent ray (mu = 1, upward) at each wavelength
        if (h.kind == 0) ray_off += (2 * n_mu + 1) * d.n_act;
        d.nu0 = h.nu0; d.A = h.A; d.Bul = h.Bul; d.Blu = h.Blu; d.alpha0 = h.alpha0; d.coll_val = h.coll_val;
        d.gamma = h.gamma; d.hnu4pi = kH * h.nu0 / (4.0 * kPI);
        d.c_el = h.c_el;
        d.n_zc = static_cast<int>(h.zq.size());
        d.zc_off = static_cast<int>(zq.size());
        zq.insert(zq.end(), h.zq.begin(), h.zq.end());
        zshift.insert(zshift.end(), h.zshift.begin(), h.zshift.end());
        zstr.insert(zstr.end(), h.zstr.begin(), h.zstr.end());
        d.prd = h.kind == 0 && h.prd;
        d.psi_off = H.psi_off[t];
        d.g_off = -1;
        if (d.prd) {
            d.g_off = D.g_cols;
            D.g_cols += d.n_act * d.n_act;
            prd_t.push_back(t);
        }
        d.wsum = 0.0;
        for (double w : h.w) d.wsum += w;
        act_j.insert(act_j.end(), h.act.begin(), h.act.end());
        act_w.insert(act_w.end(), h.w.begin(), h.w.end());
        tr[t] = d;
    }
    if (ray_off != H.ray_cols) { set_error("internal: ray table mismatch"); return RH15D_EINVAL; }
    D.n_prd = static_cast<int>(prd_t.size());
    for (const auto &d : tr)
        if (d.prd && d.n_act > kMaxPrdFreq) {
            set_error("a PRD line has %d wavelengths (limit %d)", d.n_act, kMaxPrdFreq);
            return RH15D_EINVAL;
        }
    for (const auto &d : tr)
        if (d.kind == 0 && (2 * n_mu + 1) * d.n_act > kMaxLineRays) {
            set_error("a line has %d rays per depth (limit %d)", (2 * n_mu + 1) * d.n_act, kMaxLineRays);
            return RH15D_EINVAL;
        }
    int rc = RH15D_OK;
    std::vector<double> E(atom->E), g(atom->g);
    std::vector<int> st(atom->stage);
#define UP(vec, dst) do { if ((rc = upload(atom, vec, dst)) != RH15D_OK) return rc; } while (0)
    UP(E, &D.E); UP(g, &D.g); UP(st, &D.stage); UP(tr, &D.tr);
    UP(zq, &D.zq); UP(zshift, &D.zshift); UP(zstr, &D.zstr);
    std::vector<double> lam(atom->lam), nu(atom->nu);
    UP(lam, &D.lam); UP(nu, &D.nu); UP(act_j, &D.act_j); UP(act_w, &D.act_w);
    UP(H.mu, &D.mu); UP(H.wmu, &D.wmu);
    std::vector<int> jo(atom->jact_off), jt(atom->jact_t), jja(atom->jact_t.size());
    for (int j = 0; j < D.NL; j++)
        for (int i = jo[j]; i < jo[j + 1]; i++) {
            const auto &act = atom->tr[jt[i]].act;
            jja[i] = static_cast<int>(std::lower_bound(act.begin(), act.end(), j) - act.begin());
        }
    UP(jo, &D.jact_off); UP(jt, &D.jact_t); UP(jja, &D.jact_ja);
    // per line ray: frequency, signed direction cosine (+ up), quadrature
    // weight W = w_nu w_mu / 2 (0 for the vertical emergent rays, which are
    // not in the normalisation) and the ray's place in the profile table.
    // The preparation visits the rays in order of distance from the line
    // centre, so the lanes of a wavefront mostly fall in the same region of
    // the Voigt approximation.
    {
        std::vector<double> pnu, pmus, pw;
        std::vector<float> pdnu, pmusf;
        std::vector<int> poff(1, 0), pdst;
        for (int t = 0; t < D.n_lines; t++) {
            const auto &h = atom->tr[t];
            const int na = static_cast<int>(h.act.size()), nq = 2 * na * n_mu;
            const size_t first = pnu.size();
            for (int r = 0; r < nq + na; r++) {
                int ja, m = 0;
                double mus, w = 0.0;
                if (r < nq) {
                    const int sd = r / (na * n_mu), rem = r % (na * n_mu);
                    ja = rem / n_mu;
                    m = rem % n_mu;
                    mus = sd ? H.mu[m] : -H.mu[m];
                    w = h.w[ja] * 0.5 * H.wmu[m];
                } else {
                    ja = r - nq;
                    mus = 1.0;
                }
                pnu.push_back(atom->nu[h.act[ja]]);
                pmus.push_back(mus);
                pw.push_back(w);
                pdst.push_back(r);
            }
            std::vector<int> ord(nq + na);
            for (int r = 0; r < nq + na; r++) ord[r] = r;
            std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
                return std::fabs(pnu[first + x] - h.nu0) < std::fabs(pnu[first + y] - h.nu0);
            });
            auto permute = [&](auto &v) {
                std::vector<typename std::decay_t<decltype(v)>::value_type> w(v.begin() + first, v.end());
                for (int r = 0; r < nq + na; r++) v[first + r] = w[ord[r]];
            };
            permute(pnu); permute(pmus); permute(pw); permute(pdst);
            for (size_t r = first; r < pnu.size(); r++) {
                pdnu.push_back(static_cast<float>(pnu[r] - h.nu0));
                pmusf.push_back(static_cast<float>(pmus[r]));
            }
            poff.push_back(static_cast<int>(pnu.size()));
        }
        if (pnu.empty()) {
            pnu.push_back(0.0); pmus.push_back(0.0); pw.push_back(0.0); pdst.push_back(0);
            pdnu.push_back(0.0f); pmusf.push_back(0.0f);
        }
        UP(pnu, &D.prof_nu); UP(pmus, &D.prof_mus); UP(pw, &D.prof_w); UP(poff, &D.prof_off);
        UP(pdst, &D.prof_dst); UP(pdnu, &D.prof_dnu); UP(pmusf, &D.prof_musf);
    }
    UP(H.groups, &D.groups);
    UP(H.lane_j, &D.lanes.j); UP(H.lane_m0, &D.lanes.m0);
    UP(H.lane_lamfac, &D.lanes.lamfac); UP(H.lane_hnu_k, &D.lanes.hnu_k); UP(H.lane_2hnu3c2, &D.lanes.two_hnu3c2);
    UP(H.pbase, &D.lanes.pbase); UP(H.wj, &D.lanes.wj); UP(H.kapj, &D.lanes.kapj); UP(H.alpha, &D.lanes.alpha);
    UP(H.psb, &D.lanes.psb); UP(H.lane_ist, &D.lanes.ist);
    {
        std::vector<int> pt(prd_t), si(H.st_idx);
        if (pt.empty()) pt.push_back(-1);
        UP(pt, &D.prd_t); UP(si, &D.st_idx);
    }
    UP(H.p_off, &D.p_off); UP(H.p_key, &D.p_key); UP(H.q_off, &D.q_off); UP(H.q_key, &D.q_key);
    D.n_xpairs = static_cast<int>(H.x_t.size());
    UP(H.x_t, &D.x_t); UP(H.x_t2, &D.x_t2); UP(H.x_off, &D.x_off); UP(H.x_key, &D.x_key);
    {
        const int L = D.L;
        std::vector<int> up(L * L, -1), dn(L * L, -1);
        for (int t = 0; t < D.T; t++) {
            const int l = atom->tr[t].l, u = atom->tr[t].u;
            if (up[u * L + l] >= 0 || dn[l * L + u] >= 0) {
                set_error("two transitions connect levels %d and %d", l, u);
                return RH15D_EINVAL;
            }
            up[u * L + l] = t;   // l -> u (excitation / ionisation)
            dn[l * L + u] = t;   // u -> l (de-excitation / recombination)
        }
        std::vector<std::vector<int>> xe(L * L);
        for (size_t x = 0; x < H.x_t.size(); x++) {
            const int lt = atom->tr[H.x_t[x]].l, ut = atom->tr[H.x_t[x]].u, u2 = atom->tr[H.x_t2[x]].u;
            xe[ut * L + u2].push_back((int)x + 1);
            xe[lt * L + u2].push_back(-((int)x + 1));
        }
        std::vector<int> xo(L * L + 1, 0), xv;
        for (int e = 0; e < L * L; e++) {
            xv.insert(xv.end(), xe[e].begin(), xe[e].end());
            xo[e + 1] = static_cast<int>(xv.size());
        }
        if (xv.empty()) xv.push_back(0);
        UP(up, &D.up_t); UP(dn, &D.dn_t); UP(xo, &D.xe_off); UP(xv, &D.xe_val);
    }
#undef UP
    for (const auto &G : H.groups) {
        // per ray-step: background and Planck 7, formal step 19, source 1;
        // per transition 9 (opacity) + 8 (rates) + 2 (reductions);
        // per cross pair 3 + 1 (counted for the rays that carry the slot)
        const double rays = (double)G.n_lanes * shape.mc;
        D.rays_per_depth += rays;
        D.flops_per_depth += rays * (27.0 + 19.0 * G.n_slots + 4.0 * G.n_pairs);
        D.reads_per_depth += rays * G.n_line_slots;
        D.keys_per_depth += G.n_keys;
    }
    auto res = atom->dev.emplace(key, D);
    *out = &res.first->second;
    return RH15D_OK;
}

// The sweep shape of a solve: the caller's, else the autotuned one for this
// device, angle count and precision, else one angle per lane with mixed packing
// (the fastest shape measured for the six-level atom on MI355X).
SweepShape pick_shape(rh15d_atom *atom, const rh15d_options *o) {
    SweepShape sh;
    bool any_prd = false;
    for (const auto &t : atom->tr) any_prd |= t.kind == 0 && t.prd;
    if (o->prd && any_prd) {
        // the partial-frequency-redistribution sweep carries one angle per lane
        sh.mc = 1;
        sh.pack = o->sweep_pack > 0 ? o->sweep_pack - 1 : 1;
        return sh;
    }
    sh.mc = o->sweep_mc > 0 ? o->sweep_mc : 1;
    sh.pack = o->sweep_pack > 0 ? o->sweep_pack - 1 : 1;
    if (o->sweep_mc <= 0 && o->sweep_pack <= 0) {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            std::lock_guard<std::mutex> lock(atom->mu_);
            auto it = atom->tuned.find({{dev, o->n_mu}, o->precision});
            if (it != atom->tuned.end()) sh = it->second;
        }
    }
    return sh;
}

struct Layout {
    size_t off_doff, off_lnr, off_kbg, off_gr, off_norm, off_phi, off_part, off_rec, off_popsf, off_rad, off_nse, off_dk,
        off_flag, off_ring, off_slots, off_dprev, off_ctr, off_lists, off_psi, off_ist, off_gtab, off_rho, total;
};
constexpr int kSlotInts = 6;   // per-slot int arrays: column, state, iteration, Ng count, Ng head, bad input

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(const DevAtom &D, int64_t n_columns, int S, int ND, bool fp32, bool ng, bool prd) {
    const size_t R = fp32 ? 4 : 8;
    const size_t P = (size_t)S * ND;
    Layout l{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    l.off_doff = take((n_columns + 1) * 8);
    l.off_lnr = take(P * D.L * 8);
    l.off_kbg = take(P * 8);
    l.off_gr = take(P * std::max(D.n_cont, 1) * 8);
    l.off_norm = take(P * std::max(D.n_lines, 1) * 8);
    l.off_phi = take(P * std::max(D.ray_cols, 1) * R);
    l.off_part = take(P * D.n_keys * R);
    l.off_rec = take(P * rec_width(D.n_cont) * R);
    l.off_popsf = take(fp32 ? P * D.L * 4 : 8);
    l.off_rad = take(P * D.L * D.L * 8);
    l.off_nse = take(P * D.L * 8);
    l.off_dk = take(P * 8);
    l.off_flag = take(P * 4);
    l.off_ring = take(ng ? 4 * P * D.L * 8 : 8);
    l.off_slots = take((size_t)S * kSlotInts * 4);
    l.off_dprev = take((size_t)S * 8);
    l.off_ctr = take(CTR_COUNT * 4);
    l.off_lists = take((size_t)S * 2 * 4);
    // partial frequency redistribution
    l.off_psi = take(prd ? P * D.psi_cols * R : 8);
    l.off_ist = take(prd ? P * D.ist_cols * R : 8);
    l.off_gtab = take(prd ? P * D.g_cols * R : 8);
    l.off_rho = take(prd ? P * (D.psi_cols / (2 * D.n_mu + 1)) * 8 : 8);
    l.total = o;
    return l;
}

int validate(const rh15d_atom *atom, const rh15d_columns *cols, const rh15d_options *o) {
    if (!atom || !cols || !o) { set_error("null argument"); return RH15D_EINVAL; }
    if (cols->n_columns < 0 || (cols->n_columns > 0 && !cols->depth_offset)) { set_error("bad column count or offsets"); return RH15D_EINVAL; }
    if (cols->n_columns > (int64_t)1 << 30) { set_error("too many columns"); return RH15D_EINVAL; }
    if (o->n_mu < 1 || o->n_mu > RH15D_MAX_MU) { set_error("n_mu must be in 1..%d", RH15D_MAX_MU); return RH15D_EINVAL; }
    if (o->ng_order != 0 && o->ng_order != 2) { set_error("ng_order must be 0 or 2"); return RH15D_EINVAL; }
    if (o->max_iter < 0) { set_error("max_iter must be >= 0"); return RH15D_EINVAL; }
    if (o->precision != RH15D_FP64 && o->precision != RH15D_FP32) { set_error("unknown precision"); return RH15D_EINVAL; }
    if (o->start < 0 || o->start > 3) { set_error("unknown start"); return RH15D_EINVAL; }
    if (!(o->tol_fp >= 0.0) || !std::isfinite(o->tol_fp)) { set_error("tol_fp must be finite and >= 0"); return RH15D_EINVAL; }
    if (o->esc_iter < 0 || o->esc_iter > 100) { set_error("esc_iter must be in 0..100"); return RH15D_EINVAL; }
    if (o->prd != 0 && o->prd != 1) { set_error("prd must be 0 or 1"); return RH15D_EINVAL; }
    if (!std::isfinite(o->prd_eps0)) { set_error("prd_eps0 must be finite"); return RH15D_EINVAL; }
    if (o->prd && o->sweep_mc > 1) { set_error("partial frequency redistribution needs sweep_mc 0 or 1"); return RH15D_EINVAL; }
    if (o->scheduler != RH15D_SCHED_CHUNKED && o->scheduler != RH15D_SCHED_SLOTS) { set_error("unknown scheduler"); return RH15D_EINVAL; }
    if (o->batch_columns < 0) { set_error("batch_columns must be >= 0"); return RH15D_EINVAL; }
    if (o->sweep_mc < 0 || (o->sweep_mc > 0 && o->n_mu % o->sweep_mc != 0) ||
        (o->sweep_mc > 0 && o->sweep_mc != 1 && o->sweep_mc != 3 && o->sweep_mc != 5)) {
        set_error("sweep_mc must be 0 (automatic) or 1, 3, 5 dividing n_mu"); return RH15D_EINVAL;
    }
    if (o->sweep_pack < 0 || o->sweep_pack > 2) { set_error("sweep_pack must be 0, 1 or 2"); return RH15D_EINVAL; }
    if (o->start == RH15D_START_PROVIDED && !cols->init_pops) { set_error("start=PROVIDED needs init_pops"); return RH15D_EINVAL; }
    if (!(o->tol >= 0.0)) { set_error("tol must be >= 0"); return RH15D_EINVAL; }
    if (!(o->crs_f0 >= 0.0) || !std::isfinite(o->crs_f0)) { set_error("crs_f0 must be finite and >= 0"); return RH15D_EINVAL; }
    if (cols->depth_offset && cols->depth_offset[0] != 0) { set_error("depth_offset[0] must be 0"); return RH15D_EINVAL; }
    for (int64_t c = 0; c < cols->n_columns; c++) {
        const int64_t n = cols->depth_offset[c + 1] - cols->depth_offset[c];
        if (n < 2 || n > RH15D_MAX_DEPTH) { set_error("column %lld has %lld depth points (need 2..%d)", (long long)c, (long long)n, RH15D_MAX_DEPTH); return RH15D_EINVAL; }
    }
    if (cols->n_columns > 0 && (!cols->z || !cols->T || !cols->n_e || !cols->n_H || !cols->v_z || !cols->v_turb)) {
        set_error("null column array"); return RH15D_EINVAL;
    }
    if ((cols->B != nullptr) != (cols->B_incl != nullptr) || (cols->B != nullptr) != (cols->B_azim != nullptr)) {
        set_error("the magnetic field needs all of B, B_incl and B_azim, or none"); return RH15D_EINVAL;
    }
    return RH15D_OK;
}

int max_depth(const rh15d_columns *cols) {
    int64_t nd = 2;
    for (int64_t c = 0; c < cols->n_columns; c++) nd = std::max(nd, cols->depth_offset[c + 1] - cols->depth_offset[c]);
    return (int)nd;
}

// Partial frequency redistribution is on when asked for and the atom has PRD lines.
bool prd_active(const DevAtom &D, const rh15d_options *o) { return o->prd != 0 && D.n_prd > 0; }

// Resident columns: the caller's choice, else as many as fit a 40 GiB
// working set (the device has 288 GB of HBM), at most 8192.
int slot_count(const DevAtom &D, const rh15d_columns *cols, const rh15d_options *o, int ND,
               size_t budget = size_t(40) << 30) {
    const int64_t n = std::max<int64_t>(cols->n_columns, 1);
    if (o->batch_columns > 0) return (int)std::min<int64_t>(o->batch_columns, n);
    const Layout one = make_layout(D, 0, 1, ND, o->precision == RH15D_FP32, o->ng_order == 2, prd_active(D, o));
    int64_t S = std::max<int64_t>(1, (int64_t)(budget / one.total));
    return (int)std::min<int64_t>(std::min<int64_t>(S, 8192), n);
}

unsigned grid_for(int64_t work, int per_block, unsigned cap) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + per_block - 1) / per_block, cap));
}

template <int L>
void launch_se_l(RunArgs &a, bool fp32, int kind, hipStream_t st) {
    if (kind != SE_ITERATION) {
        const dim3 grid(grid_for((int64_t)a.S * a.ND, 256, 16384));
        if (kind == SE_ESCAPE) hipLaunchKernelGGL((k_se_start<L, SE_ESCAPE>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_se_start<L, SE_ZERO_RADIATION>), grid, dim3(256), 0, st, a);
        return;
    }
    const unsigned blocks = grid_for((int64_t)a.S * a.ND, 256, 1u << 30);
    if (fp32) hipLaunchKernelGGL(k_rad_rates<float>, dim3(blocks, L * L), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(k_rad_rates<double>, dim3(blocks, L * L), dim3(256), 0, st, a);
    if (fp32) hipLaunchKernelGGL((k_se<float, L>), dim3(blocks), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_se<double, L>), dim3(blocks), dim3(256), 0, st, a);
}

void launch_se(RunArgs &a, bool fp32, int kind, hipStream_t st) {
    switch (a.A.L) {
        case 2: launch_se_l<2>(a, fp32, kind, st); break;
        case 3: launch_se_l<3>(a, fp32, kind, st); break;
        case 4: launch_se_l<4>(a, fp32, kind, st); break;
        case 5: launch_se_l<5>(a, fp32, kind, st); break;
        case 6: launch_se_l<6>(a, fp32, kind, st); break;
        case 7: launch_se_l<7>(a, fp32, kind, st); break;
        default: launch_se_l<8>(a, fp32, kind, st); break;
    }
}

template <typename R, int MODE, int NS, int NC, int MC, bool PRD>
void launch_sweep_range(const RunArgs &a, hipStream_t st) {
    const int id = group_class(NS, NC);
    const int gb = a.A.g_begin[id], ge = a.A.g_begin[id + 1];
    if (ge <= gb) return;
    const R *popsb = sizeof(R) == 8 ? reinterpret_cast<const R *>(a.pops) : reinterpret_cast<const R *>(a.popsf);
    hipLaunchKernelGGL((k_sweep<R, MODE, NS, NC, MC, PRD>), dim3((ge - gb + 3) / 4, a.S), dim3(256), 0, st, a, gb,
                       ge, reinterpret_cast<const R *>(a.rec), reinterpret_cast<const R *>(a.phi), popsb,
                       reinterpret_cast<R *>(a.part));
}

// every (slots, continua) class of NS slots, in class order
template <typename R, int MODE, int NS, int MC, bool PRD>
void launch_sweep_ns(const RunArgs &a, hipStream_t st) {
    launch_sweep_range<R, MODE, NS, 0, MC, PRD>(a, st);
    launch_sweep_range<R, MODE, NS, 1, MC, PRD>(a, st);
    if constexpr (NS >= 2) launch_sweep_range<R, MODE, NS, 2, MC, PRD>(a, st);
    if constexpr (NS >= 3) launch_sweep_range<R, MODE, NS, 3, MC, PRD>(a, st);
    if constexpr (NS >= 4) launch_sweep_range<R, MODE, NS, 4, MC, PRD>(a, st);
}

// The launches for the different slot counts touch disjoint rate sums, so
// they may run concurrently: each goes to a side stream forked from (and
// joined back into) the launch stream, and one launch's tail of finishing
// wavefronts overlaps the others' work.  Inside a captured iteration the
// fork and join become parallel branches of the graph.
struct SideStreams {
    bool on = false;
    hipStream_t s[kMaxSlots] = {};
    hipEvent_t fork = nullptr, join[kMaxSlots] = {};
    int init() {
        for (int i = 0; i < kMaxSlots; i++) {
            HIP_TRY(hipStreamCreateWithFlags(&s[i], hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&join[i], hipEventDisableTiming));
        }
        HIP_TRY(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        on = true;
        return RH15D_OK;
    }
    ~SideStreams() {
        for (int i = 0; i < kMaxSlots; i++) {
            if (s[i]) (void)hipStreamDestroy(s[i]);
            if (join[i]) (void)hipEventDestroy(join[i]);
        }
        if (fork) (void)hipEventDestroy(fork);
    }
};

template <typename R, int MODE, int MC, bool PRD = false>
void launch_sweep_mc(const RunArgs &a, hipStream_t st, SideStreams *side) {
    int used = 0;
    for (int ns = 1; ns <= kMaxSlots; ns++)
        used += a.A.g_begin[group_class(ns + 1, 0)] > a.A.g_begin[group_class(ns, 0)];
    if (!side || !side->on || used < 2) {
        launch_sweep_ns<R, MODE, 1, MC, PRD>(a, st);
        launch_sweep_ns<R, MODE, 2, MC, PRD>(a, st);
        launch_sweep_ns<R, MODE, 3, MC, PRD>(a, st);
        launch_sweep_ns<R, MODE, 4, MC, PRD>(a, st);
        return;
    }
    (void)hipEventRecord(side->fork, st);
    for (int i = 0; i < kMaxSlots; i++) (void)hipStreamWaitEvent(side->s[i], side->fork, 0);
    launch_sweep_ns<R, MODE, 1, MC, PRD>(a, side->s[0]);
    launch_sweep_ns<R, MODE, 2, MC, PRD>(a, side->s[1]);
    launch_sweep_ns<R, MODE, 3, MC, PRD>(a, side->s[2]);
    launch_sweep_ns<R, MODE, 4, MC, PRD>(a, side->s[3]);
    for (int i = 0; i < kMaxSlots; i++) {
        (void)hipEventRecord(side->join[i], side->s[i]);
        (void)hipStreamWaitEvent(st, side->join[i], 0);
    }
}

template <typename R, int MODE>
void launch_sweep(const RunArgs &a, hipStream_t st, SideStreams *side) {
    // partial frequency redistribution: one angle per lane (the solve forces it)
    if (a.prd) { launch_sweep_mc<R, MODE, 1, true>(a, st, side); return; }
    switch (a.A.mc) {
        case 5: launch_sweep_mc<R, MODE, 5>(a, st, side); break;
        case 3: launch_sweep_mc<R, MODE, 3>(a, st, side); break;
        default: launch_sweep_mc<R, MODE, 1>(a, st, side); break;
    }
}

struct Launcher {
    RunArgs a;
    bool fp32;
    int start;
    bool want_spec, want_psi, want_stokes;
    hipStream_t st;
    SideStreams *side = nullptr;

    void refill_phase(Timer *tm) {
        hipLaunchKernelGGL(k_refill, dim3(1), dim3(kRefillThreads), 0, st, a);
        const int64_t pts = (int64_t)a.S * a.ND;
        if (fp32) hipLaunchKernelGGL(k_prep_depth<float>, dim3(grid_for(pts, 256, 16384)), dim3(256), 0, st, a);
        else hipLaunchKernelGGL(k_prep_depth<double>, dim3(grid_for(pts, 256, 16384)), dim3(256), 0, st, a);
        if (a.A.n_lines > 0) {
            const unsigned pb = grid_for(pts * a.A.n_lines, 4, 65536);
            if (fp32) hipLaunchKernelGGL(k_prep_profile<float>, dim3(pb), dim3(256), 0, st, a);
            else hipLaunchKernelGGL(k_prep_profile<double>, dim3(pb), dim3(256), 0, st, a);
        }
        if (a.prd) {
            // one 64-lane workgroup per item, grid-stride (most iterations refill few slots)
            const unsigned tb = grid_for(pts * a.A.n_prd, 1, 16384);
            if (fp32) hipLaunchKernelGGL(k_prd_tables<float>, dim3(tb), dim3(64), 0, st, a);
            else hipLaunchKernelGGL(k_prd_tables<double>, dim3(tb), dim3(64), 0, st, a);
        }
        if (start == RH15D_START_ZERO_RADIATION) launch_se(a, fp32, SE_ZERO_RADIATION, st);
        if (start == RH15D_START_ESCAPE)
            for (int i = 0; i < a.esc_iter; i++) {
                hipLaunchKernelGGL(k_escape_beta, dim3(grid_for((int64_t)a.S * a.A.T, 256, 4096)), dim3(256), 0, st, a);
                launch_se(a, fp32, SE_ESCAPE, st);
            }
        hipLaunchKernelGGL(k_init_slots, dim3(grid_for(a.S, 256, 1024)), dim3(256), 0, st, a);
        (void)tm;
    }

    void iteration(Timer *tm) {
        if (tm) tm->mark(2, st);
        if (fp32) launch_sweep<float, MODE_RATES>(a, st, side);
        else launch_sweep<double, MODE_RATES>(a, st, side);
        if (tm) tm->mark(3, st);
        launch_se(a, fp32, SE_ITERATION, st);
        if (tm) tm->mark(4, st);
        hipLaunchKernelGGL(k_converge, dim3(a.S), dim3(kConvThreads), 0, st, a);
        if (a.prd) {
            // rho of the slots still iterating, then their emission profiles
            const int64_t pts = (int64_t)a.S * a.ND;
            const unsigned rb = grid_for(pts * a.A.n_prd, 4, 65536);
            const unsigned pb = grid_for(pts * a.A.psi_cols, 256, 65536);
            if (fp32) {
                hipLaunchKernelGGL(k_prd_rho<float>, dim3(rb), dim3(256), 0, st, a);
                hipLaunchKernelGGL(k_prd_psi<float>, dim3(pb), dim3(256), 0, st, a);
            } else {
                hipLaunchKernelGGL(k_prd_rho<double>, dim3(rb), dim3(256), 0, st, a);
                hipLaunchKernelGGL(k_prd_psi<double>, dim3(pb), dim3(256), 0, st, a);
            }
        }
        if (tm) tm->mark(5, st);
        if (want_spec) {
            const unsigned eb = grid_for((int64_t)a.S * a.A.NL, 256, 8192);
            if (fp32)
                hipLaunchKernelGGL((k_emergent<float, float>), dim3(eb), dim3(256), 0, st, a,
                                   reinterpret_cast<const float *>(a.rec), reinterpret_cast<const float *>(a.phi), a.popsf);
            else
                hipLaunchKernelGGL((k_emergent<double, double>), dim3(eb), dim3(256), 0, st, a,
                                   reinterpret_cast<const double *>(a.rec), reinterpret_cast<const double *>(a.phi),
                                   a.pops);
        }
        if (want_stokes)
            hipLaunchKernelGGL(k_stokes, dim3(grid_for((int64_t)a.S * a.A.NL, 256, 8192)), dim3(256), 0, st, a);
        if (want_psi) {
            if (fp32) launch_sweep<float, MODE_PSI>(a, st, side);
            else launch_sweep<double, MODE_PSI>(a, st, side);
            const unsigned gb = grid_for((int64_t)a.S * a.ND * a.A.T, 256, 16384);
            if (a.psi) {
                if (fp32) hipLaunchKernelGGL(k_psi_gather<float>, dim3(gb), dim3(256), 0, st, a);
                else hipLaunchKernelGGL(k_psi_gather<double>, dim3(gb), dim3(256), 0, st, a);
            }
        }
        if (tm) tm->mark(6, st);
        refill_phase(tm);
        if (tm) tm->mark(7, st);
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *rh15d_last_error(void) { return rh15d::last_error(); }

int rh15d_load_atom(const char *path, rh15d_atom **out) {
    if (!path || !out) { set_error("null argument"); return RH15D_EINVAL; }
    *out = nullptr;
    auto *a = new rh15d_atom();
    std::string err;
    int rc = parse_atom_file(path, a, err);
    if (rc != RH15D_OK) { set_error("%s: %s", path, err.c_str()); delete a; return rc; }
    *out = a;
    return RH15D_OK;
}

void rh15d_free_atom(rh15d_atom *atom) {
    if (!atom) return;
    for (void *p : atom->dev_allocs) (void)hipFree(p);
    delete atom;
}

int rh15d_atom_get_info(const rh15d_atom *atom, rh15d_atom_info *info) {
    if (!atom || !info) { set_error("null argument"); return RH15D_EINVAL; }
    info->n_levels = atom->L;
    info->n_lines = atom->n_lines;
    info->n_continua = atom->n_cont;
    info->n_transitions = static_cast<int>(atom->tr.size());
    info->n_lambda = static_cast<int>(atom->lam.size());
    return RH15D_OK;
}

int rh15d_atom_lambda(const rh15d_atom *atom, double *lambda_host) {
    if (!atom || !lambda_host) { set_error("null argument"); return RH15D_EINVAL; }
    std::memcpy(lambda_host, atom->lam.data(), atom->lam.size() * sizeof(double));
    return RH15D_OK;
}

int rh15d_last_stats(rh15d_stats *stats) {
    if (!stats) { set_error("null argument"); return RH15D_EINVAL; }
    *stats = g_stats;
    return RH15D_OK;
}

int rh15d_default_options(rh15d_options *o) {
    if (!o) { set_error("null argument"); return RH15D_EINVAL; }
    o->precision = RH15D_FP64;
    o->n_mu = 5;
    o->tol = 1e-4;
    o->max_iter = 200;
    o->ng_order = 2;
    o->ng_delay = 5;
    o->ng_period = 4;
    o->start = RH15D_START_LTE;
    o->coll_scale = 1.0;
    o->crs_f0 = 1.0;
    o->scheduler = RH15D_SCHED_CHUNKED;
    o->batch_columns = 0;
    o->profile = 0;
    o->sweep_mc = 0;
    o->sweep_pack = 0;
    o->tol_fp = 0.0;
    o->esc_iter = 3;
    o->prd = 0;
    o->prd_eps0 = 0.0;
    return RH15D_OK;
}

int rh15d_workspace_size(const rh15d_atom *atom_c, const rh15d_columns *cols, const rh15d_options *o, size_t *bytes) {
    int rc = validate(atom_c, cols, o);
    if (rc != RH15D_OK) return rc;
    if (!bytes) { set_error("null argument"); return RH15D_EINVAL; }
    DevAtom *D = nullptr;
    rh15d_atom *atom_m = const_cast<rh15d_atom *>(atom_c);
    if ((rc = get_dev_atom(atom_m, o->n_mu, pick_shape(atom_m, o), &D)) != RH15D_OK) return rc;
    const int ND = max_depth(cols);
    const int S = slot_count(*D, cols, o, ND);
    *bytes = make_layout(*D, cols->n_columns, S, ND, o->precision == RH15D_FP32, o->ng_order == 2,
                         prd_active(*D, o)).total;
    return RH15D_OK;
}

}  // extern "C"

namespace rh15d {

// The solve.  fixed_ws: the workspace is a fixed device region of
// workspace_bytes that the slot count must fit, and nothing is allocated
// (no device, pinned-host or graph memory, no side streams, no events).
int solve_columns_impl(const rh15d_atom *atom_c, const rh15d_columns *cols, const rh15d_options *o,
                       const rh15d_outputs *out, void *workspace, size_t workspace_bytes, void *hip_stream,
                       bool fixed_ws) {
    int rc = validate(atom_c, cols, o);
    if (rc != RH15D_OK) return rc;
    if (!out || (cols->n_columns > 0 && (!out->pops || !out->n_iter || !out->status))) {
        set_error("null output array"); return RH15D_EINVAL;
    }
    if (fixed_ws && o->profile) { set_error("profiling needs events: not available without allocation"); return RH15D_EINVAL; }
    g_stats = rh15d_stats{};
    if (cols->n_columns == 0) return RH15D_OK;
    rh15d_atom *atom = const_cast<rh15d_atom *>(atom_c);
    DevAtom *D = nullptr;
    if ((rc = get_dev_atom(atom, o->n_mu, pick_shape(atom, o), &D, !fixed_ws)) != RH15D_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const bool fp32 = o->precision == RH15D_FP32;
    const int ND = max_depth(cols);
    const bool prd = prd_active(*D, o);
    int S = fixed_ws ? slot_count(*D, cols, o, ND, workspace_bytes) : slot_count(*D, cols, o, ND);
    // a fixed region also holds the column offsets: fewer slots if needed
    while (fixed_ws && o->batch_columns <= 0 && S > 1 &&
           make_layout(*D, cols->n_columns, S, ND, fp32, o->ng_order == 2, prd).total > workspace_bytes)
        S--;
    const Layout lay = make_layout(*D, cols->n_columns, S, ND, fp32, o->ng_order == 2, prd);
    if (workspace && workspace_bytes < lay.total) {
        if (fixed_ws)
            set_error("these columns need %zu bytes of workspace (at least one resident column and the column "
                      "offsets), more than the %zu bytes of the fixed region", lay.total, workspace_bytes);
        else
            set_error("workspace too small: %zu < %zu", workspace_bytes, lay.total);
        return RH15D_ENOMEM;
    }
    void *own = nullptr;
    if (!workspace) {
        HIP_TRY(hipMalloc(&own, lay.total));
        workspace = own;
    }
    char *ws = static_cast<char *>(workspace);
    int *h_ctr = nullptr;
    int result = RH15D_OK;
    auto fail = [&](hipError_t e, const char *what) {
        if (result == RH15D_OK) set_error("%s: %s", what, hipGetErrorString(e));
        result = RH15D_EDEVICE;
    };
    // the done-counter read back every few iterations: pinned host memory,
    // or with a fixed workspace this thread's own pageable buffer
    thread_local int h_ctr_fixed[CTR_COUNT];
    hipError_t e = hipSuccess;
    if (fixed_ws) {
        h_ctr = h_ctr_fixed;
    } else {
        e = hipHostMalloc(reinterpret_cast<void **>(&h_ctr), CTR_COUNT * sizeof(int), hipHostMallocDefault);
        if (e != hipSuccess) { fail(e, "hipHostMalloc"); if (own) (void)hipFree(own); return result; }
    }
    auto free_host = [&]() { if (!fixed_ws) (void)hipHostFree(h_ctr); };

    RunArgs a{};
    a.A = *D;
    a.doff = reinterpret_cast<const int64_t *>(ws + lay.off_doff);
    a.n_columns = cols->n_columns;
    a.S = S; a.ND = ND;
    a.chunked = o->scheduler == RH15D_SCHED_CHUNKED;
    a.rec_w = rec_width(D->n_cont);
    a.z = cols->z; a.T = cols->T; a.ne = cols->n_e; a.nH = cols->n_H; a.vz = cols->v_z; a.vt = cols->v_turb;
    a.init = cols->init_pops;
    a.Bf = cols->B; a.Bincl = cols->B_incl; a.Bazim = cols->B_azim;
    a.stokes = out->stokes;
    a.psi_ray = out->psi_ray;
    a.pops = out->pops; a.history = out->history; a.spectrum = out->spectrum; a.psi = out->psi_star;
    a.n_iter = out->n_iter; a.status = out->status;
    int *slots = reinterpret_cast<int *>(ws + lay.off_slots);
    a.slot_col = slots; a.slot_state = slots + S; a.slot_it = slots + 2 * S; a.ng_count = slots + 3 * S;
    a.ng_head = slots + 4 * S;
    a.slot_bad = slots + 5 * S;
    a.slot_dprev = reinterpret_cast<double *>(ws + lay.off_dprev);
    a.ctr = reinterpret_cast<int *>(ws + lay.off_ctr);
    a.retire_list = reinterpret_cast<int *>(ws + lay.off_lists);
    a.refill_list = a.retire_list + S;
    a.lnr = reinterpret_cast<double *>(ws + lay.off_lnr);
    a.kbg = reinterpret_cast<double *>(ws + lay.off_kbg);
    a.gr = reinterpret_cast<double *>(ws + lay.off_gr);
    a.norm = reinterpret_cast<double *>(ws + lay.off_norm);
    a.phi = ws + lay.off_phi;
    a.part = ws + lay.off_part;
    a.rec = ws + lay.off_rec;
    a.popsf = fp32 ? reinterpret_cast<float *>(ws + lay.off_popsf) : nullptr;
    a.rad = reinterpret_cast<double *>(ws + lay.off_rad);
    a.nse = reinterpret_cast<double *>(ws + lay.off_nse);
    a.dk = reinterpret_cast<double *>(ws + lay.off_dk);
    a.flag = reinterpret_cast<int *>(ws + lay.off_flag);
    a.ring = reinterpret_cast<double *>(ws + lay.off_ring);
    a.max_iter = o->max_iter; a.ng_order = o->ng_order; a.ng_delay = o->ng_delay; a.ng_period = o->ng_period;
    a.start = o->start; a.tol = o->tol; a.coll_scale = o->coll_scale; a.crs_f0 = o->crs_f0;
    a.tol_fp = o->tol_fp; a.esc_iter = o->esc_iter;
    a.prd = prd ? 1 : 0; a.prd_eps0 = o->prd_eps0;
    a.emis = ws + lay.off_psi; a.ist = ws + lay.off_ist; a.gtab = ws + lay.off_gtab;
    a.rho = reinterpret_cast<double *>(ws + lay.off_rho);

    Launcher run{a, fp32, o->start, out->spectrum != nullptr, out->psi_star != nullptr || out->psi_ray != nullptr,
                 out->stokes != nullptr, st};
    Timer tm;
    if ((rc = tm.init(o->profile != 0)) != RH15D_OK) { free_host(); if (own) (void)hipFree(own); return rc; }
    // the sweep's classes run concurrently on side streams, or one after
    // another on the caller's stream with a fixed workspace
    SideStreams side;
    if (!fixed_ws && (rc = side.init()) != RH15D_OK) { free_host(); if (own) (void)hipFree(own); return rc; }
    run.side = &side;
    Timer *tp = tm.on ? &tm : nullptr;
    tm.mark(0, st);
    e = hipMemcpyAsync(const_cast<int64_t *>(a.doff), cols->depth_offset, (cols->n_columns + 1) * sizeof(int64_t),
                       hipMemcpyHostToDevice, st);
    if (e != hipSuccess) fail(e, "copy depth offsets");
    hipLaunchKernelGGL(k_setup, dim3(grid_for(S, 256, 1024)), dim3(256), 0, st, run.a);
    run.refill_phase(nullptr);

    // One iteration is a fixed sequence of launches whose amounts of work
    // live on the device; the slot scheduler captures it once as a graph.
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    const bool try_graph = o->scheduler == RH15D_SCHED_SLOTS && !tm.on && st != nullptr && !fixed_ws;
    if (try_graph && result == RH15D_OK) {
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            run.iteration(nullptr);
            if (hipStreamEndCapture(st, &graph) != hipSuccess || !graph ||
                hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
                exec = nullptr;
        }
        (void)hipGetLastError();
    }
    const int64_t rounds = (cols->n_columns + S - 1) / S;
    const int64_t bound = (rounds + 1) * ((int64_t)o->max_iter + 2) + 4;
    const int per_check = tm.on ? 1 : (exec ? 4 : 2);
    int64_t iters = 0;
    while (result == RH15D_OK) {
        for (int r = 0; r < per_check; r++, iters++) {
            if (exec) {
                e = hipGraphLaunch(exec, st);
                if (e != hipSuccess) { fail(e, "graph launch"); break; }
                g_stats.graph_launches++;
            } else {
                run.iteration(tp);
            }
        }
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(h_ctr, a.ctr, CTR_COUNT * sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) { fail(e, "iteration"); break; }
        if (tm.on) {
            g_stats.sweep_ms += tm.ms(2, 3);
            g_stats.se_ms += tm.ms(3, 4);
            g_stats.converge_ms += tm.ms(4, 5);
            g_stats.final_ms += tm.ms(5, 6);
            g_stats.prep_ms += tm.ms(6, 7);
            g_stats.sweep_launches++;
        }
        if (h_ctr[CTR_EMITTED] >= cols->n_columns) break;
        if (iters > bound) { set_error("iteration loop did not drain the column queue"); result = RH15D_EDEVICE; break; }
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    tm.mark(1, st);
    if (result == RH15D_OK) {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) fail(e, "synchronize");
    }
    if (result == RH15D_OK && tm.on) {
        g_stats.total_ms = tm.ms(0, 1);
        std::vector<int32_t> nit(cols->n_columns);
        e = hipMemcpy(nit.data(), out->n_iter, nit.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            fail(e, "read n_iter");
        } else {
            const double rsize = fp32 ? 4.0 : 8.0;
            for (int64_t c = 0; c < cols->n_columns; c++) {
                const double pts = (double)nit[c] * (double)(cols->depth_offset[c + 1] - cols->depth_offset[c]);
                g_stats.column_iterations += nit[c];
                g_stats.ray_steps += (int64_t)(pts * D->rays_per_depth);
                g_stats.sweep_flops += pts * D->flops_per_depth;
                g_stats.sweep_bytes += pts * (D->reads_per_depth + D->keys_per_depth) * rsize;
            }
        }
    }
    free_host();
    if (own) (void)hipFree(own);
    return result;
}

}  // namespace rh15d

extern "C" {

int rh15d_solve_columns(const rh15d_atom *atom_c, const rh15d_columns *cols, const rh15d_options *o,
                        const rh15d_outputs *out, void *workspace, size_t workspace_bytes, void *hip_stream) {
    return rh15d::solve_columns_impl(atom_c, cols, o, out, workspace, workspace_bytes, hip_stream, false);
}

int rh15d_autotune(rh15d_atom *atom, const rh15d_columns *cols, const rh15d_options *opt, void *hip_stream,
                   rh15d_tune_result *res) {
    int rc = validate(atom, cols, opt);
    if (rc != RH15D_OK) return rc;
    if (!res || cols->n_columns < 1) { set_error("null result or no columns"); return RH15D_EINVAL; }
    *res = rh15d_tune_result{};
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int64_t P = cols->depth_offset[cols->n_columns], n = cols->n_columns;
    const int L = atom->L;
    double *pops = nullptr;
    int32_t *nit = nullptr, *status = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int result = RH15D_OK;
    auto fail = [&](hipError_t e, const char *what) {
        if (result == RH15D_OK) set_error("%s: %s", what, hipGetErrorString(e));
        result = RH15D_EDEVICE;
    };
    hipError_t e = hipMalloc(&pops, (size_t)P * L * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&nit, n * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&status, n * sizeof(int32_t));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) fail(e, "autotune set-up");
    rh15d_outputs out{};
    out.pops = pops;
    out.n_iter = nit;
    out.status = status;
    double best = 1e300;
    for (int mc : {1, 3, 5}) {
        if (result != RH15D_OK || opt->n_mu % mc != 0) continue;
        for (int pack : {1, 2}) {
            if (result != RH15D_OK) break;
            rh15d_options o = *opt;
            o.sweep_mc = mc;
            o.sweep_pack = pack;
            o.profile = 0;
            // first call builds the shape's tables and warms the caches; the second is timed
            if ((rc = rh15d_solve_columns(atom, cols, &o, &out, nullptr, 0, hip_stream)) != RH15D_OK) { result = rc; break; }
            if ((e = hipEventRecord(e0, st)) != hipSuccess) { fail(e, "event"); break; }
            if ((rc = rh15d_solve_columns(atom, cols, &o, &out, nullptr, 0, hip_stream)) != RH15D_OK) { result = rc; break; }
            if ((e = hipEventRecord(e1, st)) != hipSuccess) { fail(e, "event"); break; }
            if ((e = hipEventSynchronize(e1)) != hipSuccess) { fail(e, "event"); break; }
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { fail(e, "event"); break; }
            const int c = res->n_candidates++;
            res->cand_mc[c] = mc;
            res->cand_pack[c] = pack;
            res->ms[c] = ms;
            if (ms < best) {
                best = ms;
                res->sweep_mc = mc;
                res->sweep_pack = pack;
            }
        }
    }
    if (result == RH15D_OK) {
        int dev = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess) {
            fail(e, "hipGetDevice");
        } else {
            std::lock_guard<std::mutex> lock(atom->mu_);
            atom->tuned[{{dev, opt->n_mu}, opt->precision}] = SweepShape{res->sweep_mc, res->sweep_pack - 1};
        }
    }
    (void)hipFree(pops);
    (void)hipFree(nit);
    (void)hipFree(status);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return result;
}

int rh15d_departures(const rh15d_atom *atom_c, const rh15d_columns *cols, const double *pops, float *log_b,
                     void *hip_stream) {
    if (!atom_c || !cols || !pops || !log_b || cols->n_columns < 0 || !cols->depth_offset || !cols->T || !cols->n_e ||
        !cols->n_H) {
        set_error("null argument or negative column count"); return RH15D_EINVAL;
    }
    rh15d_atom *atom = const_cast<rh15d_atom *>(atom_c);
    DevAtom *D = nullptr;
    int rc = get_dev_atom(atom, 1, SweepShape{}, &D);
    if (rc != RH15D_OK) return rc;
    const int64_t n = cols->depth_offset[cols->n_columns];
    if (n == 0) return RH15D_OK;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(k_departures, dim3(grid_for(n, 256, 65535)), dim3(256), 0, st, *D, n, cols->T, cols->n_e,
                       cols->n_H, pops, log_b);
    HIP_TRY(hipGetLastError());
    return RH15D_OK;
}

int rh15d_pops_from_departures(const rh15d_atom *atom_c, const rh15d_columns *cols, const float *log_b, double shrink,
                               double *pops, void *hip_stream) {
    if (!(shrink >= 0.0)) { set_error("shrink must be >= 0"); return RH15D_EINVAL; }
    if (!atom_c || !cols || !pops || !log_b || cols->n_columns < 0 || !cols->depth_offset || !cols->T || !cols->n_e ||
        !cols->n_H) {
        set_error("null argument or negative column count"); return RH15D_EINVAL;
    }
    rh15d_atom *atom = const_cast<rh15d_atom *>(atom_c);
    DevAtom *D = nullptr;
    int rc = get_dev_atom(atom, 1, SweepShape{}, &D);
    if (rc != RH15D_OK) return rc;
    const int64_t n = cols->depth_offset[cols->n_columns];
    if (n == 0) return RH15D_OK;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(k_pops_from_departures, dim3(grid_for(n, 256, 65535)), dim3(256), 0, st, *D, n, cols->T,
                       cols->n_e, cols->n_H, log_b, shrink, pops);
    HIP_TRY(hipGetLastError());
    return RH15D_OK;
}

}  // extern "C"
