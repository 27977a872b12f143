// Grid optimisation of atmosphere columns (Sec. 2.3, "Grid optimisation"):
// each column is re-interpolated onto a new depth grid with more points
// where temperature, vertical velocity or optical depth change fast, one
// column per wavefront.
//
// Reading (the paper gives no formula).  The interval between input points
// k-1 and k gets the length
//   d_k = sqrt((w_z dz_k / H)^2 + (w_T d ln T_k)^2 + (w_v dv_k)^2
//              + (w_tau d ln(tau_k + tau_min))^2),
// H the column's height range, tau the optical depth from the top in the
// atom's background at its reference wavelength (trapezoid rule in z, zero
// without a background), tau_min = 1e-5.  The new points divide the summed
// length M into equal parts, first and last input point kept exactly; every
// variable is linear in M inside an interval: z, v_z, v_turb as they are,
// T, n_e, n_H in their logarithms.
//
// A wavefront carries one column: lane l owns the consecutive input points
// [l ch, (l+1) ch), ch = ceil(N / 64).  Two wavefront scans (optical depth,
// then the length) leave M in LDS; every output point then finds its
// interval by bisection in M.  The work is a few transcendental functions
// per input point and a read of six input and a write of six output values
// per point: bound by HBM for long columns, by launch latency for few.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "rh15d_internal.h"

using namespace rh15d;

namespace {

constexpr double kTauMin = 1.0e-5;
// LDS of one block when the input columns are staged (up to 1170 points)
constexpr size_t kStageLds = 64 * 1024;

struct GridArgs {
    const int64_t *in_off, *out_off;  // [n_columns + 1] each, device
    const double *z, *T, *ne, *nH, *vz, *vt;
    double *zo, *To, *neo, *nHo, *vzo, *vto;
    int32_t *status;
    double wz, wT, wv, wtau;
    double c_bg;      // background coefficient; 0 without the background law
    int64_t n_columns;
    int max_in;       // longest input column of the launch
};

// Exclusive prefix sum over the wavefront.  Every shuffle runs with all 64
// lanes active: a lane that reads from a lane outside the execution mask
// gets no defined value, so the shuffles are never put under a condition.
__device__ __forceinline__ double scan_excl(double v, int lane) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    const double prev = __shfl_up(v, 1, kWave);
    return lane > 0 ? prev : 0.0;
}

__device__ __forceinline__ double bg_opacity(double c_bg, double T, double ne, double nH) {
    if (c_bg == 0.0) return 0.0;
    return c_bg * nH * ne * pow(T, -1.5) * exp(kBgTheta / T);
}

// kStage: the column's six input fields are first copied to LDS with
// coalesced loads (six arrays of g.max_in values after M), so that the
// three passes over the column and the interpolation read LDS instead of
// re-reading HBM; used when the longest input column of the launch fits.
template <bool kStage>
__global__ __launch_bounds__(kWave) void k_optimize_grid(GridArgs g) {
    extern __shared__ double M[];  // [max input points of the launch] (+ 6 staged fields)
    const int lane = threadIdx.x;
    for (int64_t c = blockIdx.x; c < g.n_columns; c += gridDim.x) {
        const int64_t i0 = g.in_off[c], o0 = g.out_off[c];
        const int N = (int)(g.in_off[c + 1] - i0), n_out = (int)(g.out_off[c + 1] - o0);
        const double *z, *T, *ne, *nH, *vz, *vt;
        if (kStage) {
            double *S = M + g.max_in;
            for (int k = lane; k < N; k += kWave) {
                S[k] = g.z[i0 + k];
                S[g.max_in + k] = g.T[i0 + k];
                S[2 * g.max_in + k] = g.ne[i0 + k];
                S[3 * g.max_in + k] = g.nH[i0 + k];
                S[4 * g.max_in + k] = g.vz[i0 + k];
                S[5 * g.max_in + k] = g.vt[i0 + k];
            }
            __syncthreads();
            z = S; T = S + g.max_in; ne = S + 2 * g.max_in; nH = S + 3 * g.max_in; vz = S + 4 * g.max_in;
            vt = S + 5 * g.max_in;
        } else {
            z = g.z + i0; T = g.T + i0; ne = g.ne + i0; nH = g.nH + i0; vz = g.vz + i0; vt = g.vt + i0;
        }
        // input checks, as the solve makes them (microturbulence only finite)
        int bad = N < 2;
        for (int k = lane; k < N; k += kWave) {
            if (!(T[k] > 0.0 && ne[k] > 0.0 && nH[k] > 0.0) || !isfinite(T[k] + ne[k] + nH[k] + vz[k] + vt[k] + z[k]))
                bad = 1;
            if (k > 0 && !(z[k] < z[k - 1])) bad = 1;
        }
        bad = __any(bad);
        double total = 0.0;
        if (!bad) {
            const int ch = (N + kWave - 1) / kWave;
            const int lo = min(N, lane * ch), hi = min(N, lo + ch);
            const int k0 = max(lo, 1);
            // optical depth: local partial sums of the trapezoid increments
            double s = 0.0;
            if (k0 < hi) {
                double kp = bg_opacity(g.c_bg, T[k0 - 1], ne[k0 - 1], nH[k0 - 1]);
                for (int k = k0; k < hi; k++) {
                    const double kk = bg_opacity(g.c_bg, T[k], ne[k], nH[k]);
                    s += 0.5 * (kp + kk) * (z[k - 1] - z[k]);
                    M[k] = s;
                    kp = kk;
                }
            }
            const double tau0 = scan_excl(s, lane);  // tau at point k0 - 1
            // interval lengths, local partial sums
            const double H = z[0] - z[N - 1];
            double tp = tau0, m = 0.0;
            for (int k = k0; k < hi; k++) {
                const double tk = tau0 + M[k];
                const double dz = g.wz * (z[k - 1] - z[k]) / H;
                const double dT = g.wT * (log(T[k]) - log(T[k - 1]));
                const double dv = g.wv * (vz[k] - vz[k - 1]);
                const double dt = g.wtau * (log(tk + kTauMin) - log(tp + kTauMin));
                m += sqrt(dz * dz + dT * dT + dv * dv + dt * dt);
                M[k] = m;
                tp = tk;
            }
            const double m0 = scan_excl(m, lane);
            for (int k = k0; k < hi; k++) M[k] += m0;
            if (lane == 0) M[0] = 0.0;
            __syncthreads();
            total = M[N - 1];
            if (!(total > 0.0 && isfinite(total))) bad = 1;
        }
        double *zo = g.zo + o0, *To = g.To + o0, *neo = g.neo + o0, *nHo = g.nHo + o0, *vzo = g.vzo + o0,
               *vto = g.vto + o0;
        if (bad) {
            for (int j = lane; j < n_out; j += kWave)
                zo[j] = To[j] = neo[j] = nHo[j] = vzo[j] = vto[j] = NAN;
        } else {
            for (int j = lane; j < n_out; j += kWave) {
                if (j == 0 || j == n_out - 1) {
                    const int k = j == 0 ? 0 : N - 1;
                    zo[j] = z[k]; To[j] = T[k]; neo[j] = ne[k]; nHo[j] = nH[k]; vzo[j] = vz[k]; vto[j] = vt[k];
                    continue;
                }
                const double target = total * (double)j / (double)(n_out - 1);
                // first k >= 1 with M[k] >= target (the last interval at most)
                int a = 1, b = N - 1;
                while (a < b) {
                    const int mid = (a + b) >> 1;
                    if (M[mid] < target) a = mid + 1; else b = mid;
                }
                const int k = a;
                const double f = (target - M[k - 1]) / (M[k] - M[k - 1]);
                zo[j] = z[k - 1] + f * (z[k] - z[k - 1]);
                To[j] = exp(log(T[k - 1]) + f * (log(T[k]) - log(T[k - 1])));
                neo[j] = exp(log(ne[k - 1]) + f * (log(ne[k]) - log(ne[k - 1])));
                nHo[j] = exp(log(nH[k - 1]) + f * (log(nH[k]) - log(nH[k - 1])));
                vzo[j] = vz[k - 1] + f * (vz[k] - vz[k - 1]);
                vto[j] = vt[k - 1] + f * (vt[k] - vt[k - 1]);
            }
        }
        if (lane == 0) g.status[c] = bad ? RH15D_BAD_INPUT : 0;
        __syncthreads();  // M is reused by the next column of this block
    }
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));                  \
            return RH15D_EDEVICE;                                                      \
        }                                                                              \
    } while (0)

}  // namespace

extern "C" {

int rh15d_default_grid_options(rh15d_grid_options *opt) {
    if (!opt) { set_error("null options"); return RH15D_EINVAL; }
    opt->w_z = 1.0;
    opt->w_T = 2.0;
    opt->w_v = 2.0e-4;
    opt->w_tau = 0.2;
    return RH15D_OK;
}

int rh15d_optimize_grid(const rh15d_atom *atom, const rh15d_columns *in, const rh15d_grid_options *opt,
                        const rh15d_grid_output *out, void *hip_stream) {
    if (!atom || !in || !opt || !out || in->n_columns < 0) {
        set_error("null argument or negative column count"); return RH15D_EINVAL;
    }
    const int64_t n = in->n_columns;
    if (n == 0) return RH15D_OK;
    if (!in->depth_offset || !out->depth_offset || !in->z || !in->T || !in->n_e || !in->n_H || !in->v_z ||
        !in->v_turb || !out->z || !out->T || !out->n_e || !out->n_H || !out->v_z || !out->v_turb || !out->status) {
        set_error("null column array"); return RH15D_EINVAL;
    }
    const double w[4] = {opt->w_z, opt->w_T, opt->w_v, opt->w_tau};
    bool any = false;
    for (double x : w) {
        if (!(x >= 0.0 && std::isfinite(x))) { set_error("grid weights must be finite and >= 0"); return RH15D_EINVAL; }
        any = any || x > 0.0;
    }
    if (!any) { set_error("all grid weights are zero"); return RH15D_EINVAL; }
    if (in->depth_offset[0] != 0 || out->depth_offset[0] != 0) {
        set_error("depth_offset[0] must be 0"); return RH15D_EINVAL;
    }
    int64_t max_in = 0;
    for (int64_t c = 0; c < n; c++) {
        const int64_t ni = in->depth_offset[c + 1] - in->depth_offset[c];
        const int64_t no = out->depth_offset[c + 1] - out->depth_offset[c];
        if (ni < 0 || ni > RH15D_GRID_MAX_INPUT) {
            set_error("column %lld: %lld input points (0..%d)", (long long)c, (long long)ni, RH15D_GRID_MAX_INPUT);
            return RH15D_EINVAL;
        }
        if (no < 2 || no > RH15D_MAX_DEPTH) {
            set_error("column %lld: %lld output points (2..%d)", (long long)c, (long long)no, RH15D_MAX_DEPTH);
            return RH15D_EINVAL;
        }
        max_in = std::max(max_in, ni);
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    int64_t *doff = nullptr;
    HIP_TRY(hipMallocAsync(reinterpret_cast<void **>(&doff), 2 * (n + 1) * sizeof(int64_t), st));
    // the offsets are read from the caller's host arrays before the call
    // returns (a synchronous upload: the call waits for earlier work on
    // the stream)
    hipError_t e = hipMemcpyAsync(doff, in->depth_offset, (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(doff + n + 1, out->depth_offset, (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFreeAsync(doff, st);
        set_error("upload of the depth offsets: %s", hipGetErrorString(e));
        return RH15D_EDEVICE;
    }
    GridArgs g;
    g.in_off = doff;
    g.out_off = doff + n + 1;
    g.z = in->z; g.T = in->T; g.ne = in->n_e; g.nH = in->n_H; g.vz = in->v_z; g.vt = in->v_turb;
    g.zo = out->z; g.To = out->T; g.neo = out->n_e; g.nHo = out->n_H; g.vzo = out->v_z; g.vto = out->v_turb;
    g.status = out->status;
    g.wz = w[0]; g.wT = w[1]; g.wv = w[2]; g.wtau = w[3];
    g.c_bg = atom->bg_kind == 1 ? atom->c_bg : 0.0;
    g.n_columns = n;
    g.max_in = (int)std::max<int64_t>(max_in, 1);
    const unsigned blocks = (unsigned)std::min<int64_t>(n, 1 << 20);
    const size_t lds = (size_t)g.max_in * sizeof(double);
    if (7 * lds <= kStageLds)
        hipLaunchKernelGGL(k_optimize_grid<true>, dim3(blocks), dim3(kWave), 7 * lds, st, g);
    else
        hipLaunchKernelGGL(k_optimize_grid<false>, dim3(blocks), dim3(kWave), lds, st, g);
    e = hipGetLastError();
    (void)hipFreeAsync(doff, st);
    if (e != hipSuccess) { set_error("grid optimisation launch: %s", hipGetErrorString(e)); return RH15D_EDEVICE; }
    return RH15D_OK;
}

}  // extern "C"
