// Learned start solution for MALI: a small MLP that predicts the natural-log
// departure coefficients ln(n_i / n*_i) of every level at a depth point from
// the local thermodynamic stencil.  The paper (Sec. 2.3) shows that the
// start solution decides how many iterations a column needs; the network
// only supplies that start, MALI still iterates to convergence.
//
// Network: 36 inputs (a 9-point depth stencil, offsets 0, +-2, +-8, +-32,
// +-128, of ln T, ln n_e, ln n_H and v_z / 10 km/s, z-scored) -> n_layers x n_hidden (SiLU) -> n_out.
// Dense layers run on CDNA matrix cores: gfx950's v_mfma_f32_16x16x32_bf16
// (16 x 16 outputs, 32-deep K per instruction) with FP32 accumulation.  Weights are rounded to BF16 when staged
// in LDS; forward activations enter as two BF16 terms (hi + lo), backward
// products round both operands to BF16.  Master weights, gradients and Adam
// moments are FP32.
#include <hip/hip_runtime.h>

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

constexpr int kStencil = 9;
constexpr int kFeat = 4 * kStencil;   // 36
constexpr int64_t kChunk = 1 << 18;   // samples per forward pass of a long inference
constexpr int kMaxSplit = 64;         // most sample chunks of a weight-gradient product
constexpr int kMseBlocks = 256;       // workgroups (and loss partials) of the squared-error kernel

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Operands of v_mfma_f32_16x16x32_bf16: lane l holds row (A) or column (B)
// l % 16 and the 8 consecutive K indices 8 (l / 16) .. 8 (l / 16) + 7 of the
// 32-deep block; the 16 x 16 FP32 result sits in lane l as rows
// 4 (l / 16) .. 4 (l / 16) + 3 of column l % 16.
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 bf16x8_of(const unsigned short (&v)[8]) {
    bf16x8 r;
#pragma unroll
    for (int t = 0; t < 8; t++) r[t] = __builtin_bit_cast(__bf16, v[t]);
    return r;
}

__device__ __forceinline__ unsigned short to_bf16(float f) {
    unsigned int u = __builtin_bit_cast(unsigned int, f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float sigmoid(float z) { return 1.f / (1.f + __expf(-z)); }

// Z = op(A)[M x K] op(B)[K x N] (+ bias[n]) (* silu'(D[m][n]) if D); H =
// silu(Z) if act.  FP32 in HBM, BF16 in LDS, FP32 accumulation.
// op(A)[m][k] = TA ? A[k lda + m] : A[m lda + k], op(B)[k][n] = TB ?
// B[n ldb + k] : B[k ldb + n].  Z and H (leading dimension ldc) are each
// optional.  Split K: workgroup z of the grid takes k in [z kchunk,
// (z + 1) kchunk) and writes its partial product at Z + z zstride.  A
// 64 x 64 tile per workgroup of four wavefronts, each a 32 x 32 block of
// 2 x 2 MFMA tiles.
constexpr int kBM = 64, kBN = 64, kBK = 32;

__device__ __forceinline__ float silu_grad(float z) {
    const float s = sigmoid(z);
    return s * (1.f + z * (1.f - s));
}

__device__ __forceinline__ float from_bf16(unsigned short h) {
    return __builtin_bit_cast(float, (unsigned int)h << 16);
}

// SA: op(A) enters as two BF16 terms, hi = bf16(a) and lo = bf16(a - hi),
// multiplied by the same BF16 B tile (two MFMAs): about 16 significant bits
// for the activations of the forward pass, whose rounding noise would
// otherwise set the floor of the network's output error; the weights (B)
// stay BF16.
template <bool TA, bool TB, bool SA>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float *A, int lda, const float *B, int ldb,
                                              const float *bias, const float *D, float *Z, float *H, int ldc, int act,
                                              int kchunk, int64_t zstride) {
    __shared__ unsigned short As[kBM][kBK + 4];
    __shared__ unsigned short Al[SA ? kBM : 1][kBK + 4];
    __shared__ unsigned short Bs[kBK][kBN + 4];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
    if (Z) Z += blockIdx.z * zstride;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kbeg; k0 < kend; k0 += kBK) {
        for (int e = tid; e < kBM * kBK; e += 256) {
            // TA: consecutive threads take consecutive m (A is k-major)
            const int r = TA ? e % kBM : e / kBK, c = TA ? e / kBM : e % kBK;
            const int m = m0 + r, k = k0 + c;
            float v = 0.f;
            if (m < M && k < kend) v = TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
            const unsigned short hi = to_bf16(v);
            As[r][c] = hi;
            if (SA) Al[r][c] = to_bf16(v - from_bf16(hi));
        }
        for (int e = tid; e < kBK * kBN; e += 256) {
            // TB: consecutive threads take consecutive k (B is n-major)
            const int r = TB ? e % kBK : e / kBN, c = TB ? e / kBK : e % kBN;
            const int k = k0 + r, n = n0 + c;
            float v = 0.f;
            if (k < kend && n < N) v = TB ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n];
            Bs[r][c] = to_bf16(v);
        }
        __syncthreads();
        static_assert(kBK == 32, "one 32-deep MFMA block per K tile");
        {
            const int kb = 8 * (lane >> 4);
            bf16x8 af[2], al[2], bfr[2];
#pragma unroll
            for (int i = 0; i < 2; i++) {
                const int row = wm + i * 16 + (lane & 15), col = wn + i * 16 + (lane & 15);
                unsigned short va[8], vl[8], vb[8];
#pragma unroll
                for (int t = 0; t < 8; t++) {
                    va[t] = As[row][kb + t];
                    vl[t] = SA ? Al[row][kb + t] : (unsigned short)0;
                    vb[t] = Bs[kb + t][col];
                }
                af[i] = bf16x8_of(va);
                al[i] = bf16x8_of(vl);
                bfr[i] = bf16x8_of(vb);
            }
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    if (SA) acc[i][j] = mfma32(al[i], bfr[j], acc[i][j]);
                    acc[i][j] = mfma32(af[i], bfr[j], acc[i][j]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
                const int n = n0 + wn + j * 16 + (lane & 15);
                if (m < M && n < N) {
                    float z = acc[i][j][r] + (bias ? bias[n] : 0.f);
                    if (D) z *= silu_grad(D[(size_t)m * ldc + n]);
                    if (Z) Z[(size_t)m * ldc + n] = z;
                    if (H) H[(size_t)m * ldc + n] = act ? z * sigmoid(z) : z;
                }
            }
}

// dY = 2 (Y - T) / (n N); per-block partial sums of the squared error.
// ctr (a replayed training step, else NULL): the target rows start at row
// ctr[0] * n of T.
__global__ void k_mse(const float *Y, const float *T, float *dY, int64_t n, int N, double *partial,
                      const int *ctr) {
    __shared__ double sh[256];
    if (ctr) T += (int64_t)ctr[0] * n * N;
    double s = 0.0;
    const double scale = 2.0 / ((double)n * N);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * N; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = Y[i] - T[i];
        dY[i] = (float)(scale * d);
        s += (double)d * d;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// part[z][j] = sum of dZ[i][j] over rows i of chunk z (rows in order)
__global__ void k_colsum_partial(const float *dZ, int64_t n, int N, int64_t chunk, float *part) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int64_t i0 = blockIdx.y * chunk, i1 = min(n, i0 + chunk);
    float s = 0.f;
    for (int64_t i = i0; i < i1; i++) s += dZ[i * N + j];
    part[(int64_t)blockIdx.y * N + j] = s;
}

// out[i] = sum over z of part[z stride + i], z in order
__global__ void k_reduce_splits(const float *part, int nsplit, int64_t stride, int64_t count, float *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int z = 0; z < nsplit; z++) s += part[z * stride + i];
        out[i] = (float)s;
    }
}

// ---------------------------------------------------------------------------
// fused inference: every layer of a tile of samples in one workgroup, the
// activations kept in LDS between layers (no round trip through HBM)
// ---------------------------------------------------------------------------
constexpr int kFuseRows = 32;           // samples per workgroup
constexpr int kFuseMaxW = 256;          // widest layer the fused kernel takes
constexpr int kFuseLd = kFuseMaxW + 8;  // LDS row stride in BF16 elements
constexpr int kMaxDense = 10;

// One dense layer of the fused kernel; the array lives in device memory
// (written once when the network is created), so the kernel reads it with
// scalar loads instead of indexing a by-value argument array.
struct FusedLayer {
    int kp, np, nout, pad;              // fan-in padded to 32, fan-out padded to 16, fan-out
    const unsigned short *w;            // weights packed as MFMA B fragments
    const float *b;                     // biases (FP32 master copy)
};

// B fragments of a [K][N] weight matrix for v_mfma_f32_16x16x32_bf16:
// block (kb, nb) holds, for lane l, W[32 kb + 8 (l / 16) + t][16 nb + l % 16],
// t = 0..7, as 8 consecutive BF16 values; zero outside the matrix.
__global__ void k_pack_b(const float *W, int K, int N, int KB, int NB, unsigned short *out) {
    const int64_t total = (int64_t)KB * NB * 512;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(e & 7), lane = (int)((e >> 3) & 63);
        const int64_t f = e >> 9;
        const int nb = (int)(f % NB), kb = (int)(f / NB);
        const int k = kb * 32 + 8 * (lane >> 4) + t, c = nb * 16 + (lane & 15);
        out[e] = (k < K && c < N) ? to_bf16(W[(size_t)k * N + c]) : (unsigned short)0;
    }
}

// The same arithmetic as the layer-by-layer path (normalised input; per
// 32-deep K block the LO then the HI half of the activations times the BF16
// weights; bias, SiLU), so the outputs agree bit for bit.  Wavefront w owns
// the output blocks of 16 columns w, w + 4, ...; the weight fragments of the
// next K block are loaded while the current block's MFMAs run.  Activation
// columns between a layer's width and the next layer's 32-padded fan-in are
// written as zeros.
__global__ __launch_bounds__(256) void k_mlp_fused(const FusedLayer *__restrict__ layers, int n_layers,
                                                   const float *feat, const float *mean, const float *istd, int64_t n,
                                                   float *out) {
    constexpr int RB = kFuseRows / 16;  // row blocks of 16 samples
    __shared__ __align__(16) unsigned short Hh[kFuseRows][kFuseLd];
    __shared__ __align__(16) unsigned short Hl[kFuseRows][kFuseLd];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t row0 = (int64_t)blockIdx.x * kFuseRows;
    const int kp0 = layers[0].kp;
    for (int e = tid; e < kFuseRows * kp0; e += 256) {
        const int r = e / kp0, c = e % kp0;
        float v = 0.f;
        if (c < kFeat && row0 + r < n) v = (feat[(row0 + r) * kFeat + c] - mean[c]) * istd[c];
        const unsigned short hi = to_bf16(v);
        Hh[r][c] = hi;
        Hl[r][c] = to_bf16(v - from_bf16(hi));
    }
    __syncthreads();
    const int nout_last = layers[n_layers - 1].nout;
    for (int l = 0; l < n_layers; l++) {
        const FusedLayer &ly = layers[l];
        const int KB = ly.kp / 32, NB = ly.np / 16, nout = ly.nout;
        const bool last = l == n_layers - 1;
        // output blocks written: the layer's, and for a hidden layer up to
        // the next layer's 32-padded fan-in (zeros past the width)
        const int NBW = last ? NB : (NB + 1) / 2 * 2;
        const uint4 *wf = reinterpret_cast<const uint4 *>(ly.w);
        f32x4 acc[RB][4];
#pragma unroll
        for (int i = 0; i < RB; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        uint4 bnext[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int nb = wave + 4 * j;
            bnext[j] = nb < NB ? wf[(int64_t)nb * 64 + lane] : uint4{0u, 0u, 0u, 0u};
        }
        for (int kb = 0; kb < KB; kb++) {
            uint4 bcur[4];
#pragma unroll
            for (int j = 0; j < 4; j++) bcur[j] = bnext[j];
            if (kb + 1 < KB) {
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int nb = wave + 4 * j;
                    if (nb < NB) bnext[j] = wf[((int64_t)(kb + 1) * NB + nb) * 64 + lane];
                }
            }
            const int k = kb * 32 + 8 * (lane >> 4);
            bf16x8 ah[RB], al[RB];
#pragma unroll
            for (int i = 0; i < RB; i++) {
                const int row = i * 16 + (lane & 15);
                ah[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(&Hh[row][k]));
                al[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(&Hl[row][k]));
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if (wave + 4 * j < NB) {
                    const bf16x8 bv = __builtin_bit_cast(bf16x8, bcur[j]);
#pragma unroll
                    for (int i = 0; i < RB; i++) {
                        acc[i][j] = mfma32(al[i], bv, acc[i][j]);
                        acc[i][j] = mfma32(ah[i], bv, acc[i][j]);
                    }
                }
            }
        }
        __syncthreads();  // every wavefront has read this layer's input
        const float *bias = ly.b;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int nb = wave + 4 * j;
            if (nb >= NBW) continue;
            const int col = nb * 16 + (lane & 15);
            const float bc = col < nout ? bias[col] : 0.f;
#pragma unroll
            for (int i = 0; i < RB; i++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int row = i * 16 + 4 * (lane >> 4) + r;
                    if (last) {
                        if (col < nout_last && row0 + row < n) out[(row0 + row) * nout_last + col] = acc[i][j][r] + bc;
                    } else {
                        unsigned short hi = 0, lo = 0;
                        if (col < nout) {
                            const float z = acc[i][j][r] + bc;
                            const float h = z * sigmoid(z);
                            hi = to_bf16(h);
                            lo = to_bf16(h - from_bf16(hi));
                        }
                        Hh[row][col] = hi;
                        Hl[row][col] = lo;
                    }
                }
        }
        __syncthreads();
    }
}

// sched (a replayed training step, else NULL): the step's learning rate and
// bias corrections are sched[3 ctr[0] + 0, 1, 2].
__global__ void k_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, const float *sched, const int *ctr) {
    if (sched) {
        const float *q = sched + 3 * (int64_t)ctr[0];
        lr = q[0];
        c1 = q[1];
        c2 = q[2];
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// Loss of a replayed training step: the squared-error partials summed in
// order (as the host does for a single step), into losses[ctr[0]].
__global__ void k_step_loss(const double *partial, int nb, int64_t n, int N, const int *ctr, float *losses) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nb; b++) s += partial[b];
    losses[ctr[0]] = (float)(s / ((double)n * N));
}

// The cursor of replayed training steps: set, then advanced after each step.
__global__ void k_set_counter(int *ctr, int v) { ctr[0] = v; }
__global__ void k_advance_counter(int *ctr) { ctr[0] += 1; }

// Raw stencil features of sample points (global depth indices; NULL = all
// points in order), columns ragged with offsets doff: ln T, ln n_e, ln n_H and
// v_z / 10 km/s at the depth offsets kStencilOffset from the point, clamped to
// the column (edge replication).  The offsets grow geometrically so that the
// nine points see both the local gradients and the column's structure a few
// hundred points away, including how far the point lies from either end.
__constant__ int kStencilOffset[kStencil] = {-128, -32, -8, -2, 0, 2, 8, 32, 128};

__global__ void k_features(const int64_t *doff, int64_t n_columns, const double *T, const double *ne,
                           const double *nH, const double *vz, const int64_t *samples, int64_t n, float *out) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = samples ? samples[s] : s;
        int64_t lo = 0, hi = n_columns - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (doff[mid] <= g) lo = mid; else hi = mid - 1;
        }
        const int64_t g0 = doff[lo], N = doff[lo + 1] - g0, k = g - g0;
        for (int j = 0; j < kStencil; j++) {
            int64_t kk = k + kStencilOffset[j];
            kk = kk < 0 ? 0 : (kk >= N ? N - 1 : kk);
            const int64_t q = g0 + kk;
            float *f = out + s * kFeat + j * 4;
            f[0] = (float)log(T[q]);
            f[1] = (float)log(ne[q]);
            f[2] = (float)log(nH[q]);
            f[3] = (float)(vz[q] * 1e-4);
        }
    }
}

// (x - mean) / std per feature
// ctr (a replayed training step, else NULL): the rows start at row ctr[0] * n of x.
__global__ void k_normalize(const float *x, const float *mean, const float *istd, float *y, int64_t n,
                            const int *ctr) {
    if (ctr) x += (int64_t)ctr[0] * n * kFeat;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * kFeat; i += (int64_t)gridDim.x * blockDim.x) {
        const int f = (int)(i % kFeat);
        y[i] = (x[i] - mean[f]) * istd[f];
    }
}

// Per-feature sums and sums of squares: block partials, then one block in order.
__global__ void k_feat_partial(const float *x, int64_t n, double *partial) {
    __shared__ double sh[256];
    for (int f = 0; f < kFeat; f++) {
        double s = 0.0, q = 0.0;
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
            const double v = x[i * kFeat + f];
            s += v;
            q += v * v;
        }
        for (int pass = 0; pass < 2; pass++) {
            sh[threadIdx.x] = pass ? q : s;
            __syncthreads();
            for (int o = 128; o > 0; o >>= 1) {
                if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
                __syncthreads();
            }
            if (threadIdx.x == 0) partial[((size_t)blockIdx.x * kFeat + f) * 2 + pass] = sh[0];
            __syncthreads();
        }
    }
}

__global__ void k_feat_finish(const double *partial, int nblocks, int64_t n, float *mean, float *stdv) {
    const int f = threadIdx.x;
    if (f >= kFeat) return;
    double s = 0.0, q = 0.0;
    for (int b = 0; b < nblocks; b++) {
        s += partial[((size_t)b * kFeat + f) * 2];
        q += partial[((size_t)b * kFeat + f) * 2 + 1];
    }
    const double m = s / n;
    const double var = q / n - m * m;
    mean[f] = (float)m;
    stdv[f] = (float)sqrt(var > 1e-12 ? var : 1e-12);
}

unsigned blocks_for(int64_t n, unsigned cap = 65535) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

struct rh15d_mlp {
    int n_hidden = 256, n_layers = 3, n_out = 6;
    std::vector<int> dims;             // n_in, hidden..., n_out
    std::vector<size_t> w_off, b_off;  // offsets into the flat parameter vector
    size_t n_params = 0;
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;  // device, FP32
    float *mean = nullptr, *istd = nullptr;                                 // device [36]
    std::vector<float> h_mean, h_std;
    int64_t step = 0;
    // activations for up to `cap` samples
    int64_t cap = 0;
    float *x = nullptr;                     // normalised inputs [cap][36]
    std::vector<float *> Z, H, dH;          // per layer
    float *wpart = nullptr, *bpart = nullptr;  // split-K partial gradients
    unsigned short *packed = nullptr;          // BF16 weights as MFMA B fragments (fused inference)
    std::vector<size_t> pk_off;
    FusedLayer *layers = nullptr;              // device descriptors of the fused kernel
    double *partial = nullptr;              // reductions
    int dev = 0;
    // rh15d_mlp_train_batches: one training step captured as a HIP graph on
    // the handle's own stream and replayed once per batch; a device cursor
    // selects the batch and the step's Adam scalars (sched).
    hipStream_t tstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t texec = nullptr;
    const float *g_feat = nullptr, *g_target = nullptr;  // what the captured step reads and writes
    float *g_losses = nullptr;
    int64_t g_batch = 0;
    int *ctr = nullptr;
    float *sched = nullptr;                 // device [sched_cap][3]: lr, c1, c2
    int64_t sched_cap = 0;
    std::vector<float> h_sched;
};

namespace {

void free_acts(rh15d_mlp *p) {
    (void)hipFree(p->x);
    for (auto *q : p->Z) (void)hipFree(q);
    for (auto *q : p->H) (void)hipFree(q);
    for (auto *q : p->dH) (void)hipFree(q);
    (void)hipFree(p->wpart);
    (void)hipFree(p->bpart);
    p->Z.clear(); p->H.clear(); p->dH.clear();
    p->x = nullptr;
    p->wpart = p->bpart = nullptr;
    p->cap = 0;
}

int ensure_cap(rh15d_mlp *p, int64_t n) {
    if (n <= p->cap) return RH15D_OK;
    free_acts(p);
    const int L = (int)p->dims.size() - 1;
    HIP_TRY(hipMalloc(&p->x, n * kFeat * sizeof(float)));
    p->Z.assign(L, nullptr); p->H.assign(L, nullptr); p->dH.assign(L, nullptr);
    for (int l = 0; l < L; l++) {
        const size_t bytes = (size_t)n * p->dims[l + 1] * sizeof(float);
        HIP_TRY(hipMalloc(&p->Z[l], bytes));
        HIP_TRY(hipMalloc(&p->H[l], bytes));
        HIP_TRY(hipMalloc(&p->dH[l], bytes));
    }
    size_t mn = 0, nmax = 0;
    for (int l = 0; l < L; l++) {
        mn = std::max(mn, (size_t)p->dims[l] * p->dims[l + 1]);
        nmax = std::max(nmax, (size_t)p->dims[l + 1]);
    }
    HIP_TRY(hipMalloc(&p->wpart, kMaxSplit * mn * sizeof(float)));
    HIP_TRY(hipMalloc(&p->bpart, kMaxSplit * nmax * sizeof(float)));
    p->cap = n;
    return RH15D_OK;
}

struct Epilogue {
    const float *bias = nullptr;  // + bias[n]
    const float *dact = nullptr;  // * silu'(dact[m][n])
    float *Z = nullptr, *H = nullptr;
    bool act = false;             // H = silu(Z)
    bool split_a = false;         // A as BF16 hi + lo (forward pass)
};

void gemm(bool ta, bool tb, int M, int N, int K, const float *A, int lda, const float *B, int ldb, const Epilogue &e,
          int ldc, hipStream_t st, int nsplit = 1, int kchunk = 0, int64_t zstride = 0) {
    const dim3 grid((N + kBN - 1) / kBN, (M + kBM - 1) / kBM, nsplit);
    const int a = e.act ? 1 : 0;
    if (nsplit == 1) kchunk = K;
#define RH15D_GEMM(TA_, TB_, SA_)                                                                                \
    hipLaunchKernelGGL((k_gemm<TA_, TB_, SA_>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, e.bias, e.dact, \
                       e.Z, e.H, ldc, a, kchunk, zstride)
    if (!ta && !tb) {
        if (e.split_a) RH15D_GEMM(false, false, true);
        else RH15D_GEMM(false, false, false);
    } else if (ta && !tb) RH15D_GEMM(true, false, false);
    else if (!ta && tb) RH15D_GEMM(false, true, false);
    else RH15D_GEMM(true, true, false);
#undef RH15D_GEMM
}

// Split of the sample dimension for the weight-gradient products, whose
// outputs are small (fan_in x fan_out) and whose sums run over all samples:
// enough workgroups to fill the chip, chunks a multiple of the K tile.
void split_for(int64_t n, int M, int N, int *nsplit, int *chunk) {
    const int tiles = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
    int s = (int)std::min<int64_t>(kMaxSplit, std::max<int64_t>(1, (1024 + tiles - 1) / tiles));
    s = (int)std::min<int64_t>(s, std::max<int64_t>(1, n / 128));
    int64_t c = (n + s - 1) / s;
    c = (c + kBK - 1) / kBK * kBK;
    *chunk = (int)c;
    *nsplit = (int)((n + c - 1) / c);
}

// Forward pass of n samples (raw features in HBM).  Training keeps every
// layer's pre-activation Z and activation H for the backward pass and leaves
// the output in p->Z.back(); inference keeps only H (the bias and SiLU are
// applied in the GEMM epilogue) and writes the output layer to `out`.
void forward(rh15d_mlp *p, const float *feat, int64_t n, bool training, float *out, hipStream_t st,
             const int *ctr = nullptr) {
    hipLaunchKernelGGL(k_normalize, dim3(blocks_for(n * kFeat)), dim3(256), 0, st, feat, p->mean, p->istd, p->x, n,
                       ctr);
    const int L = (int)p->dims.size() - 1;
    const float *in = p->x;
    for (int l = 0; l < L; l++) {
        const int K = p->dims[l], N = p->dims[l + 1];
        const bool last = l == L - 1;
        float *Z = training ? p->Z[l] : nullptr;
        float *H = last ? (training ? nullptr : out) : p->H[l];
        Epilogue e;
        e.bias = p->params + p->b_off[l];
        e.Z = Z;
        e.H = H;
        e.act = !last;
        e.split_a = true;
        gemm(false, false, (int)n, N, K, in, K, p->params + p->w_off[l], N, e, N, st);
        in = p->H[l];
    }
}

int backward(rh15d_mlp *p, const float *target, int64_t n, float *loss, hipStream_t st, const int *ctr = nullptr) {
    const int L = (int)p->dims.size() - 1;
    const int nout = p->dims[L];
    const int nb = kMseBlocks;
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, st, p->Z[L - 1], target, p->dH[L - 1], n, nout, p->partial,
                       ctr);
    for (int l = L - 1; l >= 0; l--) {
        const int K = p->dims[l], N = p->dims[l + 1];
        const float *dZ = p->dH[l];  // includes silu'(Z[l]) for hidden layers (epilogue below)
        const float *in = l == 0 ? p->x : p->H[l - 1];
        // dW = in^T dZ and db = column sums of dZ, split over the samples, then reduced in order
        int ns, chunk;
        split_for(n, K, N, &ns, &chunk);
        Epilogue ew;
        ew.Z = p->wpart;
        gemm(true, false, K, N, (int)n, in, K, dZ, N, ew, N, st, ns, chunk, (int64_t)K * N);
        hipLaunchKernelGGL(k_colsum_partial, dim3((N + 255) / 256, ns), dim3(256), 0, st, dZ, n, N, (int64_t)chunk,
                           p->bpart);
        hipLaunchKernelGGL(k_reduce_splits, dim3(blocks_for((int64_t)K * N, 4096)), dim3(256), 0, st, p->wpart, ns,
                           (int64_t)K * N, (int64_t)K * N, p->grads + p->w_off[l]);
        hipLaunchKernelGGL(k_reduce_splits, dim3(blocks_for(N)), dim3(256), 0, st, p->bpart, ns, (int64_t)N, (int64_t)N,
                           p->grads + p->b_off[l]);
        if (l > 0) {
            // dZ[l-1] = (dZ W^T) * silu'(Z[l-1])
            Epilogue eb;
            eb.dact = p->Z[l - 1];
            eb.Z = p->dH[l - 1];
            gemm(false, true, (int)n, K, N, dZ, N, p->params + p->w_off[l], N, eb, K, st);
        }
    }
    if (loss) {
        std::vector<double> part(nb);
        HIP_TRY(hipMemcpyAsync(part.data(), p->partial, nb * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        double s = 0.0;
        for (double x : part) s += x;
        *loss = (float)(s / ((double)n * nout));
    }
    HIP_TRY(hipGetLastError());
    return RH15D_OK;
}

}  // namespace

extern "C" {

int rh15d_mlp_create(int n_hidden, int n_layers, int n_out, uint64_t seed, rh15d_mlp **out) {
    if (!out || n_hidden < 1 || n_hidden > 4096 || n_layers < 1 || n_layers > 8 || n_out < 1 || n_out > 64) {
        set_error("bad MLP shape"); return RH15D_EINVAL;
    }
    *out = nullptr;
    auto *p = new rh15d_mlp();
    p->n_hidden = n_hidden; p->n_layers = n_layers; p->n_out = n_out;
    p->dims.push_back(kFeat);
    for (int l = 0; l < n_layers; l++) p->dims.push_back(n_hidden);
    p->dims.push_back(n_out);
    for (size_t l = 0; l + 1 < p->dims.size(); l++) {
        p->w_off.push_back(p->n_params);
        p->n_params += (size_t)p->dims[l] * p->dims[l + 1];
        p->b_off.push_back(p->n_params);
        p->n_params += p->dims[l + 1];
    }
    // He-uniform weights (bound sqrt(6 / fan_in)), zero biases, from a seeded splitmix64
    std::vector<float> h(p->n_params, 0.f);
    uint64_t s = seed;
    for (size_t l = 0; l + 1 < p->dims.size(); l++) {
        const double bound = std::sqrt(6.0 / p->dims[l]);
        for (size_t i = 0; i < (size_t)p->dims[l] * p->dims[l + 1]; i++) {
            const double u = (splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
            h[p->w_off[l] + i] = (float)((2.0 * u - 1.0) * bound);
        }
    }
    p->h_mean.assign(kFeat, 0.f);
    p->h_std.assign(kFeat, 1.f);
    std::vector<float> ones(kFeat, 1.f), zeros(kFeat, 0.f);
    hipError_t e = hipGetDevice(&p->dev);
    auto bytes = p->n_params * sizeof(float);
    if (e == hipSuccess) e = hipMalloc(&p->params, bytes);
    if (e == hipSuccess) e = hipMalloc(&p->grads, bytes);
    if (e == hipSuccess) e = hipMalloc(&p->m, bytes);
    if (e == hipSuccess) e = hipMalloc(&p->v, bytes);
    if (e == hipSuccess) e = hipMalloc(&p->mean, kFeat * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&p->istd, kFeat * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&p->partial, 256 * kFeat * 2 * sizeof(double));
    size_t pk = 0;
    for (size_t l = 0; l + 1 < p->dims.size(); l++) {
        p->pk_off.push_back(pk);
        pk += (size_t)((p->dims[l] + 31) / 32 * 32) * ((p->dims[l + 1] + 15) / 16 * 16);
    }
    if (e == hipSuccess) e = hipMalloc(&p->packed, pk * sizeof(unsigned short));
    if (e == hipSuccess) e = hipMalloc(&p->layers, (p->dims.size() - 1) * sizeof(FusedLayer));
    if (e == hipSuccess) {
        std::vector<FusedLayer> ly(p->dims.size() - 1);
        for (size_t l = 0; l + 1 < p->dims.size(); l++) {
            ly[l].kp = (p->dims[l] + 31) / 32 * 32;
            ly[l].np = (p->dims[l + 1] + 15) / 16 * 16;
            ly[l].nout = p->dims[l + 1];
            ly[l].w = p->packed + p->pk_off[l];
            ly[l].b = p->params + p->b_off[l];
        }
        e = hipMemcpy(p->layers, ly.data(), ly.size() * sizeof(FusedLayer), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemcpy(p->params, h.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p->grads, 0, bytes);
    if (e == hipSuccess) e = hipMemset(p->m, 0, bytes);
    if (e == hipSuccess) e = hipMemset(p->v, 0, bytes);
    if (e == hipSuccess) e = hipMemcpy(p->mean, zeros.data(), kFeat * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->istd, ones.data(), kFeat * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        set_error("MLP allocation failed: %s", hipGetErrorString(e));
        rh15d_mlp_free(p);
        return RH15D_EDEVICE;
    }
    *out = p;
    return RH15D_OK;
}

void rh15d_mlp_free(rh15d_mlp *p) {
    if (!p) return;
    free_acts(p);
    (void)hipFree(p->params); (void)hipFree(p->grads); (void)hipFree(p->m); (void)hipFree(p->v);
    (void)hipFree(p->mean); (void)hipFree(p->istd); (void)hipFree(p->partial); (void)hipFree(p->packed);
    (void)hipFree(p->layers);
    if (p->tstream) (void)hipStreamSynchronize(p->tstream);
    if (p->texec) (void)hipGraphExecDestroy(p->texec);
    if (p->ev_in) (void)hipEventDestroy(p->ev_in);
    if (p->ev_out) (void)hipEventDestroy(p->ev_out);
    if (p->tstream) (void)hipStreamDestroy(p->tstream);
    (void)hipFree(p->ctr);
    (void)hipFree(p->sched);
    delete p;
}

int rh15d_mlp_n_params(const rh15d_mlp *p, int64_t *n) {
    if (!p || !n) { set_error("null argument"); return RH15D_EINVAL; }
    *n = (int64_t)p->n_params;
    return RH15D_OK;
}

int rh15d_mlp_get_params(const rh15d_mlp *p, float *host) {
    if (!p || !host) { set_error("null argument"); return RH15D_EINVAL; }
    HIP_TRY(hipMemcpy(host, p->params, p->n_params * sizeof(float), hipMemcpyDeviceToHost));
    return RH15D_OK;
}

int rh15d_mlp_set_params(rh15d_mlp *p, const float *host) {
    if (!p || !host) { set_error("null argument"); return RH15D_EINVAL; }
    HIP_TRY(hipMemcpy(p->params, host, p->n_params * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(p->m, 0, p->n_params * sizeof(float)));
    HIP_TRY(hipMemset(p->v, 0, p->n_params * sizeof(float)));
    p->step = 0;
    return RH15D_OK;
}

int rh15d_mlp_get_grads(const rh15d_mlp *p, float *host) {
    if (!p || !host) { set_error("null argument"); return RH15D_EINVAL; }
    HIP_TRY(hipMemcpy(host, p->grads, p->n_params * sizeof(float), hipMemcpyDeviceToHost));
    return RH15D_OK;
}

int rh15d_mlp_get_normalization(const rh15d_mlp *p, float *mean, float *stdv) {
    if (!p || !mean || !stdv) { set_error("null argument"); return RH15D_EINVAL; }
    std::memcpy(mean, p->h_mean.data(), kFeat * sizeof(float));
    std::memcpy(stdv, p->h_std.data(), kFeat * sizeof(float));
    return RH15D_OK;
}

int rh15d_mlp_set_normalization(rh15d_mlp *p, const float *mean, const float *stdv) {
    if (!p || !mean || !stdv) { set_error("null argument"); return RH15D_EINVAL; }
    std::vector<float> is(kFeat);
    for (int f = 0; f < kFeat; f++) {
        if (!(stdv[f] > 0.f)) { set_error("feature scale must be positive"); return RH15D_EINVAL; }
        is[f] = 1.f / stdv[f];
    }
    p->h_mean.assign(mean, mean + kFeat);
    p->h_std.assign(stdv, stdv + kFeat);
    HIP_TRY(hipMemcpy(p->mean, mean, kFeat * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->istd, is.data(), kFeat * sizeof(float), hipMemcpyHostToDevice));
    return RH15D_OK;
}

int rh15d_mlp_features(const rh15d_columns *cols, const int64_t *samples, int64_t n, float *feat, void *stream) {
    if (!cols || !feat || n < 0 || cols->n_columns < 1 || !cols->depth_offset || !cols->T || !cols->n_e || !cols->n_H ||
        !cols->v_z) {
        set_error("null argument or no columns"); return RH15D_EINVAL;
    }
    if (!samples && n != cols->depth_offset[cols->n_columns]) {
        set_error("without sample indices n must be the total depth %lld", (long long)cols->depth_offset[cols->n_columns]);
        return RH15D_EINVAL;
    }
    if (n == 0) return RH15D_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int64_t *doff = nullptr;
    HIP_TRY(hipMallocAsync(reinterpret_cast<void **>(&doff), (cols->n_columns + 1) * sizeof(int64_t), st));
    HIP_TRY(hipMemcpyAsync(doff, cols->depth_offset, (cols->n_columns + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_features, dim3(blocks_for(n)), dim3(256), 0, st, doff, cols->n_columns, cols->T, cols->n_e,
                       cols->n_H, cols->v_z, samples, n, feat);
    HIP_TRY(hipFreeAsync(doff, st));
    HIP_TRY(hipGetLastError());
    return RH15D_OK;
}

int rh15d_mlp_fit_normalization(rh15d_mlp *p, const float *feat, int64_t n, void *stream) {
    if (!p || !feat || n < 2) { set_error("bad argument"); return RH15D_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    float *dm = nullptr;
    HIP_TRY(hipMallocAsync(reinterpret_cast<void **>(&dm), 2 * kFeat * sizeof(float), st));
    hipLaunchKernelGGL(k_feat_partial, dim3(256), dim3(256), 0, st, feat, n, p->partial);
    hipLaunchKernelGGL(k_feat_finish, dim3(1), dim3(64), 0, st, p->partial, 256, n, dm, dm + kFeat);
    std::vector<float> h(2 * kFeat);
    HIP_TRY(hipMemcpyAsync(h.data(), dm, 2 * kFeat * sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipFreeAsync(dm, st));
    return rh15d_mlp_set_normalization(p, h.data(), h.data() + kFeat);
}

int rh15d_mlp_forward(rh15d_mlp *p, const float *feat, int64_t n, float *out, void *stream) {
    if (!p || !feat || !out || n < 0) { set_error("null argument"); return RH15D_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int L = (int)p->dims.size() - 1;
    if (p->n_hidden % 16 == 0 && p->n_hidden <= kFuseMaxW && p->n_out <= 16 && L <= kMaxDense) {
        if (n == 0) return RH15D_OK;
        // the weights change with every Adam step or set_params: pack them for this call
        for (int l = 0; l < L; l++) {
            const int K = p->dims[l], N = p->dims[l + 1], KB = (K + 31) / 32, NB = (N + 15) / 16;
            hipLaunchKernelGGL(k_pack_b, dim3(blocks_for((int64_t)KB * NB * 512)), dim3(256), 0, st,
                               p->params + p->w_off[l], K, N, KB, NB, p->packed + p->pk_off[l]);
        }
        hipLaunchKernelGGL(k_mlp_fused, dim3((unsigned)((n + kFuseRows - 1) / kFuseRows)), dim3(256), 0, st,
                           p->layers, L, feat, p->mean, p->istd, n, out);
        HIP_TRY(hipGetLastError());
        return RH15D_OK;
    }
    int rc = ensure_cap(p, std::min<int64_t>(std::max<int64_t>(n, 1), kChunk));
    if (rc != RH15D_OK) return rc;
    const int nout = p->dims.back();
    for (int64_t s0 = 0; s0 < n; s0 += kChunk) {
        const int64_t m = std::min<int64_t>(kChunk, n - s0);
        forward(p, feat + s0 * kFeat, m, false, out + s0 * nout, st);
    }
    HIP_TRY(hipGetLastError());
    return RH15D_OK;
}

int rh15d_mlp_gradients(rh15d_mlp *p, const float *feat, const float *target, int64_t n, float *loss, void *stream) {
    if (!p || !feat || !target || n < 1 || n > kChunk) { set_error("bad argument (1 <= n <= %lld)", (long long)kChunk); return RH15D_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = ensure_cap(p, n);
    if (rc != RH15D_OK) return rc;
    forward(p, feat, n, true, nullptr, st);
    return backward(p, target, n, loss, st);
}

int rh15d_mlp_train_step(rh15d_mlp *p, const float *feat, const float *target, int64_t n, float lr, float *loss,
                         void *stream) {
    int rc = rh15d_mlp_gradients(p, feat, target, n, loss, stream);
    if (rc != RH15D_OK) return rc;
    if (!(lr >= 0.f)) { set_error("learning rate must be >= 0"); return RH15D_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    p->step++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)p->step), c2 = 1.f - std::pow(b2, (float)p->step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for((int64_t)p->n_params)), dim3(256), 0, st, p->params, p->grads, p->m, p->v,
                       (int64_t)p->n_params, lr, b1, b2, 1e-8f, c1, c2, nullptr, nullptr);
    HIP_TRY(hipGetLastError());
    return RH15D_OK;
}

int rh15d_mlp_train_batches(rh15d_mlp *p, const float *feat, const float *target, int64_t batch, int n_batches,
                            const float *lr, float *losses, void *stream) {
    if (!p || !feat || !target || !lr || batch < 1 || batch > kChunk || n_batches < 0) {
        set_error("bad argument (1 <= batch <= %lld, n_batches >= 0)", (long long)kChunk);
        return RH15D_EINVAL;
    }
    for (int b = 0; b < n_batches; b++)
        if (!(lr[b] >= 0.f)) { set_error("learning rate %d must be >= 0", b); return RH15D_EINVAL; }
    if (n_batches == 0) return RH15D_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t cap0 = p->cap;
    int rc = ensure_cap(p, batch);
    if (rc != RH15D_OK) return rc;
    auto drop_graph = [&]() {
        if (p->texec) (void)hipGraphExecDestroy(p->texec);
        p->texec = nullptr;
    };
    if (!p->tstream) {
        HIP_TRY(hipStreamCreateWithFlags(&p->tstream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming));
        HIP_TRY(hipMalloc(&p->ctr, sizeof(int)));
    }
    // the previous call's replays read h_sched (copied) and sched: let them finish
    HIP_TRY(hipStreamSynchronize(p->tstream));
    if (p->cap != cap0) drop_graph();   // activation buffers moved
    if (p->sched_cap < n_batches) {
        drop_graph();
        (void)hipFree(p->sched);
        p->sched = nullptr;
        p->sched_cap = 0;
        HIP_TRY(hipMalloc(&p->sched, (size_t)n_batches * 3 * sizeof(float)));
        p->sched_cap = n_batches;
    }
    if (p->texec && (p->g_feat != feat || p->g_target != target || p->g_batch != batch || p->g_losses != losses))
        drop_graph();
    // the Adam scalars of every step, as rh15d_mlp_train_step computes them
    const float b1 = 0.9f, b2 = 0.999f;
    p->h_sched.resize((size_t)n_batches * 3);
    for (int b = 0; b < n_batches; b++) {
        const float step = (float)(p->step + 1 + b);
        p->h_sched[3 * b] = lr[b];
        p->h_sched[3 * b + 1] = 1.f - std::pow(b1, step);
        p->h_sched[3 * b + 2] = 1.f - std::pow(b2, step);
    }
    // after the caller's work on its stream
    HIP_TRY(hipEventRecord(p->ev_in, st));
    HIP_TRY(hipStreamWaitEvent(p->tstream, p->ev_in, 0));
    HIP_TRY(hipMemcpyAsync(p->sched, p->h_sched.data(), (size_t)n_batches * 3 * sizeof(float), hipMemcpyHostToDevice,
                           p->tstream));
    hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, p->tstream, p->ctr, 0);
    if (!p->texec) {
        const int L = (int)p->dims.size() - 1;
        HIP_TRY(hipStreamBeginCapture(p->tstream, hipStreamCaptureModeThreadLocal));
        forward(p, feat, batch, true, nullptr, p->tstream, p->ctr);
        rc = backward(p, target, batch, nullptr, p->tstream, p->ctr);
        if (losses)
            hipLaunchKernelGGL(k_step_loss, dim3(1), dim3(64), 0, p->tstream, p->partial, kMseBlocks, batch, p->dims[L],
                               p->ctr, losses);
        hipLaunchKernelGGL(k_adam, dim3(blocks_for((int64_t)p->n_params)), dim3(256), 0, p->tstream, p->params,
                           p->grads, p->m, p->v, (int64_t)p->n_params, 0.f, b1, b2, 1e-8f, 1.f, 1.f, p->sched, p->ctr);
        hipLaunchKernelGGL(k_advance_counter, dim3(1), dim3(1), 0, p->tstream, p->ctr);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(p->tstream, &graph);
        if (rc != RH15D_OK) { if (graph) (void)hipGraphDestroy(graph); return rc; }
        if (ec != hipSuccess) { set_error("training step capture failed: %s", hipGetErrorString(ec)); return RH15D_EDEVICE; }
        const hipError_t ei = hipGraphInstantiate(&p->texec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            p->texec = nullptr;
            set_error("training step graph: %s", hipGetErrorString(ei));
            return RH15D_EDEVICE;
        }
        p->g_feat = feat;
        p->g_target = target;
        p->g_batch = batch;
        p->g_losses = losses;
    }
    for (int b = 0; b < n_batches; b++) HIP_TRY(hipGraphLaunch(p->texec, p->tstream));
    p->step += n_batches;
    HIP_TRY(hipEventRecord(p->ev_out, p->tstream));
    HIP_TRY(hipStreamWaitEvent(st, p->ev_out, 0));
    HIP_TRY(hipGetLastError());
    return RH15D_OK;
}

}  // extern "C"
