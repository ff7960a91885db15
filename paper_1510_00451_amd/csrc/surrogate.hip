// Learned surrogate of the local solve (not part of the paper's method):
// patch spectrum features, a 33 -> 256 -> 256 -> 256 -> 3 GELU network on the
// matrix cores (BF16 operands, FP32 accumulation), its training step (forward,
// relative Frobenius loss on a Cholesky head for K - K_b, backward, Adam on FP32 master
// weights) and ensemble inference with a fallback gate.
#include <math.h>

#include "band_core.h"
#include "shmm_internal.h"

namespace shmm {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {   // round to nearest, ties to even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);   // Inf / NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ------------------------------------------------------------------ features

struct BlockSync {
    __device__ void operator()() const { __syncthreads(); }
};

constexpr int kFeatRows = 8;   // rows (pass A) or columns (pass B) per workgroup

// Pass A: FFT along x of Z = vx + i vy for kFeatRows rows of one patch.
__global__ __launch_bounds__(256) void k_feat_rows(const shmm_domain *dom, const int32_t *list, int n,
                                                   const float *vx, const float *vy, c32 *work) {
    extern __shared__ c32 lds[];
    const int li = blockIdx.y;
    const shmm_domain D = dom[list[li]];
    const int r0 = blockIdx.x * kFeatRows;
    c32 *a = lds, *b = lds + kFeatRows * n;
    for (int t = threadIdx.x; t < kFeatRows * n; t += blockDim.x) {
        const int r = t / n, i = t - r * n;
        const int64_t c = D.offset + (int64_t)(r0 + r) * n + i;
        a[t] = c32{vx[c], vy[c]};
    }
    __syncthreads();
    // kFeatRows independent transforms: give each a slice of the threads
    const int per = blockDim.x / kFeatRows, row = threadIdx.x / per, tid = threadIdx.x - row * per;
    c32 *res = fft_inverse(a + row * n, b + row * n, n, tid, per, BlockSync{});
    // every row took the same number of passes, so res sits in the same buffer for all
    c32 *out = work + ((int64_t)li * n + r0) * n;
    for (int t = tid; t < n; t += per) out[(int64_t)row * n + t] = res[t];
}

// Pass B: FFT along y of kFeatRows columns; the spectrum A(k) of Z overwrites
// the pass-A rows in place (each workgroup owns its columns).
__global__ __launch_bounds__(256) void k_feat_cols(int n, c32 *work) {
    extern __shared__ c32 lds[];
    const int li = blockIdx.y;
    const int c0 = blockIdx.x * kFeatRows;
    c32 *a = lds, *b = lds + kFeatRows * n;
    c32 *src = work + (int64_t)li * n * n;
    for (int t = threadIdx.x; t < kFeatRows * n; t += blockDim.x) {
        const int col = t / n, j = t - col * n;
        a[t] = src[(int64_t)j * n + c0 + col];
    }
    __syncthreads();
    const int per = blockDim.x / kFeatRows, col = threadIdx.x / per, tid = threadIdx.x - col * per;
    c32 *res = fft_inverse(a + col * n, b + col * n, n, tid, per, BlockSync{});
    for (int t = tid; t < n; t += per) src[(int64_t)t * n + c0 + col] = res[t];
}

constexpr int kFeatThreads = 256;

// One workgroup per patch.  With A(k) = Vx(k) + i Vy(k) (Vx, Vy the transforms
// of the real fields), Vx(k) = (A(k) + conj A(-k))/2 and Vy(k) = (A(k) -
// conj A(-k))/(2i).  Channel energies per mode: |Vx|^2, |Vy|^2, |Vx+Vy|^2/2,
// |Vx-Vy|^2/2, each over |k_phys|^2 = q^2 (2 pi / L)^2; octave bin
// b = floor(log2 q), 0 <= b < 8, over every mode of the patch but the mean.
// Each thread sums a fixed stride of the modes, then one thread per bin adds
// the threads' partial sums in thread order: bitwise reproducible.  The
// features are the logarithms of the bin sums over det K_b.
__global__ __launch_bounds__(kFeatThreads) void k_feat_bins(const shmm_domain *dom, const int32_t *list, int n,
                                                            const c32 *work, const double *Kb, float *features) {
    __shared__ float part[SHMM_SURR_BINS][kFeatThreads];
    __shared__ float E[SHMM_SURR_BINS];
    const int li = blockIdx.x;
    const int64_t d = list[li];
    const int N = dom[d].N;
    const c32 *A = work + (int64_t)li * n * n;
    const float scale = (float)((double)n / (double)N * (double)n / (double)N / ((double)n * n * n * n));
    const int half = n / 2, mask = n - 1;
    float acc[SHMM_SURR_BINS];
#pragma unroll
    for (int c = 0; c < SHMM_SURR_BINS; ++c) acc[c] = 0.0f;
    for (int m = threadIdx.x; m < n * n; m += kFeatThreads) {
        const int jr = m / n, ic = m - jr * n;
        const int k1 = ic < half ? ic : ic - n, k2 = jr < half ? jr : jr - n;
        const int q2 = k1 * k1 + k2 * k2;
        const int b = q2 >= 1 ? (31 - __builtin_clz((unsigned)q2)) >> 1 : -1;
        if (b < 0 || b >= 8) continue;
        const c32 p = A[m];
        const c32 r = A[(int64_t)((-k2) & mask) * n + ((-k1) & mask)];
        const float vxr = 0.5f * (p.x + r.x), vxi = 0.5f * (p.y - r.y);
        const float vyr = 0.5f * (p.y + r.y), vyi = -0.5f * (p.x - r.x);
        const float pr = vxr + vyr, pi = vxi + vyi, mr = vxr - vyr, mi = vxi - vyi;
        const float wq = scale / (float)q2;
        const float e0 = (vxr * vxr + vxi * vxi) * wq, e1 = (vyr * vyr + vyi * vyi) * wq;
        const float e2 = 0.5f * (pr * pr + pi * pi) * wq, e3 = 0.5f * (mr * mr + mi * mi) * wq;
#pragma unroll
        for (int bb = 0; bb < 8; ++bb) {      // register accumulators: no dynamic index
            const bool h = b == bb;
            acc[bb] += h ? e0 : 0.0f;
            acc[8 + bb] += h ? e1 : 0.0f;
            acc[16 + bb] += h ? e2 : 0.0f;
            acc[24 + bb] += h ? e3 : 0.0f;
        }
    }
#pragma unroll
    for (int c = 0; c < SHMM_SURR_BINS; ++c) part[c][threadIdx.x] = acc[c];
    __syncthreads();
    if (threadIdx.x < SHMM_SURR_BINS) {
        float sum = 0.0f;
        for (int t = 0; t < kFeatThreads; ++t) sum += part[threadIdx.x][t];
        E[threadIdx.x] = sum;
    }
    __syncthreads();
    const double logdet = log(Kb[3 * d] * Kb[3 * d + 2] - Kb[3 * d + 1] * Kb[3 * d + 1]);
    if (threadIdx.x < SHMM_SURR_BINS) {
        float tot = 0.0f;
        for (int i = 0; i < 16; ++i) tot += E[i];
        const float floor = 1e-8f * tot + 1e-30f;
        features[(int64_t)li * SHMM_SURR_IN + threadIdx.x] = logf(E[threadIdx.x] + floor) - (float)logdet;
    }
    if (threadIdx.x == SHMM_SURR_BINS) features[(int64_t)li * SHMM_SURR_IN + SHMM_SURR_BINS] = (float)(0.5 * logdet);
    if (threadIdx.x == SHMM_SURR_BINS + 1) {
        // anisotropy of the base: the traceless part of log K_b, whose (1,1)
        // and (1,2) entries are g(rho) q / m and g(rho) K12 / m with m the mean
        // and r the half gap of the eigenvalues, rho = r / m, g = atanh(rho) / rho
        const double k11 = Kb[3 * d], k12 = Kb[3 * d + 1], k22 = Kb[3 * d + 2];
        const double m = 0.5 * (k11 + k22), q = 0.5 * (k11 - k22);
        const double rho = sqrt(q * q + k12 * k12) / m;
        const double g = rho < 1e-4 ? 1.0 + rho * rho / 3.0 : atanh(rho) / rho;
        features[(int64_t)li * SHMM_SURR_IN + SHMM_SURR_BINS + 1] = (float)(g * q / m);
        features[(int64_t)li * SHMM_SURR_IN + SHMM_SURR_BINS + 2] = (float)(g * k12 / m);
    }
}

// ------------------------------------------------------------------ GEMM

enum { EPI_F32 = 0, EPI_BIAS_F32 = 1, EPI_BIAS_GELU = 2, EPI_GELU_GRAD = 3 };

struct GemmArgs {
    int M, N, K;
    const uint16_t *A;
    int64_t sam, sak;
    const uint16_t *B;
    int64_t sbk, sbn;
    int epi;
    const float *bias;     // [N]
    float *outf;           // FP32 output (pre-activation, gradient, or result)
    int64_t ldo;
    uint16_t *outh;        // BF16 output (activation or gradient), may be null
    int64_t ldh;
    const float *z;        // saved pre-activations for EPI_GELU_GRAD
    int64_t ldz;
    float *partial;        // split K: [gridDim.z][M][N] raw sums (EPI_F32 only), or null
    int kchunk;            // K per slice when split
};

constexpr int TM = 64, TN = 64, TK = 64, LDK = TK + 8;   // LDS row pitch 144 B (16-byte aligned rows)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// How a workgroup stages one operand tile from global memory: element by
// element (any strides), or 16-byte vectors of 8 elements along the
// operand's contiguous dimension (K, or M / N), when that dimension has unit
// stride, the other stride is a multiple of 8 and the base is 16-byte aligned.
enum { LD_SCALAR = 0, LD_VEC_K = 1, LD_VEC_MN = 2 };

// Tile [rows][TK] of an operand X with X(r, k) at base[r * sr + k * sk],
// stored to LDS as dst[r][k] (row pitch LDK) for rows r0 + [0, 64) < R and
// k in [k0, k0 + TK) within [k0, kend); zero elsewhere.  256 threads.
template <int MODE>
__device__ __forceinline__ void stage_tile(uint16_t (*dst)[LDK], const uint16_t *__restrict__ base, int64_t sr,
                                           int64_t sk, int r0, int R, int k0, int kend) {
    const int t = threadIdx.x;
    if constexpr (MODE == LD_VEC_K) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int idx = t + 256 * j;
            const int r = idx >> 3, kk = (idx & 7) * 8;
            const int gr = r0 + r, gk = k0 + kk;
            uint4 v = {0u, 0u, 0u, 0u};
            if (gr < R && gk + 7 < kend) {
                v = *reinterpret_cast<const uint4 *>(base + gr * sr + gk);
            } else if (gr < R) {
                uint16_t e[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) e[i] = gk + i < kend ? base[gr * sr + gk + i] : (uint16_t)0;
                v.x = e[0] | ((uint32_t)e[1] << 16);
                v.y = e[2] | ((uint32_t)e[3] << 16);
                v.z = e[4] | ((uint32_t)e[5] << 16);
                v.w = e[6] | ((uint32_t)e[7] << 16);
            }
            *reinterpret_cast<uint4 *>(&dst[r][kk]) = v;
        }
    } else if constexpr (MODE == LD_VEC_MN) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int idx = t + 256 * j;
            const int k = idx >> 3, rr = (idx & 7) * 8;
            const int gk = k0 + k, gr = r0 + rr;
            uint16_t e[8];
            if (gk < kend && gr + 7 < R) {
                const uint4 v = *reinterpret_cast<const uint4 *>(base + gk * sk + gr);
                e[0] = (uint16_t)v.x; e[1] = (uint16_t)(v.x >> 16);
                e[2] = (uint16_t)v.y; e[3] = (uint16_t)(v.y >> 16);
                e[4] = (uint16_t)v.z; e[5] = (uint16_t)(v.z >> 16);
                e[6] = (uint16_t)v.w; e[7] = (uint16_t)(v.w >> 16);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) e[i] = (gk < kend && gr + i < R) ? base[gk * sk + gr + i] : (uint16_t)0;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) dst[rr + i][k] = e[i];
        }
    } else {
        for (int idx = t; idx < 64 * TK; idx += 256) {
            const int r = idx / TK, k = idx - r * TK;
            const int gr = r0 + r, gk = k0 + k;
            dst[r][k] = (gr < R && gk < kend) ? base[gr * sr + gk * sk] : (uint16_t)0;
        }
    }
}

// C[M][N] = A[M][K] B[K][N]: BF16 operands from arbitrary strides, FP32
// accumulation on gfx950's v_mfma_f32_16x16x32_bf16.  64 x 64 tile per
// workgroup, four wavefronts of 32 x 32 (2 x 2 matrix-core tiles), K in steps
// of 64 staged through LDS (A as [m][k], B as [n][k]: k contiguous, so each
// lane's 8 operand elements are one 16-byte LDS read).  Operand layout of the
// 16x16x32 instruction: lane l holds A[l % 16][8 (l / 16) + i] and
// B[8 (l / 16) + i][l % 16], i < 8, and receives D[4 (l / 16) + r][l % 16], r < 4.
template <int MA, int MB>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
    __shared__ __align__(16) uint16_t As[TM][LDK];
    __shared__ __align__(16) uint16_t Bt[TN][LDK];
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int kbeg = g.partial ? blockIdx.z * g.kchunk : 0;
    const int kend = g.partial ? min(g.K, kbeg + g.kchunk) : g.K;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
        stage_tile<MA>(As, g.A, g.sam, g.sak, m0, g.M, k0, kend);
        stage_tile<MB>(Bt, g.B, g.sbn, g.sbk, n0, g.N, k0, kend);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; kk += 32) {
            const int kq = kk + 8 * (lane >> 4);
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *reinterpret_cast<const bf16x8 *>(&As[wm * 32 + i * 16 + (lane & 15)][kq]);
                b[i] = *reinterpret_cast<const bf16x8 *>(&Bt[wn * 32 + i * 16 + (lane & 15)][kq]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                const int col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row >= g.M || col >= g.N) continue;
                float v = acc[i][j][r];
                if (g.partial) {
                    g.partial[((int64_t)blockIdx.z * g.M + row) * g.N + col] = v;
                    continue;
                }
                if (g.epi == EPI_BIAS_F32 || g.epi == EPI_BIAS_GELU) v += g.bias[col];
                if (g.epi == EPI_GELU_GRAD) v *= gelu_grad(g.z[row * g.ldz + col]);
                if (g.outf) g.outf[row * g.ldo + col] = v;
                if (g.outh) g.outh[row * g.ldh + col] = to_bf16(g.epi == EPI_BIAS_GELU ? gelu(v) : v);
            }
}

// staging mode of an operand with X(r, k) at base[r * sr + k * sk] (host side)
int load_mode(const uint16_t *base, int64_t sr, int64_t sk) {
    if (((uintptr_t)base & 15) != 0) return LD_SCALAR;
    if (sk == 1 && sr % 8 == 0) return LD_VEC_K;
    if (sr == 1 && sk % 8 == 0) return LD_VEC_MN;
    return LD_SCALAR;
}

template <int MA>
void launch_gemm_b(int mb, dim3 grid, const GemmArgs &g, hipStream_t s) {
    switch (mb) {
        case LD_VEC_K: hipLaunchKernelGGL((k_gemm_bf16<MA, LD_VEC_K>), grid, dim3(256), 0, s, g); break;
        case LD_VEC_MN: hipLaunchKernelGGL((k_gemm_bf16<MA, LD_VEC_MN>), grid, dim3(256), 0, s, g); break;
        default: hipLaunchKernelGGL((k_gemm_bf16<MA, LD_SCALAR>), grid, dim3(256), 0, s, g); break;
    }
}

void launch_gemm_kernel(dim3 grid, const GemmArgs &g, hipStream_t s) {
    const int ma = load_mode(g.A, g.sam, g.sak), mb = load_mode(g.B, g.sbn, g.sbk);
    switch (ma) {
        case LD_VEC_K: launch_gemm_b<LD_VEC_K>(mb, grid, g, s); break;
        case LD_VEC_MN: launch_gemm_b<LD_VEC_MN>(mb, grid, g, s); break;
        default: launch_gemm_b<LD_SCALAR>(mb, grid, g, s); break;
    }
}

// out[r][c] = sum over the slices z = 0, 1, ... of partial[z][r][c], in that order.
__global__ void k_splitk_sum(const float *partial, int slices, int M, int N, float *out, int64_t ldo) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)M * N) return;
    const int row = (int)(t / N), col = (int)(t - (int64_t)row * N);
    float v = 0.0f;
    for (int z = 0; z < slices; ++z) v += partial[(int64_t)z * M * N + t];
    out[row * ldo + col] = v;
}

constexpr int kSplitSlices = 16;   // K slices of the weight-gradient products
constexpr int kSplitMinK = 2048;   // split K from this length on (few output tiles)

int gemm(GemmArgs g, hipStream_t s, float *split_work = nullptr) {
    if (g.M <= 0 || g.N <= 0) return SHMM_OK;
    const dim3 tiles((unsigned)((g.N + TN - 1) / TN), (unsigned)((g.M + TM - 1) / TM));
    // few output tiles over a long K (weight gradients: K = batch): split K
    // into slices, then add the slices in a fixed order
    if (split_work && g.epi == EPI_F32 && tiles.x * tiles.y < 64 && g.K >= kSplitMinK) {
        g.kchunk = (g.K / kSplitSlices + TK - 1) / TK * TK;
        const int slices = (g.K + g.kchunk - 1) / g.kchunk;
        g.partial = split_work;
        launch_gemm_kernel(dim3(tiles.x, tiles.y, (unsigned)slices), g, s);
        SHMM_HIP_CHECK(hipGetLastError());
        const int64_t cnt = (int64_t)g.M * g.N;
        hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                           (const float *)split_work, slices, g.M, g.N, g.outf, g.ldo);
        SHMM_HIP_CHECK(hipGetLastError());
        return SHMM_OK;
    }
    g.partial = nullptr;
    g.kchunk = 0;
    launch_gemm_kernel(tiles, g, s);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

// ------------------------------------------------------------------ network pieces

struct Layout {
    int64_t W[4], b[4];
    int in[4], out[4];
};

Layout layout() {
    Layout L;
    const int dims[5] = {SHMM_SURR_IN, SHMM_SURR_WIDTH, SHMM_SURR_WIDTH, SHMM_SURR_WIDTH, SHMM_SURR_OUT};
    int64_t off = 0;
    for (int l = 0; l < 4; ++l) {
        L.in[l] = dims[l];
        L.out[l] = dims[l + 1];
        L.W[l] = off;
        off += (int64_t)dims[l] * dims[l + 1];
        L.b[l] = off;
        off += dims[l + 1];
    }
    return L;
}

__global__ void k_standardize(const float *x, int64_t B, const float *mu, const float *sigma, uint16_t *xh) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * SHMM_SURR_IN) return;
    const int c = (int)(t % SHMM_SURR_IN);
    xh[t] = to_bf16((x[t] - mu[c]) / sigma[c]);
}

// Head K = K_b + sqrt(det K_b) L L^T (the enhancement K - K_b is positive
// semi-definite); optional loss and output gradient.
__global__ void k_head(const float *o, const double *Kb, int64_t B, double *K_out, const double *K_true,
                       float *go, double *loss_part) {
    __shared__ double red[256];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double ls = 0.0;
    if (t < B) {
        const double s = sqrt(Kb[3 * t] * Kb[3 * t + 2] - Kb[3 * t + 1] * Kb[3 * t + 1]);
        const double l11 = exp((double)o[3 * t]), l21 = o[3 * t + 1], l22 = exp((double)o[3 * t + 2]);
        const double k11 = Kb[3 * t] + s * l11 * l11, k12 = Kb[3 * t + 1] + s * l11 * l21,
                     k22 = Kb[3 * t + 2] + s * (l21 * l21 + l22 * l22);
        if (K_out) {
            K_out[3 * t] = k11;
            K_out[3 * t + 1] = k12;
            K_out[3 * t + 2] = k22;
        }
        if (K_true) {
            const double t11 = K_true[3 * t], t12 = K_true[3 * t + 1], t22 = K_true[3 * t + 2];
            const double d11 = k11 - t11, d12 = k12 - t12, d22 = k22 - t22;
            const double nrm = t11 * t11 + 2.0 * t12 * t12 + t22 * t22;
            ls = (d11 * d11 + 2.0 * d12 * d12 + d22 * d22) / nrm;
            const double g11 = 2.0 * d11 / nrm / (double)B, g12 = 4.0 * d12 / nrm / (double)B,
                         g22 = 2.0 * d22 / nrm / (double)B;
            go[3 * t] = (float)(g11 * 2.0 * s * l11 * l11 + g12 * s * l11 * l21);
            go[3 * t + 1] = (float)(g12 * s * l11 + g22 * 2.0 * s * l21);
            go[3 * t + 2] = (float)(g22 * 2.0 * s * l22 * l22);
        }
    }
    if (loss_part) {
        red[threadIdx.x] = ls;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
    }
}

__global__ void k_to_bf16(const float *src, uint16_t *dst, int64_t count) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) dst[t] = to_bf16(src[t]);
}

constexpr int kColSlices = 16;

// Column sums of dz [B][n] (the bias gradient) in a fixed order: workgroup
// (x, z) sums 64 columns over row slice z, four row lanes then lane 0..3 in
// order; k_colsum_final adds the slices in order.
__global__ __launch_bounds__(256) void k_colsum_part(const float *dz, int64_t B, int n, float *part) {
    __shared__ float red[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), lane = threadIdx.x >> 6;
    const int64_t chunk = (B + kColSlices - 1) / kColSlices;
    const int64_t r0 = blockIdx.y * chunk, r1 = min(B, r0 + chunk);
    float v = 0.0f;
    if (c < n)
        for (int64_t r = r0 + lane; r < r1; r += 4) v += dz[r * n + c];
    red[lane][threadIdx.x & 63] = v;
    __syncthreads();
    if (lane == 0 && c < n) {
        const int i = threadIdx.x & 63;
        part[(int64_t)blockIdx.y * n + c] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
    }
}

__global__ void k_colsum_final(const float *part, int n, float *out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    float v = 0.0f;
    for (int z = 0; z < kColSlices; ++z) v += part[(int64_t)z * n + c];
    out[c] = v;
}

__global__ void k_loss_total(const double *part, int parts, int64_t B, double *loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int p = 0; p < parts; ++p) s += part[p];
        *loss = s / (double)B;
    }
}

constexpr int kNormParts = 128;

// Global gradient norm, fixed order: workgroup b sums the squares of entries
// b, b + 128 * 256 ... per thread, then a tree; k_norm_final adds the parts
// in order (FP64), writes the norm to loss[1] and the clipping scale
// min(1, clip / norm) (1 when clip <= 0).
__global__ __launch_bounds__(256) void k_sqsum(const float *g, int64_t count, float *part) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        s += g[i] * g[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_norm_final(const float *part, int parts, float clip, double *loss, float *scale) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < parts; ++i) s += (double)part[i];
    const double norm = sqrt(s);
    loss[1] = norm;
    *scale = (clip > 0.0f && norm > (double)clip) ? (float)((double)clip / norm) : 1.0f;
}

// Adam (Kingma & Ba) with bias correction on the FP32 masters, on the
// gradient times the clipping scale; refreshes BF16 copies.
__global__ void k_adam(float *p, float *m, float *v, const float *g, const float *scale, int64_t count, float lr,
                       float c1, float c2, uint16_t *ph) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const float gt = g[t] * scale[0];
    const float mt = 0.9f * m[t] + 0.1f * gt;
    const float vt = 0.999f * v[t] + 0.001f * gt * gt;
    m[t] = mt;
    v[t] = vt;
    const float pt = p[t] - lr * (mt / c1) / (sqrtf(vt / c2) + 1e-8f);
    p[t] = pt;
    ph[t] = to_bf16(pt);
}

// Ensemble mean, relative spread and the fallback flag.
// Ensemble mean, spread and gate.  A patch is flagged when a feature lies
// outside [lo, hi], when the largest member deviation from the mean exceeds
// tau (relative Frobenius), or when the predicted enhancement
// |K_mean - K_b|_F / |K_b|_F exceeds emax.
__global__ void k_gate(const double *Km, int E, int64_t B, const float *x, const double *Kb, const float *lo,
                       const float *hi, double tau, double emax, double *K_out, uint8_t *flag,
                       double *spread_out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B) return;
    double m[3] = {0.0, 0.0, 0.0};
    for (int e = 0; e < E; ++e)
        for (int q = 0; q < 3; ++q) m[q] += Km[((int64_t)e * B + t) * 3 + q];
    for (int q = 0; q < 3; ++q) m[q] /= (double)E;
    const double fm = sqrt(m[0] * m[0] + 2.0 * m[1] * m[1] + m[2] * m[2]);
    double sp = 0.0;
    for (int e = 0; e < E; ++e) {
        const double *k = Km + ((int64_t)e * B + t) * 3;
        const double a = k[0] - m[0], b = k[1] - m[1], c = k[2] - m[2];
        const double f = sqrt(a * a + 2.0 * b * b + c * c) / fm;
        sp = f > sp ? f : sp;
    }
    bool out = false;
    for (int c = 0; c < SHMM_SURR_IN; ++c) {
        const float v = x[t * SHMM_SURR_IN + c];
        if (!(v >= lo[c] && v <= hi[c])) out = true;
    }
    const double *kb = Kb + 3 * t;
    const double d0 = m[0] - kb[0], d1 = m[1] - kb[1], d2 = m[2] - kb[2];
    const double enh = sqrt(d0 * d0 + 2.0 * d1 * d1 + d2 * d2) /
                       sqrt(kb[0] * kb[0] + 2.0 * kb[1] * kb[1] + kb[2] * kb[2]);
    for (int q = 0; q < 3; ++q) K_out[3 * t + q] = m[q];
    flag[t] = (uint8_t)((sp > tau || out || !(fm > 0.0) || !(enh <= emax)) ? 1 : 0);
    if (spread_out) spread_out[t] = sp;
}

}  // namespace

size_t surrogate_feature_workspace(int n, int64_t nlist) { return (size_t)nlist * n * n * sizeof(c32); }

int launch_patch_features(const shmm_domain *d_dom, const int32_t *d_list, int32_t nlist, int n,
                          const float *vx, const float *vy, const double *Kb, float *features, void *work,
                          hipStream_t s) {
    if (nlist <= 0) return SHMM_OK;
    if (n < kFeatRows || n > 256) return SHMM_ERANGE;
    c32 *fw = (c32 *)work;
    const dim3 grid((unsigned)(n / kFeatRows), (unsigned)nlist);
    hipLaunchKernelGGL(k_feat_rows, grid, dim3(256), 2 * kFeatRows * n * sizeof(c32), s, d_dom, d_list, n, vx,
                       vy, fw);
    SHMM_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_feat_cols, grid, dim3(256), 2 * kFeatRows * n * sizeof(c32), s, n, fw);
    SHMM_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_feat_bins, dim3((unsigned)nlist), dim3(kFeatThreads), 0, s, d_dom, d_list, n, (const c32 *)fw, Kb,
                       features);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

// Workspace of one forward/backward at batch B (bytes), laid out by `carve`.
struct NetWork {
    uint16_t *h[4];      // bf16 activations: h[0] = standardised input [B][33], h[1..3] [B][256]
    float *z[3];         // pre-activations of the hidden layers [B][256]
    float *o;            // outputs [B][3]
    float *go;           // output gradient [B][3]
    float *dz;           // FP32 gradient of the current layer [B][256]
    uint16_t *dzh;       // its bf16 copy
    float *dz2;          // second buffer for the next layer's gradient
    double *loss_part;   // [ceil(B / 256)]
    float *grad;         // [SHMM_SURR_PARAMS_PADDED]
    float *split;        // split-K slices [kSplitSlices][256][256]
    float *colpart;      // column-sum slices [kColSlices][256]
    float *gpart;        // gradient-norm parts [kNormParts], then the clipping scale
};

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

size_t surrogate_net_workspace(int64_t B) {
    size_t s = 0;
    s += align256((size_t)B * SHMM_SURR_IN * 2);
    for (int l = 1; l < 4; ++l) s += align256((size_t)B * SHMM_SURR_WIDTH * 2);
    for (int l = 0; l < 3; ++l) s += align256((size_t)B * SHMM_SURR_WIDTH * 4);
    s += 2 * align256((size_t)B * 3 * 4);
    s += 2 * align256((size_t)B * SHMM_SURR_WIDTH * 4) + align256((size_t)B * SHMM_SURR_WIDTH * 2);
    s += align256((size_t)((B + 255) / 256) * 8);
    s += align256((size_t)SHMM_SURR_PARAMS_PADDED * 4);
    s += align256((size_t)kSplitSlices * SHMM_SURR_WIDTH * SHMM_SURR_WIDTH * 4);
    s += align256((size_t)kColSlices * SHMM_SURR_WIDTH * 4);
    s += align256((size_t)(kNormParts + 1) * 4);
    return s;
}

static NetWork carve(void *work, int64_t B) {
    char *p = (char *)work;
    NetWork w;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += align256(bytes);
        return (void *)r;
    };
    w.h[0] = (uint16_t *)take((size_t)B * SHMM_SURR_IN * 2);
    for (int l = 1; l < 4; ++l) w.h[l] = (uint16_t *)take((size_t)B * SHMM_SURR_WIDTH * 2);
    for (int l = 0; l < 3; ++l) w.z[l] = (float *)take((size_t)B * SHMM_SURR_WIDTH * 4);
    w.o = (float *)take((size_t)B * 3 * 4);
    w.go = (float *)take((size_t)B * 3 * 4);
    w.dz = (float *)take((size_t)B * SHMM_SURR_WIDTH * 4);
    w.dz2 = (float *)take((size_t)B * SHMM_SURR_WIDTH * 4);
    w.dzh = (uint16_t *)take((size_t)B * SHMM_SURR_WIDTH * 2);
    w.loss_part = (double *)take((size_t)((B + 255) / 256) * 8);
    w.grad = (float *)take((size_t)SHMM_SURR_PARAMS_PADDED * 4);
    w.split = (float *)take((size_t)kSplitSlices * SHMM_SURR_WIDTH * SHMM_SURR_WIDTH * 4);
    w.colpart = (float *)take((size_t)kColSlices * SHMM_SURR_WIDTH * 4);
    w.gpart = (float *)take((size_t)(kNormParts + 1) * 4);
    return w;
}

// member pointers inside one model block
struct Model {
    float *p;          // FP32 parameters
    float *mu, *sigma; // standardisation
    uint16_t *ph;      // bf16 parameters
};

static Model model_at(void *base) {
    Model m;
    m.p = (float *)base;
    m.mu = m.p + SHMM_SURR_PARAMS_PADDED;
    m.sigma = m.mu + 64;
    m.ph = (uint16_t *)(m.mu + 128);
    return m;
}

static int net_forward(const Model &m, const float *x, int64_t B, const NetWork &w, hipStream_t s) {
    const Layout L = layout();
    const int64_t nin = B * SHMM_SURR_IN;
    hipLaunchKernelGGL(k_standardize, dim3((unsigned)((nin + 255) / 256)), dim3(256), 0, s, x, B, m.mu,
                       m.sigma, w.h[0]);
    SHMM_HIP_CHECK(hipGetLastError());
    int rc;
    for (int l = 0; l < 4; ++l) {
        GemmArgs g;
        g.M = (int)B;
        g.N = L.out[l];
        g.K = L.in[l];
        g.A = w.h[l];
        g.sam = L.in[l];
        g.sak = 1;
        g.B = m.ph + L.W[l];
        g.sbk = 1;
        g.sbn = L.in[l];
        g.bias = m.p + L.b[l];
        g.z = nullptr;
        g.ldz = 0;
        if (l < 3) {
            g.epi = EPI_BIAS_GELU;
            g.outf = w.z[l];
            g.ldo = L.out[l];
            g.outh = w.h[l + 1];
            g.ldh = L.out[l];
        } else {
            g.epi = EPI_BIAS_F32;
            g.outf = w.o;
            g.ldo = 3;
            g.outh = nullptr;
            g.ldh = 0;
        }
        if ((rc = gemm(g, s))) return rc;
    }
    return SHMM_OK;
}

int surrogate_train_step(void *model, float *adam, const float *x, const double *Kb, const double *Kt,
                         int64_t B, float lr, float clip, int32_t t, double *loss, float *grad_out, void *work,
                         hipStream_t s) {
    const Layout L = layout();
    const Model m = model_at(model);
    const NetWork w = carve(work, B);
    int rc = net_forward(m, x, B, w, s);
    if (rc) return rc;
    const unsigned hb = (unsigned)((B + 255) / 256);
    hipLaunchKernelGGL(k_head, dim3(hb), dim3(256), 0, s, (const float *)w.o, Kb, B, (double *)nullptr, Kt, w.go,
                       w.loss_part);
    SHMM_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(64), 0, s, (const double *)w.loss_part, (int)hb, B, loss);
    SHMM_HIP_CHECK(hipGetLastError());
    // backward: dz of layer 3 is the output gradient
    const float *dz = w.go;
    float *next = w.dz;
    for (int l = 3; l >= 0; --l) {
        const int n_out = L.out[l], n_in = L.in[l];
        const int64_t cnt = B * n_out;
        hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, dz, w.dzh, cnt);
        SHMM_HIP_CHECK(hipGetLastError());
        // dW_l = dz^T h_l   ([out][B] x [B][in])
        GemmArgs g;
        g.M = n_out;
        g.N = n_in;
        g.K = (int)B;
        g.A = w.dzh;
        g.sam = 1;
        g.sak = n_out;
        g.B = w.h[l];
        g.sbk = n_in;
        g.sbn = 1;
        g.epi = EPI_F32;
        g.bias = nullptr;
        g.outf = w.grad + L.W[l];
        g.ldo = n_in;
        g.outh = nullptr;
        g.ldh = 0;
        g.z = nullptr;
        g.ldz = 0;
        if ((rc = gemm(g, s, w.split))) return rc;
        hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)((n_out + 63) / 64), (unsigned)kColSlices), dim3(256), 0,
                           s, dz, B, n_out, w.colpart);
        SHMM_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_colsum_final, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, s,
                           (const float *)w.colpart, n_out, w.grad + L.b[l]);
        SHMM_HIP_CHECK(hipGetLastError());
        if (l == 0) break;
        // dz_{l-1} = (dz W_l) * gelu'(z_{l-1})   ([B][out] x [out][in])
        GemmArgs h;
        h.M = (int)B;
        h.N = n_in;
        h.K = n_out;
        h.A = w.dzh;
        h.sam = n_out;
        h.sak = 1;
        h.B = m.ph + L.W[l];
        h.sbk = n_in;
        h.sbn = 1;
        h.epi = EPI_GELU_GRAD;
        h.bias = nullptr;
        h.outf = next;
        h.ldo = n_in;
        h.outh = nullptr;
        h.ldh = 0;
        h.z = w.z[l - 1];
        h.ldz = n_in;
        if ((rc = gemm(h, s))) return rc;
        dz = next;
        next = (next == w.dz) ? w.dz2 : w.dz;
    }
    hipLaunchKernelGGL(k_sqsum, dim3(kNormParts), dim3(256), 0, s, (const float *)w.grad, (int64_t)SHMM_SURR_PARAMS,
                       w.gpart);
    SHMM_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, s, (const float *)w.gpart, kNormParts, clip, loss,
                       w.gpart + kNormParts);
    SHMM_HIP_CHECK(hipGetLastError());
    const float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((SHMM_SURR_PARAMS + 255) / 256)), dim3(256), 0, s, m.p, adam,
                       adam + SHMM_SURR_PARAMS_PADDED, (const float *)w.grad, (const float *)(w.gpart + kNormParts),
                       (int64_t)SHMM_SURR_PARAMS, lr, c1, c2, m.ph);
    SHMM_HIP_CHECK(hipGetLastError());
    if (grad_out)
        SHMM_HIP_CHECK(hipMemcpyAsync(grad_out, w.grad, SHMM_SURR_PARAMS * sizeof(float),
                                      hipMemcpyDeviceToDevice, s));
    return SHMM_OK;
}

int surrogate_refresh_bf16(void *model, hipStream_t s) {
    const Model m = model_at(model);
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((SHMM_SURR_PARAMS + 255) / 256)), dim3(256), 0, s,
                       (const float *)m.p, m.ph, (int64_t)SHMM_SURR_PARAMS);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

int surrogate_infer(const void *models, int32_t E, const float *x, const double *Kb, int64_t B,
                    const float *lo, const float *hi, double tau, double emax, double *K_out, uint8_t *flags,
                    double *spread, double *K_members, void *work, hipStream_t s) {
    const NetWork w = carve(work, B);
    double *Km = K_members;
    int rc;
    for (int e = 0; e < E; ++e) {
        const Model m = model_at((char *)models + (size_t)e * SHMM_SURR_MODEL_BYTES);
        if ((rc = net_forward(m, x, B, w, s))) return rc;
        hipLaunchKernelGGL(k_head, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, (const float *)w.o, Kb, B,
                           Km + (size_t)e * B * 3, (const double *)nullptr, (float *)nullptr, (double *)nullptr);
        SHMM_HIP_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_gate, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, (const double *)Km, E, B, x, Kb,
                       lo, hi, tau, emax, K_out, flags, spread);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

// ------------------------------------------------------------------ dataset statistics

namespace {

// Column c of x [B][33]: FP64 mean, standard deviation (divisor B - 1),
// minimum and maximum, one workgroup per column.  Thread t takes rows t,
// t + 256, ...; partial sums meet in a fixed tree, so the result does not
// depend on scheduling.  Two passes (the mean, then the squared deviations).
__global__ __launch_bounds__(256) void k_feature_stats(const float *__restrict__ x, int64_t B,
                                                       double *__restrict__ stats) {
    __shared__ double red[256];
    __shared__ double lo[256], hi[256];
    const int c = blockIdx.x, t = threadIdx.x;
    double sum = 0.0, mn = INFINITY, mx = -INFINITY;
    for (int64_t r = t; r < B; r += 256) {
        const double v = (double)x[r * SHMM_SURR_IN + c];
        sum += v;
        mn = v < mn ? v : mn;
        mx = v > mx ? v : mx;
    }
    red[t] = sum;
    lo[t] = mn;
    hi[t] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            red[t] += red[t + w];
            lo[t] = lo[t + w] < lo[t] ? lo[t + w] : lo[t];
            hi[t] = hi[t + w] > hi[t] ? hi[t + w] : hi[t];
        }
        __syncthreads();
    }
    const double mean = red[0] / (double)B;
    __syncthreads();
    double sq = 0.0;
    for (int64_t r = t; r < B; r += 256) {
        const double d = (double)x[r * SHMM_SURR_IN + c] - mean;
        sq += d * d;
    }
    red[t] = sq;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) {
        stats[c] = mean;
        stats[SHMM_SURR_IN + c] = sqrt(red[0] / (double)(B - 1));
        stats[2 * SHMM_SURR_IN + c] = lo[0];
        stats[3 * SHMM_SURR_IN + c] = hi[0];
    }
}

// Rescaled copy of labelled local problems: velocity and diffusivity scaled
// together by c = 10^log10c[b] leave the corrector unchanged, so K and K_b
// scale by c, the band features (squared Peclet numbers) stay and feature 32
// (log sqrt det K_b) moves by ln c.
__global__ void k_rescale(const float *__restrict__ x, const double *__restrict__ Kb, const double *__restrict__ K,
                          const double *__restrict__ log10c, int64_t B, float *__restrict__ xo,
                          double *__restrict__ Kbo, double *__restrict__ Ko) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double c = exp(log10c[b] * 2.302585092994045684);
    for (int i = 0; i < SHMM_SURR_IN; ++i) {
        const float v = x[b * SHMM_SURR_IN + i];
        xo[b * SHMM_SURR_IN + i] = i == SHMM_SURR_BINS ? (float)((double)v + log(c)) : v;
    }
    for (int q = 0; q < 3; ++q) {
        Kbo[3 * b + q] = Kb[3 * b + q] * c;
        Ko[3 * b + q] = K[3 * b + q] * c;
    }
}

}  // namespace

namespace {

// Chain-aware gate (the surrogate inside Algorithm 3): a finer level's result
// enters its parent's base K_net = K_star - K_off + K_in after K_off is
// subtracted, so its absolute error must stay well below the parent's K_in.
// Flags domain d when spread_d |K_hat_d|_F (the ensemble's largest member
// deviation, absolute) exceeds tol lambda_min(K_in of d's parent); domains
// without a parent keep their flag.
// Bound on the absolute error of an accepted estimate: its predicted change of
// the base plus the ensemble's spread in absolute terms.  The members agree on
// what the features cannot resolve, so the spread alone misses the systematic
// part; where it was measured (finest-level patches) the error stayed below
// the predicted change.  The reference is the smallest K_in of every
// ancestor: an error in a result shifts its parent's base K_net = K_star -
// K_off + K_in, and through the parent's result (nearly its base where the
// enhancement is small) the base of every level above it, down to the
// coarsest, where K_in is kappa I.
__global__ void k_chain_gate(const shmm_domain *__restrict__ dom, int64_t first, int64_t count,
                             const double *__restrict__ K_hat, const double *__restrict__ K_base,
                             const double *__restrict__ spread, const double *__restrict__ K_in, double tol,
                             uint8_t *__restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    int32_t a = dom[first + i].parent;
    if (a < 0) return;
    double lam = INFINITY;
    for (int hops = 0; a >= 0 && hops < 64; ++hops, a = dom[a].parent) {   // levels are far fewer than 64
        const double *kp = K_in + 3 * (int64_t)a;
        const double m = 0.5 * (kp[0] + kp[2]), q = 0.5 * (kp[0] - kp[2]);
        lam = fmin(lam, m - sqrt(q * q + kp[1] * kp[1]));
    }
    const double *k = K_hat + 3 * i, *kb = K_base + 3 * i;
    const double fro = sqrt(k[0] * k[0] + 2.0 * k[1] * k[1] + k[2] * k[2]);
    const double d0 = k[0] - kb[0], d1 = k[1] - kb[1], d2 = k[2] - kb[2];
    const double change = sqrt(d0 * d0 + 2.0 * d1 * d1 + d2 * d2);
    if (!(change + spread[i] * fro <= tol * lam)) flags[i] = 1;
}

}  // namespace

int launch_chain_gate(const shmm_domain *dom, int64_t first, int64_t count, const double *K_hat,
                      const double *K_base, const double *spread, const double *K_in, double tol, uint8_t *flags,
                      hipStream_t s) {
    if (count <= 0) return SHMM_OK;
    hipLaunchKernelGGL(k_chain_gate, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, dom, first, count, K_hat,
                       K_base, spread, K_in, tol, flags);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

int launch_feature_stats(const float *x, int64_t B, double *stats, hipStream_t s) {
    hipLaunchKernelGGL(k_feature_stats, dim3(SHMM_SURR_IN), dim3(256), 0, s, x, B, stats);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

int launch_surrogate_rescale(const float *x, const double *Kb, const double *K, const double *log10c, int64_t B,
                             float *xo, double *Kbo, double *Ko, hipStream_t s) {
    if (B <= 0) return SHMM_OK;
    hipLaunchKernelGGL(k_rescale, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, x, Kb, K, log10c, B, xo,
                       Kbo, Ko);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

}  // namespace shmm
