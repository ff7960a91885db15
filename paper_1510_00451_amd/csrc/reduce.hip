// Effective diffusivity (the K formula after eq:homo; HMM step 3) and the
// level combination of Algorithms 1-3, in FP64.
#include "shmm_internal.h"

namespace shmm {

namespace {

constexpr int kRedThreads = 256;
constexpr int kRedVals = 11;   // p11 p12 p21 p22 m1 m2 e11 e12 e21 e22 bad

// Fixed-order butterfly over the 64 lanes of a wavefront.
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(kRedThreads) void k_moments(
    const shmm_domain *__restrict__ dom, int64_t first, const float *__restrict__ f1,
    const float *__restrict__ f2, const float *__restrict__ w, int64_t cells_total,
    const double *__restrict__ Kb, double *__restrict__ K_out, double *__restrict__ K_energy,
    double *__restrict__ mass, int32_t *__restrict__ status, const int32_t *__restrict__ list, int32_t inner) {
    __shared__ double part[kRedThreads / 64][kRedVals];
    const int64_t d = list ? (int64_t)list[blockIdx.x] : first + blockIdx.x;
    const shmm_domain D = dom[d];
    const int n = D.n, mask = n - 1;
    // averaging window: the centred m x m cells (the whole patch when inner
    // is 0 or not below n)
    const int m = inner > 0 && inner < n ? inner : n, x0 = (n - m) / 2, cells = m * m;
    const int64_t o = D.offset;
    const double K11 = Kb[3 * d], K12 = Kb[3 * d + 1], K22 = Kb[3 * d + 2];
    const double ih2 = 1.0 / (D.h * D.h);
    const float *w1 = w + o, *w2 = w + cells_total + o;
    double v[kRedVals];
#pragma unroll
    for (int q = 0; q < kRedVals; ++q) v[q] = 0.0;
    for (int i = threadIdx.x; i < cells; i += kRedThreads) {
        const int yi = i / m, y = x0 + yi, x = x0 + (i - yi * m), c = y * n + x;
        const int xe = (x + 1) & mask, xw = (x - 1) & mask, yn = (y + 1) & mask, ys = (y - 1) & mask;
        const double a1 = f1[o + c], a2 = f2[o + c];
        const double u1 = w1[c], u2 = w2[c];
        v[0] += a1 * u1;
        v[1] += a1 * u2;
        v[2] += a2 * u1;
        v[3] += a2 * u2;
        v[4] += u1;
        v[5] += u2;
        double D1, D2;
        {
            const float *u = w1;
            D1 = (K11 * ((double)u[y * n + xe] - 2.0 * u1 + (double)u[y * n + xw]) +
                  K22 * ((double)u[yn * n + x] - 2.0 * u1 + (double)u[ys * n + x]) +
                  0.5 * K12 * (((double)u[yn * n + xe] - (double)u[yn * n + xw]) -
                               ((double)u[ys * n + xe] - (double)u[ys * n + xw]))) * ih2;
            u = w2;
            D2 = (K11 * ((double)u[y * n + xe] - 2.0 * u2 + (double)u[y * n + xw]) +
                  K22 * ((double)u[yn * n + x] - 2.0 * u2 + (double)u[ys * n + x]) +
                  0.5 * K12 * (((double)u[yn * n + xe] - (double)u[yn * n + xw]) -
                               ((double)u[ys * n + xe] - (double)u[ys * n + xw]))) * ih2;
        }
        v[6] += u1 * D1;
        v[7] += u1 * D2;
        v[8] += u2 * D1;
        v[9] += u2 * D2;
        if (!isfinite(u1) || !isfinite(u2)) v[10] = 1.0;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kRedVals; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) part[wave][q] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[kRedVals];
        for (int q = 0; q < kRedVals; ++q) {
            t[q] = 0.0;
            for (int wv = 0; wv < kRedThreads / 64; ++wv) t[q] += part[wv][q];
        }
        const double inv = 1.0 / (double)cells;
        K_out[3 * d + 0] = K11 + t[0] * inv;
        K_out[3 * d + 1] = K12 + 0.5 * (t[1] + t[2]) * inv;
        K_out[3 * d + 2] = K22 + t[3] * inv;
        if (K_energy) {
            K_energy[3 * d + 0] = K11 - t[6] * inv;
            K_energy[3 * d + 1] = K12 - 0.5 * (t[7] + t[8]) * inv;
            K_energy[3 * d + 2] = K22 - t[9] * inv;
        }
        if (mass) {
            mass[2 * d + 0] = t[4];
            mass[2 * d + 1] = t[5];
        }
        const bool bad = t[10] != 0.0 || !isfinite(t[0]) || !isfinite(t[1]) || !isfinite(t[2]) ||
                         !isfinite(t[3]);
        if (status && bad) status[d] |= SHMM_DOM_NONFINITE;
    }
}

// Change of both correctors over the last chunk of steps, for the adaptive
// stop of the local solves: out[8 i + q] for domain first + i holds the sums
// over its cells of (w_j - w_prev_j)^2 (q = 0, 1), f_j^2 (q = 2, 3) and
// f_i w_j (q = 4 + 2 (i - 1) + (j - 1)), FP64 in a fixed order; then
// w_prev <- w.  w_prev covers the listed domains only: [2][prev_cells], cell
// c of domain first + i at d.offset - prev_base + c, or with a list (domains
// of one size) cell c of list entry i at i n^2 + c.
constexpr int kDeltaVals = 8;

__global__ __launch_bounds__(kRedThreads) void k_chunk_delta(
    const shmm_domain *__restrict__ dom, int64_t first, const float *__restrict__ f1,
    const float *__restrict__ f2, const float *__restrict__ w, int64_t cells_total, float *__restrict__ w_prev,
    int64_t prev_cells, int64_t prev_base, const int32_t *__restrict__ list, double *__restrict__ out) {
    __shared__ double part[kRedThreads / 64][kDeltaVals];
    const shmm_domain D = dom[list ? (int64_t)list[blockIdx.x] : first + blockIdx.x];
    const int cells = D.n * D.n;
    const int64_t o = D.offset, po = list ? (int64_t)blockIdx.x * cells : D.offset - prev_base;
    double v[kDeltaVals];
#pragma unroll
    for (int q = 0; q < kDeltaVals; ++q) v[q] = 0.0;
    for (int c = threadIdx.x; c < cells; c += kRedThreads) {
        const float a = w[o + c], b = w[cells_total + o + c];
        const double da = (double)a - (double)w_prev[po + c];
        const double db = (double)b - (double)w_prev[prev_cells + po + c];
        const double g1 = f1[o + c], g2 = f2[o + c];
        v[0] += da * da;
        v[1] += db * db;
        v[2] += g1 * g1;
        v[3] += g2 * g2;
        v[4] += g1 * (double)a;
        v[5] += g1 * (double)b;
        v[6] += g2 * (double)a;
        v[7] += g2 * (double)b;
        w_prev[po + c] = a;
        w_prev[prev_cells + po + c] = b;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kDeltaVals; ++q) {
        const double t = wave_sum(v[q]);
        if (lane == 0) part[wave][q] = t;
    }
    __syncthreads();
    if (threadIdx.x < kDeltaVals) {
        double t = 0.0;
        for (int wv = 0; wv < kRedThreads / 64; ++wv) t += part[wv][threadIdx.x];
        out[kDeltaVals * (int64_t)blockIdx.x + threadIdx.x] = t;
    }
}

// Algorithm 1: line-wise shear formula (eq:shearhomoY for the columns of the
// off-12 band, eq:shearhomoX for the rows of the off-21 band), then the
// harmonic mean across lines; the other diagonal entry and K12 pass through.
__device__ inline void offdiag(const double *K, const double *s, int n, int dir, double *out) {
    double acc = 0.0;
    if (dir == 0) {
        for (int i = 0; i < n; ++i) acc += 1.0 / (K[0] + s[i] / K[2]);
        out[0] = (double)n / acc;
        out[1] = K[1];
        out[2] = K[2];
    } else {
        for (int i = 0; i < n; ++i) acc += 1.0 / (K[2] + s[i] / K[0]);
        out[0] = K[0];
        out[1] = K[1];
        out[2] = (double)n / acc;
    }
}

__device__ inline double lam_min(const double *K) {
    const double m = 0.5 * (K[0] + K[2]), q = 0.5 * (K[0] - K[2]);
    return m - sqrt(q * q + K[1] * K[1]);
}

__global__ void k_chain(const shmm_domain *__restrict__ dom, const InstDev *__restrict__ insts,
                        const int32_t *__restrict__ child_start, const int32_t *__restrict__ child_idx,
                        int64_t first, int64_t count, int32_t mode, const double *__restrict__ lines,
                        double *K_in, double *K_off, double *K_base, const double *__restrict__ K_solve,
                        double *R, int32_t *status) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const int64_t d = first + t;
    const shmm_domain D = dom[d];
    const InstDev I = insts[D.instance];
    const bool finest = D.level == I.L - 1;
    const double *s12 = lines + D.line_offset, *s21 = s12 + D.n;
    double a[3], b[3];
    if (mode == 0) {
        double kin[3];
        if (D.level == 0) {
            kin[0] = I.kappa; kin[1] = 0.0; kin[2] = I.kappa;
        } else {
            for (int q = 0; q < 3; ++q) kin[q] = K_off[3 * (int64_t)D.parent + q];
        }
        for (int q = 0; q < 3; ++q) K_in[3 * d + q] = kin[q];
        if (!finest) {
            offdiag(kin, s12, D.n, 0, a);
            offdiag(kin, s21, D.n, 1, b);
            for (int q = 0; q < 3; ++q) K_off[3 * d + q] = a[q] + b[q] - kin[q];
        }
    } else if (mode == 1) {
        if (finest) {
            for (int q = 0; q < 3; ++q) K_base[3 * d + q] = K_in[3 * d + q];
            return;
        }
        double ks[3] = {0.0, 0.0, 0.0};
        const int c0 = child_start[d], c1 = child_start[d + 1];
        for (int c = c0; c < c1; ++c)
            for (int q = 0; q < 3; ++q) ks[q] += R[3 * (int64_t)child_idx[c] + q];
        double kb[3];
        for (int q = 0; q < 3; ++q) kb[q] = ks[q] / (double)(c1 - c0) - K_off[3 * d + q] + K_in[3 * d + q];
        const double floor = lam_min(K_in + 3 * d);
        if (!(lam_min(kb) >= floor) || !(kb[0] > 0.0)) {
            // clamp the eigenvalues of the symmetric 2x2 to at least lambda_min(K_in)
            const double m = 0.5 * (kb[0] + kb[2]), q = 0.5 * (kb[0] - kb[2]);
            const double r = sqrt(q * q + kb[1] * kb[1]);
            double l1 = m + r, l2 = m - r;
            double cth = 1.0, sth = 0.0;
            if (r > 0.0) {
                const double ang = 0.5 * atan2(2.0 * kb[1], kb[0] - kb[2]);
                cth = cos(ang);
                sth = sin(ang);
            }
            l1 = l1 > floor ? l1 : floor;
            l2 = l2 > floor ? l2 : floor;
            if (!isfinite(l1) || !isfinite(l2)) l1 = l2 = floor, cth = 1.0, sth = 0.0;
            kb[0] = l1 * cth * cth + l2 * sth * sth;
            kb[1] = (l1 - l2) * cth * sth;
            kb[2] = l1 * sth * sth + l2 * cth * cth;
            if (status) status[d] |= SHMM_DOM_NOT_SPD;
        }
        for (int q = 0; q < 3; ++q) K_base[3 * d + q] = kb[q];
    } else if (mode == 3) {
        // macro diffusivity: the level without its own diagonal band
        const double *kn = K_base + 3 * d;
        if (finest) {
            for (int q = 0; q < 3; ++q) R[3 * d + q] = kn[q];
            return;
        }
        offdiag(kn, s12, D.n, 0, a);
        offdiag(kn, s21, D.n, 1, b);
        for (int q = 0; q < 3; ++q) R[3 * d + q] = a[q] + b[q] - kn[q];
    } else {
        if (finest) {
            for (int q = 0; q < 3; ++q) R[3 * d + q] = K_solve[3 * d + q];
            return;
        }
        const double *kn = K_base + 3 * d;
        offdiag(kn, s12, D.n, 0, a);
        offdiag(kn, s21, D.n, 1, b);
        for (int q = 0; q < 3; ++q) R[3 * d + q] = K_solve[3 * d + q] + a[q] + b[q] - 2.0 * kn[q];
    }
}

__global__ void k_mark(int32_t *status, const int32_t *list, int64_t count, int32_t bits) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) status[list[t]] |= bits;
}

// Non-finite check of the corrector fields of listed domains of one size n:
// one workgroup per domain reads both correctors (float4) and ORs
// SHMM_DOM_NONFINITE into the domain's status word if any value is NaN/Inf.
__global__ __launch_bounds__(256) void k_nonfinite(const shmm_domain *__restrict__ dom,
                                                   const int32_t *__restrict__ list, int n,
                                                   const float *__restrict__ w, int64_t cells,
                                                   int32_t *status) {
    const int32_t d = list[blockIdx.x];
    const int64_t o = dom[d].offset;
    const int64_t nn = (int64_t)n * n;
    int bad = 0;
    if ((o & 3) == 0 && (cells & 3) == 0 && (nn & 3) == 0) {
        const float4 *a = reinterpret_cast<const float4 *>(w + o);
        const float4 *b = reinterpret_cast<const float4 *>(w + cells + o);
        for (int64_t c = threadIdx.x; c < nn / 4; c += blockDim.x) {
            const float4 x = a[c], y = b[c];
            bad |= !isfinite(x.x) | !isfinite(x.y) | !isfinite(x.z) | !isfinite(x.w);
            bad |= !isfinite(y.x) | !isfinite(y.y) | !isfinite(y.z) | !isfinite(y.w);
        }
    } else {
        for (int64_t c = threadIdx.x; c < nn; c += blockDim.x)
            bad |= !isfinite(w[o + c]) | !isfinite(w[cells + o + c]);
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0 && bad) atomicOr(status + d, (int32_t)SHMM_DOM_NONFINITE);
}

}  // namespace

int launch_mark_status(int32_t *status, const int32_t *list, int64_t count, int32_t bits, hipStream_t s) {
    if (count <= 0) return SHMM_OK;
    hipLaunchKernelGGL(k_mark, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, status, list, count, bits);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

int launch_mark_nonfinite(const shmm_domain *d_dom, const int32_t *d_list, int32_t nlist, int n, const float *w,
                          int64_t cells_total, int32_t *status, hipStream_t s) {
    if (nlist <= 0 || !status) return SHMM_OK;
    hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)nlist), dim3(256), 0, s, d_dom, d_list, n, w, cells_total,
                       status);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

int launch_effective_diffusivity(const shmm_domain *d_dom, int64_t first, int64_t count,
                                 const float *f1, const float *f2, const float *w,
                                 int64_t cells_total, const double *Kb, double *K_out,
                                 double *K_energy, double *mass, int32_t *status, hipStream_t s) {
    if (count <= 0) return SHMM_OK;
    hipLaunchKernelGGL(k_moments, dim3((unsigned)count), dim3(kRedThreads), 0, s, d_dom, first, f1, f2,
                       w, cells_total, Kb, K_out, K_energy, mass, status, (const int32_t *)nullptr, 0);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

int launch_effective_diffusivity_window(const shmm_domain *d_dom, int64_t first, int64_t count, int32_t inner,
                                        const float *f1, const float *f2, const float *w, int64_t cells_total,
                                        const double *Kb, double *K_out, int32_t *status, hipStream_t s) {
    if (count <= 0) return SHMM_OK;
    hipLaunchKernelGGL(k_moments, dim3((unsigned)count), dim3(kRedThreads), 0, s, d_dom, first, f1, f2, w,
                       cells_total, Kb, K_out, (double *)nullptr, (double *)nullptr, status,
                       (const int32_t *)nullptr, inner);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

int launch_chunk_delta(const shmm_domain *d_dom, int64_t first, const int32_t *d_list, int64_t count, const float *f1,
                       const float *f2, const float *w, int64_t cells_total, float *w_prev, int64_t prev_cells,
                       int64_t prev_base, double *out, hipStream_t s) {
    if (count <= 0) return SHMM_OK;
    hipLaunchKernelGGL(k_chunk_delta, dim3((unsigned)count), dim3(kRedThreads), 0, s, d_dom, first, f1, f2, w,
                       cells_total, w_prev, prev_cells, prev_base, d_list, out);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

int launch_effective_diffusivity_list(const shmm_domain *d_dom, const int32_t *d_list, int64_t count,
                                      const float *f1, const float *f2, const float *w, int64_t cells_total,
                                      const double *Kb, double *K_out, int32_t *status, hipStream_t s) {
    if (count <= 0) return SHMM_OK;
    hipLaunchKernelGGL(k_moments, dim3((unsigned)count), dim3(kRedThreads), 0, s, d_dom, (int64_t)0, f1, f2, w,
                       cells_total, Kb, K_out, (double *)nullptr, (double *)nullptr, status, d_list, 0);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

int launch_level_chain(const shmm_domain *d_dom, const InstDev *d_inst, const int32_t *d_child_start,
                       const int32_t *d_child_idx, int64_t first, int64_t count, int32_t mode,
                       const double *lines, double *K_in, double *K_off, double *K_base,
                       const double *K_solve, double *R, int32_t *status, hipStream_t s) {
    if (count <= 0) return SHMM_OK;
    hipLaunchKernelGGL(k_chain, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, s, d_dom, d_inst,
                       d_child_start, d_child_idx, first, count, mode, lines, K_in, K_off, K_base,
                       K_solve, R, status);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

}  // namespace shmm
