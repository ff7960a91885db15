// Band filter kernels (Section 3.1): band tags, pruned separable FFT synthesis
// of psi, vx, vy at the patch nodes, cell forcings, and line energies of the
// off-diagonal bands.
#include <algorithm>

#include "band_core.h"

namespace shmm {

namespace {

struct BlockSync {
    __device__ void operator()() const { __syncthreads(); }
};

constexpr int kBandThreads = 256;

__global__ void k_band_tags(InstDev inst, int8_t *tags) {
    const int span = 2 * inst.kmax + 1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)span * span) return;
    const int k2 = (int)(idx / span) - inst.kmax, k1 = (int)(idx % span) - inst.kmax;
    if (k1 == 0 && k2 == 0) {
        tags[idx] = -1;
        return;
    }
    const int l = band_level(k1, k2, inst.thresh, inst.L);
    tags[idx] = (int8_t)(4 * l + band_part(k1, k2, l, inst.thresh, inst.L));
}

__global__ __launch_bounds__(kBandThreads) void k_band_pass1(BandParams p) {
    extern __shared__ c32 lds[];
    band_pass1_block(p, blockIdx.x, lds, lds + p.P1, threadIdx.x, blockDim.x, BlockSync{});
}

__global__ __launch_bounds__(kBandThreads) void k_band_pass2(BandParams p) {
    extern __shared__ c32 lds[];
    band_pass2_block(p, blockIdx.x, lds, lds + p.P2, threadIdx.x, blockDim.x, BlockSync{});
}

// f1 = cell average of the x-face velocities, f2 = of the y-face velocities.
__global__ void k_forcing(const shmm_domain *dom, int64_t first, int n, const float *vx,
                          const float *vy, float *f1, float *f2) {
    const int64_t d = first + blockIdx.y;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t)n * n) return;
    const int64_t o = dom[d].offset;
    const int j = (int)(c / n), i = (int)(c % n);
    const int ie = (i + 1) & (n - 1), jn = (j + 1) & (n - 1);
    f1[o + c] = 0.5f * (vx[o + c] + vx[o + (int64_t)j * n + ie]);
    f2[o + c] = 0.5f * (vy[o + c] + vy[o + (int64_t)jn * n + i]);
}

// The patch is treated as periodic: the faces on its last row and column use
// the wrapped node values (x-face row n-1 pairs node rows n-1 and 0; y-face
// column n-1 pairs node columns n-1 and 0).  Needed only when the band is not
// periodic on the patch; otherwise the synthesised differences already agree.
__global__ void k_seam(const shmm_domain *dom, int64_t first, int n, const float *psi,
                       const int64_t psi_base, float *vx, float *vy) {
    const int64_t d = first + blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = dom[d].offset;
    const float ih = (float)(1.0 / dom[d].h);
    const float *P = psi + (o - psi_base);
    const int64_t last = (int64_t)(n - 1) * n;
    vx[o + last + i] = -(P[i] - P[last + i]) * ih;
    vy[o + (int64_t)i * n + (n - 1)] = (P[(int64_t)i * n] - P[(int64_t)i * n + (n - 1)]) * ih;
}

// Windowed patches: the face velocities of the tapered stream function
// W psi, W = w(x) w(y) on the nodes of each patch, with w 0 on the seam node,
// rising as sin^2 over `taper` nodes and 1 inside (symmetric under
// i -> n - i), so that the periodic extension of W psi is smooth.  The faces
// are differences of that one node field (zero discrete divergence).
__device__ inline float taper_weight(int i, int n, int taper) {
    const int e = i < n - i ? i : n - i;
    if (e >= taper) return 1.0f;
    const double s = sin(0.5 * M_PI * (double)e / (double)taper);
    return (float)(s * s);
}

__global__ void k_taper_faces(const shmm_domain *dom, int64_t first, int n, int taper, const float *psi,
                              float *vx, float *vy) {
    const int64_t d = first + blockIdx.y;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t)n * n) return;
    const int64_t o = dom[d].offset;
    const float ih = (float)(1.0 / dom[d].h);
    const int j = (int)(c / n), i = (int)(c % n);
    const int jn = (j + 1) & (n - 1), ie = (i + 1) & (n - 1);
    const float wj = taper_weight(j, n, taper), wi = taper_weight(i, n, taper);
    const float p = wj * wi * psi[o + c];
    const float pn = taper_weight(jn, n, taper) * wi * psi[o + (int64_t)jn * n + i];
    const float pe = wj * taper_weight(ie, n, taper) * psi[o + (int64_t)j * n + ie];
    vx[o + c] = -(pn - p) * ih;
    vy[o + c] = (pe - p) * ih;
}

// Gershgorin bound of the advection operator of each patch:
// max over cells of (|vx_W| + |vx_E| + |vy_S| + |vy_N|) / 2.
__global__ __launch_bounds__(256) void k_vmax(const shmm_domain *dom, int64_t first, int n, const float *vx,
                                              const float *vy, double *vmax) {
    __shared__ float red[256];
    const int64_t d = first + blockIdx.x;
    const int64_t o = dom[d].offset;
    const int mask = n - 1;
    float m = 0.0f;
    for (int c = threadIdx.x; c < n * n; c += blockDim.x) {
        const int j = c / n, i = c - j * n;
        const float s = fabsf(vx[o + c]) + fabsf(vx[o + (int64_t)j * n + ((i + 1) & mask)]) + fabsf(vy[o + c]) +
                        fabsf(vy[o + (int64_t)((j + 1) & mask) * n + i]);
        m = fmaxf(m, s);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) vmax[d] = 0.5 * (double)red[0];
}

// One thread per (outer wavenumber, line): neighbouring lanes take
// neighbouring lines of the same outer wavenumber, so they read the same
// coefficients.  part[kidx][line].
__global__ void k_line_rows(BandParams p, int cnt, double *part) {
    const int lines = 2 * p.M * p.n;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)cnt * lines) return;
    const int kidx = (int)(t / lines), line = (int)(t - (int64_t)kidx * lines);
    const int per_dir = p.M * p.n;
    const int dir = line / per_dir, r = line - dir * per_dir;
    part[t] = line_row_energy(p, dir, r / p.n, r % p.n, kidx);
}

// Per line: the outer contributions added in increasing k_o (fixed order).
__global__ void k_line_sum(BandParams p, int cnt, const double *part) {
    const int lines = 2 * p.M * p.n;
    const int line = blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= lines) return;
    double total = 0.0;
    for (int kidx = 0; kidx < cnt; ++kidx) total += part[(int64_t)kidx * lines + line];
    const int per_dir = p.M * p.n;
    const int dir = line / per_dir, r = line - dir * per_dir;
    line_store(p, dir, r / p.n, r % p.n, total);
}

int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

int launch_band_tags(const InstDev &inst, int8_t *d_tags, hipStream_t s) {
    const int64_t total = (int64_t)(2 * inst.kmax + 1) * (2 * inst.kmax + 1);
    hipLaunchKernelGGL(k_band_tags, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, inst, d_tags);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

static void fill_params(BandParams &p, const InstDev &inst, const Group &g) {
    p.inst = inst;
    p.level = g.level;
    p.N = g.N;
    p.n = g.n;
    p.M = g.M;
    p.kb1 = g.kb1;
    p.kb2 = g.kb2;
    p.P1 = next_pow2(2 * g.kb2 + 1);
    p.R1 = g.N / p.P1;
    p.P2 = next_pow2(g.kb1 + 1);
    p.R2 = g.N / p.P2;
    p.first = g.first;
}

static size_t line_part_offset(const Group &g) {
    return (size_t)3 * (g.kb1 + 1) * g.M * g.n * sizeof(c32) + (size_t)g.count * g.n * g.n * sizeof(float);
}

size_t band_filter_workspace(const InstDev &inst, const Group &g) {
    // G[3][kb1 + 1][M n], psi of the group's cells when the caller wants none,
    // then the line-energy contributions [outer wavenumbers][2 M n] (FP64)
    return line_part_offset(g) + (size_t)line_outer_count(inst, g.level) * 2 * g.M * g.n * sizeof(double);
}

int launch_window_patches(const shmm_domain *d_dom, int64_t first, int64_t count, int n, int taper,
                          const float *d_psi, float *d_vx, float *d_vy, float *d_f1, float *d_f2, double *d_vmax,
                          hipStream_t s) {
    if (count <= 0 || taper <= 0) return SHMM_OK;
    const int cells = n * n;
    for (int64_t c0 = 0; c0 < count; c0 += 65535) {
        const int64_t cn = std::min<int64_t>(65535, count - c0);
        const dim3 grid((unsigned)((cells + 255) / 256), (unsigned)cn);
        hipLaunchKernelGGL(k_taper_faces, grid, dim3(256), 0, s, d_dom, first + c0, n, taper, d_psi, d_vx, d_vy);
        SHMM_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_forcing, grid, dim3(256), 0, s, d_dom, first + c0, n, (const float *)d_vx,
                           (const float *)d_vy, d_f1, d_f2);
        SHMM_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_vmax, dim3((unsigned)cn), dim3(256), 0, s, d_dom, first + c0, n, (const float *)d_vx,
                           (const float *)d_vy, d_vmax);
        SHMM_HIP_CHECK(hipGetLastError());
    }
    return SHMM_OK;
}

int launch_band_filter(const InstDev &inst, const Group &g, const shmm_domain *d_dom, float *d_psi,
                       float *d_vx, float *d_vy, float *d_f1, float *d_f2, double *d_lines,
                       double *d_vmax, void *work, size_t work_bytes, hipStream_t s) {
    BandParams p;
    fill_params(p, inst, g);
    if (p.P1 > 4096 || p.P2 > 4096 || p.P1 > g.N || p.P2 > g.N) return SHMM_ERANGE;
    if (work_bytes < band_filter_workspace(inst, g)) return SHMM_ENOMEM;
    p.dom = d_dom;
    p.I0 = g.d_I0;
    p.J0 = g.d_J0;
    p.G = (c32 *)work;
    // psi is needed for the seam faces of non-periodic patches
    float *psi_buf = d_psi;
    int64_t psi_base = 0;
    if (!d_psi && !g.periodic) {
        psi_base = g.cell_first;
        psi_buf = (float *)((char *)work + (size_t)3 * (g.kb1 + 1) * g.M * g.n * sizeof(c32));
        p.out[0] = psi_buf - psi_base;
    } else {
        p.out[0] = d_psi;
    }
    p.out[1] = d_vx;
    p.out[2] = d_vy;
    p.chan_first = (d_psi || !g.periodic) ? 0 : 1;
    p.lines = d_lines;
    const size_t lds1 = 2 * (size_t)p.P1 * sizeof(c32), lds2 = 2 * (size_t)p.P2 * sizeof(c32);
    hipLaunchKernelGGL(k_band_pass1, dim3((unsigned)((g.kb1 + 1) * p.R1)), dim3(kBandThreads), lds1,
                       s, p);
    SHMM_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_band_pass2, dim3((unsigned)(g.M * g.n * p.R2)), dim3(kBandThreads), lds2, s,
                       p);
    SHMM_HIP_CHECK(hipGetLastError());
    if (!g.periodic) {
        hipLaunchKernelGGL(k_seam, dim3((unsigned)((g.n + 63) / 64), (unsigned)g.count), dim3(64), 0, s,
                           d_dom, g.first, g.n, (const float *)psi_buf, psi_base, d_vx, d_vy);
        SHMM_HIP_CHECK(hipGetLastError());
    }
    const int cells = g.n * g.n;
    hipLaunchKernelGGL(k_forcing, dim3((unsigned)((cells + 255) / 256), (unsigned)g.count), dim3(256),
                       0, s, d_dom, g.first, g.n, d_vx, d_vy, d_f1, d_f2);
    SHMM_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_vmax, dim3((unsigned)g.count), dim3(256), 0, s, d_dom, g.first, g.n, (const float *)d_vx,
                       (const float *)d_vy, d_vmax);
    SHMM_HIP_CHECK(hipGetLastError());
    const int lines = 2 * g.M * g.n;
    const int cnt = line_outer_count(inst, g.level);
    double *part = (double *)((char *)work + line_part_offset(g));
    if (cnt > 0) {
        const int64_t rows = (int64_t)cnt * lines;
        hipLaunchKernelGGL(k_line_rows, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, p, cnt, part);
        SHMM_HIP_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_line_sum, dim3((unsigned)((lines + 255) / 256)), dim3(256), 0, s, p, cnt,
                       (const double *)part);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

}  // namespace shmm
