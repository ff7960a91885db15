// Band filter (Section 3.1): per-block logic of the pruned separable Fourier
// synthesis and of the off-diagonal line energies.
//
// Each function is the work of one thread block, written as a loop over the
// block's threads (tid = 0 .. nt-1) with a barrier functor between passes, so
// the kernels in band.hip run it with the hardware barrier and a host harness
// can run the same code with nt = 1 and no barrier.
#pragma once

#include <math.h>
#include <stdint.h>

#include "shmm_internal.h"

namespace shmm {

struct c32 {
    float x, y;
};

__host__ __device__ inline c32 cmul(c32 a, c32 b) {
    return c32{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__host__ __device__ inline void sincospi_f32(float x, float *s, float *c) {
#ifdef __HIP_DEVICE_COMPILE__
    sincospif(x, s, c);
#else
    *s = (float)sin(M_PI * (double)x);
    *c = (float)cos(M_PI * (double)x);
#endif
}

__host__ __device__ inline void sincospi_f64(double x, double *s, double *c) {
#ifdef __HIP_DEVICE_COMPILE__
    sincospi(x, s, c);
#else
    *s = sin(M_PI * x);
    *c = cos(M_PI * x);
#endif
}

// Unnormalised inverse DFT of length P (a power of two),
//   out[j] = sum_k in[k] exp(+2 pi i k j / P),
// by Stockham autosort passes of radix 4 (radix 2 for a leftover factor).
// Pass with sub-transform length Ns: butterfly j reads in[j + r P/R],
// r < R, twiddles it by exp(2 pi i (j mod Ns) r / (Ns R)), and writes the R-point
// DFT to out[(j div Ns) Ns R + (j mod Ns) + m Ns].  a and b are ping-pong
// buffers; the result buffer is returned.
template <class Sync>
__host__ __device__ c32 *fft_inverse(c32 *a, c32 *b, int P, int tid, int nt, Sync sync) {
    for (int Ns = 1; Ns < P;) {
        const int radix = ((P / Ns) % 4 == 0) ? 4 : 2;
        const int nb = P / radix;
        for (int j = tid; j < nb; j += nt) {
            const int k = j & (Ns - 1);
            const int base = (j - k) * radix + k;
            if (radix == 4) {
                c32 v0 = a[j], v1 = a[j + nb], v2 = a[j + 2 * nb], v3 = a[j + 3 * nb];
                if (k) {
                    const float f = (float)k / (float)(2 * Ns);  // angle / pi of r = 1
                    float s, c;
                    sincospi_f32(f, &s, &c);
                    v1 = cmul(v1, c32{c, s});
                    sincospi_f32(2.0f * f, &s, &c);
                    v2 = cmul(v2, c32{c, s});
                    sincospi_f32(3.0f * f, &s, &c);
                    v3 = cmul(v3, c32{c, s});
                }
                const c32 s02{v0.x + v2.x, v0.y + v2.y}, d02{v0.x - v2.x, v0.y - v2.y};
                const c32 s13{v1.x + v3.x, v1.y + v3.y}, d13{v1.x - v3.x, v1.y - v3.y};
                b[base] = c32{s02.x + s13.x, s02.y + s13.y};
                b[base + Ns] = c32{d02.x - d13.y, d02.y + d13.x};           // d02 + i d13
                b[base + 2 * Ns] = c32{s02.x - s13.x, s02.y - s13.y};
                b[base + 3 * Ns] = c32{d02.x + d13.y, d02.y - d13.x};       // d02 - i d13
            } else {
                c32 v0 = a[j], v1 = a[j + nb];
                if (k) {
                    float s, c;
                    sincospi_f32((float)k / (float)Ns, &s, &c);
                    v1 = cmul(v1, c32{c, s});
                }
                b[base] = c32{v0.x + v1.x, v0.y + v1.y};
                b[base + Ns] = c32{v0.x - v1.x, v0.y - v1.y};
            }
        }
        sync();
        c32 *t = a;
        a = b;
        b = t;
        Ns *= radix;
    }
    return a;
}

// Parameters of the synthesis of one (instance, level) group.
//
// The level's diagonal band B has |k1| <= kb1, |k2| <= kb2 and psi is real, so
//   psi(x, y) = Re[ g_0(y) + 2 sum_{k1 > 0} g_{k1}(y) e^{i k1 x} ],
//   g_{k1}(y) = sum_{k2} c(k1, k2) e^{i k2 y}.
// Both sums are needed only at the patch nodes, a subset of the level grid
// x = 2 pi I / N.  A length-N DFT whose input is supported on |k| <= K is
// evaluated at I = I_a R + I_b (R = N / P, P >= 2K + 1) as R DFTs of length P of
// the inputs c(k) e^{2 pi i k I_b / N}; outputs not on a patch are dropped.
// Channels: 0 = psi at the nodes, 1 = vx, 2 = vy, whose coefficients are
// c(k) times the exact difference symbols -(e^{i k2 h} - 1)/h and
// (e^{i k1 h} - 1)/h (computed in FP64 before rounding).
struct BandParams {
    InstDev inst;
    int32_t level;
    int32_t N, n, M;
    int32_t kb1, kb2;
    int32_t P1, R1, P2, R2;
    int32_t chan_first;         // 0 if psi is wanted, else 1
    int64_t first;              // first domain of the group in the table
    const shmm_domain *dom;     // the table
    const int32_t *I0;          // [M] node origin of lattice column qx
    const int32_t *J0;          // [M] node origin of lattice row qy
    c32 *G;                     // [3][kb1 + 1][M n] pass-1 output
    float *out[3];              // psi (may be null), vx, vy: packed per domain
    double *lines;              // packed line energies
};

// Pass 1 (along x2): block (k1, J_b).  a, b hold P1 complex values each.
template <class Sync>
__host__ __device__ void band_pass1_block(const BandParams &p, int blk, c32 *a, c32 *b, int tid,
                                          int nt, Sync sync) {
    const int k1 = blk / p.R1;
    const int Jb = blk % p.R1;
    const int span = 2 * p.inst.kmax + 1;
    const int slots = p.M * p.n;
    const double h = 2.0 * M_PI / (double)p.N;
    for (int ch = p.chan_first; ch < 3; ++ch) {
        for (int t = tid; t < p.P1; t += nt) a[t] = c32{0.0f, 0.0f};
        sync();
        for (int k2 = -p.kb2 + tid; k2 <= p.kb2; k2 += nt) {
            if (band_level(k1, k2, p.inst.thresh, p.inst.L) != p.level) continue;
            if (band_part(k1, k2, p.level, p.inst.thresh, p.inst.L) != SHMM_DIAG) continue;
            if (k1 > p.inst.kmax || k2 > p.inst.kmax || k2 < -p.inst.kmax) continue;
            const int64_t idx = (int64_t)(k2 + p.inst.kmax) * span + (k1 + p.inst.kmax);
            double re = p.inst.psi_hat[2 * idx], im = p.inst.psi_hat[2 * idx + 1];
            if (ch > 0) {
                // e^{i theta} - 1 = -2 sin^2(theta/2) + i sin(theta), theta = k h = 2 pi k / N
                const int k = ch == 1 ? k2 : k1;
                double s, c;
                sincospi_f64((double)k / (double)p.N, &s, &c);
                double mr = -2.0 * s * s / h, mi = 2.0 * s * c / h;
                if (ch == 1) { mr = -mr; mi = -mi; }
                const double tr = re * mr - im * mi, ti = re * mi + im * mr;
                re = tr;
                im = ti;
            }
            int64_t r = ((int64_t)k2 * Jb) % p.N;
            if (r < 0) r += p.N;
            double ts, tc;
            sincospi_f64(2.0 * (double)r / (double)p.N, &ts, &tc);
            a[(k2 + p.P1) & (p.P1 - 1)] = c32{(float)(re * tc - im * ts), (float)(re * ts + im * tc)};
        }
        sync();
        c32 *res = fft_inverse(a, b, p.P1, tid, nt, sync);
        c32 *G = p.G + ((int64_t)ch * (p.kb1 + 1) + k1) * slots;
        for (int t = tid; t < slots; t += nt) {
            const int qy = t / p.n, j = t - qy * p.n;
            const int J = (p.J0[qy] + j) % p.N;
            if (J % p.R1 != Jb) continue;
            G[t] = res[J / p.R1];
        }
        sync();
    }
}

// Pass 2 (along x1): block (slot, I_b).  a, b hold P2 complex values each.
template <class Sync>
__host__ __device__ void band_pass2_block(const BandParams &p, int blk, c32 *a, c32 *b, int tid,
                                          int nt, Sync sync) {
    const int slot = blk / p.R2;
    const int Ib = blk % p.R2;
    const int slots = p.M * p.n;
    const int qy = slot / p.n, j = slot - qy * p.n;
    for (int ch = p.chan_first; ch < 3; ++ch) {
        for (int t = tid; t < p.P2; t += nt) a[t] = c32{0.0f, 0.0f};
        sync();
        const c32 *G = p.G + (int64_t)ch * (p.kb1 + 1) * slots;
        for (int k1 = tid; k1 <= p.kb1; k1 += nt) {
            const c32 g = G[(int64_t)k1 * slots + slot];
            const float wgt = k1 == 0 ? 1.0f : 2.0f;
            const int64_t r = ((int64_t)k1 * Ib) % p.N;
            float s, c;
            sincospi_f32(2.0f * (float)r / (float)p.N, &s, &c);
            const c32 v = cmul(g, c32{c, s});
            a[k1] = c32{wgt * v.x, wgt * v.y};
        }
        sync();
        c32 *res = fft_inverse(a, b, p.P2, tid, nt, sync);
        float *out = p.out[ch];
        for (int t = tid; t < slots; t += nt) {
            const int qx = t / p.n, i = t - qx * p.n;
            const int I = (p.I0[qx] + i) % p.N;
            if (I % p.R2 != Ib) continue;
            const shmm_domain &d = p.dom[p.first + (int64_t)qy * p.M + qx];
            out[d.offset + (int64_t)j * p.n + i] = res[I / p.R2].x;
        }
        sync();
    }
}

// Number of outer wavenumbers of a level's off-diagonal bands: |k_o| in
// (a_l, kmax] on both signs (0 at the last level).
__host__ __device__ inline int line_outer_count(const InstDev &inst, int lev) {
    if (lev >= inst.L - 1) return 0;
    const int out_lo = inst.thresh[lev] + 1;
    return inst.kmax >= out_lo ? 2 * (inst.kmax - out_lo + 1) : 0;
}

// Contribution of one outer wavenumber to the energy of one line (Algorithm 1
// with eq:shearhomoY / eq:shearhomoX, by Parseval): |sum over the inner
// wavenumbers of psi_hat e^{i k_in x}|^2.  dir 0 = column x1 = pi (2 (I0[q] +
// i) + 1) / N of the off-12 band (inner index k1, outer k2); dir 1 = row of the
// off-21 band (inner k2, outer k1).  kidx enumerates the outer wavenumbers in
// increasing order (-kmax .. -out_lo, then out_lo .. kmax).
__host__ __device__ inline double line_row_energy(const BandParams &p, int dir, int q, int i, int kidx) {
    const int lev = p.level, kmax = p.inst.kmax;
    const int in_lo = lev == 0 ? 0 : p.inst.thresh[lev - 1] + 1;
    const int in_hi = p.inst.thresh[lev] < kmax ? p.inst.thresh[lev] : kmax;
    const int out_lo = p.inst.thresh[lev] + 1;
    if (in_lo > in_hi) return 0.0;
    const int half = kmax - out_lo + 1;
    const int ko = kidx < half ? -kmax + kidx : out_lo + (kidx - half);
    const int span = 2 * kmax + 1;
    const int64_t twoI1 = 2 * (int64_t)((dir == 0 ? p.I0[q] : p.J0[q]) + i) + 1;
    const int64_t twoN = 2 * (int64_t)p.N;
    const int64_t rs = twoI1 % twoN;
    double ss, sc;
    sincospi_f64((double)rs / (double)p.N, &ss, &sc);   // e^{i x}
    int64_t r0 = ((-(int64_t)in_hi) * twoI1) % twoN;
    if (r0 < 0) r0 += twoN;
    double er, ei;
    sincospi_f64((double)r0 / (double)p.N, &ei, &er);   // e^{-i in_hi x}
    double sr = 0.0, si = 0.0;
    for (int ki = -in_hi; ki <= in_hi; ++ki) {
        const int aki = ki < 0 ? -ki : ki;
        if (aki >= in_lo) {
            const int k1 = dir == 0 ? ki : ko, k2 = dir == 0 ? ko : ki;
            const int64_t idx = (int64_t)(k2 + kmax) * span + (k1 + kmax);
            const double pr = p.inst.psi_hat[2 * idx], pi = p.inst.psi_hat[2 * idx + 1];
            sr += pr * er - pi * ei;
            si += pr * ei + pi * er;
        }
        const double nr = er * sc - ei * ss, ni = er * ss + ei * sc;
        er = nr;
        ei = ni;
    }
    return sr * sr + si * si;
}

// Write the energy of one line to every domain of the group that contains it.
__host__ __device__ inline void line_store(const BandParams &p, int dir, int q, int i, double total) {
    for (int o = 0; o < p.M; ++o) {
        const int64_t local = dir == 0 ? (int64_t)o * p.M + q : (int64_t)q * p.M + o;
        const shmm_domain &d = p.dom[p.first + local];
        p.lines[d.line_offset + (dir == 0 ? 0 : p.n) + i] = total;
    }
}

// Energy of one line: the outer contributions added in increasing k_o.
__host__ __device__ inline void line_energy_one(const BandParams &p, int dir, int q, int i) {
    double total = 0.0;
    const int cnt = line_outer_count(p.inst, p.level);
    for (int kidx = 0; kidx < cnt; ++kidx) total += line_row_energy(p, dir, q, i, kidx);
    line_store(p, dir, q, i, total);
}

}  // namespace shmm
