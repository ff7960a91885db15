// Local solves (HMM steps 1-2 of Section 2.2; the two reconstructions with
// orthogonal gradients of the numerical homogenization K[psi, K; D]).
//
// Each corrector obeys w' = div(v w + K_b grad w) + f on a periodic n x n
// patch.  With a = dt v / (2h) on the faces, the dt-scaled right-hand side at
// cell (x, y) is
//   dt F = dt f + cc w_C + aE w_E - aW w_W + aN w_N - aS w_S
//        + cxx (w_E + w_W) + cyy (w_N + w_S) + cxy ((w_NE - w_NW) - (w_SE - w_SW))
// (centred flux-form advection with div v = 0 dropped from the centre term;
// K11 dxx + K22 dyy + 2 K12 dxdy diffusion), advanced by classic RK4.
//
// Kernels, by patch size (variants are chosen per size through the tuner):
// * resident (n <= 128): one workgroup per (domain, corrector) holds the whole
//   patch.  The RK stage input is double-buffered in LDS (one barrier per
//   stage); every thread owns a column strip of R cells and keeps their state,
//   the RK accumulator, a compensation term (Kahan summation of the step
//   increments, so FP32 does not stall near the quasi-stationary state) and
//   its face coefficients in registers.  HBM is touched only to load the
//   patch and to store the final state.  Two arithmetic forms: the split form
//   above (k_solve_resident) and the coefficient form (k_solve_resident_e,
//   the default, with the stage input read a row ahead at 64^2 and 128^2),
//   plus a row-per-wavefront variant (k_solve_rows).
// * n = 256: full-width bands of rows plus a ring of redundant cells, kept
//   resident for all steps and exchanging their rings with the neighbouring
//   bands (k_solve_ring in solve_ring.hip, the default), or relaunched every
//   few steps with their state in workspace between launches (k_solve_band,
//   and k_solve_tiled on square tiles).
// * per-stage launches (k_solve_stage): any other size.
#include <algorithm>

#include "shmm_internal.h"
#include "solve_stage.h"

namespace shmm {

namespace {

// One RK stage over a thread's strip.  KIND 0: r = dt (L y + f);
// KIND 1: q = r + cw dt L y; KIND 2: q1 = r + dt/2 L y, w <- w + q1 (compensated).
template <int NN, int R, int FIELD, int KIND>
__device__ __forceinline__ void rk_stage(const float *__restrict__ C, int offW, int offE, int offS,
                                         int offN, float *__restrict__ out, const SolveConsts &k,
                                         float cw, float (&aE)[R], float (&b)[R + 1],
                                         float (&wv)[R], float (&comp)[R], float (&rr)[R]) {
    // Keep the face coefficients opaque to loop-invariant code motion:
    // quantities derived from them (west face, forcing) are recomputed each
    // stage instead of being hoisted into R more registers each.
#pragma unroll
    for (int r = 0; r < R; ++r) asm volatile("" : "+v"(aE[r]));
#pragma unroll
    for (int r = 0; r <= R; ++r) asm volatile("" : "+v"(b[r]));
    const float *Wc = C + offW;
    const float *Ec = C + offE;
    float sW = Wc[offS], sC = C[offS], sE = Ec[offS];
    float cW = Wc[0], cC = C[0], cE = Ec[0];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int rn = (r + 1 < R) ? (r + 1) * NN : offN;
        const float nW = Wc[rn], nC = C[rn], nE = Ec[rn];
        // the west face follows from the discrete divergence-free identity
        // aE - aW + aN - aS = 0 of the synthesised face velocities
        const float aW = aE[r] + (b[r + 1] - b[r]);
        float t = k.cc * cC;
        t = fmaf(aE[r], cE, t);
        t = fmaf(-aW, cW, t);
        t = fmaf(b[r + 1], nC, t);
        t = fmaf(-b[r], sC, t);
        t = fmaf(k.cxx, cE + cW, t);
        t = fmaf(k.cyy, nC + sC, t);
        t = fmaf(k.cxy, (nE - nW) - (sE - sW), t);
        float o;
        if (KIND == 0) {
            const float ff = FIELD == 0 ? k.fh * (aE[r] + aW) : k.fh * (b[r] + b[r + 1]);
            rr[r] = t + ff;
            o = rr[r];
        } else if (KIND == 1) {
            o = fmaf(cw, t, rr[r]);
        } else {
            const float q1 = fmaf(0.5f, t, rr[r]);
            const float yk = q1 - comp[r];
            const float tk = wv[r] + yk;
            comp[r] = (tk - wv[r]) - yk;
            wv[r] = tk;
            o = tk;
        }
        out[r * NN] = o;
        sW = cW; sC = cC; sE = cE;
        cW = nW; cC = nC; cE = nE;
    }
}

template <int NN, int R, int FIELD>
__device__ __forceinline__ void solve_body(float *__restrict__ buf, const shmm_domain *__restrict__ dom,
                                           const int32_t *__restrict__ list,
                                           const float *__restrict__ vx, const float *__restrict__ vy,
                                           const double *__restrict__ Kb, float *__restrict__ w,
                                           int64_t cells_total, int32_t step_begin, int32_t steps) {
    constexpr int MASK = NN - 1;
    constexpr int PLANE = NN * NN;
    const int64_t d = list[blockIdx.x >> 1];
    const shmm_domain D = dom[d];
    const int64_t s_end64 = (int64_t)step_begin + steps;
    const int32_t s_end = (int32_t)(s_end64 < D.nsteps ? s_end64 : D.nsteps);
    if (step_begin >= s_end) return;

    const int tid = threadIdx.x;
    const int x = tid & MASK;
    const int y0 = (tid / NN) * R;
    // neighbour offsets inside a row (periodic) and across the strip ends
    const int offW = x == 0 ? MASK : -1;
    const int offE = x == MASK ? -MASK : 1;
    const int offS = y0 == 0 ? (NN - 1) * NN : -NN;                 // row before the strip
    const int offN = y0 + R == NN ? (R - NN) * NN : R * NN;          // row after the strip
    const SolveConsts k = solve_consts(D, Kb, d);
    const int64_t o = D.offset;
    const float *vxo = vx + o + y0 * NN + x;
    const float *vyo = vy + o + y0 * NN + x;

    // aE: east x-face, b[r]: south y-face of row r (b[r + 1] is its north face)
    float aE[R], b[R + 1], wv[R], comp[R], rr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        aE[r] = k.a * vxo[r * NN + offE];
        b[r] = k.a * vyo[r * NN];
    }
    b[R] = k.a * vyo[offN];
    float *wf = w + (int64_t)FIELD * cells_total + o + y0 * NN + x;
    float *lo = buf + y0 * NN + x, *hi = lo + PLANE;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        wv[r] = wf[r * NN];
        comp[r] = 0.0f;
        rr[r] = 0.0f;
        lo[r * NN] = wv[r];
    }
    __syncthreads();

    // Classic RK4 for the linear autonomous system w' = L w + f in its Horner
    // form: r = dt (L w + f); q3 = r + (dt/4) L r; q2 = r + (dt/3) L q3;
    // q1 = r + (dt/2) L q2; w <- w + q1.  Stage inputs alternate between the
    // two LDS planes, one barrier per stage.
    for (int32_t s = step_begin; s < s_end; ++s) {
        rk_stage<NN, R, FIELD, 0>(lo, offW, offE, offS, offN, hi, k, 0.0f, aE, b, wv, comp, rr);
        __syncthreads();
        rk_stage<NN, R, FIELD, 1>(hi, offW, offE, offS, offN, lo, k, 0.25f, aE, b, wv, comp, rr);
        __syncthreads();
        rk_stage<NN, R, FIELD, 1>(lo, offW, offE, offS, offN, hi, k, 1.0f / 3.0f, aE, b, wv, comp, rr);
        __syncthreads();
        rk_stage<NN, R, FIELD, 2>(hi, offW, offE, offS, offN, lo, k, 0.5f, aE, b, wv, comp, rr);
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) wf[r * NN] = wv[r];
}

// Workgroup 2 i + j advances corrector j of patch list[i]: both correctors of
// every patch of the phase run in one launch.
template <int NN, int R>
__global__ __launch_bounds__(NN *NN / R) void k_solve_resident(
    const shmm_domain *__restrict__ dom, const int32_t *__restrict__ list,
    const float *__restrict__ vx, const float *__restrict__ vy, const double *__restrict__ Kb,
    float *__restrict__ w, int64_t cells_total, int32_t step_begin, int32_t steps) {
    __shared__ float buf[2 * NN * NN];
    if (blockIdx.x & 1)
        solve_body<NN, R, 1>(buf, dom, list, vx, vy, Kb, w, cells_total, step_begin, steps);
    else
        solve_body<NN, R, 0>(buf, dom, list, vx, vy, Kb, w, cells_total, step_begin, steps);
}

// Resident kernel, coefficient form (rk_stage_e).
template <int NN, int R, int FIELD, int CL, bool FRAME = false, bool PIPE = false>
__device__ __forceinline__ void solve_body_e(float *__restrict__ buf, const shmm_domain *__restrict__ dom,
                                             const int32_t *__restrict__ list,
                                             const float *__restrict__ vx, const float *__restrict__ vy,
                                             const double *__restrict__ Kb, float *__restrict__ w,
                                             int64_t cells_total, int32_t step_begin, int32_t steps) {
    constexpr int MASK = NN - 1;
    constexpr int PLANE = NN * NN;
    const int64_t d = list[blockIdx.x >> 1];
    const shmm_domain D = dom[d];
    const int64_t s_end64 = (int64_t)step_begin + steps;
    const int32_t s_end = (int32_t)(s_end64 < D.nsteps ? s_end64 : D.nsteps);
    if (step_begin >= s_end) return;

    const int tid = threadIdx.x;
    const int x = tid & MASK;
    const int y0 = (tid / NN) * R;
    const int offW = x == 0 ? MASK : -1;
    const int offE = x == MASK ? -MASK : 1;
    const int offS = y0 == 0 ? (NN - 1) * NN : -NN;
    const int offN = y0 + R == NN ? (R - NN) * NN : R * NN;
    SolveConsts k = solve_consts(D, Kb, d);
    // the constants are uniform across the workgroup: keep them in scalar registers
    k.cc = uniform(k.cc);
    k.cxy = uniform(k.cxy);
    k.fh = uniform(k.fh);
    const float two_cyy = uniform(2.0f * k.cyy);
    const int64_t o = D.offset;
    const float *vxo = vx + o + y0 * NN + x;
    const float *vyo = vy + o + y0 * NN + x;

    float eE[R], eW[R], nb[R + 1], wv[R], comp[R], rr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        eE[r] = k.cxx + k.a * vxo[r * NN + offE];
        eW[r] = k.cxx - k.a * vxo[r * NN];
        nb[r] = k.cyy + k.a * vyo[r * NN];
    }
    nb[R] = k.cyy + k.a * vyo[offN];
    float *wf = w + (int64_t)FIELD * cells_total + o + y0 * NN + x;
    float *lo = buf + y0 * NN + x, *hi = lo + PLANE;
    constexpr int T = NN * NN / R;
    float *cl = buf + 2 * PLANE + tid;   // CL rows of compensation, stride T
#pragma unroll
    for (int r = 0; r < R; ++r) {
        wv[r] = wf[r * NN];
        comp[r] = 0.0f;
        rr[r] = 0.0f;
        lo[r * NN] = wv[r];
        if (r < CL) cl[r * T] = 0.0f;
    }
    __syncthreads();
    constexpr bool OP = NN >= 128;
    for (int32_t s = step_begin; s < s_end; ++s) {
        rk_stage_e<NN, R, FIELD, 0, OP, CL, FRAME, PIPE>(lo, offW, offE, offS, offN, hi, k, two_cyy, 0.0f, eE, eW, nb, wv, comp,
                                            rr, cl, T, y0, x == MASK);
        __syncthreads();
        rk_stage_e<NN, R, FIELD, 1, OP, CL, FRAME, PIPE>(hi, offW, offE, offS, offN, lo, k, two_cyy, 0.25f, eE, eW, nb, wv, comp,
                                            rr, cl, T, y0, x == MASK);
        __syncthreads();
        rk_stage_e<NN, R, FIELD, 1, OP, CL, FRAME, PIPE>(lo, offW, offE, offS, offN, hi, k, two_cyy, 1.0f / 3.0f, eE, eW, nb, wv,
                                            comp, rr, cl, T, y0, x == MASK);
        __syncthreads();
        rk_stage_e<NN, R, FIELD, 2, OP, CL, FRAME, PIPE>(hi, offW, offE, offS, offN, lo, k, two_cyy, 0.5f, eE, eW, nb, wv, comp,
                                            rr, cl, T, y0, x == MASK);
        __syncthreads();
    }
    // a fresh base pointer: the row addresses are rebuilt here instead of
    // being held in registers through the step loop
    asm volatile("" : "+v"(wf));
#pragma unroll
    for (int r = 0; r < R; ++r) wf[r * NN] = wv[r];
}

template <int NN, int R, int CL = 0, bool FRAME = false, bool PIPE = false>
__global__ __launch_bounds__(NN *NN / R) void k_solve_resident_e(
    const shmm_domain *__restrict__ dom, const int32_t *__restrict__ list,
    const float *__restrict__ vx, const float *__restrict__ vy, const double *__restrict__ Kb,
    float *__restrict__ w, int64_t cells_total, int32_t step_begin, int32_t steps) {
    __shared__ float buf[2 * NN * NN + CL * (NN * NN / R)];
    if (blockIdx.x & 1)
        solve_body_e<NN, R, 1, CL, FRAME, PIPE>(buf, dom, list, vx, vy, Kb, w, cells_total, step_begin, steps);
    else
        solve_body_e<NN, R, 0, CL, FRAME, PIPE>(buf, dom, list, vx, vy, Kb, w, cells_total, step_begin, steps);
}

// Row-resident variant for patches whose row fits one wavefront (n = 64 C):
// lane l owns columns [C l, C l + C) of R consecutive rows; a wavefront owns
// whole rows, so the x-neighbours across lanes come from wave-wide DPP
// rotations (which also realise the periodic wrap) and the stage input stays
// in registers.  Only the first and last row of each wavefront's strip go
// through LDS (double-buffered), read by the wavefronts above and below.
__device__ __forceinline__ float from_prev_lane(float v) {   // lane i <- lane (i - 1) mod 64
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x13C, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_next_lane(float v) {   // lane i <- lane (i + 1) mod 64
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x134, 0xF, 0xF, false));
}

template <int C>
struct RowTuple {
    float w, v[C], e;   // west neighbour, own cells, east neighbour
};

template <int C>
__device__ __forceinline__ RowTuple<C> make_tuple(const float (&v)[C]) {
    RowTuple<C> t;
#pragma unroll
    for (int c = 0; c < C; ++c) t.v[c] = v[c];
    t.w = from_prev_lane(v[C - 1]);
    t.e = from_next_lane(v[0]);
    return t;
}

template <int C>
__device__ __forceinline__ float left_of(const RowTuple<C> &t, int c) { return c == 0 ? t.w : t.v[c - 1]; }
template <int C>
__device__ __forceinline__ float right_of(const RowTuple<C> &t, int c) { return c == C - 1 ? t.e : t.v[c + 1]; }

template <int NN, int C, int R, int FIELD, int KIND>
__device__ __forceinline__ void row_stage(const float *__restrict__ edge_in, float *__restrict__ edge_out,
                                          int wave, int x0, const SolveConsts &k, float cw,
                                          float (&aE)[R][C], float (&b)[R + 1][C], float (&y)[R][C],
                                          float (&wv)[R][C], float (&comp)[R][C], float (&rr)[R][C]) {
    constexpr int WAVES = NN / R;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) asm volatile("" : "+v"(aE[r][c]));
#pragma unroll
    for (int r = 0; r <= R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) asm volatile("" : "+v"(b[r][c]));
    // row above the strip: last row of the previous wavefront (periodic)
    const int up = (wave + WAVES - 1) % WAVES, down = (wave + 1) % WAVES;
    float tmp[C];
#pragma unroll
    for (int c = 0; c < C; ++c) tmp[c] = edge_in[(up * 2 + 1) * NN + x0 + c];
    RowTuple<C> S = make_tuple<C>(tmp);
    RowTuple<C> M = make_tuple<C>(y[0]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        RowTuple<C> N;
        if (r + 1 < R) {
            N = make_tuple<C>(y[r + 1]);
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) tmp[c] = edge_in[(down * 2 + 0) * NN + x0 + c];
            N = make_tuple<C>(tmp);
        }
        // west face of the first owned cell: east face of the previous lane's last cell
        const float aW0 = from_prev_lane(aE[r][C - 1]);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float ae = aE[r][c], aw = c == 0 ? aW0 : aE[r][c - 1];
            const float bs = b[r][c], bn = b[r + 1][c];
            const float cC = M.v[c], cE = right_of(M, c), cW = left_of(M, c);
            const float nC = N.v[c], nE = right_of(N, c), nW = left_of(N, c);
            const float sC = S.v[c], sE = right_of(S, c), sW = left_of(S, c);
            float t = k.cc * cC;
            t = fmaf(ae, cE, t);
            t = fmaf(-aw, cW, t);
            t = fmaf(bn, nC, t);
            t = fmaf(-bs, sC, t);
            t = fmaf(k.cxx, cE + cW, t);
            t = fmaf(k.cyy, nC + sC, t);
            t = fmaf(k.cxy, (nE - nW) - (sE - sW), t);
            float o;
            if (KIND == 0) {
                const float ff = FIELD == 0 ? k.fh * (ae + aw) : k.fh * (bs + bn);
                rr[r][c] = t + ff;
                o = rr[r][c];
            } else if (KIND == 1) {
                o = fmaf(cw, t, rr[r][c]);
            } else {
                const float q1 = fmaf(0.5f, t, rr[r][c]);
                const float yk = q1 - comp[r][c];
                const float tk = wv[r][c] + yk;
                comp[r][c] = (tk - wv[r][c]) - yk;
                wv[r][c] = tk;
                o = tk;
            }
            y[r][c] = o;
        }
        S = M;
        M = N;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        edge_out[(wave * 2 + 0) * NN + x0 + c] = y[0][c];
        edge_out[(wave * 2 + 1) * NN + x0 + c] = y[R - 1][c];
    }
}

template <int NN, int C, int R, int FIELD>
__device__ __forceinline__ void rows_body(float *__restrict__ edges, const shmm_domain *__restrict__ dom,
                                          const int32_t *__restrict__ list, const float *__restrict__ vx,
                                          const float *__restrict__ vy, const double *__restrict__ Kb,
                                          float *__restrict__ w, int64_t cells_total, int32_t step_begin,
                                          int32_t steps) {
    constexpr int WAVES = NN / R;
    constexpr int EDGE = WAVES * 2 * NN;   // one buffer of boundary rows
    const int64_t d = list[blockIdx.x >> 1];
    const shmm_domain D = dom[d];
    const int64_t s_end64 = (int64_t)step_begin + steps;
    const int32_t s_end = (int32_t)(s_end64 < D.nsteps ? s_end64 : D.nsteps);
    if (step_begin >= s_end) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x0 = lane * C, y0 = wave * R;
    const SolveConsts k = solve_consts(D, Kb, d);
    const int64_t o = D.offset;
    float aE[R][C], b[R + 1][C], y[R][C], wv[R][C], comp[R][C], rr[R][C];
#pragma unroll
    for (int r = 0; r <= R; ++r) {
        const int yy = (y0 + r) & (NN - 1);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            b[r][c] = k.a * vy[o + yy * NN + x0 + c];
            if (r < R) aE[r][c] = k.a * vx[o + yy * NN + ((x0 + c + 1) & (NN - 1))];
        }
    }
    float *wf = w + (int64_t)FIELD * cells_total + o;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            wv[r][c] = wf[(y0 + r) * NN + x0 + c];
            y[r][c] = wv[r][c];
            comp[r][c] = 0.0f;
            rr[r][c] = 0.0f;
        }
    float *e0 = edges, *e1 = edges + EDGE;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        e0[(wave * 2 + 0) * NN + x0 + c] = y[0][c];
        e0[(wave * 2 + 1) * NN + x0 + c] = y[R - 1][c];
    }
    __syncthreads();
    for (int32_t s = step_begin; s < s_end; ++s) {
        row_stage<NN, C, R, FIELD, 0>(e0, e1, wave, x0, k, 0.0f, aE, b, y, wv, comp, rr);
        __syncthreads();
        row_stage<NN, C, R, FIELD, 1>(e1, e0, wave, x0, k, 0.25f, aE, b, y, wv, comp, rr);
        __syncthreads();
        row_stage<NN, C, R, FIELD, 1>(e0, e1, wave, x0, k, 1.0f / 3.0f, aE, b, y, wv, comp, rr);
        __syncthreads();
        row_stage<NN, C, R, FIELD, 2>(e1, e0, wave, x0, k, 0.5f, aE, b, y, wv, comp, rr);
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) wf[(y0 + r) * NN + x0 + c] = wv[r][c];
}

template <int NN, int C, int R>
__global__ __launch_bounds__(64 * (NN / R)) void k_solve_rows(
    const shmm_domain *__restrict__ dom, const int32_t *__restrict__ list,
    const float *__restrict__ vx, const float *__restrict__ vy, const double *__restrict__ Kb,
    float *__restrict__ w, int64_t cells_total, int32_t step_begin, int32_t steps) {
    __shared__ float edges[2 * (NN / R) * 2 * NN];
    if (blockIdx.x & 1)
        rows_body<NN, C, R, 1>(edges, dom, list, vx, vy, Kb, w, cells_total, step_begin, steps);
    else
        rows_body<NN, C, R, 0>(edges, dom, list, vx, vy, Kb, w, cells_total, step_begin, steps);
}

template <int NN, int C, int R>
int launch_rows(const shmm_domain *d_dom, const int32_t *d_list, int32_t nlist, const float *vx,
                const float *vy, const double *Kb, float *w, int64_t cells_total, int32_t step_begin,
                int32_t steps, hipStream_t s) {
    static_assert(NN == 64 * C, "a row must fill one wavefront");
    hipLaunchKernelGGL((k_solve_rows<NN, C, R>), dim3((unsigned)(2 * nlist)), dim3(64 * (NN / R)), 0, s,
                       d_dom, d_list, vx, vy, Kb, w, cells_total, step_begin, steps);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

// Overlapped tiles for patches too large for one CU (n = 256): a workgroup
// advances a TW x TW tile of one corrector by HALO / 4 RK4 steps, computing on
// the tile plus a HALO-cell ring (each stage consumes one ring of valid
// cells, so after 4 s stages everything at least 4 s cells inside the region
// is exact) and writes back the tile.  The state (w and its compensation)
// lives in list-local workspace planes between launches, ping-ponged so no
// workgroup overwrites cells another one still reads.  The stage arithmetic
// is the coefficient-form resident stage; cells on the region's border see
// clamped neighbours and lie outside the written tile.  A patch whose plan
// has ended leaves both planes alone: k_solve_tiles_fini picks its last state
// by the parity of the launches that advanced it.
template <int TW, int HALO, int R, int FIELD>
__device__ __forceinline__ void tiled_body(float *__restrict__ buf, const shmm_domain *__restrict__ dom,
                                           const int32_t *__restrict__ list, int n,
                                           const float *__restrict__ vx, const float *__restrict__ vy,
                                           const double *__restrict__ Kb, const float *__restrict__ w_in,
                                           const float *__restrict__ c_in, float *__restrict__ w_out,
                                           float *__restrict__ c_out, int64_t list_cells, int32_t step0,
                                           int32_t s_cap) {
    constexpr int W = TW + 2 * HALO;
    constexpr int PLANE = W * W;
    const int tiles = n / TW;
    const int tx = blockIdx.x % tiles, ty = blockIdx.x / tiles;
    const int li = blockIdx.y >> 1;
    const int64_t d = list[li];
    const shmm_domain D = dom[d];
    const int32_t lim = s_cap < D.nsteps ? s_cap : D.nsteps;
    if (step0 >= lim) return;
    const int32_t s_end = step0 + HALO / 4 < lim ? step0 + HALO / 4 : lim;
    const int mask = n - 1;

    const int tid = threadIdx.x;
    const int x = tid % W;
    const int y0 = (tid / W) * R;
    const int offW = x == 0 ? 0 : -1;
    const int offE = x == W - 1 ? 0 : 1;
    const int offS = y0 == 0 ? 0 : -W;
    const int offN = y0 + R == W ? (R - 1) * W : R * W;
    SolveConsts k = solve_consts(D, Kb, d);
    k.cc = uniform(k.cc);
    k.cxy = uniform(k.cxy);
    k.fh = uniform(k.fh);
    const float two_cyy = uniform(2.0f * k.cyy);
    const int gx = (tx * TW - HALO + x) & mask;
    const int gxe = (gx + 1) & mask;
    const int gy0 = ty * TW - HALO + y0;
    // uniform base pointers and 32-bit offsets inside one patch plane
    const float *vxp = vx + D.offset, *vyp = vy + D.offset;
    const int64_t ws = (int64_t)FIELD * list_cells + (int64_t)li * n * n;
    const float *wp = w_in + ws, *cp = c_in + ws;

    float eE[R], eW[R], nb[R + 1], wv[R], comp[R], rr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = ((gy0 + r) & mask) * n;
        eE[r] = k.cxx + k.a * vxp[row + gxe];
        eW[r] = k.cxx - k.a * vxp[row + gx];
        nb[r] = k.cyy + k.a * vyp[row + gx];
        wv[r] = wp[row + gx];
        comp[r] = cp[row + gx];
        rr[r] = 0.0f;
    }
    nb[R] = k.cyy + k.a * vyp[((gy0 + R) & mask) * n + gx];
    float *lo = buf + y0 * W + x, *hi = lo + PLANE;
#pragma unroll
    for (int r = 0; r < R; ++r) lo[r * W] = wv[r];
    __syncthreads();
    for (int32_t s = step0; s < s_end; ++s) {
        rk_stage_e<W, R, FIELD, 0, false>(lo, offW, offE, offS, offN, hi, k, two_cyy, 0.0f, eE, eW, nb, wv, comp, rr);
        __syncthreads();
        rk_stage_e<W, R, FIELD, 1, false>(hi, offW, offE, offS, offN, lo, k, two_cyy, 0.25f, eE, eW, nb, wv, comp, rr);
        __syncthreads();
        rk_stage_e<W, R, FIELD, 1, false>(lo, offW, offE, offS, offN, hi, k, two_cyy, 1.0f / 3.0f, eE, eW, nb, wv, comp,
                                   rr);
        __syncthreads();
        rk_stage_e<W, R, FIELD, 2, false>(hi, offW, offE, offS, offN, lo, k, two_cyy, 0.5f, eE, eW, nb, wv, comp, rr);
        __syncthreads();
    }
    if (x < HALO || x >= HALO + TW) return;
    float *wo = w_out + ws, *co = c_out + ws;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int yy = y0 + r;
        if (yy < HALO || yy >= HALO + TW) continue;
        const int at = ((gy0 + r) & mask) * n + gx;
        wo[at] = wv[r];
        co[at] = comp[r];
    }
}

template <int TW, int HALO, int R>
__global__ __launch_bounds__((TW + 2 * HALO) * (TW + 2 * HALO) / R) void k_solve_tiled(
    const shmm_domain *__restrict__ dom, const int32_t *__restrict__ list, int n,
    const float *__restrict__ vx, const float *__restrict__ vy, const double *__restrict__ Kb,
    const float *__restrict__ w_in, const float *__restrict__ c_in, float *__restrict__ w_out,
    float *__restrict__ c_out, int64_t list_cells, int32_t step0, int32_t s_cap) {
    __shared__ float buf[2 * (TW + 2 * HALO) * (TW + 2 * HALO)];
    if (blockIdx.y & 1)
        tiled_body<TW, HALO, R, 1>(buf, dom, list, n, vx, vy, Kb, w_in, c_in, w_out, c_out, list_cells, step0,
                                   s_cap);
    else
        tiled_body<TW, HALO, R, 0>(buf, dom, list, n, vx, vy, Kb, w_in, c_in, w_out, c_out, list_cells, step0,
                                   s_cap);
}

// Full-width bands (n = 256): the same scheme with a region of whole rows,
// TH rows of the patch plus a HALO-row ring above and below, so x stays
// periodic inside the region and only the rows carry redundant work.  NN x
// (TH + 2 HALO) cells with R-cell column strips, as in the resident kernel
// (CL rows of compensation in LDS).  When TH does not divide NN the last band
// is moved up to end at the last row; it then shares rows with the band
// before it, and both write the same values there (a cell at least HALO rows
// inside both regions goes through the same operations on the same inputs).
template <int NN, int TH, int HALO, int R, int CL, int FIELD>
__device__ __forceinline__ void band_body(float *__restrict__ buf, const shmm_domain *__restrict__ dom,
                                          const int32_t *__restrict__ list, int li, int band,
                                          const float *__restrict__ vx, const float *__restrict__ vy,
                                          const double *__restrict__ Kb, const float *__restrict__ w_in,
                                          const float *__restrict__ c_in, float *__restrict__ w_out,
                                          float *__restrict__ c_out, int64_t list_cells, int32_t step0,
                                          int32_t s_cap) {
    constexpr int MASK = NN - 1;
    constexpr int H = TH + 2 * HALO;
    constexpr int PLANE = NN * H;
    constexpr int T = PLANE / R;
    const int64_t d = list[li];
    const shmm_domain D = dom[d];
    const int32_t lim = s_cap < D.nsteps ? s_cap : D.nsteps;
    if (step0 >= lim) return;
    const int32_t s_end = step0 + HALO / 4 < lim ? step0 + HALO / 4 : lim;
    const int band_top = band * TH < NN - TH ? band * TH : NN - TH;

    const int tid = threadIdx.x;
    const int x = tid & MASK;
    const int y0 = (tid / NN) * R;
    const int offW = x == 0 ? MASK : -1;
    const int offE = x == MASK ? -MASK : 1;
    const int offS = y0 == 0 ? 0 : -NN;
    const int offN = y0 + R == H ? (R - 1) * NN : R * NN;
    SolveConsts k = solve_consts(D, Kb, d);
    k.cc = uniform(k.cc);
    k.cxy = uniform(k.cxy);
    k.fh = uniform(k.fh);
    const float two_cyy = uniform(2.0f * k.cyy);
    const int xe = (x + 1) & MASK;
    const int gy0 = band_top - HALO + y0;
    const float *vxp = vx + D.offset, *vyp = vy + D.offset;
    const int64_t ws = (int64_t)FIELD * list_cells + (int64_t)li * NN * NN;
    const float *wp = w_in + ws, *cp = c_in + ws;
    float *cl = buf + 2 * PLANE + tid;

    float eE[R], eW[R], nb[R + 1], wv[R], comp[R], rr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = ((gy0 + r) & MASK) * NN;
        eE[r] = k.cxx + k.a * vxp[row + xe];
        eW[r] = k.cxx - k.a * vxp[row + x];
        nb[r] = k.cyy + k.a * vyp[row + x];
        wv[r] = wp[row + x];
        if (r < CL) {
            cl[r * T] = cp[row + x];
            comp[r] = 0.0f;
        } else {
            comp[r] = cp[row + x];
        }
        rr[r] = 0.0f;
    }
    nb[R] = k.cyy + k.a * vyp[((gy0 + R) & MASK) * NN + x];
    float *lo = buf + y0 * NN + x, *hi = lo + PLANE;
#pragma unroll
    for (int r = 0; r < R; ++r) lo[r * NN] = wv[r];
    __syncthreads();
    constexpr bool OP = R >= 32;
    for (int32_t s = step0; s < s_end; ++s) {
        rk_stage_e<NN, R, FIELD, 0, OP, CL>(lo, offW, offE, offS, offN, hi, k, two_cyy, 0.0f, eE, eW, nb, wv, comp,
                                            rr, cl, T);
        __syncthreads();
        rk_stage_e<NN, R, FIELD, 1, OP, CL>(hi, offW, offE, offS, offN, lo, k, two_cyy, 0.25f, eE, eW, nb, wv, comp,
                                            rr, cl, T);
        __syncthreads();
        rk_stage_e<NN, R, FIELD, 1, OP, CL>(lo, offW, offE, offS, offN, hi, k, two_cyy, 1.0f / 3.0f, eE, eW, nb, wv,
                                            comp, rr, cl, T);
        __syncthreads();
        rk_stage_e<NN, R, FIELD, 2, OP, CL>(hi, offW, offE, offS, offN, lo, k, two_cyy, 0.5f, eE, eW, nb, wv, comp,
                                            rr, cl, T);
        __syncthreads();
    }
    // recompute the row addresses here rather than keep R of them live
    // through the step loop
    int gy = gy0, xs = x;
    asm volatile("" : "+v"(gy), "+v"(xs));
    float *wo = w_out + ws, *co = c_out + ws;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int yy = y0 + r;
        if (yy < HALO || yy >= HALO + TH) continue;
        const int at = ((gy + r) & MASK) * NN + xs;
        wo[at] = wv[r];
        co[at] = r < CL ? cl[r * T] : comp[r];
    }
}

// One-dimensional grid, 2 * bands workgroups per patch (band-major, the two
// correctors of a band side by side).  xcd_map: workgroup i runs on XCD
// i mod 8 (round-robin dispatch), so patch 8 q + j takes the slots of XCD j
// from 2 * bands * q on; a patch's bands and correctors then run together
// on one XCD and share its L2 for the face velocities and the ring rows.
// The grid is padded to a multiple of 8 patches; padding slots return.
template <int NN, int TH>
constexpr int band_count() { return (NN + TH - 1) / TH; }

template <int NN, int TH, int HALO, int R, int CL>
__global__ __launch_bounds__(NN *(TH + 2 * HALO) / R) void k_solve_band(
    const shmm_domain *__restrict__ dom, const int32_t *__restrict__ list, int32_t count, int32_t xcd_map,
    const float *__restrict__ vx, const float *__restrict__ vy, const double *__restrict__ Kb,
    const float *__restrict__ w_in, const float *__restrict__ c_in, float *__restrict__ w_out,
    float *__restrict__ c_out, int64_t list_cells, int32_t step0, int32_t s_cap) {
    __shared__ float buf[2 * NN * (TH + 2 * HALO) + CL * (NN * (TH + 2 * HALO) / R)];
    constexpr int PER = 2 * band_count<NN, TH>();
    const int i = blockIdx.x;
    int li, k;
    if (xcd_map) {
        const int slot = i >> 3;
        li = (slot / PER) * 8 + (i & 7);
        k = slot % PER;
    } else {
        li = i / PER;
        k = i % PER;
    }
    if (li >= count) return;
    if (k & 1)
        band_body<NN, TH, HALO, R, CL, 1>(buf, dom, list, li, k >> 1, vx, vy, Kb, w_in, c_in, w_out, c_out,
                                          list_cells, step0, s_cap);
    else
        band_body<NN, TH, HALO, R, CL, 0>(buf, dom, list, li, k >> 1, vx, vy, Kb, w_in, c_in, w_out, c_out,
                                          list_cells, step0, s_cap);
}

template <int NN, int TH, int HALO, int R, int CL>
int launch_band(const shmm_domain *d_dom, const int32_t *d_list, int32_t cn, const float *vx, const float *vy,
                const double *Kb, const float *w_in, const float *c_in, float *w_out, float *c_out,
                int64_t list_cells, int32_t step, int32_t s_end, hipStream_t s) {
    constexpr int PER = 2 * band_count<NN, TH>();
    // the XCD mapping once every XCD gets at least 8 patches
    const int32_t xcd_map = cn >= 64 ? 1 : 0;
    const int64_t wgs = xcd_map ? (int64_t)PER * 8 * ((cn + 7) / 8) : (int64_t)PER * cn;
    hipLaunchKernelGGL((k_solve_band<NN, TH, HALO, R, CL>), dim3((unsigned)wgs), dim3(NN * (TH + 2 * HALO) / R), 0,
                       s, d_dom, d_list, cn, xcd_map, vx, vy, Kb, w_in, c_in, w_out, c_out, list_cells, step, s_end);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

// Copy each patch's last state back to its corrector.  The launches from
// step_begin advanced a patch ceil((min(s_end, nsteps) - step_begin) / per)
// times; an even count leaves its state in y0 (the plane the first launch
// read), an odd count in y1.
__global__ void k_solve_tiles_fini(const shmm_domain *__restrict__ dom, const int32_t *__restrict__ list, int n,
                                   const float *__restrict__ y0, const float *__restrict__ y1,
                                   float *__restrict__ w, int64_t cells_total, int64_t list_cells,
                                   int32_t step_begin, int32_t s_end, int32_t per) {
    const int li = blockIdx.y >> 1;
    const int field = blockIdx.y & 1;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n * n) return;
    const shmm_domain D = dom[list[li]];
    const int32_t lim = s_end < D.nsteps ? s_end : D.nsteps;
    const int32_t launches = lim > step_begin ? (lim - step_begin + per - 1) / per : 0;
    const float *src = (launches & 1) ? y1 : y0;
    w[(int64_t)field * cells_total + D.offset + c] = src[(int64_t)field * list_cells + (int64_t)li * n * n + c];
}

// Fallback for other patch sizes: one launch per RK stage, state in global
// memory, classic RK4 stage by stage (k1..k4 accumulated) with the same
// operator and the same compensated update.
__global__ __launch_bounds__(256) void k_solve_stage(
    const shmm_domain *__restrict__ dom, const int32_t *__restrict__ list, int n,
    const float *__restrict__ vx, const float *__restrict__ vy, const double *__restrict__ Kb,
    float *__restrict__ w, int64_t cells_total, const float *__restrict__ ycur,
    float *__restrict__ ynext, float *__restrict__ acc, float *__restrict__ comp,
    int64_t list_cells, int32_t step, int st, int frame) {
    const int li = blockIdx.y >> 1;
    const int field = blockIdx.y & 1;
    const int64_t d = list[li];
    const shmm_domain D = dom[d];
    if (step >= D.nsteps) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n * n) return;
    const int mask = n - 1;
    const int y = c / n, x = c - y * n;
    const int xe = (x + 1) & mask, xw = (x - 1) & mask, yn = (y + 1) & mask, ys = (y - 1) & mask;
    const SolveConsts k = solve_consts(D, Kb, d);
    const int64_t o = D.offset;
    const int64_t ws = (int64_t)field * list_cells + (int64_t)li * n * n;
    const float *Y = ycur + ws;
    const float aE = k.a * vx[o + y * n + xe], aW = k.a * vx[o + c];
    const float bS = k.a * vy[o + c], bN = k.a * vy[o + yn * n + x];
    const float cC = Y[c], cE = Y[y * n + xe], cW = Y[y * n + xw];
    const float nC = Y[yn * n + x], nE = Y[yn * n + xe], nW = Y[yn * n + xw];
    const float sC = Y[ys * n + x], sE = Y[ys * n + xe], sW = Y[ys * n + xw];
    const float ff = field == 0 ? k.fh * (aE + aW) : k.fh * (bS + bN);
    float t = fmaf(k.cc, cC, ff);
    t = fmaf(aE, cE, t);
    t = fmaf(-aW, cW, t);
    t = fmaf(bN, nC, t);
    t = fmaf(-bS, sC, t);
    t = fmaf(k.cxx, cE + cW, t);
    t = fmaf(k.cyy, nC + sC, t);
    t = fmaf(k.cxy, (nE - nW) - (sE - sW), t);
    // zero-frame local problem: the last row and column stay at zero
    if (frame && (x == mask || y == mask)) t = 0.0f;
    float *wf = w + (int64_t)field * cells_total + o;
    const float wc = wf[c];
    float out;
    if (st == 0) {
        acc[ws + c] = t;
        out = fmaf(0.5f, t, wc);
    } else if (st < 3) {
        acc[ws + c] = fmaf(2.0f, t, acc[ws + c]);
        out = fmaf(st == 2 ? 1.0f : 0.5f, t, wc);
    } else {
        const float inc = (acc[ws + c] + t) * (1.0f / 6.0f);
        const float cp = comp[ws + c];
        const float yk = inc - cp;
        const float tk = wc + yk;
        comp[ws + c] = (tk - wc) - yk;
        wf[c] = tk;
        out = tk;
    }
    ynext[ws + c] = out;
}

__global__ void k_solve_stage_init(const shmm_domain *__restrict__ dom,
                                   const int32_t *__restrict__ list, int n,
                                   const float *__restrict__ w, int64_t cells_total,
                                   float *__restrict__ ycur, float *__restrict__ comp,
                                   int64_t list_cells) {
    const int li = blockIdx.y >> 1;
    const int field = blockIdx.y & 1;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n * n) return;
    const shmm_domain D = dom[list[li]];
    const int64_t ws = (int64_t)field * list_cells + (int64_t)li * n * n;
    ycur[ws + c] = w[(int64_t)field * cells_total + D.offset + c];
    comp[ws + c] = 0.0f;
}

template <int NN, int R>
int launch_resident(const shmm_domain *d_dom, const int32_t *d_list, int32_t nlist, const float *vx,
                    const float *vy, const double *Kb, float *w, int64_t cells_total,
                    int32_t step_begin, int32_t steps, hipStream_t s) {
    hipLaunchKernelGGL((k_solve_resident<NN, R>), dim3((unsigned)(2 * nlist)), dim3(NN * NN / R), 0, s,
                       d_dom, d_list, vx, vy, Kb, w, cells_total, step_begin, steps);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

template <int NN, int R, int CL = 0, bool FRAME = false, bool PIPE = false>
int launch_resident_e(const shmm_domain *d_dom, const int32_t *d_list, int32_t nlist, const float *vx,
                      const float *vy, const double *Kb, float *w, int64_t cells_total,
                      int32_t step_begin, int32_t steps, hipStream_t s) {
    hipLaunchKernelGGL((k_solve_resident_e<NN, R, CL, FRAME, PIPE>), dim3((unsigned)(2 * nlist)), dim3(NN * NN / R), 0, s,
                       d_dom, d_list, vx, vy, Kb, w, cells_total, step_begin, steps);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

}  // namespace

bool local_solve_resident(int n) { return n == 8 || n == 16 || n == 32 || n == 64 || n == 128; }

int local_solve_variants(int n) { return n == 64 ? 7 : n == 128 ? 9 : n == 256 ? 8 : 1; }

namespace {
// Zero both corrector fields of the listed domains (one workgroup row per domain).
__global__ __launch_bounds__(256) void k_zero_fields(const shmm_domain *dom, const int32_t *list, int n, float *w,
                                                     int64_t cells) {
    const int64_t o = dom[list[blockIdx.y]].offset;
    const int64_t nn = (int64_t)n * n;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nn; c += (int64_t)gridDim.x * blockDim.x) {
        w[o + c] = 0.0f;
        w[cells + o + c] = 0.0f;
    }
}
}  // namespace

int launch_zero_fields(const shmm_domain *d_dom, const int32_t *d_list, int32_t nlist, int n, float *d_w,
                       int64_t cells, hipStream_t s) {
    const unsigned bx = (unsigned)std::min<int64_t>(16, ((int64_t)n * n + 255) / 256);
    for (int32_t c0 = 0; c0 < nlist; c0 += 65535) {
        const int32_t cn = std::min<int32_t>(65535, nlist - c0);
        hipLaunchKernelGGL(k_zero_fields, dim3(bx, (unsigned)cn), dim3(256), 0, s, d_dom, d_list + c0, n, d_w,
                           cells);
        SHMM_HIP_CHECK(hipGetLastError());
    }
    return SHMM_OK;
}

size_t local_solve_workspace(int n, int64_t list_cells, bool frame) {
    (void)frame;   // zero-frame solves of resident sizes stay resident too
    if (local_solve_resident(n)) return 0;
    return (size_t)4 * 2 * list_cells * sizeof(float);   // ycur, ynext, acc, comp; 2 fields
}

int launch_local_solve(const shmm_domain *d_dom, const int32_t *d_list, int32_t nlist, int n,
                       int32_t max_steps, const float *vx, const float *vy, const float *f1,
                       const float *f2, const double *Kb, float *w, int64_t cells_total,
                       int32_t step_begin, int32_t steps, int64_t list_cells, void *work,
                       int variant, hipStream_t s, bool frame, uint32_t ring_spin_cap) {
    (void)f1;
    (void)f2;   // the forcing is rebuilt from the face velocities in registers
    if (nlist <= 0) return SHMM_OK;
    // the zero-frame local problem: the resident coefficient-form kernels
    // with the frame held at zero up to 128^2, the ring-exchange bands at
    // 256^2 (other variants and sizes stage by stage)
    if (frame) {
        switch (n) {
            case 8: return launch_resident_e<8, 2, 0, true>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            case 16: return launch_resident_e<16, 4, 0, true>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            case 32: return launch_resident_e<32, 8, 0, true>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            case 64: return launch_resident_e<64, 16, 0, true>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            case 128: return launch_resident_e<128, 32, 8, true>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            default: break;
        }
    }
    switch (frame ? 0 : n) {
        case 8: return launch_resident_e<8, 2>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
        case 16: return launch_resident_e<16, 4>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
        case 32: return launch_resident_e<32, 8>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
        case 64:
            if (variant == 1) return launch_rows<64, 1, 16>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            if (variant == 2) return launch_rows<64, 1, 8>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            if (variant == 3) return launch_resident_e<64, 16>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            if (variant == 4) return launch_resident_e<64, 8>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            if (variant == 5) return launch_resident_e<64, 16, 0, false, true>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            if (variant == 6) return launch_resident_e<64, 8, 0, false, true>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            return launch_resident<64, 16>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
        case 128:
            if (variant == 1) return launch_rows<128, 2, 16>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            if (variant == 2) return launch_rows<128, 2, 8>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            if (variant == 3) return launch_resident_e<128, 32>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            if (variant == 4) return launch_resident_e<128, 16>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            if (variant == 5) return launch_resident_e<128, 32, 8>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            if (variant == 6) return launch_resident_e<128, 32, 16>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            if (variant == 7) return launch_resident_e<128, 32, 8, false, true>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            if (variant == 8) return launch_resident_e<128, 32, 16, false, true>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
            return launch_resident<128, 32>(d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, step_begin, steps, s);
        default: break;
    }
    float *ws = (float *)work;
    float *ycur = ws, *ynext = ws + 2 * list_cells, *acc = ws + 4 * list_cells,
          *comp = ws + 6 * list_cells;
    const int64_t s_end64 = (int64_t)step_begin + steps;
    const int32_t s_end = (int32_t)(s_end64 < max_steps ? s_end64 : max_steps);
    if (n == 256 && (variant == 6 || variant == 7)) {   // persistent bands with a ring exchange (solve_ring.hip)
        // each patch stops at min(step_begin + steps, its plan) inside the
        // kernel, so the launch does not depend on the host's plan (a
        // captured graph stays valid when the plans change)
        const int32_t s_cap = (int32_t)std::min<int64_t>(s_end64, 2147483647);
        return launch_ring_solve(d_dom, d_list, nlist, n, vx, vy, Kb, w, cells_total, step_begin, s_cap, work,
                                 local_solve_workspace(n, list_cells), s, frame, ring_spin_cap, variant == 7);
    }
    if (n == 256 && variant != 2 && !frame) {
        // Overlapped regions, HALO / 4 steps per launch.  Full-width bands:
        // variant 0 32 rows with 8 above and below (768 threads), 1 the same
        // with 1024 threads, 3 24 rows with 12 (3 steps per launch), 4 16
        // rows with 8 (256 threads, two workgroups per CU); 5 square 64^2
        // tiles with a ring of 8 (640 threads).  Lists split at 16384
        // patches (grid.y < 65536).
        const int32_t per = variant == 3 ? 3 : 2;
        for (int32_t c0 = 0; c0 < nlist; c0 += 16384) {
            const int32_t cn = std::min<int32_t>(16384, nlist - c0);
            const int64_t off = (int64_t)c0 * n * n;
            const int32_t *cl = d_list + c0;
            float *const y0 = ycur + off, *const y1 = ynext + off;
            float *yc = y0, *yn = y1, *cc = comp + off, *cx = acc + off;
            const dim3 cg((unsigned)((n * n + 255) / 256), (unsigned)(2 * cn));
            hipLaunchKernelGGL(k_solve_stage_init, cg, dim3(256), 0, s, d_dom, cl, n, w, cells_total, y0, cc,
                               list_cells);
            SHMM_HIP_CHECK(hipGetLastError());
            for (int32_t step = step_begin; step < s_end; step += per) {
                const float *ycc = yc, *ccc = cc;
                int rc = SHMM_OK;
                switch (variant) {
                    case 1:
                        rc = launch_band<256, 32, 8, 12, 0>(d_dom, cl, cn, vx, vy, Kb, ycc, ccc, yn, cx, list_cells,
                                                           step, s_end, s);
                        break;
                    case 3:
                        rc = launch_band<256, 24, 12, 16, 0>(d_dom, cl, cn, vx, vy, Kb, ycc, ccc, yn, cx, list_cells,
                                                             step, s_end, s);
                        break;
                    case 4:
                        rc = launch_band<256, 16, 8, 32, 8>(d_dom, cl, cn, vx, vy, Kb, ycc, ccc, yn, cx, list_cells,
                                                           step, s_end, s);
                        break;
                    case 5:
                        hipLaunchKernelGGL((k_solve_tiled<64, 8, 10>), dim3(16, (unsigned)(2 * cn)), dim3(640), 0, s,
                                           d_dom, cl, n, vx, vy, Kb, ycc, ccc, yn, cx, list_cells, step, s_end);
                        break;
                    default:
                        rc = launch_band<256, 32, 8, 16, 0>(d_dom, cl, cn, vx, vy, Kb, ycc, ccc, yn, cx, list_cells,
                                                           step, s_end, s);
                        break;
                }
                if (rc) return rc;
                SHMM_HIP_CHECK(hipGetLastError());
                std::swap(yc, yn);
                std::swap(cc, cx);
            }
            hipLaunchKernelGGL(k_solve_tiles_fini, cg, dim3(256), 0, s, d_dom, cl, n, (const float *)y0,
                               (const float *)y1, w, cells_total, list_cells, step_begin, s_end, per);
            SHMM_HIP_CHECK(hipGetLastError());
        }
        return SHMM_OK;
    }
    if (2 * (int64_t)nlist > 65535) return SHMM_ERANGE;
    const dim3 grid((unsigned)((n * n + 255) / 256), (unsigned)(2 * nlist));
    hipLaunchKernelGGL(k_solve_stage_init, grid, dim3(256), 0, s, d_dom, d_list, n, w, cells_total,
                       ycur, comp, list_cells);
    SHMM_HIP_CHECK(hipGetLastError());
    // generic path: one launch per RK stage
    for (int32_t step = step_begin; step < s_end; ++step) {
        for (int st = 0; st < 4; ++st) {
            hipLaunchKernelGGL(k_solve_stage, grid, dim3(256), 0, s, d_dom, d_list, n, vx, vy, Kb, w,
                               cells_total, ycur, ynext, acc, comp, list_cells, step, st, frame ? 1 : 0);
            SHMM_HIP_CHECK(hipGetLastError());
            float *t = ycur;
            ycur = ynext;
            ynext = t;
        }
    }
    return SHMM_OK;
}

}  // namespace shmm
