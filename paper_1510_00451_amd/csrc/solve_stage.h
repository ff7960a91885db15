// Shared pieces of the local-solve kernels: the dt-scaled stencil constants
// of a domain and one RK stage of the coefficient form over a thread's
// column strip (the operator and the Horner form of RK4 are described at the
// top of solve.hip).
#pragma once

#include "shmm_internal.h"

namespace shmm {
namespace {

struct SolveConsts {
    float cxx, cyy, cxy, cc, a, fh;
};

__device__ inline SolveConsts solve_consts(const shmm_domain &D, const double *Kb, int64_t d) {
    const double h = D.h, dt = D.dt, h2 = h * h;
    const double K11 = Kb[3 * d], K12 = Kb[3 * d + 1], K22 = Kb[3 * d + 2];
    SolveConsts c;
    c.cxx = (float)(dt * K11 / h2);
    c.cyy = (float)(dt * K22 / h2);
    c.cxy = (float)(dt * K12 / (2.0 * h2));
    c.cc = (float)(-2.0 * dt * (K11 + K22) / h2);
    c.a = (float)(dt / (2.0 * h));
    c.fh = (float)h;
    return c;
}

__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Coefficient form of the stage.  With eE = cxx + aE, eW = cxx - aW,
// eN = cyy + aN and eS = cyy - aS the dt-scaled operator is
//   cc w_C + eE w_E + eW w_W + eN w_N + eS w_S + cxy ((w_NE - w_NW) - (w_SE - w_SW)),
// five products instead of the split advection and diffusion terms.  A thread
// keeps eE, eW and nb[r] = cyy + (south face of row r) for its strip, so
// eN of row r is nb[r + 1] and eS is 2 cyy - nb[r]; the forcing is
// h (eE - eW) (first corrector) or h (eN - eS) (second).  The x-difference of
// a row, w_E - w_W, is formed once and used by the rows above and below.
// OPAQUE: hide the coefficients from loop-invariant motion, so that derived
// values are recomputed each stage instead of hoisted into R more registers
// each.  Needed at n = 128, where hoisting spills; smaller patches are faster
// with the derived values hoisted.
// CL: the compensation of the first CL rows of the strip lives in LDS
// (cl[r * cstride]) instead of registers, to relieve register pressure.
// FRAME: the zero-frame local problem; the cells of the patch's last column
// (xlast) and last row (strip row y0 + r = NN - 1) keep a zero derivative.
// PIPE: read the stage input one row further ahead (row r + 2 while row r is
// computed) and keep each pair of rows' reads in front of the previous pair's
// arithmetic with a scheduling barrier, so the LDS latency overlaps the
// arithmetic instead of being waited for at the top of every pair; same
// arithmetic, same results.
template <int NN, int R, int FIELD, int KIND, bool OPAQUE, int CL = 0, bool FRAME = false, bool PIPE = false>
__device__ __forceinline__ void rk_stage_e(const float *__restrict__ C, int offW, int offE, int offS,
                                           int offN, float *__restrict__ out, const SolveConsts &k,
                                           float two_cyy, float cw, float (&eE)[R], float (&eW)[R],
                                           float (&nb)[R + 1], float (&wv)[R], float (&comp)[R],
                                           float (&rr)[R], float *__restrict__ cl = nullptr,
                                           int cstride = 0, int y0 = 0, bool xlast = false) {
    if (OPAQUE) {
#pragma unroll
        for (int r = 0; r < R; ++r) asm volatile("" : "+v"(eE[r]), "+v"(eW[r]));
#pragma unroll
        for (int r = 0; r <= R; ++r) asm volatile("" : "+v"(nb[r]));
    }
    const float *Wc = C + offW;
    const float *Ec = C + offE;
    float sC = C[offS];
    float dS = Ec[offS] - Wc[offS];
    float cW = Wc[0], cC = C[0], cE = Ec[0];
    float qW = 0.0f, qC = 0.0f, qE = 0.0f;       // PIPE: the row after the next
    if (PIPE) {
        const int r1 = 1 < R ? NN : offN;
        qW = Wc[r1]; qC = C[r1]; qE = Ec[r1];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float nW, nC, nE;
        if (PIPE) {
            nW = qW; nC = qC; nE = qE;
            if (r + 2 <= R) {
                const int rp = (r + 2 < R) ? (r + 2) * NN : offN;
                qW = Wc[rp]; qC = C[rp]; qE = Ec[rp];
            }
            if (r & 1) __builtin_amdgcn_sched_barrier(0);
        } else {
            const int rn = (r + 1 < R) ? (r + 1) * NN : offN;
            nW = Wc[rn]; nC = C[rn]; nE = Ec[rn];
        }
        const float dN = nE - nW;
        const float eS = two_cyy - nb[r];
        float t = k.cc * cC;
        t = fmaf(eE[r], cE, t);
        t = fmaf(eW[r], cW, t);
        t = fmaf(nb[r + 1], nC, t);
        t = fmaf(eS, sC, t);
        t = fmaf(k.cxy, dN - dS, t);
        float keep = 1.0f;
        if (FRAME) {
            keep = (xlast || y0 + r == NN - 1) ? 0.0f : 1.0f;
            t *= keep;
        }
        float o;
        if (KIND == 0) {
            rr[r] = FIELD == 0 ? fmaf(k.fh, eE[r] - eW[r], t) : fmaf(k.fh, nb[r + 1] - eS, t);
            if (FRAME) rr[r] *= keep;
            o = rr[r];
        } else if (KIND == 1) {
            o = fmaf(cw, t, rr[r]);
        } else {
            const float q1 = fmaf(0.5f, t, rr[r]);
            const float cp = r < CL ? cl[r * cstride] : comp[r];
            const float yk = q1 - cp;
            const float tk = wv[r] + yk;
            const float cn = (tk - wv[r]) - yk;
            if (r < CL)
                cl[r * cstride] = cn;
            else
                comp[r] = cn;
            wv[r] = tk;
            o = tk;
        }
        out[r * NN] = o;
        sC = cC;
        dS = cE - cW;
        cW = nW; cC = nC; cE = nE;
    }
}

}  // namespace
}  // namespace shmm
