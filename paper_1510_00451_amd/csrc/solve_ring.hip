// Persistent ring-exchange bands for patches too large for one CU (n = 256).
//
// The overlapped-band path reloads each region (state, compensation and face
// velocities) from global memory every HALO / 4 steps, and that reload is
// most of its time.  Here a group of 2 NN / TH workgroups, every full-width
// band of both correctors of one patch, stays resident for all of the
// patch's steps: the state, the compensation and the face coefficients of
// each region remain in registers and LDS.  After every HALO / 4 steps each
// thread of a band publishes its cells of the HALO rows nearest the band's two
// edges (state and compensation) to a slab in global memory and polls the
// cells of its ring rows in the two neighbouring bands' slabs until they are
// written: the slabs start empty (a reserved NaN bit pattern), and a taken
// word is emptied again.  After the last window of a patch the bands instead
// signal round counters and wait for their neighbours', so that no band
// writes its final rows before both neighbours have loaded the patch.  Slab
// words and counters are written and read only as relaxed device-scope
// atomics, which are coherent across the device by themselves; the ordering
// comes from each thread's store completion wait before it publishes again
// and from the neighbours' dependence on each other's rows.  No device-scope
// fence is needed, so no cache is written back or invalidated per round.  The
// stage arithmetic of every owned cell is that of the overlapped bands on the
// same inputs, so both paths give identical results.
//
// Co-residency: the grid never exceeds what the device holds at once (one
// workgroup per CU), so every workgroup of a group is eventually running
// whatever else shares the device; groups then loop over the patches of the
// list.  Each wait is bounded: a workgroup that waits longer than the spin
// limit (tens of seconds) writes NaN into its owned rows of this and every
// later patch of its group, without waiting again, so every wave exits and
// the failure shows as a non-finite corrector (SHMM_DOM_NONFINITE in the
// status of the local solve) and a non-finite estimate.  The spin limit is
// a context setting (SHMM_TUNE_RING_SPIN_CAP).
#include <algorithm>

#include "shmm_internal.h"
#include "solve_stage.h"

namespace shmm {

namespace {

template <int NN, int TH, int HALO>
struct RingShape {
    static_assert(NN % TH == 0, "bands must tile the patch");
    static_assert(TH >= 2 * HALO, "the two published row sets of a band must not overlap");
    static_assert(HALO % 4 == 0, "a ring of HALO rows carries HALO / 4 RK4 steps");
    static constexpr int BANDS = NN / TH;
    static constexpr int PER = 2 * BANDS;         // workgroups per group
    static constexpr int H = TH + 2 * HALO;       // rows of a region
    // floats per (member, round parity): state then compensation, each the
    // HALO lowest owned rows followed by the HALO highest owned rows
    static constexpr int SLAB = 4 * HALO * NN;
};

// Slab traffic of one strip of rows [ST R, ST R + R) of a region, with ST a
// compile-time strip index so that the row tests fold away.  Publish: the
// owned rows within HALO of the region's lower ring go to slab rows
// [0, HALO), those within HALO of its upper ring to [HALO, 2 HALO); the
// compensation follows the state at slab row 2 HALO.
template <int NN, int TH, int HALO, int R, int ST>
__device__ __forceinline__ void publish_strip(float *__restrict__ mine, const float (&wv)[R],
                                              const float (&comp)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int yy = ST * R + r;
        int q;
        if (yy >= HALO && yy < 2 * HALO)
            q = yy - HALO;
        else if (yy >= TH && yy < TH + HALO)
            q = HALO + (yy - TH);
        else
            continue;
        __hip_atomic_store(mine + q * NN, wv[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(mine + (2 * HALO + q) * NN, comp[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Bit pattern of a slab word that holds nothing yet: a NaN with every
// payload bit set, which no arithmetic of the solve produces from finite data
// (a NaN that arises in a solve has the default payload and passes through).
// Only a non-finite input carrying this very pattern can publish it; the
// neighbour's wait then runs to the spin limit and gives up, which ends in
// the same NaN corrector and status bit that such an input gives anyway.
constexpr uint32_t kSlabEmpty = 0xFFFFFFFFu;

// Ring rows of the strip straight from the neighbours' slabs, polled until
// every word of them has been written (none reads kSlabEmpty), then emptied
// again for the round that next uses this slab parity.  A poll reads one word
// of each neighbour until both are written, and all of the words only then,
// so a band that waits long loads little.  At most spin_cap polls (0: give
// up without polling); returns false when it gives up.  Strips without ring
// rows return at once.
template <int NN, int TH, int HALO, int R, int ST>
__device__ __forceinline__ bool take_strip_polled(uint32_t *__restrict__ fs, uint32_t *__restrict__ fn,
                                                  float *__restrict__ lo, float (&wv)[R], float (&comp)[R],
                                                  uint32_t spin_cap) {
    constexpr bool kRing = ST * R < HALO || ST * R + R > TH + HALO;
    if constexpr (!kRing) {
        return true;
    } else {
        // the first ring word of each neighbour this strip reads (compile time)
        constexpr int kFirstS = ST * R < HALO ? HALO + ST * R : -1;
        constexpr int kFirstN = ST * R + R > TH + HALO ? (ST * R > TH + HALO ? ST * R : TH + HALO) - TH - HALO : -1;
        uint32_t a[R], c[R];
        for (uint32_t it = 0;; ++it) {
            if (it >= spin_cap) return false;
            if (it > 0) __builtin_amdgcn_s_sleep(1);
            bool seen = true;
            if constexpr (kFirstS >= 0)
                seen = seen && __hip_atomic_load(fs + kFirstS * NN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kSlabEmpty;
            if constexpr (kFirstN >= 0)
                seen = seen && __hip_atomic_load(fn + kFirstN * NN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kSlabEmpty;
            if (!seen) continue;
            bool ready = true;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int yy = ST * R + r;
                const uint32_t *src;
                int q;
                if (yy < HALO) {
                    src = fs;
                    q = HALO + yy;
                } else if (yy >= TH + HALO) {
                    src = fn;
                    q = yy - TH - HALO;
                } else {
                    continue;
                }
                a[r] = __hip_atomic_load(src + q * NN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                c[r] = __hip_atomic_load(src + (2 * HALO + q) * NN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ready = ready && a[r] != kSlabEmpty && c[r] != kSlabEmpty;
            }
            if (ready) break;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int yy = ST * R + r;
            uint32_t *src;
            int q;
            if (yy < HALO) {
                src = fs;
                q = HALO + yy;
            } else if (yy >= TH + HALO) {
                src = fn;
                q = yy - TH - HALO;
            } else {
                continue;
            }
            wv[r] = __uint_as_float(a[r]);
            comp[r] = __uint_as_float(c[r]);
            lo[r * NN] = wv[r];
            __hip_atomic_store(src + q * NN, kSlabEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(src + (2 * HALO + q) * NN, kSlabEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return true;
    }
}

// The above for the runtime strip index st (uniform within a wavefront),
// dispatched to the compile-time strip ST = st.
template <int NN, int TH, int HALO, int R, int ST = 0>
__device__ __forceinline__ void publish_rows(int st, float *__restrict__ mine, const float (&wv)[R],
                                             const float (&comp)[R]) {
    if constexpr (ST < (TH + 2 * HALO) / R) {
        if (st == ST)
            publish_strip<NN, TH, HALO, R, ST>(mine, wv, comp);
        else
            publish_rows<NN, TH, HALO, R, ST + 1>(st, mine, wv, comp);
    }
}

template <int NN, int TH, int HALO, int R, int ST = 0>
__device__ __forceinline__ bool take_rows_polled(int st, uint32_t *__restrict__ fs, uint32_t *__restrict__ fn,
                                                 float *__restrict__ lo, float (&wv)[R], float (&comp)[R],
                                                 uint32_t spin_cap) {
    if constexpr (ST < (TH + 2 * HALO) / R) {
        if (st == ST)
            return take_strip_polled<NN, TH, HALO, R, ST>(fs, fn, lo, wv, comp, spin_cap);
        return take_rows_polled<NN, TH, HALO, R, ST + 1>(st, fs, fn, lo, wv, comp, spin_cap);
    }
    return true;
}

template <int NN, int TH, int HALO, int R, int FIELD, bool FRAME, bool PIPE>
__device__ __forceinline__ void ring_body(float *__restrict__ buf, int *bad, const shmm_domain *__restrict__ dom,
                                          const int32_t *__restrict__ list, int32_t count, int group,
                                          int groups, int band, const float *__restrict__ vx,
                                          const float *__restrict__ vy, const double *__restrict__ Kb,
                                          float *__restrict__ w, int64_t cells_total, float *__restrict__ slab,
                                          int32_t *__restrict__ flags, int32_t step_begin, int32_t s_cap,
                                          uint32_t spin_cap) {
    using S = RingShape<NN, TH, HALO>;
    static_assert(S::H % R == 0, "a region is a whole number of strips");
    constexpr int MASK = NN - 1;
    constexpr int H = S::H;
    constexpr int PLANE = NN * H;
    constexpr int SLAB = S::SLAB;
    const int tid = threadIdx.x;
    const int x = tid & MASK;
    const int y0 = (tid / NN) * R;
    const int offW = x == 0 ? MASK : -1;
    const int offE = x == MASK ? -MASK : 1;
    const int offS = y0 == 0 ? 0 : -NN;
    const int offN = y0 + R == H ? (R - 1) * NN : R * NN;
    const int xe = (x + 1) & MASK;
    const int me = group * S::PER + band * 2 + FIELD;
    const int south = group * S::PER + ((band + S::BANDS - 1) % S::BANDS) * 2 + FIELD;
    const int north = group * S::PER + ((band + 1) % S::BANDS) * 2 + FIELD;
    float *lo = buf + y0 * NN + x, *hi = lo + PLANE;
    int32_t epoch = 0;
    bool dead = false;

    for (int li = group; li < count; li += groups) {
        const int64_t d = list[li];
        const shmm_domain D = dom[d];
        const int32_t lim = s_cap < D.nsteps ? s_cap : D.nsteps;
        if (step_begin >= lim) continue;   // the same decision in every member of the group
        const int gy0 = band * TH - HALO + y0;
        // zero frame: the strip's first patch row (mod NN) and whether this
        // thread's column is the patch's last
        const int gy0m = gy0 & MASK;
        const bool xlast = x == MASK;
        float *wf = w + (int64_t)FIELD * cells_total + D.offset;
        if (dead) {   // a wait of this group failed: poison the owned rows
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int yy = y0 + r;
                if (yy >= HALO && yy < HALO + TH) wf[((gy0 + r) & MASK) * NN + x] = __builtin_nanf("");
            }
            continue;
        }
        float wv[R];
        {
            SolveConsts k = solve_consts(D, Kb, d);
            k.cc = uniform(k.cc);
            k.cxy = uniform(k.cxy);
            k.fh = uniform(k.fh);
            const float two_cyy = uniform(2.0f * k.cyy);
            const float *vxp = vx + D.offset, *vyp = vy + D.offset;
            float eE[R], eW[R], nb[R + 1], comp[R], rr[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int row = ((gy0 + r) & MASK) * NN;
                eE[r] = k.cxx + k.a * vxp[row + xe];
                eW[r] = k.cxx - k.a * vxp[row + x];
                nb[r] = k.cyy + k.a * vyp[row + x];
                wv[r] = wf[row + x];
                comp[r] = 0.0f;
                rr[r] = 0.0f;
            }
            nb[R] = k.cyy + k.a * vyp[((gy0 + R) & MASK) * NN + x];
#pragma unroll
            for (int r = 0; r < R; ++r) lo[r * NN] = wv[r];
            __syncthreads();
            for (int32_t s = step_begin; s < lim;) {
                const int32_t se = s + HALO / 4 < lim ? s + HALO / 4 : lim;
                for (; s < se; ++s) {
                    rk_stage_e<NN, R, FIELD, 0, false, 0, FRAME, PIPE>(lo, offW, offE, offS, offN, hi, k, two_cyy, 0.0f, eE,
                                                                 eW, nb, wv, comp, rr, nullptr, 0, gy0m, xlast);
                    __syncthreads();
                    rk_stage_e<NN, R, FIELD, 1, false, 0, FRAME, PIPE>(hi, offW, offE, offS, offN, lo, k, two_cyy, 0.25f, eE,
                                                                 eW, nb, wv, comp, rr, nullptr, 0, gy0m, xlast);
                    __syncthreads();
                    rk_stage_e<NN, R, FIELD, 1, false, 0, FRAME, PIPE>(lo, offW, offE, offS, offN, hi, k, two_cyy,
                                                                 1.0f / 3.0f, eE, eW, nb, wv, comp, rr, nullptr, 0,
                                                                 gy0m, xlast);
                    __syncthreads();
                    rk_stage_e<NN, R, FIELD, 2, false, 0, FRAME, PIPE>(hi, offW, offE, offS, offN, lo, k, two_cyy, 0.5f, eE,
                                                                 eW, nb, wv, comp, rr, nullptr, 0, gy0m, xlast);
                    __syncthreads();
                }
                // One round per window.  Between windows each thread
                // publishes its rows of the two published row sets and polls
                // its ring rows in the neighbours' slabs until they are
                // written, then empties them: one trip through memory, no
                // counter.  Its stores (rows and emptied words) are complete
                // before it publishes again (the wait sits right before the
                // publication, so the emptying stores drain during the
                // window's arithmetic), and a neighbour publishes into a slab
                // parity only after taking this band's rows of the round in
                // between, so an emptied word is never overwritten by the
                // round it came from nor read again by it.
                ++epoch;
                const bool more = s < lim;
                const int st = y0 / R;
                if (more) {
                    __builtin_amdgcn_s_waitcnt(0);
                    float *mine = slab + ((int64_t)me * 2 + (epoch & 1)) * SLAB + x;
                    publish_rows<NN, TH, HALO, R>(st, mine, wv, comp);
                    uint32_t *fs = reinterpret_cast<uint32_t *>(slab + ((int64_t)south * 2 + (epoch & 1)) * SLAB + x);
                    uint32_t *fn = reinterpret_cast<uint32_t *>(slab + ((int64_t)north * 2 + (epoch & 1)) * SLAB + x);
                    if (!take_rows_polled<NN, TH, HALO, R>(st, fs, fn, lo, wv, comp, spin_cap))
                        __hip_atomic_store(bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    __syncthreads();
                    if (*bad) {
                        dead = true;
                        break;
                    }
                    continue;
                }
                // After the last window: a band writes its final rows only
                // once both neighbours have loaded this patch, i.e. have
                // signalled this round through their counters.
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (tid == 0) {
                    __hip_atomic_store(flags + me, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    // both counters read together each pass; at most
                    // spin_cap polls (0: give up without polling)
                    uint32_t it = 0;
                    for (;;) {
                        if (it >= spin_cap) {
                            *bad = 1;
                            break;
                        }
                        const int32_t fs = __hip_atomic_load(flags + south, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const int32_t fn = __hip_atomic_load(flags + north, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (fs >= epoch && fn >= epoch) break;
                        ++it;
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                __syncthreads();
                if (*bad) {
                    dead = true;
                    break;
                }
            }
        }
        // owned rows back to the corrector (NaN after a failed wait)
        int gy = gy0, xs = x;
        asm volatile("" : "+v"(gy), "+v"(xs));
        const float poison = __builtin_nanf("");
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int yy = y0 + r;
            if (yy < HALO || yy >= HALO + TH) continue;
            const float v = wv[r];
            wf[((gy + r) & MASK) * NN + xs] = dead ? poison : v;
        }
    }
}

// Grid: groups * PER workgroups.  With a multiple of 8 groups the mapping is
// XCD-aware (workgroup i runs on XCD i mod 8): the PER members of a group
// take consecutive slots of one XCD, so their slabs and counters stay in that
// XCD's L2.
template <int NN, int TH, int HALO, int R, bool FRAME = false, bool PIPE = false>
__global__ __launch_bounds__(NN *(TH + 2 * HALO) / R) void k_solve_ring(
    const shmm_domain *__restrict__ dom, const int32_t *__restrict__ list, int32_t count,
    const float *__restrict__ vx, const float *__restrict__ vy, const double *__restrict__ Kb,
    float *__restrict__ w, int64_t cells_total, float *__restrict__ slab, int32_t *__restrict__ flags,
    int32_t step_begin, int32_t s_cap, uint32_t spin_cap) {
    using S = RingShape<NN, TH, HALO>;
    __shared__ float buf[2 * NN * S::H];
    __shared__ int bad;
    const int groups = (int)gridDim.x / S::PER;
    int group, member;
    if (groups % 8 == 0) {
        const int local = (int)blockIdx.x >> 3;
        group = ((int)blockIdx.x & 7) + 8 * (local / S::PER);
        member = local % S::PER;
    } else {
        group = (int)blockIdx.x / S::PER;
        member = (int)blockIdx.x % S::PER;
    }
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    if (member & 1)
        ring_body<NN, TH, HALO, R, 1, FRAME, PIPE>(buf, &bad, dom, list, count, group, groups, member >> 1, vx, vy, Kb, w,
                                      cells_total, slab, flags, step_begin, s_cap, spin_cap);
    else
        ring_body<NN, TH, HALO, R, 0, FRAME, PIPE>(buf, &bad, dom, list, count, group, groups, member >> 1, vx, vy, Kb, w,
                                      cells_total, slab, flags, step_begin, s_cap, spin_cap);
}

__global__ void k_zero_rounds(int32_t *flags, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = 0;
}

// Every slab word empty (kSlabEmpty) before the bands start.
__global__ void k_empty_slabs(uint32_t *slab, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        slab[i] = kSlabEmpty;
}

constexpr int kRingNN = 256, kRingTH = 32, kRingHalo = 8, kRingR = 16;

template <bool FRAME, bool PIPE>
const void *ring_kernel() {
    return reinterpret_cast<const void *>(&k_solve_ring<kRingNN, kRingTH, kRingHalo, kRingR, FRAME, PIPE>);
}

}  // namespace

int launch_ring_solve(const shmm_domain *d_dom, const int32_t *d_list, int32_t nlist, int n, const float *vx,
                      const float *vy, const double *Kb, float *w, int64_t cells_total, int32_t step_begin,
                      int32_t s_end, void *work, size_t work_bytes, hipStream_t s, bool frame,
                      uint32_t spin_cap, bool pipe) {
    using S = RingShape<kRingNN, kRingTH, kRingHalo>;
    if (n != kRingNN) return SHMM_EINVAL;
    if (nlist <= 0 || step_begin >= s_end) return SHMM_OK;
    constexpr int threads = kRingNN * S::H / kRingR;
    int dev = 0, cus = 0, occ = 0;
    SHMM_HIP_CHECK(hipGetDevice(&dev));
    SHMM_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // occupancy of the instantiation that is launched
    const void *fn = frame ? (pipe ? ring_kernel<true, true>() : ring_kernel<true, false>())
                           : (pipe ? ring_kernel<false, true>() : ring_kernel<false, false>());
    SHMM_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, threads, 0));
    // every workgroup of the grid fits on the device at once
    int64_t groups = std::min<int64_t>(nlist, (int64_t)cus * occ / S::PER);
    if (groups < 1) return SHMM_EDEVICE;
    // a multiple of 8 groups (the XCD-aware mapping) unless that adds a
    // round of patches per group
    const int64_t g8 = groups - groups % 8;
    if (g8 >= 8 && (nlist + g8 - 1) / g8 == (nlist + groups - 1) / groups) groups = g8;
    const size_t need = (size_t)groups * S::PER * (2 * S::SLAB * sizeof(float) + sizeof(int32_t));
    if (!work || work_bytes < need) return SHMM_ENOMEM;
    float *slab = (float *)work;
    int32_t *flags = (int32_t *)(slab + (size_t)groups * S::PER * 2 * S::SLAB);
    const int nflags = (int)(groups * S::PER);
    hipLaunchKernelGGL(k_zero_rounds, dim3((unsigned)((nflags + 255) / 256)), dim3(256), 0, s, flags, nflags);
    SHMM_HIP_CHECK(hipGetLastError());
    const int64_t slab_words = (int64_t)groups * S::PER * 2 * S::SLAB;
    hipLaunchKernelGGL(k_empty_slabs, dim3(1024), dim3(256), 0, s, reinterpret_cast<uint32_t *>(slab), slab_words);
    SHMM_HIP_CHECK(hipGetLastError());
    const dim3 grid((unsigned)(groups * S::PER));
    if (frame && pipe)
        hipLaunchKernelGGL((k_solve_ring<kRingNN, kRingTH, kRingHalo, kRingR, true, true>), grid, dim3(threads), 0, s,
                           d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, slab, flags, step_begin, s_end, spin_cap);
    else if (frame)
        hipLaunchKernelGGL((k_solve_ring<kRingNN, kRingTH, kRingHalo, kRingR, true, false>), grid, dim3(threads), 0,
                           s, d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, slab, flags, step_begin, s_end,
                           spin_cap);
    else if (pipe)
        hipLaunchKernelGGL((k_solve_ring<kRingNN, kRingTH, kRingHalo, kRingR, false, true>), grid, dim3(threads), 0,
                           s, d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, slab, flags, step_begin, s_end,
                           spin_cap);
    else
        hipLaunchKernelGGL((k_solve_ring<kRingNN, kRingTH, kRingHalo, kRingR, false, false>), grid, dim3(threads), 0,
                           s, d_dom, d_list, nlist, vx, vy, Kb, w, cells_total, slab, flags, step_begin, s_end,
                           spin_cap);
    SHMM_HIP_CHECK(hipGetLastError());
    return SHMM_OK;
}

}  // namespace shmm
