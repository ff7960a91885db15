// Host side of the C ABI: context, bookkeeping of the domain hierarchy, step
// planning, and the entry points that enqueue the kernels.
#include <math.h>

#include <cmath>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <vector>

#include "shmm_internal.h"

namespace shmm {

int hip_fail(hipError_t e, const char *what) {
    fprintf(stderr, "shmm: HIP error %d (%s) in %s\n", (int)e, hipGetErrorString(e), what);
    return e == hipErrorOutOfMemory ? SHMM_ENOMEM : SHMM_EDEVICE;
}

namespace {

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Validation shared by shmm_build_levels and shmm_ctx_set_problem.
int validate(const shmm_problem *p, int32_t n_inst) {
    if (!p || n_inst <= 0) return SHMM_EINVAL;
    for (int32_t q = 0; q < n_inst; ++q) {
        const shmm_problem &P = p[q];
        const int L = P.n_levels;
        if (L < 1 || L > SHMM_MAX_LEVELS) return SHMM_EINVAL;
        if (!(P.kappa > 0.0) || P.kmax < 0) return SHMM_EINVAL;
        if (!(P.dt_frac > 0.0 && P.dt_frac <= 1.0) || !(P.delta > 0.0 && P.delta < 1.0)) return SHMM_EINVAL;
        if (!P.n_cells || !P.n_global || !P.lattice || (L > 1 && !P.thresh)) return SHMM_EINVAL;
        for (int l = 0; l + 1 < L - 1; ++l)
            if (!(P.thresh[l + 1] > P.thresh[l])) return SHMM_EINVAL;
        for (int l = 0; l < L; ++l) {
            const int n = P.n_cells[l], N = P.n_global[l], M = P.lattice[l];
            if (n < 4 || !pow2(n) || n > N) return SHMM_EINVAL;
            if (M < 1 || (l > 0 && M % P.lattice[l - 1] != 0)) return SHMM_EINVAL;
            for (int c = 0; c < M; ++c) {
                const int64_t num = (int64_t)N * (2 * c + 1) - (int64_t)n * M;
                if (num % (2 * M) != 0) return SHMM_EINVAL;
            }
        }
    }
    return SHMM_OK;
}

int64_t origin(int N, int n, int M, int c) {
    const int64_t num = (int64_t)N * (2 * c + 1) - (int64_t)n * M;
    int64_t v = (num / (2 * M)) % N;
    return v < 0 ? v + N : v;
}

// Domains stored phase by phase (phase = L - 1 - level), then instance, cy, cx.
void build_table(const shmm_problem *p, int32_t n_inst, std::vector<shmm_domain> &out,
                 int64_t &cells, int64_t &lines, std::vector<int64_t> &phase_first) {
    out.clear();
    phase_first.clear();
    cells = 0;
    lines = 0;
    int maxL = 0;
    for (int32_t q = 0; q < n_inst; ++q) maxL = std::max(maxL, (int)p[q].n_levels);
    std::map<std::pair<int, int>, int64_t> first;
    for (int ph = 0; ph < maxL; ++ph) {
        phase_first.push_back((int64_t)out.size());
        for (int32_t q = 0; q < n_inst; ++q) {
            const int l = p[q].n_levels - 1 - ph;
            if (l < 0) continue;
            const int n = p[q].n_cells[l], N = p[q].n_global[l], M = p[q].lattice[l];
            first[{q, l}] = (int64_t)out.size();
            for (int cy = 0; cy < M; ++cy)
                for (int cx = 0; cx < M; ++cx) {
                    shmm_domain d;
                    memset(&d, 0, sizeof(d));
                    d.instance = q;
                    d.level = l;
                    d.cx = cx;
                    d.cy = cy;
                    d.n = n;
                    d.N = N;
                    d.I0 = (int32_t)origin(N, n, M, cx);
                    d.J0 = (int32_t)origin(N, n, M, cy);
                    d.parent = -1;
                    d.nsteps = 0;
                    d.offset = cells;
                    d.line_offset = lines;
                    d.h = 2.0 * M_PI / (double)N;
                    d.dt = -1.0;   // not planned yet
                    out.push_back(d);
                    cells += (int64_t)n * n;
                    lines += 2 * (int64_t)n;
                }
        }
    }
    phase_first.push_back((int64_t)out.size());
    for (auto &d : out) {
        if (d.level == 0) continue;
        const int M = p[d.instance].lattice[d.level], Mp = p[d.instance].lattice[d.level - 1];
        const int px = ((2 * d.cx + 1) * Mp) / (2 * M);
        const int py = ((2 * d.cy + 1) * Mp) / (2 * M);
        d.parent = (int32_t)(first[{d.instance, d.level - 1}] + (int64_t)py * Mp + px);
    }
}

// One scan of a level's diagonal band: the largest |k1|, |k2| carrying a
// coefficient, and whether every such mode is periodic on an n-cell patch of
// the level grid (k n / N integral in both directions).
void band_stats(const shmm_problem &P, int level, int n, int N, int *kb1, int *kb2, int *periodic) {
    const int K = P.kmax, span = 2 * K + 1;
    *kb1 = 0;
    *kb2 = 0;
    *periodic = 1;
    for (int b = 0; b < span; ++b)
        for (int a = 0; a < span; ++a) {
            const int k1 = a - K, k2 = b - K;
            if (k1 == 0 && k2 == 0) continue;
            const int64_t idx = (int64_t)b * span + a;
            if (P.psi_hat[2 * idx] == 0.0 && P.psi_hat[2 * idx + 1] == 0.0) continue;
            const int l = band_level(k1, k2, P.thresh, P.n_levels);
            if (l != level || band_part(k1, k2, l, P.thresh, P.n_levels) != SHMM_DIAG) continue;
            *kb1 = std::max(*kb1, abs(k1));
            *kb2 = std::max(*kb2, abs(k2));
            if (((int64_t)k1 * n) % N != 0 || ((int64_t)k2 * n) % N != 0) *periodic = 0;
        }
}

// Step plan (see shmm.h).  The expression order is part of the contract.
// rho_A = vmax / h: the Gershgorin bound of the skew advection operator.
int plan_one(const shmm_domain &d, const double *K, double vmax, double dt_frac, double delta,
             double *dt_out, int64_t *nsteps_out) {
    const double K11 = K[0], K12 = K[1], K22 = K[2];
    const double h = d.h;
    const double rho_d = (4.0 * K11 + 4.0 * K22 + 2.0 * fabs(K12)) / (h * h);
    const double rho_a = vmax / h;
    const double dt_lim = 1.0 / (rho_d / 2.785 + rho_a / 2.828);
    const double lam = 0.5 * (K11 + K22) - sqrt(0.25 * (K11 - K22) * (K11 - K22) + K12 * K12);
    if (!(lam > 0.0)) return SHMM_ENOTSPD;
    const double s = sin(M_PI / (double)d.n);
    const double decay = lam * 4.0 * s * s / (h * h);
    const double T = log(1.0 / delta) / decay;
    const double q = ceil(T / (dt_frac * dt_lim));
    if (!(q < 2147483647.0)) return SHMM_ERANGE;
    int64_t nsteps = (int64_t)q;
    if (nsteps < 1) nsteps = 1;
    *nsteps_out = nsteps;
    *dt_out = T / (double)nsteps;
    return SHMM_OK;
}

template <typename T>
int upload(T **dst, const T *src, size_t count) {
    if (*dst) {
        SHMM_HIP_CHECK(hipFree(*dst));
        *dst = nullptr;
    }
    if (count == 0) return SHMM_OK;
    SHMM_HIP_CHECK(hipMalloc((void **)dst, count * sizeof(T)));
    SHMM_HIP_CHECK(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
    return SHMM_OK;
}

}  // namespace
}  // namespace shmm

using namespace shmm;

struct RangeLists {
    std::vector<int> ns;               // distinct n in the range
    std::vector<int32_t *> d_lists;    // device list per n
    std::vector<std::vector<int32_t>> h_lists;   // host copy, in launch order
    std::vector<int32_t> counts;
    std::vector<int64_t> cells;        // cells per list
};

// Launch order of a list: longest plan first.  Workgroups of one size take
// the same time per step, one per CU for the larger sizes, and the hardware
// hands them out in order as CUs free up, so this is longest-processing-time
// list scheduling: the plans of a phase differ (the coarsest level of the
// continuous-spectrum flow spans 1.36e6 to 1.71e6 steps), and table order
// leaves the last CUs running alone for up to 5% of the phase, this order for
// under 1%.  Results do not depend on the order.
static bool order_by_plan(const std::vector<shmm_domain> &table, std::vector<int32_t> &ids) {
    std::vector<int32_t> before = ids;
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int32_t a, int32_t b) { return table[a].nsteps > table[b].nsteps; });
    return ids != before;
}

constexpr int kSideStreams = 3;   // patch sizes of one range solved concurrently

struct shmm_ctx {
    int device = 0;
    hipStream_t side[kSideStreams] = {};   // default priority
    hipEvent_t ev_fork = nullptr, ev_join[kSideStreams] = {};
    std::vector<shmm_problem> probs;
    std::vector<std::vector<double>> psi;
    std::vector<std::vector<int32_t>> geo;   // thresh | n_cells | n_global | lattice per instance
    std::vector<double *> d_psi;
    std::vector<InstDev> inst;
    InstDev *d_inst = nullptr;
    std::vector<shmm_domain> table;
    shmm_domain *d_table = nullptr;
    int64_t cells = 0, lines = 0;
    std::vector<int64_t> phase_first;
    std::vector<Group> groups;
    int32_t *d_origins = nullptr;
    int32_t *d_child_start = nullptr, *d_child_idx = nullptr;
    double *d_vmax = nullptr;                // [nd] advection bound of each patch (band filter)
    std::vector<std::vector<int>> empty;     // [inst][level]: diagonal band without coefficients
    std::map<std::pair<int64_t, int64_t>, RangeLists> lists;
    std::map<int, int> solve_variant;          // patch size n -> kernel variant
    int32_t local_bc = SHMM_LOCAL_PERIODIC;    // boundary of the local problems
    uint32_t ring_spin_cap = kRingSpinCapDefault;   // polls before a ring-exchange wait gives up
    void *work = nullptr;
    size_t work_bytes = 0;
    void *adapt = nullptr;                      // previous correctors and chunk statistics (adaptive stop)
    size_t adapt_bytes = 0;

    int ensure_adapt(size_t bytes) {
        if (bytes <= adapt_bytes) return SHMM_OK;
        if (adapt) {
            SHMM_HIP_CHECK(hipDeviceSynchronize());
            SHMM_HIP_CHECK(hipFree(adapt));
        }
        adapt = nullptr;
        adapt_bytes = 0;
        SHMM_HIP_CHECK(hipMalloc(&adapt, bytes));
        adapt_bytes = bytes;
        return SHMM_OK;
    }

    int ensure_work(size_t bytes) {
        if (bytes <= work_bytes) return SHMM_OK;
        if (work) {
            SHMM_HIP_CHECK(hipDeviceSynchronize());   // kernels may still use the old buffer
            SHMM_HIP_CHECK(hipFree(work));
        }
        work = nullptr;
        work_bytes = 0;
        SHMM_HIP_CHECK(hipMalloc(&work, bytes));
        work_bytes = bytes;
        return SHMM_OK;
    }

    void clear_lists() {
        for (auto &kv : lists)
            for (auto *p : kv.second.d_lists) (void)hipFree(p);
        lists.clear();
        for (auto &kv : seqs) (void)hipFree(kv.second);
        seqs.clear();
    }

    void release() {
        clear_lists();
        for (auto *p : d_psi) (void)hipFree(p);
        d_psi.clear();
        if (d_inst) (void)hipFree(d_inst);
        if (d_table) (void)hipFree(d_table);
        if (d_origins) (void)hipFree(d_origins);
        if (d_child_start) (void)hipFree(d_child_start);
        if (d_child_idx) (void)hipFree(d_child_idx);
        if (d_vmax) (void)hipFree(d_vmax);
        d_vmax = nullptr;
        d_inst = nullptr;
        d_table = nullptr;
        d_origins = nullptr;
        d_child_start = d_child_idx = nullptr;
    }

    // device list first, first + 1, ..., first + count - 1 (cached)
    std::map<std::pair<int64_t, int64_t>, int32_t *> seqs;
    int seq_list(int64_t first, int64_t count, int32_t **out) {
        auto key = std::make_pair(first, count);
        auto it = seqs.find(key);
        if (it == seqs.end()) {
            std::vector<int32_t> v(count);
            for (int64_t i = 0; i < count; ++i) v[i] = (int32_t)(first + i);
            int32_t *p = nullptr;
            int rc = upload(&p, v.data(), v.size());
            if (rc) return rc;
            it = seqs.emplace(key, p).first;
        }
        *out = it->second;
        return SHMM_OK;
    }

    // a device list valid until the next call (synchronous upload)
    int32_t *tmp = nullptr;
    size_t tmp_len = 0;
    int temp_list(const std::vector<int32_t> &v, int32_t **out) {
        if (v.size() > tmp_len) {
            if (tmp) {
                SHMM_HIP_CHECK(hipDeviceSynchronize());
                SHMM_HIP_CHECK(hipFree(tmp));
            }
            tmp = nullptr;
            tmp_len = 0;
            SHMM_HIP_CHECK(hipMalloc((void **)&tmp, v.size() * sizeof(int32_t)));
            tmp_len = v.size();
        }
        SHMM_HIP_CHECK(hipDeviceSynchronize());   // earlier launches may still read the old list
        SHMM_HIP_CHECK(hipMemcpy(tmp, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        *out = tmp;
        return SHMM_OK;
    }

    int range_lists(int64_t first, int64_t count, RangeLists **out) {
        auto key = std::make_pair(first, count);
        auto it = lists.find(key);
        if (it == lists.end()) {
            RangeLists rl;
            std::map<int, std::vector<int32_t>> byn;
            for (int64_t d = first; d < first + count; ++d)
                if (!empty[table[d].instance][table[d].level]) byn[table[d].n].push_back((int32_t)d);
            for (auto &kv : byn) {
                order_by_plan(table, kv.second);
                int32_t *p = nullptr;
                int rc = upload(&p, kv.second.data(), kv.second.size());
                if (rc) return rc;
                rl.ns.push_back(kv.first);
                rl.d_lists.push_back(p);
                rl.h_lists.push_back(kv.second);
                rl.counts.push_back((int32_t)kv.second.size());
                rl.cells.push_back((int64_t)kv.second.size() * kv.first * kv.first);
            }
            it = lists.emplace(key, rl).first;
        }
        *out = &it->second;
        return SHMM_OK;
    }
};

// Kernel variant per patch size when no tuning result was set: the
// LDS-staged kernel in coefficient form with pipelined reads, and at 256^2 the
// ring-exchange bands with pipelined reads (the fastest in the measurements
// on MI355X; sizes below 64 have no other variant).
static int default_solve_variant(int n) { return n == 64 ? 5 : n == 128 ? 7 : n == 256 ? 7 : 0; }

// The ring-exchange bands (n = 256, variants 6 and 7) need every workgroup of a
// group running at once; beside kernels that hold CUs for whole solves they
// would sit partly dispatched, so they run alone.
static bool runs_alone(int n, int variant) { return n == 256 && (variant == 6 || variant == 7); }

static int set_device(shmm_ctx *ctx) {
    SHMM_HIP_CHECK(hipSetDevice(ctx->device));
    return SHMM_OK;
}

static bool range_ok(shmm_ctx *ctx, int64_t first, int64_t count) {
    return ctx && first >= 0 && count >= 0 && first + count <= (int64_t)ctx->table.size();
}

// Quasi-stationary stop (HMM step 2) over the domains `ids`: contiguous in
// the table when d_list is null, else all of one size with d_list their
// device copy.  advance(s0, C) runs steps [s0, s0 + C) of every listed domain
// (capped by its plan).  After each chunk the change of both correctors over
// the chunk, the forcings and <f_i w_j> are measured in FP64.  The step
// operator contracts the error w - chi (chi the steady corrector) at least by
// rho = exp(-mu C dt) per chunk in the mean square, mu the Poincare rate of
// the step plan, so rms(w - chi) <= rho / (1 - rho) rms(w - w_prev), and every
// entry of K - K_b = <f_i w_j> is within rms(f_i) rms(w_j - chi_j) of its
// limit.  A domain stops once that is at most tol (0: its instance's delta)
// times the largest entry of its current K: its plan is cut to the steps
// taken.  Synchronises the stream after every chunk.
template <typename Advance>
static int adaptive_loop(shmm_ctx *ctx, const std::vector<int32_t> &ids, const int32_t *d_list, const float *d_f1,
                         const float *d_f2, const double *d_K_base, float *d_w, int32_t chunks, double tol,
                         hipStream_t s, Advance advance) {
    const int64_t count = (int64_t)ids.size();
    if (count == 0) return SHMM_OK;
    int32_t longest = 0;
    for (int32_t d : ids) longest = std::max(longest, ctx->table[d].nsteps);
    if (longest == 0) return SHMM_OK;
    const int32_t C = (int32_t)(((int64_t)longest + chunks - 1) / chunks);
    int64_t base = 0, rcells = 0;
    if (d_list) {
        rcells = count * (int64_t)ctx->table[ids[0]].n * ctx->table[ids[0]].n;
    } else {
        const shmm_domain &last = ctx->table[ids.back()];
        base = ctx->table[ids[0]].offset;
        rcells = last.offset + (int64_t)last.n * last.n - base;
    }
    const size_t prev_bytes = (size_t)2 * rcells * sizeof(float);
    int rc = ctx->ensure_adapt(prev_bytes + (size_t)8 * count * sizeof(double));
    if (rc) return rc;
    float *w_prev = (float *)ctx->adapt;
    double *d_stats = (double *)((char *)ctx->adapt + prev_bytes);
    const int64_t nd = (int64_t)ctx->table.size();
    std::vector<double> Kb(3 * nd), stats(8 * count);
    SHMM_HIP_CHECK(hipMemcpyAsync(Kb.data(), d_K_base, Kb.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    // w_prev <- the initial correctors (the statistics of this pass are discarded)
    if ((rc = launch_chunk_delta(ctx->d_table, ids[0], d_list, count, d_f1, d_f2, d_w, ctx->cells, w_prev, rcells,
                                 base, d_stats, s)))
        return rc;
    SHMM_HIP_CHECK(hipStreamSynchronize(s));
    for (int32_t s0 = 0; s0 < longest; s0 += C) {
        if ((rc = advance(s0, C))) return rc;
        if ((rc = launch_chunk_delta(ctx->d_table, ids[0], d_list, count, d_f1, d_f2, d_w, ctx->cells, w_prev,
                                     rcells, base, d_stats, s)))
            return rc;
        SHMM_HIP_CHECK(hipMemcpyAsync(stats.data(), d_stats, stats.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        SHMM_HIP_CHECK(hipStreamSynchronize(s));
        const int64_t done = (int64_t)s0 + C;
        bool running = false, changed = false;
        for (int64_t i = 0; i < count; ++i) {
            shmm_domain &D = ctx->table[ids[i]];
            if ((int64_t)D.nsteps <= done) continue;   // finished with this chunk, or never started
            const double *k = Kb.data() + 3 * (int64_t)ids[i];
            const double lam = 0.5 * (k[0] + k[2]) - std::sqrt(0.25 * (k[0] - k[2]) * (k[0] - k[2]) + k[1] * k[1]);
            const double sn = std::sin(M_PI / D.n);
            const double mu = lam * 4.0 * sn * sn / (D.h * D.h);
            const double rho = std::exp(-mu * (double)C * D.dt);
            const double cells = (double)D.n * D.n;
            const double *st = stats.data() + 8 * i;
            const double dw = std::sqrt(std::max(st[0], st[1]) / cells), fr = std::sqrt(std::max(st[2], st[3]) / cells);
            const double bound = fr * dw * rho / (1.0 - rho);
            const double t = tol > 0.0 ? tol : ctx->probs[D.instance].delta;
            const double K11 = k[0] + st[4] / cells, K12 = k[1] + 0.5 * (st[5] + st[6]) / cells,
                         K22 = k[2] + st[7] / cells;
            const double scale = std::max(std::fabs(K11), std::max(std::fabs(K12), std::fabs(K22)));
            if (rho < 1.0 && bound <= t * scale) {
                D.nsteps = (int32_t)done;
                changed = true;
            } else {
                running = true;
            }
        }
        if (changed) {
            if (d_list)
                SHMM_HIP_CHECK(hipMemcpy(ctx->d_table, ctx->table.data(), nd * sizeof(shmm_domain),
                                         hipMemcpyHostToDevice));
            else
                SHMM_HIP_CHECK(hipMemcpy(ctx->d_table + ids[0], ctx->table.data() + ids[0],
                                         count * sizeof(shmm_domain), hipMemcpyHostToDevice));
        }
        if (!running) break;
    }
    return SHMM_OK;
}

extern "C" {

int shmm_ctx_create(shmm_ctx **ctx, int device) {
    if (!ctx) return SHMM_EINVAL;
    int ndev = 0;
    SHMM_HIP_CHECK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return SHMM_EINVAL;
    SHMM_HIP_CHECK(hipSetDevice(device));
    // once per device: the address of the allocation-free macro step's scratch
    int rc = macro_scratch_setup(device);
    if (rc) return rc;
    shmm_ctx *c = new shmm_ctx();
    c->device = device;
    *ctx = c;
    return SHMM_OK;
}

int shmm_ctx_destroy(shmm_ctx *ctx) {
    if (!ctx) return SHMM_OK;
    (void)hipSetDevice(ctx->device);
    ctx->release();
    if (ctx->work) (void)hipFree(ctx->work);
    if (ctx->adapt) (void)hipFree(ctx->adapt);
    if (ctx->tmp) (void)hipFree(ctx->tmp);
    for (int i = 0; i < kSideStreams; ++i) {
        if (ctx->side[i]) (void)hipStreamDestroy(ctx->side[i]);
        if (ctx->ev_join[i]) (void)hipEventDestroy(ctx->ev_join[i]);
    }
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    delete ctx;
    return SHMM_OK;
}

int shmm_build_levels(const shmm_problem *p, int32_t n_inst, shmm_domain *out, int64_t *n_domains,
                      int64_t *n_cells_total, int64_t *n_lines_total) {
    int rc = validate(p, n_inst);
    if (rc) return rc;
    std::vector<shmm_domain> t;
    std::vector<int64_t> pf;
    int64_t cells = 0, lines = 0;
    build_table(p, n_inst, t, cells, lines, pf);
    if (n_domains) *n_domains = (int64_t)t.size();
    if (n_cells_total) *n_cells_total = cells;
    if (n_lines_total) *n_lines_total = lines;
    if (out) memcpy(out, t.data(), t.size() * sizeof(shmm_domain));
    return SHMM_OK;
}

int shmm_ctx_set_problem(shmm_ctx *ctx, const shmm_problem *p, int32_t n_inst) {
    if (!ctx) return SHMM_EINVAL;
    int rc = validate(p, n_inst);
    if (rc) return rc;
    if ((rc = set_device(ctx))) return rc;
    for (int32_t q = 0; q < n_inst; ++q)
        for (int l = 0; l < p[q].n_levels; ++l)
            if (!pow2(p[q].n_global[l])) return SHMM_ERANGE;
    ctx->release();
    ctx->probs.assign(p, p + n_inst);
    ctx->psi.assign(n_inst, {});
    ctx->geo.assign(n_inst, {});
    ctx->inst.assign(n_inst, InstDev());
    ctx->empty.assign(n_inst, {});
    for (int32_t q = 0; q < n_inst; ++q) {
        shmm_problem &P = ctx->probs[q];
        const int L = P.n_levels;
        const size_t span = 2 * (size_t)P.kmax + 1;
        ctx->psi[q].assign(P.psi_hat, P.psi_hat + 2 * span * span);
        auto &g = ctx->geo[q];
        g.assign(4 * SHMM_MAX_LEVELS, 0);
        for (int l = 0; l + 1 < L; ++l) g[l] = P.thresh[l];
        for (int l = 0; l < L; ++l) {
            g[SHMM_MAX_LEVELS + l] = P.n_cells[l];
            g[2 * SHMM_MAX_LEVELS + l] = P.n_global[l];
            g[3 * SHMM_MAX_LEVELS + l] = P.lattice[l];
        }
        P.psi_hat = ctx->psi[q].data();
        P.thresh = g.data();
        P.n_cells = g.data() + SHMM_MAX_LEVELS;
        P.n_global = g.data() + 2 * SHMM_MAX_LEVELS;
        P.lattice = g.data() + 3 * SHMM_MAX_LEVELS;
        double *dp = nullptr;
        if ((rc = upload(&dp, ctx->psi[q].data(), ctx->psi[q].size()))) return rc;
        ctx->d_psi.push_back(dp);
        InstDev &I = ctx->inst[q];
        I.kappa = P.kappa;
        I.psi_hat = dp;
        I.kmax = P.kmax;
        I.L = L;
        for (int l = 0; l < SHMM_MAX_LEVELS; ++l) I.thresh[l] = l + 1 < L ? P.thresh[l] : 0;
        for (int l = 0; l < L; ++l) ctx->empty[q].push_back(0);
    }
    if ((rc = upload(&ctx->d_inst, ctx->inst.data(), ctx->inst.size()))) return rc;
    build_table(ctx->probs.data(), n_inst, ctx->table, ctx->cells, ctx->lines, ctx->phase_first);
    if ((rc = upload(&ctx->d_table, ctx->table.data(), ctx->table.size()))) return rc;
    {
        std::vector<double> zero(ctx->table.size() ? ctx->table.size() : 1, -1.0);
        if ((rc = upload(&ctx->d_vmax, zero.data(), zero.size()))) return rc;
    }
    // groups (instance, level) and the band extents; lattice origins per group
    ctx->groups.clear();
    std::vector<int32_t> origins;
    const int64_t nd = (int64_t)ctx->table.size();
    for (int64_t d = 0; d < nd;) {
        const shmm_domain &D = ctx->table[d];
        Group g;
        g.inst = D.instance;
        g.level = D.level;
        g.first = d;
        g.n = D.n;
        g.N = D.N;
        g.M = ctx->probs[D.instance].lattice[D.level];
        g.count = (int64_t)g.M * g.M;
        band_stats(ctx->probs[D.instance], D.level, g.n, g.N, &g.kb1, &g.kb2, &g.periodic);
        ctx->empty[D.instance][D.level] = (g.kb1 == 0 && g.kb2 == 0) ? 1 : 0;
        g.cell_first = D.offset;
        if (2 * std::max(g.kb1, g.kb2) + 1 > g.N) return SHMM_ERANGE;
        g.d_I0 = (const int32_t *)(intptr_t)origins.size();   // fixed up after upload
        for (int c = 0; c < g.M; ++c) origins.push_back(ctx->table[d + c].I0);
        for (int c = 0; c < g.M; ++c) origins.push_back(ctx->table[d + (int64_t)c * g.M].J0);
        ctx->groups.push_back(g);
        d += g.count;
    }
    if ((rc = upload(&ctx->d_origins, origins.data(), origins.size()))) return rc;
    for (auto &g : ctx->groups) {
        const intptr_t base = (intptr_t)g.d_I0;
        g.d_I0 = ctx->d_origins + base;
        g.d_J0 = ctx->d_origins + base + g.M;
    }
    // children lists (CSR) for Algorithm 3
    std::vector<std::vector<int32_t>> ch(nd);
    for (int64_t d = 0; d < nd; ++d)
        if (ctx->table[d].parent >= 0) ch[ctx->table[d].parent].push_back((int32_t)d);
    std::vector<int32_t> start(nd + 1, 0), idx;
    for (int64_t d = 0; d < nd; ++d) {
        start[d] = (int32_t)idx.size();
        idx.insert(idx.end(), ch[d].begin(), ch[d].end());
    }
    start[nd] = (int32_t)idx.size();
    if ((rc = upload(&ctx->d_child_start, start.data(), start.size()))) return rc;
    if (idx.empty()) idx.push_back(0);
    if ((rc = upload(&ctx->d_child_idx, idx.data(), idx.size()))) return rc;
    return SHMM_OK;
}

int shmm_ctx_table(shmm_ctx *ctx, const shmm_domain **table, int64_t *n_domains,
                   int64_t *n_cells_total, int64_t *n_lines_total, const int64_t **phase_first,
                   int32_t *n_phases) {
    if (!ctx) return SHMM_EINVAL;
    if (table) *table = ctx->table.data();
    if (n_domains) *n_domains = (int64_t)ctx->table.size();
    if (n_cells_total) *n_cells_total = ctx->cells;
    if (n_lines_total) *n_lines_total = ctx->lines;
    if (phase_first) *phase_first = ctx->phase_first.data();
    if (n_phases) *n_phases = (int32_t)ctx->phase_first.size() - 1;
    return SHMM_OK;
}

int shmm_band_tags(shmm_ctx *ctx, int32_t inst, int8_t *d_tags, void *stream) {
    if (!ctx || inst < 0 || inst >= (int32_t)ctx->inst.size() || !d_tags) return SHMM_EINVAL;
    int rc = set_device(ctx);
    if (rc) return rc;
    return launch_band_tags(ctx->inst[inst], d_tags, (hipStream_t)stream);
}

int shmm_plan_steps(shmm_ctx *ctx, int64_t first, int64_t count, const double *K_base,
                    const double *vmax) {
    if (!range_ok(ctx, first, count) || !K_base) return SHMM_EINVAL;
    int rc = set_device(ctx);
    if (rc) return rc;
    std::vector<double> vm;
    if (!vmax) {   // the band filter's per-patch bounds
        vm.assign(ctx->table.size(), -1.0);
        if (count > 0) {
            SHMM_HIP_CHECK(hipDeviceSynchronize());
            SHMM_HIP_CHECK(hipMemcpy(vm.data() + first, ctx->d_vmax + first, count * sizeof(double),
                                     hipMemcpyDeviceToHost));
        }
        vmax = vm.data();
    }
    for (int64_t d = first; d < first + count; ++d) {
        shmm_domain &D = ctx->table[d];
        const shmm_problem &P = ctx->probs[D.instance];
        double dt = 0.0;
        int64_t ns = 0;
        const bool empty = ctx->empty[D.instance][D.level] != 0;
        if (!empty && !(vmax[d] >= 0.0)) return SHMM_EINVAL;   // band filter not run on this range
        rc = plan_one(D, K_base + 3 * d, empty ? 0.0 : vmax[d], P.dt_frac, P.delta, &dt, &ns);
        if (rc) return rc;
        if (ctx->empty[D.instance][D.level]) {
            // zero forcing: the corrector stays zero, nothing to integrate
            dt = 0.0;
            ns = 0;
        }
        D.dt = dt;
        D.nsteps = (int32_t)ns;
    }
    if (count > 0)
        SHMM_HIP_CHECK(hipMemcpy(ctx->d_table + first, ctx->table.data() + first,
                                 count * sizeof(shmm_domain), hipMemcpyHostToDevice));
    // launch lists of ranges that overlap the new plans: longest plan first
    // again, rewritten in place (a captured graph keeps its list pointers)
    bool synced = false;
    for (auto &kv : ctx->lists) {
        const int64_t a = kv.first.first, b = kv.first.first + kv.first.second;
        if (b <= first || a >= first + count) continue;
        RangeLists &rl = kv.second;
        for (size_t q = 0; q < rl.h_lists.size(); ++q) {
            if (!order_by_plan(ctx->table, rl.h_lists[q])) continue;
            if (!synced) {   // no solve may be reading a list while it is rewritten
                SHMM_HIP_CHECK(hipDeviceSynchronize());
                synced = true;
            }
            SHMM_HIP_CHECK(hipMemcpy(rl.d_lists[q], rl.h_lists[q].data(), rl.h_lists[q].size() * sizeof(int32_t),
                                     hipMemcpyHostToDevice));
        }
    }
    return SHMM_OK;
}

int shmm_band_filter(shmm_ctx *ctx, int64_t first, int64_t count, float *d_psi, float *d_vx,
                     float *d_vy, float *d_f1, float *d_f2, double *d_lines, void *stream) {
    if (!range_ok(ctx, first, count) || !d_vx || !d_vy || !d_f1 || !d_f2 || !d_lines)
        return SHMM_EINVAL;
    int rc = set_device(ctx);
    if (rc) return rc;
    int64_t covered = 0;
    for (const Group &g : ctx->groups) {
        if (g.first + g.count <= first || g.first >= first + count) continue;
        if (g.first < first || g.first + g.count > first + count) return SHMM_EINVAL;
        const size_t need = band_filter_workspace(ctx->inst[g.inst], g);
        if ((rc = ctx->ensure_work(need))) return rc;
        rc = launch_band_filter(ctx->inst[g.inst], g, ctx->d_table, d_psi, d_vx, d_vy, d_f1, d_f2,
                                d_lines, ctx->d_vmax, ctx->work, ctx->work_bytes, (hipStream_t)stream);
        if (rc) return rc;
        covered += g.count;
    }
    return covered == count ? SHMM_OK : SHMM_EINVAL;
}

int shmm_local_solve_batch(shmm_ctx *ctx, int64_t first, int64_t count, const float *d_vx,
                           const float *d_vy, const float *d_f1, const float *d_f2,
                           const double *d_K_base, float *d_w, int32_t step_begin, int32_t steps,
                           int32_t *d_status, void *stream) {
    if (!range_ok(ctx, first, count) || !d_vx || !d_vy || !d_K_base || !d_w || step_begin < 0 ||
        steps < 0)
        return SHMM_EINVAL;
    int rc = set_device(ctx);
    if (rc) return rc;
    for (int64_t d = first; d < first + count; ++d)
        if (ctx->table[d].nsteps < 0 || ctx->table[d].dt < 0.0) return SHMM_EINVAL;   // unplanned
    RangeLists *rl = nullptr;
    if ((rc = ctx->range_lists(first, count, &rl))) return rc;
    const size_t groups = rl->ns.size();
    // Patch sizes of the range run concurrently: the group that needs the
    // workspace (at most one size does) and the first group go on the
    // caller's stream, the others on side streams forked from and joined back
    // into it with events.  A group that runs alone (the ring-exchange bands)
    // goes first on the caller's stream, and the fork follows it.
    std::vector<int> variant(groups);
    for (size_t q = 0; q < groups; ++q) {
        const auto it = ctx->solve_variant.find(rl->ns[q]);
        variant[q] = it == ctx->solve_variant.end() ? default_solve_variant(rl->ns[q]) : it->second;
    }
    size_t need = 0;
    const bool frame = ctx->local_bc == SHMM_LOCAL_ZERO_FRAME;
    for (size_t q = 0; q < groups; ++q)
        need = std::max(need, local_solve_workspace(rl->ns[q], rl->cells[q], frame));
    if (need && (rc = ctx->ensure_work(need))) return rc;
    hipStream_t main_s = (hipStream_t)stream;
    auto max_steps_of = [&](size_t q) {
        int32_t m = 0;
        for (int64_t d = first; d < first + count; ++d)
            if (ctx->table[d].n == rl->ns[q]) m = std::max(m, ctx->table[d].nsteps);
        return m;
    };
    std::vector<size_t> rest;
    for (size_t q = 0; q < groups; ++q) {
        if (groups > 1 && runs_alone(rl->ns[q], variant[q])) {
            rc = launch_local_solve(ctx->d_table, rl->d_lists[q], rl->counts[q], rl->ns[q], max_steps_of(q), d_vx,
                                    d_vy, d_f1, d_f2, d_K_base, d_w, ctx->cells, step_begin, steps, rl->cells[q],
                                    ctx->work, variant[q], main_s, frame, ctx->ring_spin_cap);
            if (rc) return rc;
        } else {
            rest.push_back(q);
        }
    }
    int n_work = 0;
    for (size_t q : rest) n_work += local_solve_workspace(rl->ns[q], rl->cells[q], frame) ? 1 : 0;
    const bool concurrent = rest.size() > 1 && n_work <= 1;
    bool used[kSideStreams] = {};
    if (concurrent) {
        if (!ctx->ev_fork) {
            SHMM_HIP_CHECK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
            for (int i = 0; i < kSideStreams; ++i) {
                SHMM_HIP_CHECK(hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking));
                SHMM_HIP_CHECK(hipEventCreateWithFlags(&ctx->ev_join[i], hipEventDisableTiming));
            }
        }
        SHMM_HIP_CHECK(hipEventRecord(ctx->ev_fork, main_s));
    }
    int next_side = 0;
    for (size_t k = 0; k < rest.size(); ++k) {
        const size_t q = rest[k];
        hipStream_t s = main_s;
        const bool on_main = !concurrent || local_solve_workspace(rl->ns[q], rl->cells[q], frame) ||
                             (n_work == 0 && k == 0);
        if (!on_main) {
            const int i = next_side++ % kSideStreams;
            s = ctx->side[i];
            if (!used[i]) SHMM_HIP_CHECK(hipStreamWaitEvent(s, ctx->ev_fork, 0));
            used[i] = true;
        }
        rc = launch_local_solve(ctx->d_table, rl->d_lists[q], rl->counts[q], rl->ns[q], max_steps_of(q),
                                d_vx, d_vy, d_f1, d_f2, d_K_base, d_w, ctx->cells, step_begin, steps,
                                rl->cells[q], ctx->work, variant[q], s, frame, ctx->ring_spin_cap);
        if (rc) return rc;
    }
    for (int i = 0; i < kSideStreams; ++i)
        if (used[i]) {
            SHMM_HIP_CHECK(hipEventRecord(ctx->ev_join[i], ctx->side[i]));
            SHMM_HIP_CHECK(hipStreamWaitEvent(main_s, ctx->ev_join[i], 0));
        }
    // status: a corrector that is NaN/Inf after the call (a non-finite input,
    // an unstable step, or a ring-exchange band that gave up waiting)
    if (d_status)
        for (size_t q = 0; q < groups; ++q)
            if ((rc = launch_mark_nonfinite(ctx->d_table, rl->d_lists[q], rl->counts[q], rl->ns[q], d_w, ctx->cells,
                                            d_status, main_s)))
                return rc;
    return SHMM_OK;
}

int shmm_local_solve_adaptive(shmm_ctx *ctx, int64_t first, int64_t count, const float *d_vx,
                              const float *d_vy, const float *d_f1, const float *d_f2, const double *d_K_base,
                              float *d_w, int32_t chunks, double tol, int32_t *d_status, void *stream) {
    if (!range_ok(ctx, first, count) || !d_vx || !d_vy || !d_f1 || !d_f2 || !d_K_base || !d_w || chunks < 1 ||
        !(tol >= 0.0) || !std::isfinite(tol))
        return SHMM_EINVAL;
    if (count == 0) return SHMM_OK;
    for (int64_t d = first; d < first + count; ++d)
        if (ctx->table[d].nsteps < 0 || ctx->table[d].dt < 0.0) return SHMM_EINVAL;   // unplanned
    int rc = set_device(ctx);
    if (rc) return rc;
    std::vector<int32_t> ids(count);
    for (int64_t i = 0; i < count; ++i) ids[i] = (int32_t)(first + i);
    return adaptive_loop(ctx, ids, nullptr, d_f1, d_f2, d_K_base, d_w, chunks, tol, (hipStream_t)stream,
                         [&](int32_t s0, int32_t C) {
                             return shmm_local_solve_batch(ctx, first, count, d_vx, d_vy, d_f1, d_f2, d_K_base,
                                                           d_w, s0, C, d_status, stream);
                         });
}

int shmm_effective_diffusivity(shmm_ctx *ctx, int64_t first, int64_t count, const float *d_f1,
                               const float *d_f2, const float *d_w, const double *d_K_base,
                               double *d_K_out, double *d_K_energy, double *d_mass,
                               int32_t *d_status, void *stream) {
    if (!range_ok(ctx, first, count) || !d_f1 || !d_f2 || !d_w || !d_K_base || !d_K_out)
        return SHMM_EINVAL;
    int rc = set_device(ctx);
    if (rc) return rc;
    return launch_effective_diffusivity(ctx->d_table, first, count, d_f1, d_f2, d_w, ctx->cells,
                                        d_K_base, d_K_out, d_K_energy, d_mass, d_status,
                                        (hipStream_t)stream);
}

int shmm_ctx_set_local_bc(shmm_ctx *ctx, int32_t bc) {
    if (!ctx || (bc != SHMM_LOCAL_PERIODIC && bc != SHMM_LOCAL_ZERO_FRAME)) return SHMM_EINVAL;
    ctx->local_bc = bc;
    return SHMM_OK;
}

int shmm_window_patches(shmm_ctx *ctx, int64_t first, int64_t count, int32_t taper, const float *d_psi,
                        float *d_vx, float *d_vy, float *d_f1, float *d_f2, void *stream) {
    if (!range_ok(ctx, first, count) || !d_psi || !d_vx || !d_vy || !d_f1 || !d_f2 || taper < 0)
        return SHMM_EINVAL;
    if (count == 0 || taper == 0) return SHMM_OK;
    const int n = ctx->table[first].n;
    for (int64_t d = first; d < first + count; ++d)
        if (ctx->table[d].n != n) return SHMM_EINVAL;
    if (2 * taper > n) return SHMM_EINVAL;
    int rc = set_device(ctx);
    if (rc) return rc;
    return launch_window_patches(ctx->d_table, first, count, n, taper, d_psi, d_vx, d_vy, d_f1, d_f2, ctx->d_vmax,
                                 (hipStream_t)stream);
}

int shmm_effective_diffusivity_window(shmm_ctx *ctx, int64_t first, int64_t count, int32_t inner,
                                      const float *d_f1, const float *d_f2, const float *d_w,
                                      const double *d_K_base, double *d_K_out, int32_t *d_status, void *stream) {
    if (!range_ok(ctx, first, count) || !d_f1 || !d_f2 || !d_w || !d_K_base || !d_K_out || inner < 0 ||
        (inner & 1))
        return SHMM_EINVAL;
    int rc = set_device(ctx);
    if (rc) return rc;
    return launch_effective_diffusivity_window(ctx->d_table, first, count, inner, d_f1, d_f2, d_w, ctx->cells,
                                               d_K_base, d_K_out, d_status, (hipStream_t)stream);
}

int shmm_level_chain(shmm_ctx *ctx, int64_t first, int64_t count, int32_t mode,
                     const double *d_lines, double *d_K_in, double *d_K_off, double *d_K_base,
                     const double *d_K_solve, double *d_R, int32_t *d_status, void *stream) {
    if (!range_ok(ctx, first, count) || mode < 0 || mode > 3 || !d_lines || !d_K_in || !d_K_off)
        return SHMM_EINVAL;
    if (mode >= 1 && (!d_K_base || !d_R)) return SHMM_EINVAL;
    if (mode == 2 && !d_K_solve) return SHMM_EINVAL;
    int rc = set_device(ctx);
    if (rc) return rc;
    return launch_level_chain(ctx->d_table, ctx->d_inst, ctx->d_child_start, ctx->d_child_idx, first,
                              count, mode, d_lines, d_K_in, d_K_off, d_K_base, d_K_solve, d_R,
                              d_status, (hipStream_t)stream);
}

int shmm_ctx_tune(shmm_ctx *ctx, int32_t key, int32_t value) {
    if (!ctx) return SHMM_EINVAL;
    if (key == SHMM_TUNE_SOLVE_VARIANT_COUNT) return local_solve_variants(value);
    if (key == SHMM_TUNE_RING_SPIN_CAP) {
        if (value < 0) return SHMM_EINVAL;
        ctx->ring_spin_cap = (uint32_t)value;
        return SHMM_OK;
    }
    if (key > 0 && key <= 4096 && (key & (key - 1)) == 0) {
        if (value < 0 || value >= local_solve_variants(key)) return SHMM_EINVAL;
        ctx->solve_variant[key] = value;
        return SHMM_OK;
    }
    return SHMM_EINVAL;
}

int shmm_macro_step(shmm_ctx *ctx, int32_t N, int32_t bc, double g0, double g1, const void *d_vx,
                    const void *d_vy, const double *d_K, int32_t K_is_field, double dt, int32_t nsteps,
                    void *d_u, int32_t dtype, void *stream) {
    if (!ctx || N < 4 || !pow2(N) || !d_K || !d_u || (dtype != 32 && dtype != 64) || nsteps < 0)
        return SHMM_EINVAL;
    if (bc != SHMM_BC_PERIODIC && bc != SHMM_BC_DIRICHLET_X) return SHMM_EINVAL;
    if (bc == SHMM_BC_DIRICHLET_X && !(std::isfinite(g0) && std::isfinite(g1))) return SHMM_EINVAL;
    if ((d_vx == nullptr) != (d_vy == nullptr)) return SHMM_EINVAL;
    int rc = set_device(ctx);
    if (rc) return rc;
    if ((rc = ctx->ensure_work(macro_workspace(N, dtype)))) return rc;
    return launch_macro(N, bc, g0, g1, d_vx, d_vy, d_K, K_is_field, dt, nsteps, d_u, dtype, ctx->work,
                        (hipStream_t)stream);
}

int shmm_macro_step_noalloc(shmm_ctx *ctx, int32_t N, int32_t bc, double g0, double g1, const void *d_vx,
                            const void *d_vy, const double *d_K, int32_t K_is_field, double dt, int32_t nsteps,
                            void *d_u, int32_t dtype, void *stream) {
    if (!ctx || N < 4 || !pow2(N) || !d_K || !d_u || (dtype != 32 && dtype != 64) || nsteps < 0)
        return SHMM_EINVAL;
    if (bc != SHMM_BC_PERIODIC && bc != SHMM_BC_DIRICHLET_X) return SHMM_EINVAL;
    if (bc == SHMM_BC_DIRICHLET_X && !(std::isfinite(g0) && std::isfinite(g1))) return SHMM_EINVAL;
    if ((d_vx == nullptr) != (d_vy == nullptr)) return SHMM_EINVAL;
    if (N > SHMM_MACRO_NOALLOC_MAX_N) return SHMM_ERANGE;
    int rc = set_device(ctx);
    if (rc) return rc;
    size_t bytes = 0;
    void *work = macro_scratch(ctx->device, &bytes);
    if (!work) return SHMM_EDEVICE;   // shmm_ctx_create sets it up
    if (macro_workspace(N, dtype) > bytes) return SHMM_ERANGE;
    return launch_macro(N, bc, g0, g1, d_vx, d_vy, d_K, K_is_field, dt, nsteps, d_u, dtype, work,
                        (hipStream_t)stream);
}

int shmm_patch_features(shmm_ctx *ctx, int64_t first, int64_t count, const float *d_vx,
                        const float *d_vy, const double *d_K_base, float *d_features, void *stream) {
    if (!range_ok(ctx, first, count) || !d_vx || !d_vy || !d_K_base || !d_features) return SHMM_EINVAL;
    if (count == 0) return SHMM_OK;
    const int n = ctx->table[first].n;
    for (int64_t d = first; d < first + count; ++d)
        if (ctx->table[d].n != n) return SHMM_EINVAL;
    int rc = set_device(ctx);
    if (rc) return rc;
    int32_t *list = nullptr;
    if ((rc = ctx->seq_list(first, count, &list))) return rc;
    if ((rc = ctx->ensure_work(surrogate_feature_workspace(n, count)))) return rc;
    return launch_patch_features(ctx->d_table, list, (int32_t)count, n, d_vx, d_vy, d_K_base, d_features,
                                 ctx->work, (hipStream_t)stream);
}

int shmm_surrogate_refresh(shmm_ctx *ctx, void *d_model, void *stream) {
    if (!ctx || !d_model) return SHMM_EINVAL;
    int rc = set_device(ctx);
    if (rc) return rc;
    return surrogate_refresh_bf16(d_model, (hipStream_t)stream);
}

int shmm_surrogate_train_step(shmm_ctx *ctx, void *d_model, float *d_adam, const float *d_x,
                              const double *d_K_base, const double *d_K_true, int64_t B, float lr,
                              float clip, int32_t t, double *d_loss, float *d_grad, void *stream) {
    if (!ctx || !d_model || !d_adam || !d_x || !d_K_base || !d_K_true || !d_loss || B <= 0 || t < 1)
        return SHMM_EINVAL;
    if (B > (1 << 24)) return SHMM_ERANGE;
    int rc = set_device(ctx);
    if (rc) return rc;
    if ((rc = ctx->ensure_work(surrogate_net_workspace(B)))) return rc;
    return surrogate_train_step(d_model, d_adam, d_x, d_K_base, d_K_true, B, lr, clip, t, d_loss, d_grad,
                                ctx->work, (hipStream_t)stream);
}

int shmm_surrogate_infer(shmm_ctx *ctx, const void *d_models, int32_t E, const float *d_x,
                         const double *d_K_base, int64_t B, const float *d_lo, const float *d_hi,
                         double tau, double emax, double *d_K_out, uint8_t *d_flags, double *d_spread,
                         double *d_K_members, void *stream) {
    if (!ctx || !d_models || E < 1 || !d_x || !d_K_base || B < 0 || !d_lo || !d_hi || !d_K_out || !d_flags)
        return SHMM_EINVAL;
    if (B > (1 << 24)) return SHMM_ERANGE;
    if (B == 0) return SHMM_OK;
    int rc = set_device(ctx);
    if (rc) return rc;
    const size_t net = surrogate_net_workspace(B);
    const size_t km = d_K_members ? 0 : (size_t)E * B * 3 * sizeof(double);
    if ((rc = ctx->ensure_work(net + km))) return rc;
    double *Km = d_K_members ? d_K_members : (double *)((char *)ctx->work + net);
    return surrogate_infer(d_models, E, d_x, d_K_base, B, d_lo, d_hi, tau, emax, d_K_out, d_flags, d_spread, Km,
                           ctx->work, (hipStream_t)stream);
}

int shmm_surrogate_chain_gate(shmm_ctx *ctx, int64_t first, int64_t count, const double *d_K_hat,
                              const double *d_K_base, const double *d_spread, const double *d_K_in, double tol,
                              uint8_t *d_flags, void *stream) {
    if (!range_ok(ctx, first, count) || !d_K_hat || !d_K_base || !d_spread || !d_K_in || !d_flags ||
        !(tol > 0.0) || !std::isfinite(tol))
        return SHMM_EINVAL;
    int rc = set_device(ctx);
    if (rc) return rc;
    return launch_chain_gate(ctx->d_table, first, count, d_K_hat, d_K_base, d_spread, d_K_in, tol, d_flags,
                             (hipStream_t)stream);
}

int shmm_feature_stats(shmm_ctx *ctx, const float *d_x, int64_t B, double *d_stats, void *stream) {
    if (!ctx || !d_x || !d_stats || B < 2) return SHMM_EINVAL;
    int rc = set_device(ctx);
    if (rc) return rc;
    return launch_feature_stats(d_x, B, d_stats, (hipStream_t)stream);
}

int shmm_surrogate_rescale(shmm_ctx *ctx, const float *d_x, const double *d_K_base, const double *d_K_true,
                           const double *d_log10c, int64_t B, float *d_x_out, double *d_K_base_out,
                           double *d_K_true_out, void *stream) {
    if (!ctx || B < 0 || !d_x || !d_K_base || !d_K_true || !d_log10c || !d_x_out || !d_K_base_out ||
        !d_K_true_out)
        return SHMM_EINVAL;
    if (B == 0) return SHMM_OK;
    int rc = set_device(ctx);
    if (rc) return rc;
    return launch_surrogate_rescale(d_x, d_K_base, d_K_true, d_log10c, B, d_x_out, d_K_base_out, d_K_true_out,
                                    (hipStream_t)stream);
}

int shmm_fallback_solve(shmm_ctx *ctx, int64_t first, int64_t count, const uint8_t *d_flags,
                        const float *d_vx, const float *d_vy, const float *d_f1, const float *d_f2,
                        const double *d_K_base, float *d_w, double *d_K_out, int32_t chunks, double tol,
                        int32_t *d_status, void *stream) {
    if (!range_ok(ctx, first, count) || !d_flags || !d_vx || !d_vy || !d_f1 || !d_f2 || !d_K_base || !d_w ||
        !d_K_out || chunks < 0 || !(tol >= 0.0) || !std::isfinite(tol))
        return SHMM_EINVAL;
    if (count == 0) return SHMM_OK;
    int rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint8_t> flags(count);
    SHMM_HIP_CHECK(hipMemcpyAsync(flags.data(), d_flags, count, hipMemcpyDeviceToHost, s));
    SHMM_HIP_CHECK(hipStreamSynchronize(s));
    std::map<int, std::vector<int32_t>> byn;
    for (int64_t i = 0; i < count; ++i) {
        if (!flags[i]) continue;
        const shmm_domain &D = ctx->table[first + i];
        if (D.dt < 0.0) return SHMM_EINVAL;   // never planned
        byn[D.n].push_back((int32_t)(first + i));
    }
    for (auto &kv : byn) {
        const int n = kv.first;
        std::vector<int32_t> &ids = kv.second;
        int32_t max_steps = 0;
        for (int32_t d : ids) max_steps = std::max(max_steps, ctx->table[d].nsteps);
        int32_t *dl = nullptr;
        if ((rc = ctx->temp_list(ids, &dl))) return rc;
        if ((rc = launch_zero_fields(ctx->d_table, dl, (int32_t)ids.size(), n, d_w, ctx->cells, s))) return rc;
        const int64_t cells = (int64_t)ids.size() * n * n;
        const bool frame = ctx->local_bc == SHMM_LOCAL_ZERO_FRAME;
        const size_t need = local_solve_workspace(n, cells, frame);
        if (need && (rc = ctx->ensure_work(need))) return rc;
        const auto it = ctx->solve_variant.find(n);
        const int variant = it == ctx->solve_variant.end() ? default_solve_variant(n) : it->second;
        if (chunks > 0) {
            // quasi-stationary stop: the plan bounds each chunk's launches
            rc = adaptive_loop(ctx, ids, dl, d_f1, d_f2, d_K_base, d_w, chunks, tol, s, [&](int32_t s0, int32_t C) {
                int32_t longest = 0;
                for (int32_t d : ids) longest = std::max(longest, ctx->table[d].nsteps);
                return launch_local_solve(ctx->d_table, dl, (int32_t)ids.size(), n, longest, d_vx, d_vy, d_f1, d_f2,
                                          d_K_base, d_w, ctx->cells, s0, C, cells, ctx->work, variant, s, frame,
                                          ctx->ring_spin_cap);
            });
        } else {
            rc = launch_local_solve(ctx->d_table, dl, (int32_t)ids.size(), n, max_steps, d_vx, d_vy, d_f1, d_f2,
                                    d_K_base, d_w, ctx->cells, 0, 2147483647, cells, ctx->work, variant, s,
                                    frame, ctx->ring_spin_cap);
        }
        if (rc) return rc;
        rc = launch_effective_diffusivity_list(ctx->d_table, dl, (int64_t)ids.size(), d_f1, d_f2, d_w,
                                               ctx->cells, d_K_base, d_K_out, d_status, s);
        if (rc) return rc;
        if (d_status) {
            rc = launch_mark_status(d_status, dl, (int64_t)ids.size(), SHMM_DOM_FALLBACK, s);
            if (rc) return rc;
        }
    }
    return SHMM_OK;
}

}  // extern "C"
