// Internal declarations of the SHMM library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "shmm.h"

#define SHMM_HIP_CHECK(expr)                                   \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return shmm::hip_fail(e_, #expr);\
    } while (0)

namespace shmm {

int hip_fail(hipError_t e, const char *what);

// Per-instance parameters as the kernels see them.
struct InstDev {
    double kappa;
    const double *psi_hat;   // device, interleaved complex, [(2 kmax + 1)^2]
    int32_t kmax;
    int32_t L;
    int32_t thresh[SHMM_MAX_LEVELS];
};

// Which band a wavenumber belongs to (Section 3.1, closed form of the
// recursive split: the level is fixed by min(|k1|,|k2|), the part by max).
__host__ __device__ inline int band_level(int k1, int k2, const int32_t *thresh, int L) {
    int a1 = k1 < 0 ? -k1 : k1, a2 = k2 < 0 ? -k2 : k2;
    int m = a1 < a2 ? a1 : a2;
    int l = 0;
    while (l < L - 1 && m > thresh[l]) ++l;
    return l;
}

__host__ __device__ inline int band_part(int k1, int k2, int l, const int32_t *thresh, int L) {
    if (l == L - 1) return SHMM_DIAG;
    int a1 = k1 < 0 ? -k1 : k1, a2 = k2 < 0 ? -k2 : k2;
    int a = thresh[l];
    if (a1 <= a && a2 <= a) return SHMM_DIAG;
    return a1 <= a ? SHMM_OFF12 : SHMM_OFF21;
}

// One (instance, level) group of domains: a contiguous range of the table.
struct Group {
    int32_t inst, level;
    int64_t first, count;    // domain range
    int32_t n, N, M;
    int32_t kb1, kb2;        // largest |k1|, |k2| of the level's diagonal band
    int32_t periodic;        // every band mode has k n / N integral: patches are periodic
    int64_t cell_first;      // packed offset of the group's first domain
    const int32_t *d_I0;     // [M] node origin of lattice column qx (device)
    const int32_t *d_J0;     // [M] node origin of lattice row qy (device)
};

// Launchers (one translation unit each).
int launch_band_tags(const InstDev &inst, int8_t *d_tags, hipStream_t s);
int launch_band_filter(const InstDev &inst, const Group &g, const shmm_domain *d_dom,
                       float *d_psi, float *d_vx, float *d_vy, float *d_f1, float *d_f2,
                       double *d_lines, double *d_vmax, void *work, size_t work_bytes, hipStream_t s);
size_t band_filter_workspace(const InstDev &inst, const Group &g);
// windowed patches: faces of the tapered psi, their forcing and advection bounds
int launch_window_patches(const shmm_domain *d_dom, int64_t first, int64_t count, int n, int taper,
                          const float *d_psi, float *d_vx, float *d_vy, float *d_f1, float *d_f2, double *d_vmax,
                          hipStream_t s);

// polls of about a microsecond each before a ring-exchange wait gives up
// (tens of seconds)
constexpr uint32_t kRingSpinCapDefault = 1u << 25;
int launch_local_solve(const shmm_domain *d_dom, const int32_t *d_list, int32_t nlist, int n,
                       int32_t max_steps, const float *vx, const float *vy, const float *f1,
                       const float *f2, const double *Kb, float *w, int64_t cells_total,
                       int32_t step_begin, int32_t steps, int64_t list_cells, void *work,
                       int variant, hipStream_t s, bool frame = false,
                       uint32_t ring_spin_cap = kRingSpinCapDefault);
bool local_solve_resident(int n);
// persistent full-width bands of 256^2 patches with a ring exchange between
// them; work holds the exchange slabs and round counters; pipe: the stage
// input read a row further ahead (same results)
int launch_ring_solve(const shmm_domain *d_dom, const int32_t *d_list, int32_t nlist, int n, const float *vx,
                      const float *vy, const double *Kb, float *w, int64_t cells_total, int32_t step_begin,
                      int32_t s_end, void *work, size_t work_bytes, hipStream_t s, bool frame = false,
                      uint32_t spin_cap = kRingSpinCapDefault, bool pipe = false);
int local_solve_variants(int n);
// frame: the zero-frame (non-periodic) local problem (resident up to 128^2,
// ring-exchange bands at 256^2)
size_t local_solve_workspace(int n, int64_t list_cells, bool frame = false);
int launch_zero_fields(const shmm_domain *d_dom, const int32_t *d_list, int32_t nlist, int n, float *d_w,
                       int64_t cells, hipStream_t s);

int launch_effective_diffusivity_list(const shmm_domain *d_dom, const int32_t *d_list, int64_t count,
                                      const float *f1, const float *f2, const float *w, int64_t cells_total,
                                      const double *Kb, double *K_out, int32_t *status, hipStream_t s);
int launch_effective_diffusivity_window(const shmm_domain *d_dom, int64_t first, int64_t count, int32_t inner,
                                        const float *f1, const float *f2, const float *w, int64_t cells_total,
                                        const double *Kb, double *K_out, int32_t *status, hipStream_t s);
int launch_effective_diffusivity(const shmm_domain *d_dom, int64_t first, int64_t count,
                                 const float *f1, const float *f2, const float *w,
                                 int64_t cells_total, const double *Kb, double *K_out,
                                 double *K_energy, double *mass, int32_t *status, hipStream_t s);

// d_list: null for the range first..first + count - 1, else domains of one size
int launch_chunk_delta(const shmm_domain *d_dom, int64_t first, const int32_t *d_list, int64_t count, const float *f1,
                       const float *f2, const float *w, int64_t cells_total, float *w_prev, int64_t prev_cells,
                       int64_t prev_base, double *out, hipStream_t s);

int launch_level_chain(const shmm_domain *d_dom, const InstDev *d_inst, const int32_t *d_child_start,
                       const int32_t *d_child_idx, int64_t first, int64_t count, int32_t mode,
                       const double *lines, double *K_in, double *K_off, double *K_base,
                       const double *K_solve, double *R, int32_t *status, hipStream_t s);

size_t surrogate_feature_workspace(int n, int64_t nlist);
int launch_patch_features(const shmm_domain *d_dom, const int32_t *d_list, int32_t nlist, int n,
                          const float *vx, const float *vy, const double *Kb, float *features, void *work,
                          hipStream_t s);
size_t surrogate_net_workspace(int64_t B);
int surrogate_train_step(void *model, float *adam, const float *x, const double *Kb, const double *Kt,
                         int64_t B, float lr, float clip, int32_t t, double *loss, float *grad_out, void *work,
                         hipStream_t s);
int surrogate_refresh_bf16(void *model, hipStream_t s);
int surrogate_infer(const void *models, int32_t E, const float *x, const double *Kb, int64_t B,
                    const float *lo, const float *hi, double tau, double emax, double *K_out, uint8_t *flags,
                    double *spread, double *K_members, void *work, hipStream_t s);

int launch_feature_stats(const float *x, int64_t B, double *stats, hipStream_t s);
int launch_chain_gate(const shmm_domain *dom, int64_t first, int64_t count, const double *K_hat,
                      const double *K_base, const double *spread, const double *K_in, double tol, uint8_t *flags,
                      hipStream_t s);
int launch_surrogate_rescale(const float *x, const double *Kb, const double *K, const double *log10c, int64_t B,
                             float *xo, double *Kbo, double *Ko, hipStream_t s);

int launch_mark_status(int32_t *status, const int32_t *list, int64_t count, int32_t bits, hipStream_t s);
// OR SHMM_DOM_NONFINITE into the status of listed domains (one size n) whose correctors hold a NaN/Inf
int launch_mark_nonfinite(const shmm_domain *d_dom, const int32_t *d_list, int32_t nlist, int n, const float *w,
                          int64_t cells_total, int32_t *status, hipStream_t s);

int launch_macro(int32_t N, int32_t bc, double g0, double g1, const void *vx, const void *vy, const double *K,
                 int32_t K_is_field, double dt, int32_t nsteps, void *u, int32_t dtype, void *work, hipStream_t s);
size_t macro_workspace(int32_t N, int32_t dtype);
// the static scratch of the allocation-free macro step: take its address on
// `device` (which must be current) once; macro_scratch returns it (null if
// never set up) and its size
int macro_scratch_setup(int device);
void *macro_scratch(int device, size_t *bytes);

}  // namespace shmm
