/*
 * shmm.h -- C ABI of the MI355X (gfx950) implementation of the hot path of the
 * seamless heterogeneous multiscale method (SHMM) of Lee & Engquist,
 * "Multiscale numerical methods for passive advection-diffusion in
 * incompressible turbulent flow fields" (arXiv:1510.00451).
 *
 * Model problem (eq:model): u_t = v.grad u + kappa Lap u, div v = 0, with
 * v = (-d psi/dx2, d psi/dx1) from a stream function psi (Section 2.1), on the
 * periodic square [0, 2 pi]^2.  At every level of the resolution hierarchy
 * (Section 3, Figure 1) the library
 *   1. Fourier band-filters psi (Section 3.1) into the level's diagonal band,
 *      synthesised at the nodes of every local patch, and its two
 *      off-diagonal bands, reduced to line energies;
 *   2. time-integrates the two periodic corrector problems of every patch
 *      (HMM steps 1-2 of Section 2.2, numerical homogenization K[psi, K; D])
 *      with the finer level's effective diffusivity as base;
 *   3. reduces them to the 2x2 effective diffusivity (the K formula after
 *      eq:homo) and combines levels by Algorithms 1-3.
 * A macro solver (HMM step 4, eq:homo) and a learned surrogate complete it.
 *
 * Conventions shared by every entry point
 *   - All functions return int status: SHMM_OK (0) or a negative SHMM_E*.
 *     On an error the outputs are unspecified and no kernel is left running.
 *     Numerical trouble of single domains is not a call error: it is recorded
 *     in a per-domain int32 status word (SHMM_DOM_* bits).
 *   - Pointers named d_* are device pointers (hipMalloc'd or torch tensors on
 *     the current device); every other pointer is host memory.  All arrays are
 *     caller-owned, contiguous, row-major with x fastest.  The library owns
 *     only what lives inside shmm_ctx (uploaded spectra, descriptor tables,
 *     FFT and reduction workspaces).
 *   - stream is a hipStream_t (NULL = the default stream).  Device entry points
 *     only enqueue work; they do not synchronise unless stated.
 *   - Symmetric 2x2 tensors are stored as three doubles {K11, K12, K22}.
 *   - Packed per-domain fields: domain d owns cells [offset_d, offset_d + n_d^2)
 *     of every packed array, laid out [y][x].  The corrector array w holds the
 *     two correctors back to back: w[0 .. cells) for e_1, w[cells .. 2 cells)
 *     for e_2, where cells = n_cells_total.
 *   - Grid points of a patch: nodes (x0 + i h, y0 + j h); x-faces
 *     (x0 + i h, y0 + (j + 1/2) h); y-faces (x0 + (i + 1/2) h, y0 + j h); cell
 *     centres (x0 + (i + 1/2) h, y0 + (j + 1/2) h); all indices modulo n.
 */
#ifndef SHMM_H
#define SHMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SHMM_OK = 0,
    SHMM_EINVAL = -1,   /* malformed argument (kappa <= 0, n not a power of two, ...) */
    SHMM_ERANGE = -2,   /* a band above the patch Nyquist, or a size beyond a limit */
    SHMM_ENOTSPD = -3,  /* a base diffusivity that is not symmetric positive definite */
    SHMM_EDEVICE = -4,  /* a HIP runtime error */
    SHMM_ENOMEM = -5    /* a device allocation failed */
};

enum {                          /* per-domain status bits (bit 2 is reserved: the step
                                   plan never exceeds the stability bound, dt_frac <= 1) */
    SHMM_DOM_NONFINITE = 1,     /* a corrector or a moment is NaN/Inf */
    SHMM_DOM_NOT_SPD = 2,       /* K_net fell below K_in; its eigenvalues were raised */
    SHMM_DOM_FALLBACK = 8       /* surrogate flagged the patch: plain solve used */
};

enum { SHMM_DIAG = 0, SHMM_OFF12 = 1, SHMM_OFF21 = 2 };

#define SHMM_MAX_LEVELS 8

/* One flow instance and the level geometry chosen for it (eq:model, Section
 * 3, Figure 1).  Level l (0-based) uses n_cells[l]^2-cell patches with spacing
 * h_l = 2 pi / n_global[l], centred on a lattice[l] x lattice[l] lattice of
 * macro points X = 2 pi (c + 1/2) / lattice[l].  thresh holds the band edges
 * a_1 < ... < a_{L-1} (Section 3.1: alpha, alpha^2, ...).  psi_hat is host
 * memory, interleaved complex double, [(2 kmax + 1)][(2 kmax + 1)] indexed
 * [k2 + kmax][k1 + kmax], Hermitian, psi_hat(0) = 0.
 * dt_frac and delta fix the time integration of the local problems (step =
 * dt_frac of the RK4 stability bound; stop when the slowest mode has decayed
 * by delta, the quasi-stationary state of HMM step 2). */
typedef struct shmm_problem {
    double kappa;
    int32_t kmax;
    int32_t n_levels;
    const double *psi_hat;
    const int32_t *thresh;
    const int32_t *n_cells;
    const int32_t *n_global;
    const int32_t *lattice;
    double dt_frac;
    double delta;
} shmm_problem;

/* One local domain Omega at one level (Section 3, Figure 1).  Domains are
 * stored phase by phase: phase p = (L_i - 1) - level, then instance, cy, cx;
 * so each phase of the bottom-up pass and each (instance, level) group is a
 * contiguous range.  Everything but dt and nsteps is fixed by
 * shmm_build_levels; dt and nsteps are set by shmm_plan_steps. */
typedef struct shmm_domain {
    int32_t instance, level, cx, cy;
    int32_t n;          /* cells per side */
    int32_t N;          /* level grid: h = 2 pi / N */
    int32_t I0, J0;     /* node origin x0 = 2 pi I0 / N, y0 = 2 pi J0 / N */
    int32_t parent;     /* domain of the coarser level holding this centre, -1 at level 0 */
    int32_t nsteps;     /* RK4 steps of the local solve */
    int64_t offset;     /* first cell in the packed [domain][y][x] arrays */
    int64_t line_offset;/* first entry in the packed line energies (2 n per domain) */
    double h;           /* 2 pi / N */
    double dt;          /* RK4 step (-1 until planned) */
} shmm_domain;

typedef struct shmm_ctx shmm_ctx;

/* Context on one HIP device.  shmm_ctx_create makes `device` current and
 * keeps it; every later call on the context uses that device. */
int shmm_ctx_create(shmm_ctx **ctx, int device);
int shmm_ctx_destroy(shmm_ctx *ctx);

/* Bookkeeping of the hierarchy of local domains (Section 3, Figure 1: domains
 * of every level centred at the same macro points, side and spacing shrinking
 * together).  Host only, pure, bit-reproducible.  Call with out == NULL to get
 * the sizes; then with out holding *n_domains entries.  Errors: SHMM_EINVAL
 * for malformed geometry (n not a power of two, patch origin off the level
 * grid, lattice not refining its parent's, band edges not increasing,
 * kappa <= 0, dt_frac outside (0, 1], delta outside (0, 1)). */
int shmm_build_levels(const shmm_problem *p, int32_t n_inst, shmm_domain *out,
                      int64_t *n_domains, int64_t *n_cells_total, int64_t *n_lines_total);

/* Load a batch of instances into the context: builds the domain table (as
 * shmm_build_levels), uploads spectra and descriptors.  Synchronous.
 * Errors: as shmm_build_levels; SHMM_ERANGE if a level's diagonal band does
 * not fit its grid (2 K + 1 > N) or a grid is not a power of two;
 * SHMM_ENOMEM / SHMM_EDEVICE. */
int shmm_ctx_set_problem(shmm_ctx *ctx, const shmm_problem *p, int32_t n_inst);

/* Host view of the context's domain table (valid until the next
 * shmm_ctx_set_problem).  *phase_first receives n_phases + 1 range bounds. */
int shmm_ctx_table(shmm_ctx *ctx, const shmm_domain **table, int64_t *n_domains,
                   int64_t *n_cells_total, int64_t *n_lines_total,
                   const int64_t **phase_first, int32_t *n_phases);

/* Band tags of instance `inst` (Section 3.1): d_tags[(2 kmax + 1)^2] int8,
 * tag = 4 * level + part, -1 for k = 0.  Integer, bit-exact. */
int shmm_band_tags(shmm_ctx *ctx, int32_t inst, int8_t *d_tags, void *stream);

/* Step plan of the local solves of domains [first, first + count) (HMM step 2):
 * dt = T/nsteps with T = ln(1/delta) / (lambda_min(K_b) 4 sin^2(pi/n) / h^2)
 * and nsteps = ceil(T / (dt_frac / (rho_D/2.785 + rho_A/2.828))),
 * rho_D = (4 K11 + 4 K22 + 2|K12|)/h^2 and rho_A = vmax_d / h, where vmax_d is
 * max over the patch's cells of (|vx_W| + |vx_E| + |vy_S| + |vy_N|) / 2: the
 * centred advection with discretely divergence-free faces is skew-symmetric,
 * so this Gershgorin value bounds its spectral radius (seam faces of
 * non-periodic patches included).  vmax is host [n_domains] (global index) or
 * NULL to use the values the band filter computed for the range.  A patch whose
 * diagonal band holds no coefficient has zero forcing, so its corrector stays
 * zero: it gets nsteps = 0, dt = 0 and the local solve leaves it untouched.
 * K_base is host [n_domains][3].  Host arithmetic in a fixed expression order
 * (bit-exact for given inputs); updates the context's table on host and device
 * (synchronous).  The launch lists of the local solves run longest plan first:
 * when new plans change that order for a range already solved, its lists are
 * rewritten in place (so graphs that captured them stay valid) after a
 * device-wide synchronisation; the order never changes results.  Errors: SHMM_ENOTSPD if a base is not positive definite;
 * SHMM_EINVAL if vmax is NULL and the band filter has not run on the range. */
int shmm_plan_steps(shmm_ctx *ctx, int64_t first, int64_t count, const double *K_base,
                    const double *vmax);

/* Band filter of domains [first, first + count) (Section 3.1), which must be
 * whole (instance, level) groups.  For each domain writes, in FP32 at the
 * packed offsets:
 *   d_psi (optional, may be NULL): the level's diagonal band at the nodes;
 *   d_vx, d_vy: face velocities vx = -(psi(x, y + h) - psi(x, y))/h on
 *     x-faces and vy = (psi(x + h, y) - psi(x, y))/h on y-faces, synthesised
 *     directly from psi_hat times the exact difference symbol, so the discrete
 *     divergence is at FP32 rounding;
 *   d_f1, d_f2: cell averages of the face components (the forcing of the
 *     corrector problems for the reconstructions e_1, e_2);
 * and in FP64 d_lines (packed, 2 n per domain at line_offset): the off-12 band
 * energies along the n cell-centre columns, then the off-21 band energies
 * along the n cell-centre rows (Algorithm 1, by Parseval).
 * Uses an in-house radix-4/2 Stockham FFT (FP32) on the pruned band. */
int shmm_band_filter(shmm_ctx *ctx, int64_t first, int64_t count, float *d_psi, float *d_vx,
                     float *d_vy, float *d_f1, float *d_f2, double *d_lines, void *stream);

/* Windowed patches (aimed at the non-periodicity of a component on its patch,
 * which the continuous-spectrum example of Section 4 lists among the error
 * sources): replace the face velocities, forcings and advection bounds of
 * domains [first, first + count), which must share one patch size n, by
 * those of the tapered stream function W psi.  W = w(x) w(y) on the patch
 * nodes, with w(i) = sin^2(pi e / (2 taper)) for e = min(i, n - i) < taper
 * and 1 otherwise: 0 on the seam node, so the periodic extension of W psi is
 * smooth.  The faces are FP32 differences of W psi (zero discrete
 * divergence).  d_psi holds psi at the patch nodes, as shmm_band_filter
 * writes it.  taper = 0 changes nothing.  Call before shmm_plan_steps, which
 * uses the new bounds.
 * Errors: SHMM_EINVAL for a negative taper, 2 taper > n, or patch sizes that
 * differ within the range. */
int shmm_window_patches(shmm_ctx *ctx, int64_t first, int64_t count, int32_t taper, const float *d_psi,
                        float *d_vx, float *d_vy, float *d_f1, float *d_f2, void *stream);

/* Boundary of the local problems of every later local solve on the context
 * (shmm_local_solve_batch, shmm_local_solve_adaptive, shmm_fallback_solve).
 * SHMM_LOCAL_PERIODIC (the default): the patch is periodic (Section 2.2).
 * SHMM_LOCAL_ZERO_FRAME: a non-periodic local problem, aimed at the
 * non-periodicity of a component on its patch that the continuous-spectrum
 * example of Section 4 lists among the error sources: the correctors are
 * held at zero on the last row and the last column of every patch, so on the
 * remaining (n - 1)^2 cells they vanish on the boundary, and no face across
 * the patch seam is used.  These solves run on the resident kernels up to
 * 128^2, on the ring-exchange bands at 256^2 and stage by stage otherwise,
 * and are meant for oversampled patches with a windowed estimate
 * (shmm_effective_diffusivity_window).
 * Errors: SHMM_EINVAL for another value. */
#define SHMM_LOCAL_PERIODIC 0
#define SHMM_LOCAL_ZERO_FRAME 1
int shmm_ctx_set_local_bc(shmm_ctx *ctx, int32_t bc);

/* Local solves of domains [first, first + count) (HMM steps 1-2; the two
 * reconstructions with orthogonal gradients of the numerical homogenization):
 * advance both correctors w_j' = div(v w_j + K_b grad w_j) + f_j by classic
 * RK4, steps [step_begin, min(step_begin + steps, nsteps_d)) of each domain.
 * d_K_base is [n_domains][3] (global index), d_w is [2][n_cells_total] FP32
 * in/out.  FP32 stencils with a compensated state update.  Requires
 * shmm_plan_steps on the range; patches planned with zero steps are skipped.
 * d_status (may be NULL): after the call, SHMM_DOM_NONFINITE is ORed into the
 * word of every listed domain whose correctors hold a NaN or an infinity (a
 * non-finite input, or a ring-exchange band that gave up waiting for a
 * neighbour; each call re-reads the correctors of the range once to check).
 * Patches with n <= 128 stay
 * resident in LDS for the whole call; n = 256 advances in full-width bands
 * that exchange ring rows (or, as tuned, in relaunched overlapped regions)
 * and other sizes stage by stage, all through the context's workspace
 * (32 B per listed cell, grown on demand).
 * Errors: SHMM_EINVAL for a range that was never planned; SHMM_ERANGE for
 * more than 32767 patches in one call of a size that runs stage by stage:
 * sizes outside 8..256, the per-stage variant of 256^2 (tuned), and zero-frame
 * 256^2 patches on a tuned variant other than the ring-exchange bands. */
int shmm_local_solve_batch(shmm_ctx *ctx, int64_t first, int64_t count, const float *d_vx,
                           const float *d_vy, const float *d_f1, const float *d_f2,
                           const double *d_K_base, float *d_w, int32_t step_begin,
                           int32_t steps, int32_t *d_status, void *stream);

/* Local solves with the quasi-stationary stop of HMM step 2 (Section 2.2:
 * evolve until the time derivative is small).  Advances the range in chunks
 * of ceil(longest plan / chunks) steps (shmm_local_solve_batch, from step 0;
 * d_w must hold the initial correctors, normally zero) and after each chunk
 * measures, per domain in FP64, the change of both correctors over the chunk
 * and the size of the forcings.  The step operator contracts w - chi (chi
 * the steady corrector) in the mean square at least by rho = exp(-mu C dt)
 * per chunk of C steps, mu the Poincare rate of shmm_plan_steps, so every
 * entry of K - K_b = <f_i w_j> is within rms(f_i) rms(Delta w_j) rho/(1-rho)
 * of its limit.  A domain stops once that bound is at most tol times the
 * largest entry of its current K (tol = 0: the instance's delta); its plan is cut to
 * the steps taken, so shmm_ctx_table reports them.  Domains that never meet
 * the test run their full plan.  Synchronises the stream after every chunk.
 * Uses a context buffer of 8 B per cell of the range plus 64 B per domain.
 * Errors: as shmm_local_solve_batch; SHMM_EINVAL for chunks < 1 or a
 * negative or non-finite tol. */
int shmm_local_solve_adaptive(shmm_ctx *ctx, int64_t first, int64_t count, const float *d_vx,
                              const float *d_vy, const float *d_f1, const float *d_f2,
                              const double *d_K_base, float *d_w, int32_t chunks, double tol,
                              int32_t *d_status, void *stream);

/* Effective diffusivity of domains [first, first + count) (the K formula after
 * eq:homo with the corrector as chi; HMM step 3): FP64 moments of FP32 data,
 *   d_K_out   = K_b + sym(<f_i w_j>)                       [n_domains][3]
 *   d_K_energy= K_b + sym(-<w_i, D_{K_b} w_j>) (optional)   [n_domains][3]
 *   d_mass    = (sum w_1, sum w_2)             (optional)   [n_domains][2]
 * Deterministic (fixed reduction order).  Sets SHMM_DOM_NONFINITE. */
int shmm_effective_diffusivity(shmm_ctx *ctx, int64_t first, int64_t count, const float *d_f1,
                               const float *d_f2, const float *d_w, const double *d_K_base,
                               double *d_K_out, double *d_K_energy, double *d_mass,
                               int32_t *d_status, void *stream);

/* The same flux-form estimate averaged over the centred inner x inner cells
 * of each patch only (oversampled patches: the local problem is posed on a
 * patch larger than the region it describes, so that the seam of the
 * periodically treated patch lies away from the averaging window; aimed at
 * the non-periodicity of the components in a local domain, which the
 * continuous-spectrum example of Section 4 lists among the method's error
 * sources).  inner = 0, or inner >= a patch's n, averages over the whole patch,
 * as shmm_effective_diffusivity does (bit for bit).
 *   d_K_out = K_b + sym(<f_i w_j>_window)                  [n_domains][3]
 * Errors: SHMM_EINVAL for a negative or odd inner. */
int shmm_effective_diffusivity_window(shmm_ctx *ctx, int64_t first, int64_t count, int32_t inner,
                                      const float *d_f1, const float *d_f2, const float *d_w,
                                      const double *d_K_base, double *d_K_out, int32_t *d_status, void *stream);

/* Level combination (Algorithms 1-3, extended to L levels), FP64, for the
 * domains [first, first + count).  All tensor arrays are [n_domains][3]:
 *   mode 0 (top-down): K_in = kappa I at level 0, else K_off of the parent;
 *          K_off = S12(K_in) + S21(K_in) - K_in below the finest level
 *          (Algorithm 2; S12/S21 = Algorithm 1 on the line energies).
 *   mode 1 (base):     finest level: K_base = K_in; otherwise
 *          K_star = mean of the children's R, K_base = K_star - K_off + K_in
 *          (Algorithm 3, steps 2-3); a non-SPD result is clamped to
 *          lambda_min(K_in) and flagged SHMM_DOM_NOT_SPD.
 *   mode 2 (result):   finest level: R = K_solve; otherwise
 *          R = K_solve + S12(K_base) + S21(K_base) - 2 K_base (the additive
 *          rule of Algorithm 2 applied to the final step of Algorithm 3).
 *   mode 3 (macro):    R = S12(K_base) + S21(K_base) - K_base (K_base at the
 *          finest level): the level's effective diffusivity without its own
 *          diagonal band, for a macro grid that resolves that band as its
 *          advecting velocity (eq:homo with v_M; HMM step 4).  Pass a separate
 *          buffer as d_R to keep the level results.
 * Run mode 0 phase by phase from the coarsest, modes 1-2 from the finest;
 * mode 3 after mode 1 on the range. */
int shmm_level_chain(shmm_ctx *ctx, int64_t first, int64_t count, int32_t mode,
                     const double *d_lines, double *d_K_in, double *d_K_off, double *d_K_base,
                     const double *d_K_solve, double *d_R, int32_t *d_status, void *stream);

/* Kernel selection for the autotuner (no effect on results beyond rounding
 * order).  key = a patch size n (power of two): select local-solve kernel
 * variant `value` for patches of that size, 0 <= value < the count returned by
 * key = SHMM_TUNE_SOLVE_VARIANT_COUNT with value = n (a non-negative return).
 * n = 64: 0 = whole patch in LDS, column strips of 16 (split operator form);
 *   1, 2 = rows per wavefront, 16 or 8 rows per thread; 3 = whole patch in
 *   LDS, coefficient form, strips of 16; 4 = the same, strips of 8;
 *   5, 6 = 3 and 4 with the stage input read a row further ahead (pipelined
 *   LDS reads, bit-identical results; 5 is the default).
 * n = 128: 0 = split form, strips of 32; 1, 2 = rows per wavefront (16, 8);
 *   3, 4 = coefficient form, strips of 32 or 16; 5 = strips of 32 with the
 *   compensation of 8 strip rows in LDS; 6 = the same with 16 rows;
 *   7, 8 = 5 and 6 with pipelined LDS reads (bit-identical results; 7 is
 *   the default).
 * n = 256: 0 = full-width bands of 32 rows with 8-row rings, 768 threads,
 *   relaunched every 2 steps; 1 = the same at 1024 threads; 2 = one launch per
 *   RK stage; 3 = bands of 24 rows with 12-row rings (3 steps per launch);
 *   4 = bands of 16 rows, 256 threads; 5 = square 64 x 64 tiles with 8-cell
 *   rings; 6 = the bands of 0 kept resident for all steps, neighbours
 *   exchanging their ring rows every 2 steps (in a call whose range also
 *   holds other patch sizes it runs first and alone, and the other sizes
 *   follow, concurrently with one another); 7 = 6 with pipelined LDS reads
 *   (bit-identical results, also run alone; the default).
 * Other sizes have one variant.
 * Errors: SHMM_EINVAL for an unknown key or value. */
#define SHMM_TUNE_SOLVE_VARIANT_COUNT 0
/* key = SHMM_TUNE_RING_SPIN_CAP: value >= 0 is the number of polls (about a
 * microsecond each; default 2^25, tens of seconds) after which a ring-exchange
 * band stops waiting for a neighbour; 0 gives up at the first wait.  A band
 * that gives up writes NaN into its rows of the current and every later patch
 * of the call without waiting again, so every kernel still exits and the
 * failure shows as SHMM_DOM_NONFINITE (shmm_local_solve_batch).  For callers
 * that must bound a solve's wall time, and to test that path.  An empty slab
 * word is the NaN pattern 0xFFFFFFFF: a non-finite input that puts exactly
 * that pattern into a ring row makes the neighbour's wait run to this limit
 * before its (already non-finite) result comes back. */
#define SHMM_TUNE_RING_SPIN_CAP (-1)
int shmm_ctx_tune(shmm_ctx *ctx, int32_t key, int32_t value);

/* Macro solver (HMM step 4 on eq:homo with the resolved velocity kept as
 * advection): nsteps classic RK4 steps of
 *   u_t = div(v u + K(x) grad u)
 * on the N x N grid of [0, 2 pi]^2, spacing h = 2 pi / N, cells at
 * ((i + 1/2) h, (j + 1/2) h).  d_vx, d_vy are face velocities (left x-face,
 * bottom y-face of each cell; may both be NULL: pure diffusion); d_K is
 * [N*N][3] at cell centres (face value = mean of the two cells) if
 * K_is_field, else [1][3].  dtype 64: d_vx, d_vy, d_u are double; dtype 32:
 * float (K stays double).
 * bc: SHMM_BC_PERIODIC, or SHMM_BC_DIRICHLET_X (the numerical examples of
 * Section 4): u = g0 on x = 0 and u = g1 on x = 2 pi, periodic in y.  A
 * boundary x-face carries the boundary value (advection with the velocity
 * field's x-face value at x = 0, diffusion K11 of the adjacent cell over the
 * half cell, no tangential term); y-face cross terms in the first and last
 * columns use the ghost value 2 g - u.  g0, g1 are ignored when periodic.
 * Errors: SHMM_EINVAL for N < 4 or not a power of two, an unknown bc, a
 * non-finite boundary value, a dtype other than 32/64, or nsteps < 0
 * (nsteps = 0 is a no-op). */
#define SHMM_BC_PERIODIC 0
#define SHMM_BC_DIRICHLET_X 1
int shmm_macro_step(shmm_ctx *ctx, int32_t N, int32_t bc, double g0, double g1, const void *d_vx,
                    const void *d_vy, const double *d_K, int32_t K_is_field, double dt, int32_t nsteps,
                    void *d_u, int32_t dtype, void *stream);

/* The macro step of shmm_macro_step without any device allocation, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, kernels and
 * results (bit for bit) as shmm_macro_step; its three RK4 planes live in a
 * static buffer of the library (3 N^2 doubles for N up to
 * SHMM_MACRO_NOALLOC_MAX_N: 6 MiB, which every GPU the library runs on holds
 * until the process ends) instead of the context's growable workspace.  The
 * buffer needs no clearing (every plane is written before it is read).  All
 * calls on one GPU share that GPU's buffer: calls that overlap on one GPU (on
 * different streams, or from different contexts or threads) race, so
 * serialise them on one stream.
 * Errors: as shmm_macro_step; SHMM_ERANGE for N > SHMM_MACRO_NOALLOC_MAX_N. */
#define SHMM_MACRO_NOALLOC_MAX_N 512
int shmm_macro_step_noalloc(shmm_ctx *ctx, int32_t N, int32_t bc, double g0, double g1, const void *d_vx,
                            const void *d_vy, const double *d_K, int32_t K_is_field, double dt, int32_t nsteps,
                            void *d_u, int32_t dtype, void *stream);

/* ---------------------------------------------------------------------------
 * Learned surrogate of the local solve (not part of the paper's method).
 * A patch is described by 35 features.  Features 0..31 are log band energies
 * of the velocity spectrum of the patch samples (treated as periodic, DFT
 * normalised by 1/n^2) over the base: feature 8c + b is
 * log((E_cb + 1e-8 E_tot + 1e-30) / det K_b), where E_cb sums channel c times
 * (L / 2 pi)^2 / q^2 (one over the squared physical wavenumber) over the modes
 * k (patch-relative integers, q = |k|) with 2^b <= q < 2^(b+1), b = 0..7
 * (every mode of a patch of up to 256^2 but the mean); the channels are
 * |Vx|^2, |Vy|^2, |Vx + Vy|^2 / 2 and |Vx - Vy|^2 / 2, and E_tot is the sum of
 * channels 0 and 1 over the bins.  For an isotropic base kappa I the bin sums
 * over kappa are the local solve's K - K_b to first order in the Peclet
 * number (exactly for a shear flow).  Feature 32 is
 * log sqrt(det K_b).  Features 33 and 34 carry the anisotropy of the base:
 * the entries (1,1) and (1,2) of the traceless part of log K_b, that is
 * g(rho) (K11 - K22) / (K11 + K22) and g(rho) 2 K12 / (K11 + K22) with
 * rho = sqrt((K11 - K22)^2 + 4 K12^2) / (K11 + K22) and g(rho) = atanh(rho) / rho
 * (g(0) = 1): zero for an isotropic base, unchanged when K_b is scaled, and
 * turning with twice the angle of the base's principal axes.
 * A 35 -> 256 -> 256 -> 256 -> 3 GELU network maps the
 * standardised features to o, and K = K_b + sqrt(det K_b) L L^T with
 * L = [[e^o1, 0], [o2, e^o3]] (the enhancement K - K_b is positive
 * semi-definite).  Matrix products run on the matrix cores with BF16 operands
 * and FP32 accumulation.
 *
 * One ensemble member ("model") is SHMM_SURR_MODEL_BYTES of device memory:
 *   float    params[SHMM_SURR_PARAMS_PADDED]  W1 b1 W2 b2 W3 b3 W4 b4, W_l row-major [out][in]
 *   float    mu[64], sigma[64]                input standardisation (first 35 used)
 *   uint16_t bf16[SHMM_SURR_PARAMS_PADDED]    bfloat16 copy of params
 * Members of an ensemble are stored back to back.
 * ------------------------------------------------------------------------- */
#define SHMM_SURR_BINS 32
#define SHMM_SURR_IN 35
#define SHMM_SURR_WIDTH 256
#define SHMM_SURR_OUT 3
#define SHMM_SURR_PARAMS 141571
#define SHMM_SURR_PARAMS_PADDED 141824
#define SHMM_SURR_MODEL_BYTES (4 * SHMM_SURR_PARAMS_PADDED + 4 * 128 + 2 * SHMM_SURR_PARAMS_PADDED)

/* Features of domains [first, first + count), which must share one patch size
 * n (8 <= n <= 256): d_features[count][35] FP32, row i for domain first + i,
 * from the face velocities d_vx, d_vy and the bases d_K_base [n_domains][3].
 * In-house FP32 FFT; bin sums in a fixed order. */
int shmm_patch_features(shmm_ctx *ctx, int64_t first, int64_t count, const float *d_vx,
                        const float *d_vy, const double *d_K_base, float *d_features, void *stream);

/* Refresh the bfloat16 copy of a model's parameters from its FP32 params. */
int shmm_surrogate_refresh(shmm_ctx *ctx, void *d_model, void *stream);

/* One training step of one model at batch B: forward, loss
 * mean_b |K_hat - K_true|_F^2 / |K_true|_F^2 (written to d_loss[0], FP64),
 * backward, the global gradient norm (written to d_loss[1]; the gradient is
 * scaled by min(1, clip / norm) when clip > 0), and an Adam step (beta 0.9 /
 * 0.999, eps 1e-8, step t >= 1 for the bias correction, learning rate lr) on
 * the FP32 params; refreshes the bf16 copy.  d_adam holds m then v,
 * 2 * SHMM_SURR_PARAMS_PADDED floats (zero at t = 1).  d_x [B][35], d_K_base
 * and d_K_true [B][3], d_loss [2].  d_grad (optional, SHMM_SURR_PARAMS floats)
 * receives the gradient of this step before clipping. */
int shmm_surrogate_train_step(shmm_ctx *ctx, void *d_model, float *d_adam, const float *d_x,
                              const double *d_K_base, const double *d_K_true, int64_t B, float lr,
                              float clip, int32_t t, double *d_loss, float *d_grad, void *stream);

/* Ensemble inference with the fallback gate: E members at d_models; the
 * estimate is the member mean; a patch is flagged (d_flags[b] = 1) when a
 * feature lies outside [d_lo, d_hi] (35 floats each, the training range), when
 * the largest member deviation from the mean exceeds tau in relative
 * Frobenius norm, or when the predicted enhancement |K - K_b|_F / |K_b|_F
 * exceeds emax (the regime where the network was not shown accurate; pass
 * infinity to disable).  d_K_base [B][3]; d_K_out [B][3]; d_spread [B] and
 * d_K_members [E][B][3] optional.  B = 0 is a no-op; B above 2^24 is
 * SHMM_ERANGE. */
int shmm_surrogate_infer(shmm_ctx *ctx, const void *d_models, int32_t E, const float *d_x,
                         const double *d_K_base, int64_t B, const float *d_lo, const float *d_hi,
                         double tau, double emax, double *d_K_out, uint8_t *d_flags, double *d_spread,
                         double *d_K_members, void *stream);

/* Chain-aware gate for the surrogate inside the level chain (Algorithm 3):
 * a finer level's result enters its parent's base K_net = K_star - K_off +
 * K_in after K_off is subtracted, and from there (the parent's result is
 * close to its base where the enhancement is small) the bases of every level
 * above it, so its absolute error must stay well below the K_in of each
 * ancestor, the smallest being kappa I at the coarsest level.  For domain
 * first + i, i < count: sets d_flags[i] = 1 when
 * |d_K_hat[i] - d_K_base[i]|_F + d_spread[i] |d_K_hat[i]|_F (the predicted
 * change of the base plus the ensemble's largest relative member deviation,
 * as shmm_surrogate_infer writes it, times the estimate's norm) exceeds
 * tol times the smallest lambda_min(K_in) over the domain's parent and the
 * parent's ancestors; flags of domains without a parent (level 0) are left
 * as they are.  The predicted change is
 * there because the members share the error the features cannot resolve, so
 * the spread alone does not bound it.  d_K_hat, d_K_base [count][3],
 * d_spread [count], d_K_in [n_domains][3] (global index, as the level chain
 * fills it), d_flags [count].  Errors: SHMM_EINVAL for a bad range, a null
 * pointer or tol <= 0. */
int shmm_surrogate_chain_gate(shmm_ctx *ctx, int64_t first, int64_t count, const double *d_K_hat,
                              const double *d_K_base, const double *d_spread, const double *d_K_in, double tol,
                              uint8_t *d_flags, void *stream);

/* Column statistics of a feature matrix d_x [B][35] (the input
 * standardisation of the network and the range of the fallback gate): per
 * column, FP64 mean, standard deviation with the B - 1 divisor, minimum and
 * maximum over the B rows, written to d_stats [4][35] (mean, std, min, max).
 * Fixed reduction order: bitwise reproducible.  Errors: SHMM_EINVAL for
 * B < 2 or a null pointer. */
int shmm_feature_stats(shmm_ctx *ctx, const float *d_x, int64_t B, double *d_stats, void *stream);

/* Rescaled copies of labelled local problems for training: scaling velocity
 * and diffusivity together by c_b = 10^d_log10c[b] leaves the corrector of a
 * local problem unchanged, so K and K_b scale by c_b, the 32 band features
 * (energies over det K_b, squared Peclet numbers) are unchanged and feature 32
 * (log sqrt det K_b) moves by ln c_b; features 33 and 34 are scale free.
 * Inputs d_x [B][35], d_K_base and
 * d_K_true [B][3], d_log10c [B]; outputs of the same shapes (may not alias
 * the inputs).  Errors: SHMM_EINVAL for B < 0 or a null pointer. */
int shmm_surrogate_rescale(shmm_ctx *ctx, const float *d_x, const double *d_K_base, const double *d_K_true,
                           const double *d_log10c, int64_t B, float *d_x_out, double *d_K_base_out,
                           double *d_K_true_out, void *stream);

/* Plain-solve fallback for the flagged domains of [first, first + count)
 * (d_flags[i] for domain first + i): zero their correctors, run the planned
 * local solves (chunks = 0) or the quasi-stationary stop of
 * shmm_local_solve_adaptive with `chunks` and `tol` (chunks >= 1), and write
 * their effective diffusivity into d_K_out [n_domains][3] (overwriting the
 * surrogate's), setting SHMM_DOM_FALLBACK in d_status.  Reads the flags back
 * to the host (synchronises the stream).  Errors: SHMM_EINVAL for a range
 * that was never planned, chunks < 0, or a negative or non-finite tol. */
int shmm_fallback_solve(shmm_ctx *ctx, int64_t first, int64_t count, const uint8_t *d_flags,
                        const float *d_vx, const float *d_vy, const float *d_f1, const float *d_f2,
                        const double *d_K_base, float *d_w, double *d_K_out, int32_t chunks, double tol,
                        int32_t *d_status, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SHMM_H */
