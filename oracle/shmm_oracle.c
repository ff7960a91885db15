/*
 * FP64 CPU oracle for the seamless heterogeneous multiscale method (SHMM) of
 * Lee & Engquist for passive advection-diffusion in steady incompressible flow.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP path is checked against.  It shares no code with the HIP path: no
 * headers, no helpers, no tables.  Only tests, the smoke check and the CPU
 * baseline of the benchmark may load it.
 *
 * Everything is double precision, plain loops, fixed summation order.
 *
 * Grid conventions (one n x n periodic patch, spacing h):
 *   psi   at nodes         (x0 + i h, y0 + j h)          psi[j*n + i]
 *   vx    on x-faces       (x0 + i h, y0 + (j+1/2) h)    vx[j*n + i]  (left face of cell i)
 *   vy    on y-faces       (x0 + (i+1/2) h, y0 + j h)    vy[j*n + i]  (bottom face of cell j)
 *   w, u, f at cell centres (x0 + (i+1/2) h, y0 + (j+1/2) h)
 * All indices wrap modulo n.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TWO_PI 6.283185307179586476925286766559

static inline int wrap(int i, int n) { i %= n; return i < 0 ? i + n : i; }

/* ------------------------------------------------------------------------
 * Fourier synthesis of a band of the stream function (Section 3.1: the band
 * components are inverse Fourier transforms of masked coefficients).
 *
 * psi(x) = sum_k psi_hat(k) exp(i k.x), evaluated at the global grid points
 * x = 2 pi (I, J) / N for a list of integer points.  The phase k1 I + k2 J is
 * reduced exactly modulo N in integers before the cosine and sine.
 * psi_hat is interleaved (re, im), row-major [k2 + kmax][k1 + kmax];
 * mask (same shape) selects the modes of the band.
 * ---------------------------------------------------------------------- */
void orc_synth_points(const double *psi_hat, int kmax, const int8_t *mask, int64_t N,
                      int64_t npts, const int64_t *I, const int64_t *J, double *out)
{
    const int span = 2 * kmax + 1;
    /* list the band once */
    int64_t nm = 0;
    for (int a = 0; a < span * span; ++a) nm += mask[a] ? 1 : 0;
    int64_t *kk1 = (int64_t *)malloc(sizeof(int64_t) * (nm + 1));
    int64_t *kk2 = (int64_t *)malloc(sizeof(int64_t) * (nm + 1));
    double *cr = (double *)malloc(sizeof(double) * (nm + 1));
    double *ci = (double *)malloc(sizeof(double) * (nm + 1));
    int64_t m = 0;
    for (int b = 0; b < span; ++b)
        for (int a = 0; a < span; ++a) {
            int idx = b * span + a;
            if (!mask[idx]) continue;
            kk1[m] = a - kmax; kk2[m] = b - kmax;
            cr[m] = psi_hat[2 * idx]; ci[m] = psi_hat[2 * idx + 1];
            ++m;
        }
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npts; ++p) {
        double s = 0.0;
        for (int64_t q = 0; q < nm; ++q) {
            int64_t r = (kk1[q] * I[p] + kk2[q] * J[p]) % N;
            if (r < 0) r += N;
            double th = ORC_TWO_PI * (double)r / (double)N;
            s += cr[q] * cos(th) - ci[q] * sin(th);
        }
        out[p] = s;
    }
    free(kk1); free(kk2); free(cr); free(ci);
}

/* ------------------------------------------------------------------------
 * Line energies for the off-diagonal closed form (Algorithm 1 with
 * eq:shearhomoY / eq:shearhomoX).  For dir = 0 the lines are x1 = const at
 * the cell-centre columns x1 = 2 pi (I0 + i + 1/2)/N, i < n, and the value is
 * the full-period mean over x2 of the band field squared, which by Parseval is
 *      s(x1) = sum_{k2} | sum_{k1} psi_hat(k1,k2) exp(i k1 x1) |^2 .
 * For dir = 1 the roles of x1 and x2 are swapped (rows x2 = const).
 * The phase k (2 I + 1) is reduced exactly modulo 2N.
 * ---------------------------------------------------------------------- */
void orc_line_energy(const double *psi_hat, int kmax, const int8_t *mask, int64_t N,
                     int64_t I0, int n, int dir, double *out)
{
    const int span = 2 * kmax + 1;
    for (int i = 0; i < n; ++i) {
        int64_t twoI1 = 2 * (I0 + i) + 1;
        double total = 0.0;
        for (int outer = 0; outer < span; ++outer) {
            double sr = 0.0, si = 0.0;
            for (int inner = 0; inner < span; ++inner) {
                int a = dir == 0 ? inner : outer;   /* k1 index */
                int b = dir == 0 ? outer : inner;   /* k2 index */
                int idx = b * span + a;
                if (!mask[idx]) continue;
                int64_t k = (int64_t)(inner - kmax);
                int64_t r = (k * twoI1) % (2 * N);
                if (r < 0) r += 2 * N;
                double th = ORC_TWO_PI * (double)r / (double)(2 * N);
                double c = cos(th), s = sin(th);
                double pr = psi_hat[2 * idx], pi = psi_hat[2 * idx + 1];
                sr += pr * c - pi * s;
                si += pr * s + pi * c;
            }
            total += sr * sr + si * si;
        }
        out[i] = total;
    }
}

/* ------------------------------------------------------------------------
 * Right-hand side of the periodic advection-diffusion problem in
 * conservation form, u_t = div( v u + K grad u ) + f   (eq:model with
 * div v = 0, so v.grad u = div(v u); the diffusion matrix K is the base
 * diffusivity of the numerical homogenization, Section 2.2).
 *
 * Face fluxes (centred):
 *   Jx(i-1/2, j) = vx (u[i-1] + u[i])/2 + Kx11 (u[i] - u[i-1])/h
 *                + Kx12 (u[i,j+1] + u[i-1,j+1] - u[i,j-1] - u[i-1,j-1])/(4h)
 *   Jy(i, j-1/2) = vy (u[j-1] + u[j])/2 + Ky22 (u[j] - u[j-1])/h
 *                + Ky12 (u[i+1,j] + u[i+1,j-1] - u[i-1,j] - u[i-1,j-1])/(4h)
 *   F = (Jx(i+1/2) - Jx(i-1/2))/h + (Jy(j+1/2) - Jy(j-1/2))/h + f
 * kx11/kx12 live on x-faces, ky12/ky22 on y-faces (same indexing as vx/vy).
 * vx, vy or f may be NULL (zero).
 * ---------------------------------------------------------------------- */
void orc_rhs(int n, double h, const double *vx, const double *vy,
             const double *kx11, const double *kx12, const double *ky12, const double *ky22,
             const double *f, const double *u, double *out)
{
    size_t cells = (size_t)n * n;
    double *jx = (double *)malloc(sizeof(double) * cells);   /* flux through x-face i of row j */
    double *jy = (double *)malloc(sizeof(double) * cells);   /* flux through y-face j of column i */
    int *ip = (int *)malloc(sizeof(int) * n), *im = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) { ip[i] = wrap(i + 1, n); im[i] = wrap(i - 1, n); }
#define U(jj, ii) u[(size_t)(jj) * n + (ii)]
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            size_t c = (size_t)j * n + i;
            /* x-face between cell (i-1, j) and cell (i, j) */
            double ul = U(j, im[i]), ur = U(j, i);
            double a = vx ? vx[c] * 0.5 * (ul + ur) : 0.0;
            double d = kx11[c] * (ur - ul) / h
                     + kx12[c] * (U(ip[j], i) + U(ip[j], im[i]) - U(im[j], i) - U(im[j], im[i])) / (4.0 * h);
            jx[c] = a + d;
            /* y-face between cell (i, j-1) and cell (i, j) */
            double ub = U(im[j], i), ut = U(j, i);
            double b = vy ? vy[c] * 0.5 * (ub + ut) : 0.0;
            double e = ky22[c] * (ut - ub) / h
                     + ky12[c] * (U(j, ip[i]) + U(im[j], ip[i]) - U(j, im[i]) - U(im[j], im[i])) / (4.0 * h);
            jy[c] = b + e;
        }
#undef U
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            size_t c = (size_t)j * n + i;
            double r = (jx[(size_t)j * n + ip[i]] - jx[c]) / h + (jy[(size_t)ip[j] * n + i] - jy[c]) / h;
            if (f) r += f[c];
            out[c] = r;
        }
    free(jx); free(jy); free(ip); free(im);
}

/* Zero-frame local problems: the cells of the last row and the last column
 * of the patch are held at zero (their right-hand side is zero), so that the
 * corrector on the remaining (n-1)^2 cells vanishes on their boundary (a
 * non-periodic local problem; the frame separates the patch from its
 * periodic images, so no face across the patch seam is ever used). */
static void zero_frame(int n, double *r)
{
    for (int i = 0; i < n; ++i) {
        r[(size_t)(n - 1) * n + i] = 0.0;
        r[(size_t)i * n + (n - 1)] = 0.0;
    }
}

/* classic fourth-order Runge-Kutta for u' = rhs(u), nsteps steps of dt */
static void rk4_run(int n, double h, const double *vx, const double *vy,
                    const double *kx11, const double *kx12, const double *ky12,
                    const double *ky22, const double *f, double dt, int64_t nsteps,
                    double *u, int frame)
{
    size_t cells = (size_t)n * n;
    double *k1 = (double *)malloc(sizeof(double) * cells);
    double *k2 = (double *)malloc(sizeof(double) * cells);
    double *k3 = (double *)malloc(sizeof(double) * cells);
    double *k4 = (double *)malloc(sizeof(double) * cells);
    double *y = (double *)malloc(sizeof(double) * cells);
    for (int64_t s = 0; s < nsteps; ++s) {
        orc_rhs(n, h, vx, vy, kx11, kx12, ky12, ky22, f, u, k1);
        if (frame) zero_frame(n, k1);
        for (size_t c = 0; c < cells; ++c) y[c] = u[c] + 0.5 * dt * k1[c];
        orc_rhs(n, h, vx, vy, kx11, kx12, ky12, ky22, f, y, k2);
        if (frame) zero_frame(n, k2);
        for (size_t c = 0; c < cells; ++c) y[c] = u[c] + 0.5 * dt * k2[c];
        orc_rhs(n, h, vx, vy, kx11, kx12, ky12, ky22, f, y, k3);
        if (frame) zero_frame(n, k3);
        for (size_t c = 0; c < cells; ++c) y[c] = u[c] + dt * k3[c];
        orc_rhs(n, h, vx, vy, kx11, kx12, ky12, ky22, f, y, k4);
        if (frame) zero_frame(n, k4);
        for (size_t c = 0; c < cells; ++c)
            u[c] = u[c] + dt / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
    }
    free(k1); free(k2); free(k3); free(k4); free(y);
}

static void fill(double *a, size_t m, double v) { for (size_t c = 0; c < m; ++c) a[c] = v; }

/* ------------------------------------------------------------------------
 * Local solves (HMM steps 1-2, Section 2.2; two reconstructions with
 * orthogonal gradients e_1, e_2 as in the numerical homogenization
 * K[psi, K; D]).  With u = e_j.x + w_j and w_j periodic, w_j obeys
 *      w_j' = div(v w_j + K_b grad w_j) + f_j ,  w_j(0) given,
 * where f_j = div(v x_j) discretely = the cell average of the face velocity
 * component j.  Domains are independent (one OpenMP task each).
 *
 * Packed layout: domain d owns cells [off[d], off[d] + n[d]^2); w holds
 * field 1 then field 2, each of length total_cells.
 * ---------------------------------------------------------------------- */
void orc_local_solve_batch(int64_t nd, const int32_t *nn, const int64_t *off, const double *hh,
                           const double *vx, const double *vy, const double *f1,
                           const double *f2, const double *Kb, const double *dt,
                           const int64_t *nsteps, int64_t total_cells, double *w, int frame)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < 2 * nd; ++t) {
        int64_t d = t / 2;
        int field = (int)(t % 2);
        int n = nn[d];
        size_t cells = (size_t)n * n;
        const int64_t o = off[d];
        const double *f = field == 0 ? f1 + o : f2 + o;
        double *u = w + (size_t)field * total_cells + o;
        /* an identically zero forcing leaves a zero corrector at zero for all time */
        int zero = 1;
        for (size_t c = 0; c < cells; ++c) if (f[c] != 0.0 || u[c] != 0.0) { zero = 0; break; }
        if (zero) continue;
        double *kx11 = (double *)malloc(sizeof(double) * cells);
        double *kx12 = (double *)malloc(sizeof(double) * cells);
        double *ky12 = (double *)malloc(sizeof(double) * cells);
        double *ky22 = (double *)malloc(sizeof(double) * cells);
        fill(kx11, cells, Kb[3 * d + 0]);
        fill(kx12, cells, Kb[3 * d + 1]);
        fill(ky12, cells, Kb[3 * d + 1]);
        fill(ky22, cells, Kb[3 * d + 2]);
        rk4_run(n, hh[d], vx + o, vy + o, kx11, kx12, ky12, ky22, f, dt[d], nsteps[d], u, frame);
        free(kx11); free(kx12); free(ky12); free(ky22);
    }
}

/* ------------------------------------------------------------------------
 * Macro solver (HMM step 4; the homogenized equation eq:homo with the
 * resolved large-scale velocity kept as advection):
 *      u_t = div( v_M u + K(x) grad u ),  periodic N x N grid,
 * K given at cell centres (Kc[3*c] = K11, K12, K22) or constant
 * (is_field = 0: Kc holds one triple).  Face values are the arithmetic mean
 * of the two adjacent cells.  Classic RK4, nsteps of dt.
 * ---------------------------------------------------------------------- */
void orc_macro(int N, double h, const double *vx, const double *vy, const double *Kc,
               int is_field, double dt, int64_t nsteps, double *u)
{
    size_t cells = (size_t)N * N;
    double *kx11 = (double *)malloc(sizeof(double) * cells);
    double *kx12 = (double *)malloc(sizeof(double) * cells);
    double *ky12 = (double *)malloc(sizeof(double) * cells);
    double *ky22 = (double *)malloc(sizeof(double) * cells);
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            size_t c = (size_t)j * N + i;
            if (!is_field) {
                kx11[c] = Kc[0]; kx12[c] = Kc[1]; ky12[c] = Kc[1]; ky22[c] = Kc[2];
            } else {
                size_t cl = (size_t)j * N + wrap(i - 1, N);   /* left neighbour */
                size_t cb = (size_t)wrap(j - 1, N) * N + i;   /* bottom neighbour */
                kx11[c] = 0.5 * (Kc[3 * c + 0] + Kc[3 * cl + 0]);
                kx12[c] = 0.5 * (Kc[3 * c + 1] + Kc[3 * cl + 1]);
                ky12[c] = 0.5 * (Kc[3 * c + 1] + Kc[3 * cb + 1]);
                ky22[c] = 0.5 * (Kc[3 * c + 2] + Kc[3 * cb + 2]);
            }
        }
    rk4_run(N, h, vx, vy, kx11, kx12, ky12, ky22, NULL, dt, nsteps, u, 0);
    free(kx11); free(kx12); free(ky12); free(ky22);
}

/* ------------------------------------------------------------------------
 * Macro solver with the boundary conditions of the paper's numerical
 * examples (Section 4): u = g0 on x = 0 and u = g1 on x = 2 pi (Dirichlet in
 * x), periodic in y.  Cells i = 0..N-1 sit at x = (i + 1/2) h.
 *   interior x-faces (1 <= i <= N-1): the periodic flux above, with the face
 *     diffusivity the mean of the two cells;
 *   boundary x-faces: the face value is the boundary value, the normal
 *     derivative is one-sided over h/2, and the tangential derivative is zero
 *     (u is constant along the boundary):
 *       Jx(0)  = vx g0 + Kx11 (u[0] - g0) / (h/2)
 *       Jx(N)  = vx g1 + Kx11 (g1 - u[N-1]) / (h/2)
 *     with vx of the periodic velocity field at x = 0 and the diffusivity of
 *     the adjacent cell;
 *   y-faces: periodic in y; the tangential x-derivative uses ghost values
 *     u[-1] = 2 g0 - u[0] and u[N] = 2 g1 - u[N-1] (linear through the
 *     boundary value).
 * ---------------------------------------------------------------------- */
static void rhs_dirichlet_x(int N, double h, double g0, double g1, const double *vx, const double *vy,
                            const double *Kc, int is_field, const double *u, double *out)
{
    size_t cells = (size_t)N * N;
    double *jx = (double *)malloc(sizeof(double) * (size_t)N * (N + 1));   /* faces 0..N of each row */
    double *jy = (double *)malloc(sizeof(double) * cells);
#define U(jj, ii) u[(size_t)(jj) * N + (ii)]
#define KC(c, q) (is_field ? Kc[3 * (c) + (q)] : Kc[(q)])
    for (int j = 0; j < N; ++j) {
        int jp = wrap(j + 1, N), jm = wrap(j - 1, N);
        for (int i = 0; i <= N; ++i) {
            double J;
            if (i == 0) {
                size_t c = (size_t)j * N;
                J = (vx ? vx[c] * g0 : 0.0) + KC(c, 0) * (U(j, 0) - g0) / (0.5 * h);
            } else if (i == N) {
                size_t c = (size_t)j * N + (N - 1);
                J = (vx ? vx[(size_t)j * N] * g1 : 0.0) + KC(c, 0) * (g1 - U(j, N - 1)) / (0.5 * h);
            } else {
                size_t c = (size_t)j * N + i, cl = c - 1;
                double k11 = 0.5 * (KC(c, 0) + KC(cl, 0)), k12 = 0.5 * (KC(c, 1) + KC(cl, 1));
                double ul = U(j, i - 1), ur = U(j, i);
                J = (vx ? vx[c] * 0.5 * (ul + ur) : 0.0) + k11 * (ur - ul) / h
                  + k12 * (U(jp, i) + U(jp, i - 1) - U(jm, i) - U(jm, i - 1)) / (4.0 * h);
            }
            jx[(size_t)j * (N + 1) + i] = J;
        }
        for (int i = 0; i < N; ++i) {
            size_t c = (size_t)j * N + i, cb = (size_t)jm * N + i;
            double k22 = 0.5 * (KC(c, 2) + KC(cb, 2)), k12 = 0.5 * (KC(c, 1) + KC(cb, 1));
            double e_t = i + 1 < N ? U(j, i + 1) : 2.0 * g1 - U(j, N - 1);
            double e_b = i + 1 < N ? U(jm, i + 1) : 2.0 * g1 - U(jm, N - 1);
            double w_t = i > 0 ? U(j, i - 1) : 2.0 * g0 - U(j, 0);
            double w_b = i > 0 ? U(jm, i - 1) : 2.0 * g0 - U(jm, 0);
            double ub = U(jm, i), ut = U(j, i);
            jy[c] = (vy ? vy[c] * 0.5 * (ub + ut) : 0.0) + k22 * (ut - ub) / h
                  + k12 * (e_t + e_b - w_t - w_b) / (4.0 * h);
        }
    }
#undef U
#undef KC
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            size_t c = (size_t)j * N + i;
            out[c] = (jx[(size_t)j * (N + 1) + i + 1] - jx[(size_t)j * (N + 1) + i]) / h
                   + (jy[(size_t)wrap(j + 1, N) * N + i] - jy[c]) / h;
        }
    free(jx); free(jy);
}

void orc_macro_dirichlet_x(int N, double h, double g0, double g1, const double *vx, const double *vy,
                           const double *Kc, int is_field, double dt, int64_t nsteps, double *u)
{
    size_t cells = (size_t)N * N;
    double *k1 = (double *)malloc(sizeof(double) * cells);
    double *k2 = (double *)malloc(sizeof(double) * cells);
    double *k3 = (double *)malloc(sizeof(double) * cells);
    double *k4 = (double *)malloc(sizeof(double) * cells);
    double *y = (double *)malloc(sizeof(double) * cells);
    for (int64_t s = 0; s < nsteps; ++s) {
        rhs_dirichlet_x(N, h, g0, g1, vx, vy, Kc, is_field, u, k1);
        for (size_t c = 0; c < cells; ++c) y[c] = u[c] + 0.5 * dt * k1[c];
        rhs_dirichlet_x(N, h, g0, g1, vx, vy, Kc, is_field, y, k2);
        for (size_t c = 0; c < cells; ++c) y[c] = u[c] + 0.5 * dt * k2[c];
        rhs_dirichlet_x(N, h, g0, g1, vx, vy, Kc, is_field, y, k3);
        for (size_t c = 0; c < cells; ++c) y[c] = u[c] + dt * k3[c];
        rhs_dirichlet_x(N, h, g0, g1, vx, vy, Kc, is_field, y, k4);
        for (size_t c = 0; c < cells; ++c)
            u[c] = u[c] + dt / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
    }
    free(k1); free(k2); free(k3); free(k4); free(y);
}

/* Diffusion-only operator with constant K (no advection, no forcing). */
void orc_diffusion(int n, double h, const double *K, const double *u, double *out)
{
    size_t cells = (size_t)n * n;
    double *kx11 = (double *)malloc(sizeof(double) * cells);
    double *kx12 = (double *)malloc(sizeof(double) * cells);
    double *ky12 = (double *)malloc(sizeof(double) * cells);
    double *ky22 = (double *)malloc(sizeof(double) * cells);
    fill(kx11, cells, K[0]); fill(kx12, cells, K[1]); fill(ky12, cells, K[1]); fill(ky22, cells, K[2]);
    orc_rhs(n, h, NULL, NULL, kx11, kx12, ky12, ky22, NULL, u, out);
    free(kx11); free(kx12); free(ky12); free(ky22);
}

/* Full operator with constant K (advection + diffusion + optional forcing). */
void orc_operator(int n, double h, const double *vx, const double *vy, const double *K,
                  const double *f, const double *u, double *out)
{
    size_t cells = (size_t)n * n;
    double *kx11 = (double *)malloc(sizeof(double) * cells);
    double *kx12 = (double *)malloc(sizeof(double) * cells);
    double *ky12 = (double *)malloc(sizeof(double) * cells);
    double *ky22 = (double *)malloc(sizeof(double) * cells);
    fill(kx11, cells, K[0]); fill(kx12, cells, K[1]); fill(ky12, cells, K[1]); fill(ky22, cells, K[2]);
    orc_rhs(n, h, vx, vy, kx11, kx12, ky12, ky22, f, u, out);
    free(kx11); free(kx12); free(ky12); free(ky22);
}
