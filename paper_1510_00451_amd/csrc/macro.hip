// Macro solver (HMM step 4 of Section 2.2 on the homogenized equation
// eq:homo, with the resolved large-scale velocity kept as advection):
//   u_t = div(v u + K(x) grad u) on the N x N grid of [0, 2 pi]^2, classic RK4.
// Face fluxes: centred advection, K11 d1 u + K12 d2 u on x-faces and
// K12 d1 u + K22 d2 u on y-faces (tangential derivatives averaged over the two
// cells); a K field at cell centres is averaged onto the faces.
// Boundaries: periodic, or (the numerical examples of Section 4) u = g0 on
// x = 0 and g1 on x = 2 pi with y periodic.  A boundary x-face carries the
// boundary value: advection v g, diffusion K11 of the adjacent cell over the
// half cell, no tangential term (u is constant along the boundary); the
// tangential x-difference on the y-faces of the first and last columns uses
// the ghost value 2 g - u on the line through the boundary value.
#include <map>
#include <mutex>

#include "shmm_internal.h"

namespace shmm {

namespace {

template <typename T>
struct MacroArgs {
    int N;
    T h;
    const T *vx, *vy;
    const double *K;
    int K_is_field;
    T dt;
    int dirichlet_x;
    T g0, g1;
};

template <typename T>
__device__ inline void face_K(const MacroArgs<T> &a, int c, int cn, T *k11, T *k12, T *k22) {
    if (a.K_is_field) {
        *k11 = (T)(0.5 * (a.K[3 * c + 0] + a.K[3 * cn + 0]));
        *k12 = (T)(0.5 * (a.K[3 * c + 1] + a.K[3 * cn + 1]));
        *k22 = (T)(0.5 * (a.K[3 * c + 2] + a.K[3 * cn + 2]));
    } else {
        *k11 = (T)a.K[0];
        *k12 = (T)a.K[1];
        *k22 = (T)a.K[2];
    }
}

// flux through x-face f (0 <= f <= N, between cells f - 1 and f) of row j
template <typename T>
__device__ inline T flux_x(const MacroArgs<T> &a, const T *u, int f, int j) {
    const int N = a.N, m = N - 1;
    if (a.dirichlet_x && (f == 0 || f == N)) {
        const int c = j * N + (f == 0 ? 0 : m);
        const T g = f == 0 ? a.g0 : a.g1;
        const T k11 = (T)(a.K_is_field ? a.K[3 * c] : a.K[0]);
        T fl = k11 * (f == 0 ? u[c] - g : g - u[c]) / (T(0.5) * a.h);
        if (a.vx) fl += a.vx[j * N] * g;
        return fl;
    }
    const int i = f & m, il = (f - 1) & m, jn = (j + 1) & m, js = (j - 1) & m;
    const int c = j * N + i;
    T k11, k12, k22;
    face_K(a, c, j * N + il, &k11, &k12, &k22);
    const T ul = u[j * N + il], ur = u[c];
    T fl = k11 * (ur - ul) / a.h +
           k12 * (u[jn * N + i] + u[jn * N + il] - u[js * N + i] - u[js * N + il]) / (T(4) * a.h);
    if (a.vx) fl += a.vx[c] * T(0.5) * (ul + ur);
    return fl;
}

// flux through the bottom y-face of cell (i, j)
template <typename T>
__device__ inline T flux_y(const MacroArgs<T> &a, const T *u, int i, int j) {
    const int N = a.N, m = N - 1;
    const int js = (j - 1) & m;
    const int c = j * N + i, cs = js * N + i;
    T k11, k12, k22;
    face_K(a, c, cs, &k11, &k12, &k22);
    const T ub = u[cs], ut = u[c];
    T et, eb, wt, wb;   // east and west neighbours in the two rows
    if (a.dirichlet_x && i == m) {
        et = T(2) * a.g1 - ut;
        eb = T(2) * a.g1 - ub;
    } else {
        const int ie = (i + 1) & m;
        et = u[j * N + ie];
        eb = u[js * N + ie];
    }
    if (a.dirichlet_x && i == 0) {
        wt = T(2) * a.g0 - ut;
        wb = T(2) * a.g0 - ub;
    } else {
        const int iw = (i - 1) & m;
        wt = u[j * N + iw];
        wb = u[js * N + iw];
    }
    T fl = k22 * (ut - ub) / a.h + k12 * (et + eb - wt - wb) / (T(4) * a.h);
    if (a.vy) fl += a.vy[c] * T(0.5) * (ub + ut);
    return fl;
}

template <typename T>
__global__ __launch_bounds__(256) void k_macro_stage(MacroArgs<T> a, const T *__restrict__ y,
                                                     T *__restrict__ ynext, T *__restrict__ acc,
                                                     T *__restrict__ u, int st) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = a.N;
    if (c >= N * N) return;
    const int j = c / N, i = c - j * N, m = N - 1;
    const T F = (flux_x(a, y, i + 1, j) - flux_x(a, y, i, j)) / a.h +
                (flux_y(a, y, i, (j + 1) & m) - flux_y(a, y, i, j)) / a.h;
    const T t = a.dt * F;
    const T uc = u[c];
    T out;
    if (st == 0) {
        acc[c] = t;
        out = uc + T(0.5) * t;
    } else if (st < 3) {
        acc[c] += T(2) * t;
        out = uc + (st == 2 ? T(1) : T(0.5)) * t;
    } else {
        const T nu = uc + (acc[c] + t) / T(6);
        u[c] = nu;
        out = nu;
    }
    ynext[c] = out;
}

template <typename T>
__global__ void k_copy(const T *__restrict__ src, T *__restrict__ dst, int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) dst[c] = src[c];
}

template <typename T>
int run(int32_t N, int32_t bc, double g0, double g1, const void *vx, const void *vy, const double *K,
        int32_t K_is_field, double dt, int32_t nsteps, void *u, void *work, hipStream_t s) {
    MacroArgs<T> a;
    a.dirichlet_x = bc == SHMM_BC_DIRICHLET_X;
    a.g0 = (T)g0;
    a.g1 = (T)g1;
    a.N = N;
    a.h = (T)(2.0 * M_PI / (double)N);
    a.vx = (const T *)vx;
    a.vy = (const T *)vy;
    a.K = K;
    a.K_is_field = K_is_field;
    a.dt = (T)dt;
    const int cells = N * N;
    T *y0 = (T *)work, *y1 = y0 + cells, *acc = y0 + 2 * cells;
    const dim3 grid((unsigned)((cells + 255) / 256));
    hipLaunchKernelGGL(k_copy<T>, grid, dim3(256), 0, s, (const T *)u, y0, cells);
    SHMM_HIP_CHECK(hipGetLastError());
    for (int32_t step = 0; step < nsteps; ++step) {
        for (int st = 0; st < 4; ++st) {
            hipLaunchKernelGGL(k_macro_stage<T>, grid, dim3(256), 0, s, a, y0, y1, acc, (T *)u, st);
            SHMM_HIP_CHECK(hipGetLastError());
            T *t = y0;
            y0 = y1;
            y1 = t;
        }
    }
    return SHMM_OK;
}

}  // namespace

// Scratch of the allocation-free macro step (shmm_macro_step_noalloc): the
// three RK4 planes of an N x N grid, FP64, up to N = SHMM_MACRO_NOALLOC_MAX_N.
// Every GPU the library runs on holds its own copy until the process ends;
// host code reaches it only through the device address that
// macro_scratch_setup() takes with the device current.
static constexpr size_t kMacroScratchWords = (size_t)3 * SHMM_MACRO_NOALLOC_MAX_N * SHMM_MACRO_NOALLOC_MAX_N;
static __device__ __align__(256) double scratch[kMacroScratchWords];
static std::mutex scratch_lock;
static std::map<int, void *> scratch_ptr;   // device -> address of `scratch` on it

int macro_scratch_setup(int device) {
    std::lock_guard<std::mutex> g(scratch_lock);
    if (scratch_ptr.count(device)) return SHMM_OK;
    void *p = nullptr;
    SHMM_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return SHMM_EDEVICE;
    scratch_ptr[device] = p;
    return SHMM_OK;
}

void *macro_scratch(int device, size_t *bytes) {
    std::lock_guard<std::mutex> g(scratch_lock);
    const auto it = scratch_ptr.find(device);
    if (bytes) *bytes = kMacroScratchWords * sizeof(double);
    return it == scratch_ptr.end() ? nullptr : it->second;
}

size_t macro_workspace(int32_t N, int32_t dtype) {
    return (size_t)3 * N * N * (dtype == 64 ? sizeof(double) : sizeof(float));
}

int launch_macro(int32_t N, int32_t bc, double g0, double g1, const void *vx, const void *vy, const double *K,
                 int32_t K_is_field, double dt, int32_t nsteps, void *u, int32_t dtype, void *work, hipStream_t s) {
    if (dtype == 64) return run<double>(N, bc, g0, g1, vx, vy, K, K_is_field, dt, nsteps, u, work, s);
    return run<float>(N, bc, g0, g1, vx, vy, K, K_is_field, dt, nsteps, u, work, s);
}

}  // namespace shmm
