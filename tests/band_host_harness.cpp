// Runs the band-filter block code of the HIP path on the CPU (one thread per
// block, no barrier) so its FFT and pruning logic can be checked against the
// oracle without a GPU.  Test harness only.
#include <vector>

#include "band_core.h"

using namespace shmm;

extern "C" int band_host_run(const double *psi_hat, int kmax, int L, const int32_t *thresh,
                             int level, int N, int n, int M, const int32_t *I0, const int32_t *J0,
                             const shmm_domain *dom, int64_t first, int kb1, int kb2, float *psi,
                             float *vx, float *vy, double *lines) {
    BandParams p;
    p.inst.kappa = 1.0;
    p.inst.psi_hat = psi_hat;
    p.inst.kmax = kmax;
    p.inst.L = L;
    for (int l = 0; l < SHMM_MAX_LEVELS; ++l) p.inst.thresh[l] = l + 1 < L ? thresh[l] : 0;
    p.level = level;
    p.N = N;
    p.n = n;
    p.M = M;
    p.kb1 = kb1;
    p.kb2 = kb2;
    int P1 = 1, P2 = 1;
    while (P1 < 2 * kb2 + 1) P1 <<= 1;
    while (P2 < kb1 + 1) P2 <<= 1;
    p.P1 = P1;
    p.R1 = N / P1;
    p.P2 = P2;
    p.R2 = N / P2;
    p.first = first;
    p.dom = dom;
    p.I0 = I0;
    p.J0 = J0;
    std::vector<c32> G((size_t)3 * (kb1 + 1) * M * n);
    p.G = G.data();
    p.out[0] = psi;
    p.out[1] = vx;
    p.out[2] = vy;
    p.chan_first = psi ? 0 : 1;
    p.lines = lines;
    auto nosync = [] {};
    std::vector<c32> a(P1 > P2 ? P1 : P2), b(a.size());
    for (int blk = 0; blk < (kb1 + 1) * p.R1; ++blk)
        band_pass1_block(p, blk, a.data(), b.data(), 0, 1, nosync);
    for (int blk = 0; blk < M * n * p.R2; ++blk)
        band_pass2_block(p, blk, a.data(), b.data(), 0, 1, nosync);
    for (int dir = 0; dir < 2; ++dir)
        for (int q = 0; q < M; ++q)
            for (int i = 0; i < n; ++i) line_energy_one(p, dir, q, i);
    return 0;
}

// Seam faces of a patch from its node values (the device kernel k_seam).
extern "C" void seam_host(int n, double h, const float *P, float *vx, float *vy) {
    const float ih = (float)(1.0 / h);
    const int64_t last = (int64_t)(n - 1) * n;
    for (int i = 0; i < n; ++i) {
        vx[last + i] = -(P[i] - P[last + i]) * ih;
        vy[(int64_t)i * n + (n - 1)] = (P[(int64_t)i * n] - P[(int64_t)i * n + (n - 1)]) * ih;
    }
}
