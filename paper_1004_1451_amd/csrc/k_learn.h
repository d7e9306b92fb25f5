// Learned form of the first-pass interpolation: the least-squares fit of
// every F point (Algorithm 2) is computed as usual, its Gram and operator row
// give the point's 24 features, and the network (k_mlp.h) proposes a
// correction to the fitted weights on all the point's slots, trained toward
// the weights the method settles on after its recomputation pass.  The fit
// judges the proposal: it is kept when the functional of eq. LSfuncrowi at the
// corrected weights is finite and at most `judge` times the fit's own minimum;
// otherwise the fitted row is written.
#pragma once
#include "k_mlp.h"
#include "k_sparse.h"

struct __align__(16) LearnSmem {
    MlpPack w;
    unsigned short x[4][64][MLP_INP];
    unsigned short h[4][16][MLP_HLD];
    float y[4][64][4];
    float red[2][BAMG_BLK / BAMG_WAVE];
};

// Grid-stride over tiles of BAMG_BLK rows (the weights are staged in LDS once
// per workgroup).  part[2 * block + 0 / 1]: F points judged / fallbacks.
template <typename T, typename MP, typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_ls_fit_learn(int n, const ChainGeo* __restrict__ geo, int nch, int Ru, const T* __restrict__ U,
               const double* __restrict__ wall, int WS, int caliber, int* __restrict__ pc, MP* __restrict__ pv,
               T* __restrict__ inject, unsigned char* __restrict__ jcnt, const int* __restrict__ brp,
               const int* __restrict__ bci, const M* __restrict__ bv, const MlpPack* __restrict__ pk, float judge,
               float* __restrict__ part) {
    __shared__ LearnSmem S;
    mlp_stage(pk, &S.w);
    const int w = threadIdx.x / BAMG_WAVE, l = threadIdx.x % BAMG_WAVE, q = l / 16, r = l % 16;
    float nF = 0.f, nfall = 0.f;
    __syncthreads();
    for (int tile = blockIdx.x; tile * BAMG_BLK < n; tile += gridDim.x) {
        const int i = tile * BAMG_BLK + threadIdx.x;
        bool isF = false;
        LsPoint P;
        float f[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) f[k] = 0.f;
        if (i < n) {
            const int ch = find_chain(geo, nch, i);
            const ChainGeo g = geo[ch];
            const int li = i - g.off;
            const int ia = (int)g.dy.div((uint32_t)li), ib = li - ia * g.ny;
            if (grid_cpos(ia, g.nx, g.periodic) && grid_cpos(ib, g.ny, g.periodic)) {
                const int I = g.coff + ((ia + 1) >> 1) * g.ncy + ((ib + 1) >> 1);
                pc[(size_t)i * 4] = I; pv[(size_t)i * 4] = (MP)1;
#pragma unroll
                for (int s = 1; s < 4; ++s) { pc[(size_t)i * 4 + s] = -1; pv[(size_t)i * 4 + s] = (MP)0; }
                if (inject)
                    for (int k = 0; k < Ru; ++k) inject[(size_t)I * Ru + k] = U[(size_t)i * Ru + k];
                jcnt[i] = 1;
            } else {
                isF = true;
                ls_point<T>(i, g, ia, ib, Ru, 0, 1, U, U, wall + (size_t)ch * WS, caliber, P);
                point_features<M>(P, i, g, ia, ib, brp, bci, bv, f);
            }
        }
        // this thread's features as row l of its wave's input tile
#pragma unroll
        for (int k = 0; k < MLP_INP; ++k) S.x[w][l][k] = k < 24 ? f2bf(f[k]) : (unsigned short)0;
        __syncthreads();
        for (int m = 0; m < 4; ++m) {
            MlpTile Tt;
            mlp_tile_forward(S.w, &S.x[w][16 * m][0], &S.h[w][0][0], Tt);
            if (r < MLP_OUT)
#pragma unroll
                for (int a = 0; a < 4; ++a) S.y[w][16 * m + 4 * q + a][r] = Tt.y[a];
        }
        __syncthreads();
        if (isF) {
            double pm[4];
            bool finite = true;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                pm[s] = ((P.valid >> s) & 1) ? P.p[s] + (double)S.y[w][l][s] : 0.0;
                finite &= isfinite(pm[s]);
            }
            double Lm = P.sigma;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                Lm -= 2.0 * pm[s] * P.b[s];
#pragma unroll
                for (int t = 0; t < 4; ++t) Lm += pm[s] * P.G[s][t] * pm[t];
            }
            const bool keep = finite && isfinite(Lm) && Lm <= (double)judge * P.Lls;
            nF += 1.f;
            int cnt;
            if (keep) {
                cnt = write_prow<MP>(i, P.valid, P.sc, pm, pc, pv);
            } else {
                nfall += 1.f;
                cnt = write_prow<MP>(i, P.J, P.sc, P.p, pc, pv);
            }
            jcnt[i] = (unsigned char)cnt;
        }
        __syncthreads();
    }
    nF = block_sum(nF, &S.red[0][0]);
    nfall = block_sum(nfall, &S.red[1][0]);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = nF; part[2 * blockIdx.x + 1] = nfall; }
}

// acc[0..1] += sum of the per-block pairs (one thread, in block order).
__global__ void k_learn_tally(int nb, const float* __restrict__ part, double* __restrict__ acc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0, b = 0;
    for (int k = 0; k < nb; ++k) { a += part[2 * k]; b += part[2 * k + 1]; }
    acc[0] += a;
    acc[1] += b;
}

// ---------------------------------------------------------------- training pairs
// One training pair of the learned form per F point of a level: its 24
// first-pass features and the correction of its fitted slot weights (the
// final minus the first-pass weights, 4), the correction the network is to
// predict from what the first pass knows.  Only ordinary points are kept: at
// least one valid slot, every feature within +-fcap and every correction
// within +-tcap (a few degenerate points with vanishing test-vector values
// carry features and corrections orders of magnitude larger, which would
// own the squared loss); NaNs fail the test.
__device__ __forceinline__ bool pair_keep(const float* __restrict__ f, const float* __restrict__ w,
                                          const float* __restrict__ w0, float fcap, float tcap) {
    bool keep = (f[0] + f[1] + f[2] + f[3]) > 0.0f;
#pragma unroll
    for (int k = 0; k < 24; ++k) keep &= fabsf(f[k]) <= fcap;
#pragma unroll
    for (int s = 0; s < 4; ++s) keep &= fabsf(w[s] - w0[s]) <= tcap;
    return keep;
}

__global__ void k_pair_flag(int n, const float* __restrict__ feat, const float* __restrict__ w,
                            const float* __restrict__ w0, float fcap, float tcap, int* __restrict__ keep) {
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    keep[i] = pair_keep(feat + (size_t)i * 24, w + (size_t)i * 4, w0 + (size_t)i * 4, fcap, tcap) ? 1 : 0;
}

// The kept pairs of a level at rows base + pos[i] of fo (x 24) and to (x 4).
__global__ void k_pair_write(int n, const float* __restrict__ feat, const float* __restrict__ w,
                             const float* __restrict__ w0, const int* __restrict__ keep, const int* __restrict__ pos,
                             long long base, float* __restrict__ fo, float* __restrict__ to) {
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n || !keep[i]) return;
    const long long o = base + pos[i];
#pragma unroll
    for (int k = 0; k < 24; ++k) fo[o * 24 + k] = feat[(size_t)i * 24 + k];
#pragma unroll
    for (int s = 0; s < 4; ++s) to[o * 4 + s] = w[(size_t)i * 4 + s] - w0[(size_t)i * 4 + s];
}
