// Multicolour Gauss-Seidel relaxation (Section 3 names Gauss-Seidel next to
// omega-Jacobi): the points of a level are split into colours (point_colour)
// with no coupling inside a colour, and one sweep updates colour 0, 1, ... in
// order, each from the latest values of the others:
//   x_i <- x_i + w (f_i - (B x)_i) / b_ii   for every i of the colour.
// Each launch handles one colour in place; points of other colours only read.
// Products are added in CSR order in the type of the vectors.
#pragma once
#include "common.h"
#include "k_sweep.h"

// One colour of a homogeneous sweep (f = 0) on R interleaved test vectors,
// VW adjacent columns per thread (G = R / VW threads per row).
template <typename T, typename M, int VW>
__global__ void __launch_bounds__(BAMG_BLK)
k_mcgs_tv(int n, const ChainGeo* __restrict__ geo, int nch, int G, FastDiv divG, int colour, double w,
          const int* __restrict__ rp, const int* __restrict__ ci, const M* __restrict__ v, T* X) {
    const int t = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK + threadIdx.x;
    if (t >= n * G) return;
    const int i = (int)divG.div((uint32_t)t), kg = t - i * G;
    const ChainGeo g = geo[find_chain(geo, nch, i)];
    if (point_colour(g, i - g.off) != colour) return;
    const int R = G * VW;
    T acc[VW], xo[VW];
#pragma unroll
    for (int q = 0; q < VW; ++q) acc[q] = (T)0;
    M bd = (M)1;
    const int p1 = rp[i + 1];
    for (int p = rp[i]; p < p1; ++p) {
        const int j = ci[p];
        const M b = v[p];
        if (j == i) bd = b;
        T x[VW];
        VecIO<T, VW>::ld(X + (size_t)j * R + (size_t)kg * VW, x);
#pragma unroll
        for (int q = 0; q < VW; ++q) acc[q] += (T)b * x[q];
    }
    T* xi = X + (size_t)i * R + (size_t)kg * VW;
    VecIO<T, VW>::ld(xi, xo);
#pragma unroll
    for (int q = 0; q < VW; ++q) xo[q] = xo[q] + (T)w * ((T)0 - acc[q]) / (T)bd;
    VecIO<T, VW>::st(xi, xo);
}

// One colour of a sweep on B x = f, single vector, rows of the chains the
// mask keeps.
template <typename T, typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_mcgs(int n, const ChainGeo* __restrict__ geo, int nch, int colour, double w, const int* __restrict__ rp,
       const int* __restrict__ ci, const M* __restrict__ v, const T* __restrict__ F, T* X, RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, 1, n)) return;
    const int i = tile * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const ChainGeo g = geo[find_chain(geo, nch, i)];
    if (point_colour(g, i - g.off) != colour) return;
    T acc = (T)0;
    M bd = (M)1;
    const int p1 = rp[i + 1];
    for (int p = rp[i]; p < p1; ++p) {
        const int j = ci[p];
        const M b = v[p];
        if (j == i) bd = b;
        acc += (T)b * X[j];
    }
    X[i] = X[i] + (T)w * (F[i] - acc) / (T)bd;
}

// err |= 1 when an off-diagonal entry of the operator couples two points of
// one colour (the colouring would not make the sweep a Gauss-Seidel sweep).
__global__ void k_check_colours(int n, const ChainGeo* __restrict__ geo, int nch, const int* __restrict__ rp,
                                const int* __restrict__ ci, int* __restrict__ err) {
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const ChainGeo g = geo[find_chain(geo, nch, i)];
    const int ci_ = point_colour(g, i - g.off);
    int bad = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        if (j == i) continue;
        if (j < g.off || j >= g.off + g.n || point_colour(g, j - g.off) == ci_) bad = 1;
    }
    if (bad) atomicOr(err, 1);
}
