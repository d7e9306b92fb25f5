// Kernels of the outer iteration (flexible GMRES in FP64) and generic
// fixed-order reductions.
#pragma once
#include "common.h"

enum RedOp : int { RED_DOT = 0, RED_ABS = 1, RED_SUM = 2, RED_NEGSUM = 3 };

// Stage 1 of a reduction over n entries: fixed partition (grid-stride with a
// fixed grid), per-block sum in a fixed order.
template <int OP>
__global__ void k_reduce_partial(long long n, const double* __restrict__ a, const double* __restrict__ b,
                                 double* __restrict__ part) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    double s = 0;
    for (long long i = (long long)blockIdx.x * BAMG_BLK + threadIdx.x; i < n; i += (long long)gridDim.x * BAMG_BLK) {
        double v = a[i];
        if (OP == RED_DOT) s += v * b[i];
        else if (OP == RED_ABS) s += fabs(v);
        else if (OP == RED_SUM) s += v;
        else s += v < 0 ? -v : 0.0;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_reduce_final(int nparts, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    double s = 0;
    for (int j = threadIdx.x; j < nparts; j += BAMG_BLK) s += part[j];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) *out = s;
}

// Multi-dot h_b = <V_b, w> for b < nv (V: nv vectors of length n, stride n):
// stage 1 over a fixed row partition; every wavefront writes its own partial
// (no block barrier) -> part[(block*4 + wave)][nv].
__global__ void __launch_bounds__(BAMG_BLK)
k_mdot_partial(int n, int nv, const double* __restrict__ V, const double* __restrict__ w,
               double* __restrict__ part) {
    const int lane = threadIdx.x % BAMG_WAVE, wv = threadIdx.x / BAMG_WAVE;
    const int chunk = (n + gridDim.x - 1) / gridDim.x;
    const int i0 = blockIdx.x * chunk, i1 = min(n, i0 + chunk);
    const size_t slot = ((size_t)blockIdx.x * (BAMG_BLK / BAMG_WAVE) + wv) * nv;
    for (int b = 0; b < nv; ++b) {
        const double* vb = V + (size_t)b * n;
        double s = 0;
        for (int i = i0 + threadIdx.x; i < i1; i += BAMG_BLK) s += vb[i] * w[i];
        s = wave_sum(s);
        if (lane == 0) part[slot + b] = s;
    }
}

// Stage 2: h[b] = sum_blocks part[.][b]; hacc[b] += h[b] (hacc may be null).
__global__ void k_mdot_final(int nparts, int nv, const double* __restrict__ part, double* __restrict__ h,
                             double* __restrict__ hacc) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    int b = blockIdx.x;
    double s = 0;
    for (int j = threadIdx.x; j < nparts; j += BAMG_BLK) s += part[(size_t)j * nv + b];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) {
        h[b] = s;
        if (hacc) hacc[b] += s;
    }
}

// w -= sum_b h_b V_b.
__global__ void k_vupdate(int n, int nv, const double* __restrict__ V, const double* __restrict__ h,
                          double* __restrict__ w) {
    int i = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    double s = w[i];
    for (int b = 0; b < nv; ++b) s -= h[b] * V[(size_t)b * n + i];
    w[i] = s;
}

// out = a * scale where scale = num / den (device scalars; den null -> 1).
__global__ void k_scale(int n, const double* __restrict__ a, const double* __restrict__ num,
                        const double* __restrict__ den, int sqrt_den, double* __restrict__ out) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    double d = den ? (sqrt_den ? sqrt(*den) : *den) : 1.0;
    double s = (num ? *num : 1.0) / d;
    out[i] = a[i] * s;
}

__global__ void k_copy(long long n, const double* __restrict__ a, double* __restrict__ b) {
    long long i = (long long)blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// One column of the GMRES Hessenberg matrix (column-major, ld): apply the
// previous Givens rotations, form the new one, update g; est = |g[j+1]|.
// hnew2 = ||w||^2 after orthogonalisation (device scalar).
__global__ void k_givens(int j, int ld, double* __restrict__ H, const double* __restrict__ hnew2,
                         double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
                         double* __restrict__ est) {
    if (threadIdx.x != 0) return;
    double* col = H + (size_t)j * ld;
    col[j + 1] = sqrt(*hnew2);
    for (int i = 0; i < j; ++i) {
        double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    double a = col[j], b = col[j + 1];
    double r = sqrt(a * a + b * b);
    double c = r > 0 ? a / r : 1.0, s = r > 0 ? b / r : 0.0;
    cs[j] = c; sn[j] = s;
    col[j] = r; col[j + 1] = 0.0;
    g[j + 1] = -s * g[j];
    g[j] = c * g[j];
    *est = fabs(g[j + 1]);
}

// Back substitution R y = g for the k x k upper triangle of H (one thread).
__global__ void k_gmres_y(int k, int ld, const double* __restrict__ H, const double* __restrict__ g,
                          double* __restrict__ y) {
    if (threadIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int c = i + 1; c < k; ++c) s -= H[(size_t)c * ld + i] * y[c];
        y[i] = s / H[(size_t)i * ld + i];
    }
}

// x += sum_j y_j Z_j.
__global__ void k_xupdate(int n, int k, const double* __restrict__ Z, const double* __restrict__ y,
                          double* __restrict__ x) {
    int i = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    double s = x[i];
    for (int j = 0; j < k; ++j) s += y[j] * Z[(size_t)j * n + i];
    x[i] = s;
}

// g = [beta, 0, ...]; H zeroed by the caller.
__global__ void k_gmres_init(int m, const double* __restrict__ beta2, double* __restrict__ g) {
    int i = threadIdx.x;
    for (int k = i; k <= m; k += blockDim.x) g[k] = 0.0;
    if (i == 0) g[0] = sqrt(*beta2);
}

// x <- max(x, 0).
__global__ void k_clamp(int n, double* __restrict__ x) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n && x[i] < 0) x[i] = 0.0;
}

// Initial Arnoldi vector of the coarsest eigensolve (seeded, stream 7).
__global__ void k_rand_vec(int n, uint64_t seed, double* __restrict__ v) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n) v[i] = splitmix_u01(seed, 7ull, (uint64_t)i) - 0.5;
}

// c_j = sum_i T_ij (column sums of a coarse operator whose stencil lies in
// the 3x3 box): gather row i of T for every box neighbour i of j, fixed
// order.  T == identity when trp is null.
template <typename M>
__global__ void k_colsum_box(int n, FastDiv dy, int nx, int ny, int periodic, const int* __restrict__ trp,
                             const int* __restrict__ tci, const M* __restrict__ tv, double* __restrict__ c) {
    int j = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (j >= n) return;
    if (!trp) { c[j] = 1.0; return; }
    int ja = (int)dy.div((uint32_t)j), jb = j - ja * ny;
    int rows[9];
#pragma unroll
    for (int s = 0; s < 9; ++s) {
        int a = ja + s / 3 - 1, b = jb + s % 3 - 1;
        rows[s] = -1;
        if (periodic) {
            a = a < 0 ? a + nx : (a >= nx ? a - nx : a);
            b = b < 0 ? b + ny : (b >= ny ? b - ny : b);
        } else if (a < 0 || a >= nx || b < 0 || b >= ny) {
            continue;
        }
        rows[s] = a * ny + b;
    }
    double s = 0;
    // ascending row order
    for (int pass = 0; pass < 9; ++pass) {
        int best = -1;
        for (int t = 0; t < 9; ++t) {
            if (rows[t] < 0) continue;
            int rank = 0;
            for (int u = 0; u < 9; ++u) rank += rows[u] >= 0 && rows[u] < rows[t];
            if (rank == pass) best = rows[t];
        }
        if (best < 0) break;
        for (int p = trp[best]; p < trp[best + 1]; ++p)
            if (tci[p] == j) s += (double)tv[p];
    }
    c[j] = s;
}

// out[i] = V[i*R + c] widened to FP64.
template <typename T>
__global__ void k_get_col_t(int rows, int R, int c, const T* __restrict__ V, double* __restrict__ out) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < rows) out[i] = (double)V[(size_t)i * R + c];
}

// Copy column col of a dense row-major matrix (rows x ld) into out.
__global__ void k_get_col(int rows, int ld, int col, const double* __restrict__ A, double* __restrict__ out) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < rows) out[i] = A[(size_t)i * ld + col];
}

// Zero the last row and column of an n x n dense matrix.
__global__ void k_zero_border(int n, double* __restrict__ A) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n) { A[(size_t)(n - 1) * n + i] = 0.0; A[(size_t)i * n + n - 1] = 0.0; }
}

// Cast a level vector between the FP64 outer iteration and the FP32 cycle.
__global__ void k_d2f(int n, const double* __restrict__ a, float* __restrict__ b) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}
__global__ void k_f2d(int n, const float* __restrict__ a, double* __restrict__ b) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}

// ---------------------------------------------------------------- per-chain (segmented) versions
// Chain c owns rows [g[c].off, g[c].off + g[c].n) of the finest level; its
// rows are split into gridDim.x fixed chunks.  Per-chain scalars live at
// out[c * stride].

template <int OP>
__global__ void k_seg_reduce_partial(const ChainGeo* __restrict__ geo, int seg_rows, const double* __restrict__ a,
                                     const double* __restrict__ b, double* __restrict__ part) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    const ChainGeo g = geo[blockIdx.y];
    const int r0 = g.off + blockIdx.x * seg_rows, r1 = min(g.off + g.n, r0 + seg_rows);
    double s = 0;
    for (int i = r0 + threadIdx.x; i < r1; i += BAMG_BLK) {
        double v = a[i];
        if (OP == RED_DOT) s += v * b[i];
        else if (OP == RED_ABS) s += fabs(v);
        else if (OP == RED_SUM) s += v;
        else s += v < 0 ? -v : 0.0;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// Block c adds chain c's ceil(n_c / seg_rows) partials (stride P) in order.
__global__ void k_seg_reduce_final(const ChainGeo* __restrict__ geo, int seg_rows, int P,
                                   const double* __restrict__ part, double* __restrict__ out, int stride) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    const int np = (geo[blockIdx.x].n + seg_rows - 1) / seg_rows;
    double s = 0;
    for (int j = threadIdx.x; j < np; j += BAMG_BLK) s += part[(size_t)blockIdx.x * P + j];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[(size_t)blockIdx.x * stride] = s;
}

// Multi-dots per chain: part[c][chunk*4 + wave][nv] (wave partials, no
// block barrier); only chains with act[c] != 0.  Chunk = seg_rows rows.
// Dots b < nb are <V_b, w>; with nv = nb + 1 the last one is <w, w>.
__global__ void __launch_bounds__(BAMG_BLK)
k_seg_mdot_partial(const ChainGeo* __restrict__ geo, int seg_rows, int N, int nb, int nv, const int* __restrict__ act,
                   const double* __restrict__ V, const double* __restrict__ w, double* __restrict__ part) {
    const ChainGeo g = geo[blockIdx.y];
    if (!act[blockIdx.y]) return;
    const int lane = threadIdx.x % BAMG_WAVE, wv = threadIdx.x / BAMG_WAVE;
    const int i0 = g.off + blockIdx.x * seg_rows, i1 = min(g.off + g.n, i0 + seg_rows);
    if (i0 >= i1) return;
    const size_t slot = (((size_t)blockIdx.y * gridDim.x + blockIdx.x) * (BAMG_BLK / BAMG_WAVE) + wv) * nv;
    // eight dots per pass over the chunk: w is read once per eight vectors
    for (int b0 = 0; b0 < nv; b0 += 8) {
        double s[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) s[q] = 0;
        for (int i = i0 + threadIdx.x; i < i1; i += BAMG_BLK) {
            const double wi = w[i];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int b = b0 + q;
                if (b < nv) s[q] += (b < nb ? V[(size_t)b * N + i] : wi) * wi;
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double t = wave_sum(s[q]);
            if (lane == 0 && b0 + q < nv) part[slot + b0 + q] = t;
        }
    }
}

// h[c*HS + b] = sum of chain c's wave partials (its own chunk count, stride
// P chunks); hacc[c*HAS + b] += h for the basis dots b < nb.  Block (b, c).
__global__ void k_seg_mdot_final(const ChainGeo* __restrict__ geo, int seg_rows, int P, int nb, int nv,
                                 const int* __restrict__ act, const double* __restrict__ part, double* __restrict__ h,
                                 int HS, double* __restrict__ hacc, int HAS) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    const int b = blockIdx.x, c = blockIdx.y;
    if (!act[c]) return;
    const int WPB = BAMG_BLK / BAMG_WAVE;
    const int np = ((geo[c].n + seg_rows - 1) / seg_rows) * WPB;
    double s = 0;
    for (int j = threadIdx.x; j < np; j += BAMG_BLK) s += part[((size_t)c * P * WPB + j) * nv + b];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) {
        h[(size_t)c * HS + b] = s;
        if (b < nb) hacc[(size_t)c * HAS + b] += s;
    }
}

// Second Gram-Schmidt pass only where the first lost more than half of
// ||w||^2 (the test of Daniel, Gragg, Kaufman and Stewart with eta^2 = 1/2):
// after w' = w - V h, ||w'||^2 = ||w||^2 - ||h||^2 for orthonormal V.
// act2[c] = act[c] && ||w||^2 - ||h||^2 < ||w||^2 / 2  (h[c*HS + nb] = ||w||^2).
__global__ void k_seg_dgks(int nch, int nb, const int* __restrict__ act, const double* __restrict__ h, int HS,
                           int* __restrict__ act2) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nch) return;
    int need = 0;
    if (act[c]) {
        const double* hc = h + (size_t)c * HS;
        double hh = 0;
        for (int b = 0; b < nb; ++b) hh += hc[b] * hc[b];
        const double ww = hc[nb];
        need = (ww - hh) < 0.5 * ww;
    }
    act2[c] = need;
}

// Fused Gram-Schmidt passes over a row chunk of each chain (chunk and wave
// partials in the layout of k_seg_mdot_partial).
// k_seg_upd_dots: w <- w - sum_{b<nb} h_b V_b on chains with act, then the
// dots <V_b, w> of the updated w (the second pass's coefficients): each row's
// V values are loaded once into registers and serve the update and the dots.
// MAXB (>= nb) values and accumulators per thread, in registers.
#define GS_MAXB 64
template <int MAXB>
__global__ void __launch_bounds__(BAMG_BLK)
k_seg_upd_dots(const ChainGeo* __restrict__ geo, int seg_rows, int N, int nb, const int* __restrict__ act,
               const double* __restrict__ V, const double* __restrict__ h, int HS, double* __restrict__ w,
               double* __restrict__ part) {
    const ChainGeo g = geo[blockIdx.y];
    if (!act[blockIdx.y]) return;
    const int lane = threadIdx.x % BAMG_WAVE, wv = threadIdx.x / BAMG_WAVE;
    const int i0 = g.off + blockIdx.x * seg_rows, i1 = min(g.off + g.n, i0 + seg_rows);
    if (i0 >= i1) return;
    const double* hc = h + (size_t)blockIdx.y * HS;
    double acc[MAXB];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) acc[b] = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += BAMG_BLK) {
        double v[MAXB];
#pragma unroll
        for (int b = 0; b < MAXB; ++b) v[b] = b < nb ? V[(size_t)b * N + i] : 0.0;
        double s = w[i];
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
            if (b < nb) s -= hc[b] * v[b];
        w[i] = s;
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
            if (b < nb) acc[b] += v[b] * s;
    }
    const size_t slot = (((size_t)blockIdx.y * gridDim.x + blockIdx.x) * (BAMG_BLK / BAMG_WAVE) + wv) * nb;
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        if (b < nb) {
            const double t = wave_sum(acc[b]);
            if (lane == 0) part[slot + b] = t;
        }
    }
}

// k_seg_upd_norm: w <- w - sum_{b<nb} h_b V_b on chains with act2 (the second
// pass where it is needed), then the partial ||w||^2 of every chain with act
// (one value per wave, nv = 1 layout).
__global__ void __launch_bounds__(BAMG_BLK)
k_seg_upd_norm(const ChainGeo* __restrict__ geo, int seg_rows, int N, int nb, const int* __restrict__ act,
               const int* __restrict__ act2, const double* __restrict__ V, const double* __restrict__ h, int HS,
               double* __restrict__ w, double* __restrict__ part) {
    const ChainGeo g = geo[blockIdx.y];
    if (!act[blockIdx.y]) return;
    const bool upd = act2[blockIdx.y] != 0;
    const int lane = threadIdx.x % BAMG_WAVE, wv = threadIdx.x / BAMG_WAVE;
    const int i0 = g.off + blockIdx.x * seg_rows, i1 = min(g.off + g.n, i0 + seg_rows);
    if (i0 >= i1) return;
    const double* hc = h + (size_t)blockIdx.y * HS;
    double acc = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += BAMG_BLK) {
        double s = w[i];
        if (upd) {
            for (int b = 0; b < nb; ++b) s -= hc[b] * V[(size_t)b * N + i];
            w[i] = s;
        }
        acc += s * s;
    }
    acc = wave_sum(acc);
    if (lane == 0) part[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * (BAMG_BLK / BAMG_WAVE) + wv] = acc;
}

// out[c * stride] = sum of chain c's wave partials (its own chunk count, P
// chunks per chain) for chains with act; one block per chain.
__global__ void k_seg_wave_final(const ChainGeo* __restrict__ geo, int seg_rows, int P, const int* __restrict__ act,
                                 const double* __restrict__ part, double* __restrict__ out, int stride) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    const int c = blockIdx.x;
    if (!act[c]) return;
    const int WPB = BAMG_BLK / BAMG_WAVE;
    const int np = ((geo[c].n + seg_rows - 1) / seg_rows) * WPB;
    double s = 0;
    for (int j = threadIdx.x; j < np; j += BAMG_BLK) s += part[(size_t)c * P * WPB + j];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[(size_t)c * stride] = s;
}

// w -= sum_b h_b V_b on the rows of active chains.
__global__ void k_seg_vupdate(int N, const ChainGeo* __restrict__ geo, int nch, int nv, const int* __restrict__ act,
                              const double* __restrict__ V, const double* __restrict__ h, int HS,
                              double* __restrict__ w) {
    int i = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK + threadIdx.x;
    if (i >= N) return;
    const int c = find_chain(geo, nch, i);
    if (!act[c]) return;
    const double* hc = h + (size_t)c * HS;
    double s = w[i];
    for (int b = 0; b < nv; ++b) s -= hc[b] * V[(size_t)b * N + i];
    w[i] = s;
}

// out_i = a_i * num_c / den_c (den_c square-rooted when sqrt_den) on the
// rows of chains with act[c] (act null: all chains).
__global__ void k_seg_scale(int N, const ChainGeo* __restrict__ geo, int nch, const int* __restrict__ act,
                            const double* __restrict__ a, const double* __restrict__ num, const double* __restrict__ den,
                            int stride, int sqrt_den, double* __restrict__ out) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= N) return;
    const int c = find_chain(geo, nch, i);
    if (act && !act[c]) return;
    double d = den ? den[(size_t)c * stride] : 1.0;
    if (sqrt_den) d = sqrt(d);
    const double s = (num ? num[(size_t)c * stride] : 1.0) / d;
    out[i] = a[i] * s;
}

// Givens step j for every active chain (one thread each); est[c] = |g_{j+1}|.
__global__ void k_seg_givens(int nch, int j, int ld, const int* __restrict__ act, double* __restrict__ Hall, int HS,
                             const double* __restrict__ hnew2, int hstride, double* __restrict__ csall,
                             double* __restrict__ snall, double* __restrict__ gall, int GS, double* __restrict__ est) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nch || !act[c]) return;
    double* col = Hall + (size_t)c * HS + (size_t)j * ld;
    double* cs = csall + (size_t)c * GS;
    double* sn = snall + (size_t)c * GS;
    double* g = gall + (size_t)c * GS;
    col[j + 1] = sqrt(hnew2[(size_t)c * hstride]);
    for (int i = 0; i < j; ++i) {
        double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    double a = col[j], b = col[j + 1];
    double r = sqrt(a * a + b * b);
    double cc = r > 0 ? a / r : 1.0, s = r > 0 ? b / r : 0.0;
    cs[j] = cc; sn[j] = s;
    col[j] = r; col[j + 1] = 0.0;
    g[j + 1] = -s * g[j];
    g[j] = cc * g[j];
    est[c] = fabs(g[j + 1]);
}

// g = [beta_c, 0, ...] for every chain (beta2 per chain at stride).
__global__ void k_seg_gmres_init(int nch, int m, const double* __restrict__ beta2, int stride, double* __restrict__ gall,
                                 int GS) {
    int c = blockIdx.x;
    if (c >= nch) return;
    for (int k = threadIdx.x; k <= m; k += blockDim.x) gall[(size_t)c * GS + k] = 0.0;
    if (threadIdx.x == 0) gall[(size_t)c * GS] = sqrt(beta2[(size_t)c * stride]);
}

// Back substitution per chain with its own k = kd[c].
__global__ void k_seg_gmres_y(int nch, int ld, const int* __restrict__ kd, const double* __restrict__ Hall, int HS,
                              const double* __restrict__ gall, int GS, double* __restrict__ yall) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nch) return;
    const int k = kd[c];
    const double* H = Hall + (size_t)c * HS;
    const double* g = gall + (size_t)c * GS;
    double* y = yall + (size_t)c * GS;
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int q = i + 1; q < k; ++q) s -= H[(size_t)q * ld + i] * y[q];
        y[i] = s / H[(size_t)i * ld + i];
    }
}

// x += sum_{j < kd[c]} y_cj Z_j.
__global__ void k_seg_xupdate(int N, const ChainGeo* __restrict__ geo, int nch, const int* __restrict__ kd,
                              const double* __restrict__ Z, const double* __restrict__ yall, int GS,
                              double* __restrict__ x) {
    int i = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK + threadIdx.x;
    if (i >= N) return;
    const int c = find_chain(geo, nch, i);
    const int k = kd[c];
    const double* y = yall + (size_t)c * GS;
    double s = x[i];
    for (int j = 0; j < k; ++j) s += y[j] * Z[(size_t)j * N + i];
    x[i] = s;
}

// Gather / scatter between the caller's chain order and the internal one:
// out[dst_off[c] + i] = in[src_off[c] + i] for i < len[c] (block y = chain).
__global__ void k_seg_permute(const int* __restrict__ src_off, const int* __restrict__ dst_off,
                              const int* __restrict__ len, const double* __restrict__ in, double* __restrict__ out) {
    const int c = blockIdx.y;
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < len[c]; i += gridDim.x * BAMG_BLK)
        out[dst_off[c] + i] = in[src_off[c] + i];
}

// Reordered input CSR: rows of chain c move from src to dst offset; columns
// shift with them.  Pass 1 copies row lengths, pass 2 (after a scan) the
// entries.
__global__ void k_seg_csr_len(int nch, const int* __restrict__ src_off, const int* __restrict__ dst_off,
                              const int* __restrict__ len, const int* __restrict__ rp, int* __restrict__ cnt) {
    const int c = blockIdx.y;
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < len[c]; i += gridDim.x * BAMG_BLK)
        cnt[dst_off[c] + i] = rp[src_off[c] + i + 1] - rp[src_off[c] + i];
}

__global__ void k_seg_csr_fill(const int* __restrict__ src_off, const int* __restrict__ dst_off,
                               const int* __restrict__ len, const int* __restrict__ rp, const int* __restrict__ ci,
                               const double* __restrict__ v, const int* __restrict__ nrp, int* __restrict__ nci,
                               double* __restrict__ nv) {
    const int c = blockIdx.y;
    const int shift = dst_off[c] - src_off[c];
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < len[c]; i += gridDim.x * BAMG_BLK) {
        const int si = src_off[c] + i, di = dst_off[c] + i;
        int q = nrp[di];
        for (int p = rp[si]; p < rp[si + 1]; ++p, ++q) {
            nci[q] = ci[p] + shift;
            nv[q] = v[p];
        }
    }
}

// e = 0 (a fill kernel, so that a captured cycle holds no memset node).
template <typename T>
__global__ void k_fill_t(int n, T* __restrict__ e, RowMask mk) {
    if (!tile_active(mk, blockIdx.x, BAMG_BLK, 1, n)) return;
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n) e[i] = (T)0;
}
