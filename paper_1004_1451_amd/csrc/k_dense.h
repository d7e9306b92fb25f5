// Dense kernels of the coarsest level (FP64, vector ALUs).
//
// The coarsest operator B_L (n x n, rank n-1, 1^T B_L = 0) is handled through
// its Moore-Penrose inverse W = B_L^+ (Section 4.2: minimal-norm coarsest
// solve), stored dense row-major with leading dimension n:
//   1. Binv = inverse of the leading (n-1) x (n-1) block B_11 by block
//      Gauss-Jordan without pivoting (blocks of GJ_NB);
//   2. y = [-Binv b_{:,n}; 1] spans null(B_L);
//   3. W = Pi_y [[Binv, 0], [0, 0]] Pi_1 with Pi_1 = I - 1 1^T / n (projector
//      onto range(B_L) = 1^perp) and Pi_y = I - y y^T / (y^T y).
// The coarsest eigenpairs (Algorithm 3, l = L) come from Arnoldi on the
// shift-invert operator v -> u - y (c^T u)/(c^T y), u = W T v, c = T^T 1,
// whose eigenvalues on {c^T v = 0} are 1/lam for the nonzero lam.
#pragma once
#include "common.h"

#define GJ_NB 64

// Dense copy of a CSR matrix (n x n, ld n); zero first.
__global__ void k_densify(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                          const double* __restrict__ v, double* __restrict__ D) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) D[(size_t)i * n + ci[p]] = v[p];
}

template <typename M>
__global__ void k_densify_cast(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                               const M* __restrict__ v, double* __restrict__ D) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) D[(size_t)i * n + ci[p]] = (double)v[p];
}

__global__ void k_fill(long long n, double val, double* __restrict__ a) {
    long long i = (long long)blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n) a[i] = val;
}

// Max |entry| of a dense matrix: partial per block, then a fixed-order final.
__global__ void k_absmax_partial(long long n, const double* __restrict__ a, double* __restrict__ part) {
    __shared__ double sh[BAMG_BLK];
    double m = 0;
    for (long long i = (long long)blockIdx.x * BAMG_BLK + threadIdx.x; i < n; i += (long long)gridDim.x * BAMG_BLK)
        m = fmax(m, fabs(a[i]));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = BAMG_BLK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Row panel: A[k0:k0+nb, j] = Dinv * A[k0:k0+nb, j] for j outside the block.
// Block = 64 columns.
__global__ void __launch_bounds__(BAMG_BLK)
k_gj_rowpanel(int m, int ld, int k0, int nb, double* __restrict__ A) {
    __shared__ double D[GJ_NB][GJ_NB + 1];
    __shared__ double X[GJ_NB][GJ_NB + 1];
    const int tid = threadIdx.x;
    int j0 = blockIdx.x * 64;
    if (j0 >= k0 && j0 < k0 + nb) return;   // the diagonal block (aligned to 64)
    int w = min(64, m - j0);
    for (int e = tid; e < nb * nb; e += BAMG_BLK) D[e / nb][e % nb] = A[(size_t)(k0 + e / nb) * ld + k0 + e % nb];
    for (int e = tid; e < nb * 64; e += BAMG_BLK) {
        int r = e / 64, c = e % 64;
        X[r][c] = c < w ? A[(size_t)(k0 + r) * ld + j0 + c] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < nb * 64; e += BAMG_BLK) {
        int r = e / 64, c = e % 64;
        if (c >= w) continue;
        double s = 0;
        for (int k = 0; k < nb; ++k) s += D[r][k] * X[k][c];
        A[(size_t)(k0 + r) * ld + j0 + c] = s;
    }
}

// Rank-nb update of every entry outside row block and column block k:
// A[i, j] -= A[i, k-block] * A[k-block, j].  64 x 64 output tiles aligned with
// the 64-row blocks (a tile in the k row or column block has nothing to do),
// 4 x 4 per thread (256 threads); the k-block factors are staged in LDS in two
// halves of 32 (A part transposed so that both operands are read as
// contiguous 4-double runs).  34 KB of LDS lets four workgroups share a CU, so
// one workgroup's read-modify-write of its tile overlaps the others' products.
// The sum over k runs in order 0 .. nb-1.
#define GJ_T 64
#define GJ_KH 32
__global__ void __launch_bounds__(BAMG_BLK)
k_gj_update(int m, int ld, int k0, int nb, double* __restrict__ A) {
    __shared__ double AsT[GJ_KH][GJ_T + 2];
    __shared__ double Bs[GJ_KH][GJ_T + 2];
    const int tiles = ceil_div(m, GJ_T);
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int ti = t / tiles, tj = t % tiles;
    const int i0 = ti * GJ_T, j0 = tj * GJ_T;
    if (i0 == k0 || j0 == k0) return;         // inside the k row / column block
    const int tid = threadIdx.x;
    const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0;
    for (int kh = 0; kh < nb; kh += GJ_KH) {
        // A[i0 + r][k0 + kh + c] -> AsT[c][r];  A[k0 + kh + r][j0 + c] -> Bs[r][c]
        for (int e = tid; e < GJ_T * GJ_KH; e += BAMG_BLK) {
            const int r = e / GJ_KH, c = e % GJ_KH;
            AsT[c][r] = (i0 + r < m && kh + c < nb) ? A[(size_t)(i0 + r) * ld + k0 + kh + c] : 0.0;
        }
        for (int e = tid; e < GJ_KH * GJ_T; e += BAMG_BLK) {
            const int r = e / GJ_T, c = e % GJ_T;
            Bs[r][c] = (j0 + c < m && kh + r < nb) ? A[(size_t)(k0 + kh + r) * ld + j0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < GJ_KH; ++k) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = AsT[k][tr + a];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[k][tc + b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = i0 + tr + a;
        if (i >= m) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int j = j0 + tc + b;
            if (j < m) A[(size_t)i * ld + j] -= acc[a][b];
        }
    }
}

// Column panel: A[i, k-block] = -A[i, k-block] * Dinv for rows outside the
// block.  Block = 64 rows.
__global__ void __launch_bounds__(BAMG_BLK)
k_gj_colpanel(int m, int ld, int k0, int nb, double* __restrict__ A) {
    __shared__ double D[GJ_NB][GJ_NB + 1];
    __shared__ double X[64][GJ_NB + 1];
    const int tid = threadIdx.x;
    int i0 = blockIdx.x * 64;
    if (i0 == k0) return;
    int h = min(64, m - i0);
    for (int e = tid; e < nb * nb; e += BAMG_BLK) D[e / nb][e % nb] = A[(size_t)(k0 + e / nb) * ld + k0 + e % nb];
    for (int e = tid; e < 64 * nb; e += BAMG_BLK) {
        int r = e / nb, c = e % nb;
        X[r][c] = r < h ? A[(size_t)(i0 + r) * ld + k0 + c] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < 64 * nb; e += BAMG_BLK) {
        int r = e / nb, c = e % nb;
        if (r >= h) continue;
        double s = 0;
        for (int k = 0; k < nb; ++k) s += X[r][k] * D[k][c];
        A[(size_t)(i0 + r) * ld + k0 + c] = -s;
    }
}

// y = alpha * A x (+ beta * y0) for a dense row-major n x n matrix: one
// wavefront per row, fixed-order reduction.
__global__ void __launch_bounds__(BAMG_BLK)
k_gemv(int rows, int cols, int ld, const double* __restrict__ A, const double* __restrict__ x,
       double* __restrict__ y) {
    int row = blockIdx.x * (BAMG_BLK / BAMG_WAVE) + threadIdx.x / BAMG_WAVE;
    int lane = threadIdx.x % BAMG_WAVE;
    if (row >= rows) return;
    const double* a = A + (size_t)row * ld;
    double s = 0;
    for (int j = lane; j < cols; j += BAMG_WAVE) s += a[j] * x[j];
    s = wave_sum(s);
    if (lane == 0) y[row] = s;
}

// FP32 copy of the coarse inverse for the mixed-precision cycle.
__global__ void __launch_bounds__(BAMG_BLK)
k_gemv_f32(int rows, int cols, int ld, const float* __restrict__ A, const float* __restrict__ x,
           float* __restrict__ y) {
    int row = blockIdx.x * (BAMG_BLK / BAMG_WAVE) + threadIdx.x / BAMG_WAVE;
    int lane = threadIdx.x % BAMG_WAVE;
    if (row >= rows) return;
    const float* a = A + (size_t)row * ld;
    float s = 0;
    for (int j = lane; j < cols; j += BAMG_WAVE) s += a[j] * x[j];
    s = wave_sum(s);
    if (lane == 0) y[row] = s;
}

// y^T A in two stages: block (cx, ry) sums rows [ry*GT_ROWS, ...) of 256
// columns into part[ry][col]; the second stage adds the row chunks in order.
#define GT_ROWS 128
__global__ void k_gemv_t_partial(int rows, int cols, int ld, const double* __restrict__ A,
                                 const double* __restrict__ y, double* __restrict__ part) {
    int j = blockIdx.x * BAMG_BLK + threadIdx.x;
    int r0 = blockIdx.y * GT_ROWS;
    if (j >= cols) return;
    double s = 0;
    int r1 = min(rows, r0 + GT_ROWS);
    for (int i = r0; i < r1; ++i) s += y[i] * A[(size_t)i * ld + j];
    part[(size_t)blockIdx.y * cols + j] = s;
}

__global__ void k_gemv_t_final(int nchunks, int cols, const double* __restrict__ part, double* __restrict__ out) {
    int j = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (j >= cols) return;
    double s = 0;
    for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * cols + j];
    out[j] = s;
}

// Null vector from the inverse of B_11: y_1 = -Binv b_col, y_n = 1 (the GEMV
// result is passed in g).
__global__ void k_null_finish(int n, const double* __restrict__ g, double* __restrict__ y) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n - 1) y[i] = -g[i];
    if (i == n - 1) y[i] = 1.0;
}

// W <- W - s 1^T / n - y (u - (y^T s) 1^T / n)^T / (y^T y): both projections
// of the padded inverse at once (s = W 1, u = y^T W, sc[0] = y^T s,
// sc[1] = y^T y).
__global__ void k_project_w(int n, double* __restrict__ W, const double* __restrict__ s, const double* __restrict__ u,
                            const double* __restrict__ y, const double* __restrict__ sc) {
    long long e = (long long)blockIdx.x * BAMG_BLK + threadIdx.x;
    if (e >= (long long)n * n) return;
    int i = (int)(e / n), j = (int)(e % n);
    double inv_n = 1.0 / n;
    W[e] = W[e] - s[i] * inv_n - y[i] * (u[j] - sc[0] * inv_n) / sc[1];
}

// ---------------------------------------------------------------- block-tridiagonal inverse
// On the coarse grid (state s = a*ny + b, stencil within the 3x3 box) B_L is
// block tridiagonal in the grid rows a, with blocks of size b = ny, plus the
// two corner blocks (0, K) and (K, 0) when periodic (K = nx - 1).  The padded
// matrix Bh = B_L with its last row and column replaced by e_n (so that
// Bh^-1 = [[B_11^-1, 0], [0, 1]]) is factored by block LU without pivoting,
// eliminating block rows 0..K-1 in order; with the corners the fill stays in
// block column K and block row K ("arrow").  Compact factor storage, each an
// array of nx blocks of b x b (row-major):
//   Dk[k]  diagonal block, replaced by its inverse;
//   Up[k]  block (k, k+1);   Lo[k]  block (k, k-1) -> multiplier;
//   Cl[k]  block (k, K) for k < K-1;   Rw[k]  block (K, k) for k < K-1 ->
//   multiplier.
// Then Bh^-1 is formed in the dense buffer by block forward substitution on
// the identity and block back substitution.

// Extract the blocks of Bh from the dense B_L (ld n = nx*b).
__global__ void k_bt_extract(int nx, int b, const double* __restrict__ A, double* __restrict__ Dk,
                             double* __restrict__ Up, double* __restrict__ Lo, double* __restrict__ Cl,
                             double* __restrict__ Rw) {
    const int n = nx * b, K = nx - 1, bb = b * b;
    const int k = blockIdx.y, kind = blockIdx.z;
    for (int e = blockIdx.x * BAMG_BLK + threadIdx.x; e < bb; e += gridDim.x * BAMG_BLK) {
        int r = e / b, c = e % b;
        int bi, bj;
        double* dst;
        switch (kind) {
            case 0: bi = k; bj = k; dst = Dk; break;
            case 1: if (k >= K) return; bi = k; bj = k + 1; dst = Up; break;
            case 2: if (k < 1) return; bi = k; bj = k - 1; dst = Lo; break;
            case 3: if (k >= K - 1) return; bi = k; bj = K; dst = Cl; break;
            default: if (k >= K - 1) return; bi = K; bj = k; dst = Rw; break;
        }
        int gi = bi * b + r, gj = bj * b + c;
        double v = A[(size_t)gi * n + gj];
        if (gi == n - 1 || gj == n - 1) v = (gi == gj) ? 1.0 : 0.0;
        dst[(size_t)k * bb + e] = v;
    }
}

// Small dense products on b x b blocks (b <= 64), one workgroup per product:
// C = A B (mode 0, C may alias A) or C -= A B (mode 1).
struct BlkOps {
    const double* A[4];
    const double* B[4];
    double* C[4];
    int mode[4];
};
__global__ void __launch_bounds__(BAMG_BLK)
k_blk_gemm(int b, BlkOps ops) {
    __shared__ double AsT[GJ_NB][GJ_NB + 2];
    __shared__ double Bs[GJ_NB][GJ_NB + 2];
    const int q = blockIdx.x;
    const double* A = ops.A[q];
    const double* Bm = ops.B[q];
    double* C = ops.C[q];
    const int mode = ops.mode[q];
    const int tid = threadIdx.x;
    for (int e = tid; e < GJ_NB * GJ_NB; e += BAMG_BLK) {
        int r = e / GJ_NB, c = e % GJ_NB;
        bool ok = r < b && c < b;
        AsT[c][r] = ok ? A[r * b + c] : 0.0;
        Bs[r][c] = ok ? Bm[r * b + c] : 0.0;
    }
    __syncthreads();
    const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
    for (int t = 0; t < b; ++t) {
        double av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = AsT[t][tr + a];
#pragma unroll
        for (int c = 0; c < 4; ++c) bv[c] = Bs[t][tc + c];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][c] += av[a] * bv[c];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            int r = tr + a, cc = tc + c;
            if (r < b && cc < b) {
                if (mode == 0) C[r * b + cc] = acc[a][c];
                else C[r * b + cc] -= acc[a][c];
            }
        }
}

// Block row kout of the n x n buffer W (rows kout*b ..), columns of this
// workgroup's 64-column tile:  T = W[kout] - A1 W[j1] - A2 W[j2] (A1/A2 null
// = absent), then W[kout] = Dinv T (Dinv null = T).  b <= 64.
__global__ void __launch_bounds__(BAMG_BLK)
k_bt_strip(int b, int n, double* __restrict__ W, int kout, const double* __restrict__ A1, int j1,
           const double* __restrict__ A2, int j2, const double* __restrict__ Dinv) {
    __shared__ double Ms[GJ_NB][GJ_NB + 1];
    __shared__ double Xs[GJ_NB][64 + 1];
    const int tid = threadIdx.x;
    const int c0 = blockIdx.x * 64;
    const int w = min(64, n - c0);
    const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
    double T[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int r = tr + a, c = tc + q;
            T[a][q] = (r < b && c < w) ? W[(size_t)(kout * b + r) * n + c0 + c] : 0.0;
        }
    for (int term = 0; term < 2; ++term) {
        const double* M = term == 0 ? A1 : A2;
        const int jb = term == 0 ? j1 : j2;
        if (!M) continue;
        __syncthreads();
        for (int e = tid; e < b * b; e += BAMG_BLK) Ms[e / b][e % b] = M[e];
        for (int e = tid; e < b * 64; e += BAMG_BLK) {
            int r = e / 64, c = e % 64;
            Xs[r][c] = c < w ? W[(size_t)(jb * b + r) * n + c0 + c] : 0.0;
        }
        __syncthreads();
        for (int t = 0; t < b; ++t) {
            double mv[4], xv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) mv[a] = (tr + a < b) ? Ms[tr + a][t] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) xv[q] = Xs[t][tc + q];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int q = 0; q < 4; ++q) T[a][q] -= mv[a] * xv[q];
        }
    }
    if (Dinv) {
        __syncthreads();
        for (int e = tid; e < b * b; e += BAMG_BLK) Ms[e / b][e % b] = Dinv[e];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (tr + a < GJ_NB) Xs[tr + a][tc + q] = T[a][q];
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) T[a][q] = 0.0;
        for (int t = 0; t < b; ++t) {
            double mv[4], xv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) mv[a] = (tr + a < b) ? Ms[tr + a][t] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) xv[q] = Xs[t][tc + q];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int q = 0; q < 4; ++q) T[a][q] += mv[a] * xv[q];
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int r = tr + a, c = tc + q;
            if (r < b && c < w) W[(size_t)(kout * b + r) * n + c0 + c] = T[a][q];
        }
}

// W = I (n x n).
__global__ void k_identity(long long nn, int n, double* __restrict__ W) {
    long long e = (long long)blockIdx.x * BAMG_BLK + threadIdx.x;
    if (e < nn) W[e] = (e / n == e % n) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------- small vectors
// Fixed-order dot products for vectors of the coarsest level (one block).
__global__ void k_dot1(int n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    double s = 0;
    for (int i = threadIdx.x; i < n; i += BAMG_BLK) s += a[i] * b[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------- Arnoldi
// The Krylov basis Vb (n x (m+1), column j at j*n) and the Hessenberg matrix
// H ((m+1) x m, column-major ld m+1) live on the device.  One Arnoldi step is
//   w = T v_j (CSR, or copy when T = I), u = W w, u -= y (c^T u)/(c^T y),
//   two rounds of classical Gram-Schmidt, h_{j+1,j} = ||u||, v_{j+1} = u/h.
// Multi-dot: blocks = j+1, block b computes <v_b, u>.
__global__ void k_mdot(int n, int nv, const double* __restrict__ Vb, const double* __restrict__ u,
                       double* __restrict__ h) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    int b = blockIdx.x;
    if (b >= nv) return;
    double s = 0;
    for (int i = threadIdx.x; i < n; i += BAMG_BLK) s += Vb[(size_t)b * n + i] * u[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) h[b] = s;
}

// u -= sum_b h_b v_b; hacc_b += h_b.
__global__ void k_mupdate(int n, int nv, const double* __restrict__ Vb, const double* __restrict__ h,
                          double* __restrict__ u, double* __restrict__ hacc) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n) {
        double s = u[i];
        for (int b = 0; b < nv; ++b) s -= h[b] * Vb[(size_t)b * n + i];
        u[i] = s;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < nv) hacc[threadIdx.x] += h[threadIdx.x];
}

// u -= y * (c^T u) / (c^T y)   (dots precomputed: d[0] = c^T u, cy = c^T y).
__global__ void k_project_domain(int n, const double* __restrict__ y, const double* __restrict__ d,
                                 const double* __restrict__ cy, double* __restrict__ u) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n) u[i] -= y[i] * (*d / *cy);
}

// v = u / sqrt(nrm2); H[j+1, j] = sqrt(nrm2).
__global__ void k_normalize_into(int n, const double* __restrict__ u, const double* __restrict__ nrm2,
                                 double* __restrict__ v, double* __restrict__ hout) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    double nr = sqrt(*nrm2);
    if (i < n) v[i] = nr > 0 ? u[i] / nr : 0.0;
    if (i == 0) *hout = nr;
}

// ---------------------------------------------------------------- Hessenberg eigensolver
// Eigenpairs of the m x m Hessenberg matrix H_m of the Arnoldi process, with
// one wavefront (64 lanes, m <= 64), data in LDS.
//  - Eigenvalues: the Francis double-shift QR iteration of Golub and Van
//    Loan, Matrix Computations, Algorithms 7.5.1 (the implicit double-shift
//    step) and 7.5.2 (deflation of negligible subdiagonal entries), applied
//    to the active unreduced window only (no Schur vectors are needed).
//    The bulge is chased with 3-element Householder reflectors; lane j
//    updates column j of the reflected rows and lane i row i of the
//    reflected columns; the next reflector's vector comes from the lanes
//    that produced it (v_readlane), not from LDS.  A window that has not
//    deflated after 8 steps takes one step with an exceptional real double
//    shift (both shifts at the bottom diagonal entry moved by the size of
//    the two bottom subdiagonal entries); 40 m steps in all is a failure.
//  - Eigenvectors of the selected eigenvalues: inverse iteration with the
//    complex matrix H - theta I (Gaussian elimination with pivoting between
//    adjacent rows, tiny pivots replaced by 1e-14 ||H||).
#define HQR_MAXM 64
#define HQR_LD (HQR_MAXM + 1)

__device__ __forceinline__ void lds_sync() { __syncthreads(); }

// sqrt(s) for a normal s > 0 from v_rsq_f64, refined by one coupled
// Goldschmidt step for (sqrt(s), 1/(2 sqrt(s))) and one Newton correction of
// the root (within an ulp or so; far fewer dependent steps than the
// correctly rounded library square root).
__device__ __forceinline__ double sqrt_rsq(double s) {
    const double r = __builtin_amdgcn_rsq(s);
    double g = s * r, h = 0.5 * r;
    const double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    return fma(fma(-g, g, s), h, g);
}

// Householder vector of a 3-vector (x, y, z) (z = 0 for a 2-vector): with
// a = -sign(x) ||(x, y, z)||, u = (x - a, y, z) and beta = 2 / u^T u, the
// reflector I - beta u u^T maps (x, y, z) to (a, 0, 0).  beta = 0 when the
// vector is already zero below its first entry.  beta comes from u as
// formed, so the reflector is orthogonal to rounding whatever the error of
// the norm.
__device__ __forceinline__ void house3(double x, double y, double z, double& u0, double& u1, double& u2,
                                       double& beta) {
    const double tail = y * y + z * z;
    if (tail == 0.0) { u0 = 1.0; u1 = 0.0; u2 = 0.0; beta = 0.0; return; }
    const double nrm = sqrt_rsq(x * x + tail);
    const double a = x >= 0.0 ? -nrm : nrm;
    u0 = x - a; u1 = y; u2 = z;
    beta = 2.0 * cz_recip(u0 * u0 + tail);
}

// Eigenvalues of the m x m upper Hessenberg A (LDS, row-major, ld HQR_LD;
// overwritten) into (wr, wi); *fail = 1 if the iteration does not settle.
__device__ void francis_eigvals_wave(int m, double* A, double* wr, double* wi, int* fail) {
    const int lane = threadIdx.x;
    const double u = 2.220446049250313e-16;
#define HA(i, j) A[(i) * HQR_LD + (j)]
    // scale for the zero-sum fallback of the deflation test: sum of |entries|
    double fro = 0.0;
    if (lane < m)
        for (int i = 0; i <= min(lane + 1, m - 1); ++i) fro += fabs(HA(i, lane));
#pragma unroll
    for (int o = BAMG_WAVE / 2; o >= 1; o >>= 1) fro += __shfl_xor(fro, o, BAMG_WAVE);
    int hi = m - 1, stuck = 0, steps = 0;
    while (hi >= 0) {
        lds_sync();
        // lo: the bottom of the last negligible subdiagonal entry in the
        // window (GVL: |h_{i,i-1}| <= u (|h_{i-1,i-1}| + |h_ii|)); every lane
        // tests its own row, a ballot takes the largest
        int lo;
        {
            bool neg = false;
            if (lane >= 1 && lane <= hi) {
                double d = fabs(HA(lane - 1, lane - 1)) + fabs(HA(lane, lane));
                if (d == 0.0) d = fro;
                neg = fabs(HA(lane, lane - 1)) <= u * d;
            }
            const unsigned long long bal = __ballot(neg);
            lo = bal ? 63 - __clzll(bal) : 0;
        }
        if (lo == hi) {                          // a 1 x 1 block has deflated
            if (lane == 0) { wr[hi] = HA(hi, hi); wi[hi] = 0.0; }
            hi -= 1; stuck = 0;
            continue;
        }
        if (lo == hi - 1) {                      // a 2 x 2 block: its eigenvalues
            const double a = HA(hi - 1, hi - 1), b = HA(hi - 1, hi), c = HA(hi, hi - 1), d = HA(hi, hi);
            const double mid = 0.5 * (a + d), half = 0.5 * (a - d);
            const double disc = half * half + b * c;
            if (lane == 0) {
                if (disc >= 0.0) {
                    // the root of larger modulus first, the other from the
                    // determinant (no cancellation)
                    const double big = mid + (mid >= 0.0 ? sqrt(disc) : -sqrt(disc));
                    wr[hi - 1] = big;
                    wr[hi] = big != 0.0 ? (a * d - b * c) / big : 0.0;
                    wi[hi - 1] = wi[hi] = 0.0;
                } else {
                    const double im = sqrt(-disc);
                    wr[hi - 1] = wr[hi] = mid;
                    wi[hi - 1] = im; wi[hi] = -im;
                }
            }
            hi -= 2; stuck = 0;
            continue;
        }
        if (++steps > 40 * m) { if (lane == 0) *fail = 1; lds_sync(); return; }
        // the double shift: eigenvalues of the trailing 2 x 2 block through
        // their sum s and product t, or the exceptional pair
        double s, t;
        if (++stuck % 8 == 0) {
            const double r = HA(hi, hi) + fabs(HA(hi, hi - 1)) + fabs(HA(hi - 1, hi - 2));
            s = 2.0 * r; t = r * r;
        } else {
            const double a = HA(hi - 1, hi - 1), b = HA(hi - 1, hi), c = HA(hi, hi - 1), d = HA(hi, hi);
            s = a + d; t = a * d - b * c;
        }
        // first column of (H - sigma_1 I)(H - sigma_2 I) on the window
        const double h00 = HA(lo, lo), h01 = HA(lo, lo + 1), h10 = HA(lo + 1, lo), h11 = HA(lo + 1, lo + 1);
        double x = h00 * h00 + h01 * h10 - s * h00 + t;
        double y = h10 * (h00 + h11 - s);
        double z = h10 * HA(lo + 2, lo + 1);
        lds_sync();
        // every lane reads a valid row and column of the window (its own,
        // clamped); lanes outside the ranges below compute but do not store
        const int jc = min(max(lane, lo), hi);
        for (int k = lo; k <= hi - 1; ++k) {
            const bool two = k == hi - 1;        // the last reflector spans 2 rows
            const int k2 = two ? k + 1 : k + 2;  // its third row / column (read, unused, when two)
            // rows k .. k+2 of column jc, read before the reflector is formed
            const double a0 = HA(k, jc), a1 = HA(k + 1, jc), a2r = HA(k2, jc);
            double u0, u1, u2, beta;
            house3(x, y, two ? 0.0 : z, u0, u1, u2, beta);
            // rows k .. k+2 from the left, columns max(lo, k-1) .. hi
            {
                const double a2 = two ? 0.0 : a2r;
                const double w = beta * (u0 * a0 + u1 * a1 + u2 * a2);
                if (lane >= max(lo, k - 1) && lane <= hi) {
                    HA(k, lane) = a0 - w * u0;
                    HA(k + 1, lane) = a1 - w * u1;
                    if (!two) HA(k + 2, lane) = a2 - w * u2;
                }
            }
            lds_sync();
            // columns k .. k+2 from the right, rows lo .. min(k+3, hi)
            double c0;
            {
                const int i = min(jc, min(k + 3, hi));
                const double b0 = HA(i, k), b1 = HA(i, k + 1), b2r = HA(i, k2);
                const double b2 = two ? 0.0 : b2r;
                const double w = beta * (b0 * u0 + b1 * u1 + b2 * u2);
                c0 = b0 - w * u0;
                if (lane >= lo && lane <= min(k + 3, hi)) {
                    HA(lane, k) = c0;
                    HA(lane, k + 1) = b1 - w * u1;
                    if (!two) HA(lane, k + 2) = b2 - w * u2;
                }
            }
            // next reflector: column k below the diagonal, rows k+1 .. k+3
            if (!two) {
                x = readlane_f64(c0, k + 1);
                y = readlane_f64(c0, k + 2);
                z = k + 3 <= hi ? readlane_f64(c0, k + 3) : 0.0;
            }
            lds_sync();
            // entries the reflector annihilated: exactly zero below the
            // subdiagonal of column k - 1 (k > lo)
            if (k > lo && (lane == k + 1 || lane == k + 2) && lane <= hi) HA(lane, k - 1) = 0.0;
        }
    }
    lds_sync();
#undef HA
}

// Packed upper triangle (complex): row k, column j >= k.
__device__ __forceinline__ int upk(int m, int k, int j) { return k * m - (k * (k - 1)) / 2 + (j - k); }

// LU of (H - theta I) for the Hessenberg H (LDS, row-major m x m) with
// pivoting between adjacent rows, one wavefront: U (LDS, packed, 2 doubles per
// entry), the multiplier (fm[2k], fm[2k+1]) and swap flag swp[k] of step k.
// Tiny pivots are replaced by 1e-14 ||H||.
__device__ void hess_shift_factor_wave(int m, const double* __restrict__ H, double thr, double thi, double* U,
                                       double* fm, int* swp, double hnorm) {
    const int lane = threadIdx.x;
    const double tiny = 1e-14 * hnorm;
    // current row k, lane j holds entry j
    double cr = 0, ci = 0;
    if (lane < m) { cr = H[lane] - (lane == 0 ? thr : 0.0); ci = (lane == 0 ? -thi : 0.0); }
    for (int k = 0; k < m - 1; ++k) {
        double nr = 0, ni = 0;
        if (lane >= k && lane < m) {
            nr = H[(size_t)(k + 1) * m + lane] - (lane == k + 1 ? thr : 0.0);
            ni = (lane == k + 1 ? -thi : 0.0);
        }
        double ckr = readlane_f64(cr, k), cki = readlane_f64(ci, k);
        double nkr = readlane_f64(nr, k), nki = readlane_f64(ni, k);
        const bool swap = nkr * nkr + nki * nki > ckr * ckr + cki * cki;
        if (swap) {
            double tr = cr, ti = ci; cr = nr; ci = ni; nr = tr; ni = ti;
            double a = ckr, b = cki; ckr = nkr; cki = nki; nkr = a; nki = b;
        }
        if (ckr * ckr + cki * cki < tiny * tiny) {
            ckr = tiny; cki = 0.0;
            if (lane == k) { cr = tiny; ci = 0.0; }
        }
        const double rd = cz_recip(ckr * ckr + cki * cki);
        const double fr = (nkr * ckr + nki * cki) * rd, fi = (nki * ckr - nkr * cki) * rd;
        if (lane >= k && lane < m) {
            int e = upk(m, k, lane);
            U[2 * e] = cr; U[2 * e + 1] = ci;
            // next row minus f times the pivot row
            double ar = nr - (fr * cr - fi * ci), ai = ni - (fr * ci + fi * cr);
            cr = ar; ci = ai;
        } else {
            cr = 0; ci = 0;
        }
        if (lane == 0) { fm[2 * k] = fr; fm[2 * k + 1] = fi; swp[k] = swap ? 1 : 0; }
    }
    {
        int k = m - 1;
        double ckr = readlane_f64(cr, k), cki = readlane_f64(ci, k);
        if (ckr * ckr + cki * cki < tiny * tiny) { ckr = tiny; cki = 0.0; }
        if (lane == k) { int e = upk(m, k, k); U[2 * e] = ckr; U[2 * e + 1] = cki; }
    }
    lds_sync();
}

// z <- (H - theta I)^-1 z from the factors of hess_shift_factor_wave: the
// recorded swaps and multipliers in step order, then back substitution.
// Lane j keeps z_j in registers; each step broadcasts the entry it needs
// with v_readlane, and the back substitution accumulates the sums of the
// rows above column by column, so no step waits on a reduction.
__device__ void hess_shift_apply_wave(int m, const double* U, const double* fm, const int* swp, double* zr,
                                      double* zi) {
    const int lane = threadIdx.x;
    double vr = lane < m ? zr[lane] : 0.0, vi = lane < m ? zi[lane] : 0.0;
    for (int k = 0; k < m - 1; ++k) {
        const double akr = readlane_f64(vr, k), aki = readlane_f64(vi, k);
        const double bkr = readlane_f64(vr, k + 1), bki = readlane_f64(vi, k + 1);
        const bool sw = swp[k] != 0;
        const double zkr = sw ? bkr : akr, zki = sw ? bki : aki;      // z_k after the swap
        const double nkr = sw ? akr : bkr, nki = sw ? aki : bki;      // z_{k+1} after the swap
        const double fr = fm[2 * k], fi = fm[2 * k + 1];
        if (lane == k) { vr = zkr; vi = zki; }
        if (lane == k + 1) {
            vr = nkr - (fr * zkr - fi * zki);
            vi = nki - (fr * zki + fi * zkr);
        }
    }
    // back substitution: s_j accumulates sum_{t > j} U(j, t) z_t
    double sr = 0.0, si = 0.0;
    for (int i = m - 1; i >= 0; --i) {
        const int e = upk(m, i, i);
        const double ur = U[2 * e], ui = U[2 * e + 1];
        const double ar = readlane_f64(vr - sr, i), ai = readlane_f64(vi - si, i);
        const double rd = cz_recip(ur * ur + ui * ui);
        const double xr = (ar * ur + ai * ui) * rd, xi = (ai * ur - ar * ui) * rd;
        if (lane == i) { vr = xr; vi = xi; }
        if (lane < i) {
            const int f = upk(m, lane, i);
            const double wr = U[2 * f], wi = U[2 * f + 1];
            sr += wr * xr - wi * xi;
            si += wr * xi + wi * xr;
        }
    }
    lds_sync();
    if (lane < m) { zr[lane] = vr; zi[lane] = vi; }
    lds_sync();
}

// One wavefront: eigenvalues theta of H_m (the leading m x m block of the
// Hessenberg matrix stored column-major with leading dimension ld in Hh) and
// the selection of the `want` nonzero lam = 1/theta of smallest
// |lam| (largest |theta|; a conjugate pair counts as two and is never split,
// so one more at a split; among equal moduli the member with Im(lam) > 0
// first).  Outputs:
//   nsel_out[0] = selected entries, [1] = real columns they need, [2] = fail;
//   sel_lam[2e..2e+1] = lam of entry e (Im >= 0 member of a pair), and
//   sel_lam[HSEL_THETA + 2e..] = its theta (the member with Im <= 0), from
//   which hessenberg_vec_body finds the eigenvector.
#define HSEL_THETA 16
__device__ void hessenberg_select_body(int m, int ld, int want, const double* __restrict__ Hh,
                                       int* __restrict__ nsel_out, double* __restrict__ sel_lam) {
    __shared__ double A[HQR_MAXM * HQR_LD];
    __shared__ double wr[HQR_MAXM], wi[HQR_MAXM];
    __shared__ int used[HQR_MAXM];
    __shared__ int fail;
    const int lane = threadIdx.x;
    if (lane == 0) fail = 0;
    for (int i = 0; i < m; ++i)
        if (lane < m) A[i * HQR_LD + lane] = (i <= lane + 1) ? Hh[(size_t)lane * ld + i] : 0.0;
    if (lane < HQR_MAXM) used[lane] = 0;
    __threadfence_block();
    lds_sync();
    francis_eigvals_wave(m, A, wr, wi, &fail);
    lds_sync();
    int taken = 0, ne = 0, ncols = 0;
    while (taken < want && !fail && ne < HSEL_THETA / 2) {
        int best = -1;
        double bm = -1;
        for (int i = 0; i < m; ++i) {
            if (used[i]) continue;
            double mod = wr[i] * wr[i] + wi[i] * wi[i];
            if (best < 0 || mod > bm * (1 + 1e-12) || (mod >= bm * (1 - 1e-12) && wi[i] < wi[best])) { best = i; bm = mod; }
        }
        if (best < 0 || bm == 0.0) break;
        bool pair = wi[best] != 0.0;
        double thr = wr[best], thi = pair ? -fabs(wi[best]) : 0.0;
        int pj = -1;
        if (pair) {
            double bd = 1e300;
            for (int i = 0; i < m; ++i) {
                if (used[i] || i == best) continue;
                double d = (wr[i] - thr) * (wr[i] - thr) + (wi[i] + thi) * (wi[i] + thi);
                if (d < bd) { bd = d; pj = i; }
            }
        }
        lds_sync();
        if (lane == 0) { used[best] = 1; if (pj >= 0) used[pj] = 1; }
        const double den = thr * thr + thi * thi;
        if (lane == 0) {
            sel_lam[2 * ne] = thr / den;
            sel_lam[2 * ne + 1] = pair ? -thi / den : 0.0;
            sel_lam[HSEL_THETA + 2 * ne] = thr;
            sel_lam[HSEL_THETA + 2 * ne + 1] = thi;
        }
        ++ne;
        ncols += pair ? 2 : 1;
        taken += pair ? 2 : 1;
        lds_sync();
    }
    if (lane == 0) { nsel_out[0] = ne; nsel_out[1] = ncols; nsel_out[2] = fail; }
}

// One wavefront: the eigenvector of H_m (the leading m x m block, column-major
// with leading dimension ld in Hh) for the eigenvalue theta = (thr, thi), by
// three steps of inverse iteration
// with H - theta I from the start vector of ones, each normalised to
// ||z||_2 = 1; (re, im) pairs into out[2j..2j+1] (im = 0 for a real theta).
// A row-major copy of H_m stays in LDS for the elimination, which reads one
// row per step.
__device__ void hessenberg_vec_body(int m, int ld, const double* __restrict__ Hh, double thr, double thi,
                                    double* __restrict__ out) {
    __shared__ double U[HQR_MAXM * HQR_LD];
    __shared__ double Hs[HQR_MAXM * HQR_MAXM];
    __shared__ double zr[HQR_MAXM], zi[HQR_MAXM], fm[2 * HQR_MAXM];
    __shared__ int swp[HQR_MAXM];
    const int lane = threadIdx.x;
    double hn = 0;
    for (int i = 0; i < m; ++i) {
        double v = 0;
        if (lane < m) v = (i <= lane + 1) ? Hh[(size_t)lane * ld + i] : 0.0;
        if (lane < m) Hs[i * m + lane] = v;
        hn = fmax(hn, fabs(v));
    }
#pragma unroll
    for (int off = BAMG_WAVE / 2; off > 0; off >>= 1) hn = fmax(hn, __shfl_xor(hn, off, BAMG_WAVE));
    if (lane < m) { zr[lane] = 1.0; zi[lane] = 0.0; }
    __threadfence_block();
    lds_sync();
    hess_shift_factor_wave(m, Hs, thr, thi, U, fm, swp, hn);
    for (int itn = 0; itn < 3; ++itn) {
        hess_shift_apply_wave(m, U, fm, swp, zr, zi);
        double s = lane < m ? zr[lane] * zr[lane] + zi[lane] * zi[lane] : 0.0;
        s = wave_sum(s);
        s = __shfl(s, 0, BAMG_WAVE);
        const double nr = sqrt(s);
        lds_sync();
        if (lane < m) { zr[lane] /= nr; zi[lane] /= nr; }
        lds_sync();
    }
    if (lane < m) {
        out[2 * lane] = zr[lane];
        out[2 * lane + 1] = thi != 0.0 ? zi[lane] : 0.0;
    }
}

// One wavefront: the eigenvalue of the leading k x k block of a Hessenberg
// matrix H (column-major, leading dimension ld) closest to 0 and its
// eigenvector by three steps of inverse iteration with (H - theta I),
// normalised to ||eta||_2 = 1 with its largest-modulus entry (lowest index on
// ties) real and positive; the real part goes to eta[0..k-1].  A row-major
// copy of the block stays in LDS for the inverse iterations.  *fail = 1 when
// the QR iteration fails.
__device__ void hessenberg_near_zero_body(int k, const double* __restrict__ Hh, int ld, double* __restrict__ eta,
                                          int* __restrict__ fail_out) {
    __shared__ double A[HQR_MAXM * HQR_LD];
    __shared__ double Hs[HQR_MAXM * HQR_MAXM];
    __shared__ double wr[HQR_MAXM], wi[HQR_MAXM], zr[HQR_MAXM], zi[HQR_MAXM], fm[2 * HQR_MAXM];
    __shared__ int swp[HQR_MAXM];
    __shared__ int fail;
    const int lane = threadIdx.x;
    if (lane == 0) fail = 0;
    double hn = 0;
    for (int i = 0; i < k; ++i) {
        double v = 0;
        if (lane < k) v = (i <= lane + 1) ? Hh[(size_t)lane * ld + i] : 0.0;
        if (lane < k) { A[i * HQR_LD + lane] = v; Hs[i * k + lane] = v; }
        hn = fmax(hn, fabs(v));
    }
#pragma unroll
    for (int off = BAMG_WAVE / 2; off > 0; off >>= 1) hn = fmax(hn, __shfl_xor(hn, off, BAMG_WAVE));
    __threadfence_block();
    lds_sync();
    francis_eigvals_wave(k, A, wr, wi, &fail);
    lds_sync();
    int best = 0;
    double bm = wr[0] * wr[0] + wi[0] * wi[0];
    for (int i = 1; i < k; ++i) {
        const double mod = wr[i] * wr[i] + wi[i] * wi[i];
        if (mod < bm) { bm = mod; best = i; }
    }
    const double thr = wr[best], thi = wi[best];
    if (lane < k) { zr[lane] = 1.0; zi[lane] = 0.0; }
    lds_sync();
    hess_shift_factor_wave(k, Hs, thr, thi, A, fm, swp, hn);
    for (int itn = 0; itn < 3; ++itn) {
        hess_shift_apply_wave(k, A, fm, swp, zr, zi);
        double s = lane < k ? zr[lane] * zr[lane] + zi[lane] * zi[lane] : 0.0;
        s = wave_sum(s);
        s = __shfl(s, 0, BAMG_WAVE);
        const double nr = sqrt(s);
        lds_sync();
        if (lane < k) { zr[lane] /= nr; zi[lane] /= nr; }
        lds_sync();
    }
    // phase: the largest-modulus entry real and positive
    double bmod = -1;
    int bi = 0;
    for (int i = 0; i < k; ++i) {
        const double m2 = zr[i] * zr[i] + zi[i] * zi[i];
        if (m2 > bmod) { bmod = m2; bi = i; }
    }
    const double mr = zr[bi], mi = zi[bi], md = sqrt(mr * mr + mi * mi);
    if (lane < k) eta[lane] = (zr[lane] * mr + zi[lane] * mi) / md;
    if (lane == 0) *fail_out = fail;
}

// Ritz vector of entry e: v = Vb[:, 0:m] s_e (complex), into out_re / out_im.
__global__ void k_ritz(int n, int m, const double* __restrict__ Vb, const double* __restrict__ s,
                       double* __restrict__ out_re, double* __restrict__ out_im) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    double a = 0, b = 0;
    for (int j = 0; j < m; ++j) {
        double v = Vb[(size_t)j * n + i];
        a += v * s[2 * j]; b += v * s[2 * j + 1];
    }
    out_re[i] = a; out_im[i] = b;
}

// Normalise a (complex) coarsest eigenvector: ||v||_2 = 1 and the entry of
// largest re^2 + im^2 (lowest index on ties) real and positive.  One block.
// Writes the real part to column c of V (ld R) and, for a pair, the
// imaginary part to column c+1.
__global__ void k_eigvec_normalise(int n, const double* __restrict__ vr, const double* __restrict__ vi, int pair,
                                   double* __restrict__ V, int R, int c) {
    __shared__ double sh[BAMG_BLK];
    __shared__ int shi[BAMG_BLK];
    __shared__ double shs[BAMG_BLK / BAMG_WAVE];
    double s = 0, best = -1;
    int bi = 0;
    for (int i = threadIdx.x; i < n; i += BAMG_BLK) {
        double m2 = vr[i] * vr[i] + (pair ? vi[i] * vi[i] : 0.0);
        s += m2;
        if (m2 > best) { best = m2; bi = i; }
    }
    s = block_sum(s, shs);
    __syncthreads();
    sh[threadIdx.x] = best; shi[threadIdx.x] = bi;
    __syncthreads();
    for (int st = BAMG_BLK / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            double o = sh[threadIdx.x + st];
            int oi = shi[threadIdx.x + st];
            if (o > sh[threadIdx.x] || (o == sh[threadIdx.x] && oi < shi[threadIdx.x])) { sh[threadIdx.x] = o; shi[threadIdx.x] = oi; }
        }
        __syncthreads();
    }
    __shared__ double fac[2];
    if (threadIdx.x == 0) {
        int im = shi[0];
        double ar = vr[im], ai = pair ? vi[im] : 0.0;
        double mod = sqrt(ar * ar + ai * ai);
        double nrm = sqrt(s);
        // multiply by conj(v_m)/|v_m| / ||v||
        fac[0] = ar / mod / nrm; fac[1] = -ai / mod / nrm;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += BAMG_BLK) {
        double a = vr[i], b = pair ? vi[i] : 0.0;
        double nr = a * fac[0] - b * fac[1], ni = a * fac[1] + b * fac[0];
        V[(size_t)i * R + c] = nr;
        if (pair) V[(size_t)i * R + c + 1] = ni;
    }
}

// Column 0 of V: y / (c^T y).
__global__ void k_scale_into_col(int n, const double* __restrict__ y, const double* __restrict__ cy,
                                 double* __restrict__ V, int R, int c) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n) V[(size_t)i * R + c] = y[i] / *cy;
}

// Eigenvalue / column-kind tables of V from the selection (one thread).
__global__ void k_eig_tables(const int* __restrict__ nsel, const double* __restrict__ sel_lam,
                             double* __restrict__ lam, int* __restrict__ kind, int* __restrict__ ent_col) {
    if (threadIdx.x != 0) return;
    int ne = nsel[0];
    lam[0] = 0; lam[1] = 0; kind[0] = 0; ent_col[0] = 0;
    int c = 1;
    for (int e = 0; e < ne; ++e) {
        double lr = sel_lam[2 * e], li = sel_lam[2 * e + 1];
        ent_col[e + 1] = c;
        if (li != 0.0) {
            lam[2 * c] = lr; lam[2 * c + 1] = li; kind[c] = 1;
            lam[2 * c + 2] = lr; lam[2 * c + 3] = li; kind[c + 1] = 2;
            c += 2;
        } else {
            lam[2 * c] = lr; lam[2 * c + 1] = 0; kind[c] = 0;
            c += 1;
        }
    }
}
