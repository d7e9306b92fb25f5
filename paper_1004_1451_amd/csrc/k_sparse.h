// Sparse kernels of the Bootstrap AMG setup and cycle.
//
// Layouts (device):
//   B_l, T_l : CSR, int32 row_ptr / col (ascending), values of type M.
//   X (test vectors, eigenvector approximations): n x R row-major, R values of
//              one state contiguous ("interleaved").
//   P_l      : ELL-4, slot s of fine row i at 4i+s; -1 marks an empty slot;
//              used slots first, ascending coarse column.
//   Q_l      : ELL-9, slot s of coarse row I at 9I+s, fine columns ascending.
#pragma once
#include "common.h"
#include "k_sweep.h"

enum : int {
    ERR_RANGE = 1,      // column index out of range / not ascending / bad row_ptr
    ERR_NEG = 2,        // negative or non-finite entry
    ERR_WIDE = 4,       // entry joins states farther apart than the 3x3 box
    ERR_COLSUM = 8,     // |column sum - 1| > 1e-12
    ERR_ZERODIAG = 16,  // b_ii <= 0
    ERR_ELL = 32,       // a row of B_0 has more than 4 entries (no ELL-4 copy)
};

struct GridDev {
    int nx, ny, periodic;
    FastDiv dy;          // division by ny
};

// Signed offset a2 - a1 on a side of length m, wrapped into [-m/2, m/2] when
// periodic.
__device__ __forceinline__ int grid_delta(int a1, int a2, int m, int periodic) {
    int d = a2 - a1;
    if (periodic) {
        if (d > m / 2) d -= m;
        else if (d < -(m / 2)) d += m;
    }
    return d;
}

// ---------------------------------------------------------------- B = I - A
// Pass 1: validate row i of A and count the entries of row i of B (a missing
// diagonal is inserted).  Column sums accumulate with atomics: the check is a
// tolerance test, so the summation order does not matter.
__global__ void k_check_a(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                          const double* __restrict__ v, const ChainGeo* __restrict__ geo, int nch, int nnz,
                          double* __restrict__ colsum, int* __restrict__ cnt, int* __restrict__ err) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    int p0 = rp[i], p1 = rp[i + 1];
    int e = 0;
    if (p0 < 0 || p1 < p0 || p1 > nnz) { atomicOr(err, ERR_RANGE); cnt[i] = 1; return; }
    const ChainGeo g = geo[find_chain(geo, nch, i)];
    const int li = i - g.off;
    int ia = (int)g.dy.div((uint32_t)li), ib = li - ia * g.ny;
    bool has_diag = false;
    int prev = -1;
    for (int p = p0; p < p1; ++p) {
        int j = ci[p];
        double a = v[p];
        // columns stay inside the chain's own block (block-diagonal system)
        if (j < g.off || j >= g.off + g.n || j <= prev) { e |= ERR_RANGE; break; }
        prev = j;
        if (!(a >= 0.0) || !(a <= 1.0 + 1e-12)) e |= ERR_NEG;
        if (g.nx > 0) {          // nx = 0: a chain without a grid
            int lj = j - g.off;
            int ja = (int)g.dy.div((uint32_t)lj), jb = lj - ja * g.ny;
            int da = grid_delta(ia, ja, g.nx, g.periodic), db = grid_delta(ib, jb, g.ny, g.periodic);
            if (da < -1 || da > 1 || db < -1 || db > 1) e |= ERR_WIDE;
        }
        if (j == i) has_diag = true;
        atomicAdd(&colsum[j], a);
    }
    if (e) atomicOr(err, e);
    cnt[i] = (p1 - p0) + (has_diag ? 0 : 1);
}

// row_ptr alone: 0 <= rp[i] <= rp[i+1] <= nnz (checked before any kernel
// walks rows of a caller's CSR by index ranges).
__global__ void k_check_rp(int n, const int* __restrict__ rp, int nnz, int* __restrict__ err) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const int p0 = rp[i], p1 = rp[i + 1];
    if (p0 < 0 || p1 < p0 || p1 > nnz) atomicOr(err, ERR_RANGE);
}

__global__ void k_check_colsum(int n, const double* __restrict__ colsum, int* __restrict__ err) {
    int j = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (j >= n) return;
    if (!(fabs(colsum[j] - 1.0) <= 1e-12)) atomicOr(err, ERR_COLSUM);
}

// Pass 2: write row i of B = I - A and dinv_i = omega / b_ii.  With eci
// set, also the row's ELL-4 copy: the columns in eci, padded with (i, 0) as
// a CSR walk adds nothing for them, the FP64 values in ev64 and, with ev_lo
// set, their roundings to M; a row of more than 4 entries sets ERR_ELL
// instead (the copy is then not used).
template <typename M>
__global__ void k_build_b(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                          const double* __restrict__ v, const int* __restrict__ brp,
                          int* __restrict__ bci, double* __restrict__ bv, M* __restrict__ bv_lo,
                          double omega, double* __restrict__ dinv, M* __restrict__ dinv_lo,
                          int* __restrict__ eci, M* __restrict__ ev_lo, double* __restrict__ ev64,
                          int* __restrict__ err) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    int q = brp[i];
    bool done = false;
    double diag = 1.0;
    // the row's first four entries as written, for the ELL copy, in
    // registers (slot u takes the entry whose index is u)
    int ec[4] = {i, i, i, i};
    double evv[4] = {0.0, 0.0, 0.0, 0.0};
    int len = 0;
    // each entry written once, to the FP64 and (if asked) the low-precision
    // values together
    auto put = [&](int col, double val) {
        bci[q] = col;
        bv[q] = val;
        if (bv_lo) bv_lo[q] = (M)val;
        ++q;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (u == len) { ec[u] = col; evv[u] = val; }
        ++len;
    };
    const int p0 = rp[i], p1 = rp[i + 1];
    if (p1 - p0 <= 4) {
        // short rows: all loads of the row issued before the writes
        int jj[4];
        double vv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int pu = p0 + min(u, max(p1 - p0 - 1, 0));
            jj[u] = p1 > p0 ? ci[pu] : 0;
            vv[u] = p1 > p0 ? v[pu] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (u >= p1 - p0) break;
            const int j = jj[u];
            if (!done && j > i) { put(i, 1.0); done = true; }
            if (j == i) { diag = 1.0 - vv[u]; put(i, diag); done = true; }
            else put(j, -vv[u]);
        }
    } else {
        for (int p = p0; p < p1; ++p) {
            const int j = ci[p];
            if (!done && j > i) { put(i, 1.0); done = true; }
            if (j == i) { diag = 1.0 - v[p]; put(i, diag); done = true; }
            else put(j, -v[p]);
        }
    }
    if (!done) put(i, 1.0);
    if (!(diag > 0.0)) atomicOr(err, ERR_ZERODIAG);
    dinv[i] = omega / diag;
    if (dinv_lo) dinv_lo[i] = (M)(omega / diag);
    if (eci) {
        if (len > 4) {
            atomicOr(err, ERR_ELL);
        } else {
            *(int4*)(eci + (size_t)i * 4) = make_int4(ec[0], ec[1], ec[2], ec[3]);
            ((double2*)(ev64 + (size_t)i * 4))[0] = make_double2(evv[0], evv[1]);
            ((double2*)(ev64 + (size_t)i * 4))[1] = make_double2(evv[2], evv[3]);
            if (ev_lo) Ell4Val<M>::st(ev_lo + (size_t)i * 4, evv);
        }
    }
}

// dinv_i = omega / b_ii for a coarse operator (diagonal always stored, since
// every coarse row holds its own C point).
template <typename M>
__global__ void k_dinv(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                       const M* __restrict__ v, double omega, M* __restrict__ dinv, int* __restrict__ err) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    M d = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (ci[p] == i) d = v[p];
    if (!(d > (M)0)) atomicOr(err, ERR_ZERODIAG);
    dinv[i] = (M)(omega / (double)d);
}

// ---------------------------------------------------------------- scan
// Exclusive prefix sum of int32 counts in three passes (block sums, scan of
// the block sums in one block, add).  out has n+1 entries.
__global__ void k_scan_block(int n, const int* __restrict__ in, int* __restrict__ out, int* __restrict__ bsum) {
    __shared__ int sh[BAMG_BLK];
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    int v = i < n ? in[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < BAMG_BLK; off <<= 1) {
        int t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) out[i] = sh[threadIdx.x] - v;
    if (threadIdx.x == BAMG_BLK - 1) bsum[blockIdx.x] = sh[threadIdx.x];
}

// Exclusive scan of the nb block sums in place, total in *total (one
// block): thread t adds its contiguous chunk of ceil(nb / BAMG_BLK) sums,
// one block-wide scan of the chunk totals gives each chunk's offset, and the
// thread writes its chunk's prefixes (integers: the order of the additions
// does not matter).
__global__ void k_scan_sums(int nb, int* __restrict__ bsum, int* __restrict__ total) {
    __shared__ int sh[BAMG_BLK];
    const int t = threadIdx.x;
    const int per = (nb + BAMG_BLK - 1) / BAMG_BLK;
    const int lo = min(nb, t * per), hi = min(nb, lo + per);
    int own = 0;
    for (int i = lo; i < hi; ++i) own += bsum[i];
    sh[t] = own;
    __syncthreads();
    for (int off = 1; off < BAMG_BLK; off <<= 1) {
        const int v = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int run = sh[t] - own;
    for (int i = lo; i < hi; ++i) {
        const int v = bsum[i];
        bsum[i] = run;
        run += v;
    }
    if (t == BAMG_BLK - 1) *total = sh[t];
}

__global__ void k_scan_add(int n, int* __restrict__ out, const int* __restrict__ bsum, const int* __restrict__ total) {
    int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n) out[i] += bsum[blockIdx.x];
    if (i == 0) out[n] = *total;
}

// ---------------------------------------------------------------- relaxation

// sum_p v[p] * X[ci[p]*R + k] over one CSR row, in CSR order.  Index and
// value loads are issued four at a time before the dependent X loads, so a
// row costs two memory round trips instead of two per entry; padding slots
// add an exact zero, so the result equals the plain sequential sum.
// X_out = X_in + dinv (F - B X_in) on R interleaved columns (omega-Jacobi,
// Section 3).  One thread per (row, column); a wavefront covers 64/R rows and
// every stencil offset reads a contiguous run of X.  F == nullptr: homogeneous.
template <typename T, typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_sweep(int n, int R, FastDiv divR, const int* __restrict__ rp, const int* __restrict__ ci,
        const M* __restrict__ v, const M* __restrict__ dinv, const T* __restrict__ X,
        const T* __restrict__ F, T* __restrict__ Y, RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, R, n)) return;
    int t = tile * BAMG_BLK + threadIdx.x;
    if (t >= n * R) return;
    int i = (int)divR.div((uint32_t)t), k = t - i * R;
    const T xt = X[t];
    const T d = (T)dinv[i];
    const T f = F ? F[t] : (T)0;
    T acc = row_dot<T, M>(rp[i], rp[i + 1], ci, v, X, R, k, i);
    Y[t] = xt + d * (f - acc);
}

// First smoothing sweep from a zero guess: e = dinv * f.
template <typename T, typename M>
__global__ void k_jacobi_zero(int n, const M* __restrict__ dinv, const T* __restrict__ f, T* __restrict__ e,
                              RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, 1, n)) return;
    int i = tile * BAMG_BLK + threadIdx.x;
    if (i < n) e[i] = (T)dinv[i] * f[i];
}

// r = f - B e (single column).
template <typename T, typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_residual(int n, const int* __restrict__ rp, const int* __restrict__ ci, const M* __restrict__ v,
           const T* __restrict__ e, const T* __restrict__ f, T* __restrict__ r, RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, 1, n)) return;
    int i = tile * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const T fi = f ? f[i] : (T)0;
    T acc = row_dot<T, M>(rp[i], rp[i + 1], ci, v, e, 1, 0, i);
    r[i] = fi - acc;
}

// k_sweep (R = 1) and k_residual on the ELL-4 copy of B (see k_sweep_ve):
// one row per thread, the row's columns and values in one 16-byte load each,
// products added in CSR order with the same padding, so the results equal
// the CSR kernels' bit for bit.
template <typename T, typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_sweep_e(int n, const int* __restrict__ eci, const M* __restrict__ ev, const M* __restrict__ dinv,
          const T* __restrict__ X, const T* __restrict__ F, T* __restrict__ Y, RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, 1, n)) return;
    const int i = tile * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const int4 c4 = *(const int4*)(eci + (size_t)i * 4);
    M w[4];
    Ell4Val<M>::ld(ev + (size_t)i * 4, w);
    const T xt = X[i];
    const T d = (T)dinv[i];
    const T f = F ? F[i] : (T)0;
    const T x0 = X[c4.x], x1 = X[c4.y], x2 = X[c4.z], x3 = X[c4.w];
    T acc = 0;
    acc += (T)w[0] * x0;
    acc += (T)w[1] * x1;
    acc += (T)w[2] * x2;
    acc += (T)w[3] * x3;
    Y[i] = xt + d * (f - acc);
}

template <typename T, typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_residual_e(int n, const int* __restrict__ eci, const M* __restrict__ ev, const T* __restrict__ e,
             const T* __restrict__ f, T* __restrict__ r, RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, 1, n)) return;
    const int i = tile * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const int4 c4 = *(const int4*)(eci + (size_t)i * 4);
    M w[4];
    Ell4Val<M>::ld(ev + (size_t)i * 4, w);
    const T fi = f ? f[i] : (T)0;
    const T x0 = e[c4.x], x1 = e[c4.y], x2 = e[c4.z], x3 = e[c4.w];
    T acc = 0;
    acc += (T)w[0] * x0;
    acc += (T)w[1] * x1;
    acc += (T)w[2] * x2;
    acc += (T)w[3] * x3;
    r[i] = fi - acc;
}

// y = alpha * B x with FP64 vectors (values widened), used by the outer
// iteration and the coarsest eigensolve.
template <typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_spmv(int n, const int* __restrict__ rp, const int* __restrict__ ci, const M* __restrict__ v,
       const double* __restrict__ x, double alpha, double* __restrict__ y, RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, 1, n)) return;
    int i = tile * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    double acc = row_dot<double, M>(rp[i], rp[i + 1], ci, v, x, 1, 0, i);
    y[i] = alpha * acc;
}

// Coarse grid operators also live in a column-major ELL-9 form (entry k of
// row i at k ld + i, ld = the level's row count; the kernels below may run
// over a row prefix n; CSR order, padded with (i, 0)), which the Galerkin
// product writes directly: the one-row-per-thread cycle kernels load the 9
// columns and values of their rows with coalesced, independent loads.

// The multi-vector Jacobi sweep (k_sweep_v) on the column-major ELL-9 copy
// of a coarse grid level (slot k of row i at k * ld + i): one thread per
// (row, VW adjacent columns), the row's 9 columns and values read once, the
// neighbours' columns with vector loads.  Same order of the sums as the CSR
// kernel (the padding adds exact zeros there and here), so the same bits.
template <typename T, typename M, int VW, int BS>
__global__ void __launch_bounds__(BS)
k_sweep_v9(int n, int G, FastDiv divG, int ld, const int* __restrict__ cci, const M* __restrict__ cv,
           const M* __restrict__ dinv, const T* __restrict__ X, const T* __restrict__ F, T* __restrict__ Y) {
    const int t = xcd_tile(blockIdx.x, gridDim.x) * BS + threadIdx.x;
    if (t >= n * G) return;
    const int i = (int)divG.div((uint32_t)t), kg = t - i * G;
    const int R = G * VW;
    const size_t base = (size_t)i * R + (size_t)kg * VW;
    int c[9];
    M w[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) { c[k] = cci[(size_t)k * ld + i]; w[k] = cv[(size_t)k * ld + i]; }
    T xt[VW], f[VW], acc[VW];
    VecIO<T, VW>::ld(X + base, xt);
    if (F) VecIO<T, VW>::ld(F + base, f);
    else
#pragma unroll
        for (int q = 0; q < VW; ++q) f[q] = (T)0;
#pragma unroll
    for (int q = 0; q < VW; ++q) acc[q] = (T)0;
    const T d = (T)dinv[i];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        T x[VW];
        VecIO<T, VW>::ld(X + (size_t)c[k] * R + (size_t)kg * VW, x);
#pragma unroll
        for (int q = 0; q < VW; ++q) acc[q] += (T)w[k] * x[q];
    }
    T y[VW];
#pragma unroll
    for (int q = 0; q < VW; ++q) y[q] = xt[q] + d * (f[q] - acc[q]);
    VecIO<T, VW>::st(Y + base, y);
}

// sum_k v x over a row of the ELL-9 copy, k = 0..8 (the CSR order; the
// padding adds exact zeros, as the CSR kernels' padding does).
template <typename T, typename M>
__device__ __forceinline__ T row_dot9c(int ld, int i, const int* __restrict__ cci, const M* __restrict__ cv,
                                       const T* __restrict__ X) {
    int c[9];
    M w[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) { c[k] = cci[(size_t)k * ld + i]; w[k] = cv[(size_t)k * ld + i]; }
    T x[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) x[k] = X[c[k]];
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) acc += (T)w[k] * x[k];
    return acc;
}

template <typename T, typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_sweep_c9(int n, int ld, const int* __restrict__ cci, const M* __restrict__ cv, const M* __restrict__ dinv,
           const T* __restrict__ X, const T* __restrict__ F, T* __restrict__ Y, RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, 1, n)) return;
    const int i = tile * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const T xt = X[i];
    const T d = (T)dinv[i];
    const T f = F ? F[i] : (T)0;
    const T acc = row_dot9c<T, M>(ld, i, cci, cv, X);
    Y[i] = xt + d * (f - acc);
}

template <typename T, typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_residual_c9(int n, int ld, const int* __restrict__ cci, const M* __restrict__ cv, const T* __restrict__ e,
              const T* __restrict__ f, T* __restrict__ r, RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, 1, n)) return;
    const int i = tile * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const T fi = f ? f[i] : (T)0;
    r[i] = fi - row_dot9c<T, M>(ld, i, cci, cv, e);
}

// The first two smoothing sweeps of the cycle from a zero guess in one pass:
// e1 = D^-1 f (each e1_j formed as its own rounded product, as k_jacobi_zero
// stores it), then y = e1 + D^-1 (f - B e1), on the ELL-4 (row-major) or the
// ELL-9 (column-major, stride ld) copy.  Equal to k_jacobi_zero followed by
// k_sweep_e / k_sweep_c9 bit for bit, without writing and re-reading e1.
template <typename T, typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_sweep2z_e(int n, const int* __restrict__ eci, const M* __restrict__ ev, const M* __restrict__ dinv,
            const T* __restrict__ F, T* __restrict__ Y, RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, 1, n)) return;
    const int i = tile * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const int4 c4 = *(const int4*)(eci + (size_t)i * 4);
    M w[4];
    Ell4Val<M>::ld(ev + (size_t)i * 4, w);
    const int c[4] = {c4.x, c4.y, c4.z, c4.w};
    const T d = (T)dinv[i];
    const T f = F[i];
    T xt;
    {
#pragma clang fp contract(off)
        xt = d * f;              // a rounded product, as e1_i is stored
    }
    T x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = (T)dinv[c[u]] * F[c[u]];
    T acc = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += (T)w[u] * x[u];
    Y[i] = xt + d * (f - acc);
}

template <typename T, typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_sweep2z_c9(int n, int ld, const int* __restrict__ cci, const M* __restrict__ cv, const M* __restrict__ dinv,
             const T* __restrict__ F, T* __restrict__ Y, RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, 1, n)) return;
    const int i = tile * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    int c[9];
    M w[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) { c[k] = cci[(size_t)k * ld + i]; w[k] = cv[(size_t)k * ld + i]; }
    const T d = (T)dinv[i];
    const T f = F[i];
    T xt;
    {
#pragma clang fp contract(off)
        xt = d * f;              // a rounded product, as e1_i is stored
    }
    T x[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) x[k] = (T)dinv[c[k]] * F[c[k]];
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) acc += (T)w[k] * x[k];
    Y[i] = xt + d * (f - acc);
}

// dst[0] = src[0] (gathers scalars of several arrays for one read-back).
__global__ void k_copy_int(const int* __restrict__ src, int* __restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = src[0];
}

// k_spmv on the ELL-4 copy (see k_sweep_e): the same sums bit for bit.
template <typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_spmv_e(int n, const int* __restrict__ eci, const M* __restrict__ ev, const double* __restrict__ x, double alpha,
         double* __restrict__ y, RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, 1, n)) return;
    const int i = tile * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const int4 c4 = *(const int4*)(eci + (size_t)i * 4);
    M w[4];
    Ell4Val<M>::ld(ev + (size_t)i * 4, w);
    const double x0 = x[c4.x], x1 = x[c4.y], x2 = x[c4.z], x3 = x[c4.w];
    double acc = 0;
    acc += (double)w[0] * x0;
    acc += (double)w[1] * x1;
    acc += (double)w[2] * x2;
    acc += (double)w[3] * x3;
    y[i] = alpha * acc;
}

// f_c = Q r from the structure of Q alone: coarse row I takes the fine points
// of its 3x3 box whose bit is set in qmask[I], each with weight 1/|J_i|
// (jcnt), added in slot order.  Reads 2 bytes per coarse row and 1 per fine
// row instead of the 108-byte ELL row.
template <typename T>
__global__ void k_restrict_box(int nc, const ChainGeo* __restrict__ geoc, const ChainGeo* __restrict__ geof, int nch,
                               const unsigned short* __restrict__ qmask, const unsigned char* __restrict__ jcnt,
                               const T* __restrict__ r, T* __restrict__ fc, const int* __restrict__ act) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(RowMask{geoc, nch, act}, tile, BAMG_BLK, 1, nc)) return;
    int I = tile * BAMG_BLK + threadIdx.x;
    if (I >= nc) return;
    struct G2 { ChainGeo c, f; };
    const G2 gg = with_chain(geoc, nch, tile * BAMG_BLK, min(tile * BAMG_BLK + BAMG_BLK - 1, nc - 1), I,
                             [&](int c) { return G2{geoc[c], geof[c]}; });
    const ChainGeo& gc = gg.c;
    const ChainGeo& gf = gg.f;
    const int lI = I - gc.off;
    const int A = (int)gc.dy.div((uint32_t)lI), Bq = lI - A * gc.ny;
    const unsigned m = qmask[I];
    T acc = 0;
#pragma unroll
    for (int s = 0; s < 9; ++s) {
        if (!((m >> s) & 1)) continue;
        int na = grid_fine_pos(A, gf.nx, gf.periodic) + s / 3 - 1, nb = grid_fine_pos(Bq, gf.ny, gf.periodic) + s % 3 - 1;
        if (gf.periodic) {
            na = na < 0 ? na + gf.nx : (na >= gf.nx ? na - gf.nx : na);
            nb = nb < 0 ? nb + gf.ny : (nb >= gf.ny ? nb - gf.ny : nb);
        }
        const int i = gf.off + na * gf.ny + nb;
        acc += (T)(1.0 / (double)jcnt[i]) * r[i];
    }
    fc[I] = acc;
}

// e += P e_c (prolongation, ELL-4).
template <typename T, typename M>
__global__ void k_prolong_add(int n, const int* __restrict__ pc, const M* __restrict__ pv,
                              const T* __restrict__ ec, T* __restrict__ e, RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, 1, n)) return;
    int i = tile * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    // the row's 4 slots in one 16-byte load each; empty slots add nothing
    const int4 c4 = *(const int4*)(pc + (size_t)i * 4);
    const int J[4] = {c4.x, c4.y, c4.z, c4.w};
    M w[4];
    Ell4Val<M>::ld(pv + (size_t)i * 4, w);
    T x[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) x[s] = J[s] >= 0 ? ec[J[s]] : (T)0;
    T acc = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s)
        if (J[s] >= 0) acc += (T)w[s] * x[s];
    e[i] += acc;
}

// e_j + (P e_c)_j for row j, formed as k_prolong_add forms it.
template <typename T, typename M>
__device__ __forceinline__ T prolonged(int j, const int* __restrict__ pc, const M* __restrict__ pv,
                                       const T* __restrict__ ec, const T* __restrict__ e) {
    const int4 c4 = *(const int4*)(pc + (size_t)j * 4);
    const int J[4] = {c4.x, c4.y, c4.z, c4.w};
    M w[4];
    Ell4Val<M>::ld(pv + (size_t)j * 4, w);
    T x[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) x[s] = J[s] >= 0 ? ec[J[s]] : (T)0;
    T acc = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s)
        if (J[s] >= 0) acc += (T)w[s] * x[s];
    return e[j] + acc;
}

// The prolongation and the first post-smoothing sweep of the cycle in one
// pass on a coarse grid level (ELL-9 copy): Y = e' + D^-1 (f - B e') with
// e' = e + P e_c formed for the row and for each of its nine columns on the
// fly, so that e' is neither written nor read back.  The same bits as
// k_prolong_add followed by k_sweep_c9; e itself is left unchanged.
template <typename T, typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_prolong_sweep_c9(int n, int ld, const int* __restrict__ cci, const M* __restrict__ cv, const M* __restrict__ dinv,
                   const int* __restrict__ pc, const M* __restrict__ pv, const T* __restrict__ ec,
                   const T* __restrict__ e, const T* __restrict__ F, T* __restrict__ Y, RowMask mk) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (!tile_active(mk, tile, BAMG_BLK, 1, n)) return;
    const int i = tile * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    int c[9];
    M w[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) { c[k] = cci[(size_t)k * ld + i]; w[k] = cv[(size_t)k * ld + i]; }
    const T d = (T)dinv[i];
    const T f = F ? F[i] : (T)0;
    const T xt = prolonged<T, M>(i, pc, pv, ec, e);
    T x[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) x[k] = prolonged<T, M>(c[k], pc, pv, ec, e);
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) acc += (T)w[k] * x[k];
    Y[i] = xt + d * (f - acc);
}

// V_f = P V_c on R interleaved columns (interpolation of the eigenvector
// approximations, Algorithm 3).
template <typename T, typename M>
__global__ void k_interp(int n, int R, FastDiv divR, const int* __restrict__ pc, const M* __restrict__ pv,
                         const T* __restrict__ Vc, T* __restrict__ Vf) {
    int t = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK + threadIdx.x;
    if (t >= n * R) return;
    int i = (int)divR.div((uint32_t)t), k = t - i * R;
    T acc = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        int J = pc[(size_t)i * 4 + s];
        if (J >= 0) acc += (T)pv[(size_t)i * 4 + s] * Vc[(size_t)J * R + k];
    }
    Vf[t] = acc;
}

// The same product with one thread per row and all VP columns (VP a
// multiple of 4): P's row arrives in one 16-byte load for the columns and
// one or two for the values, each coarse row and the output row move in
// 16-byte pieces; the sums run over the slots in the same order.
template <typename T, typename M, int VP>
__global__ void k_interp_rows(int n, const int* __restrict__ pc, const M* __restrict__ pv,
                              const T* __restrict__ Vc, T* __restrict__ Vf) {
    static_assert(VP % 4 == 0, "row stride must be a multiple of 4");
    const int i = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const int4 c4 = *(const int4*)(pc + (size_t)i * 4);
    M w[4];
    Ell4Val<M>::ld(pv + (size_t)i * 4, w);
    const int J[4] = {c4.x, c4.y, c4.z, c4.w};
    T acc[VP];
#pragma unroll
    for (int k = 0; k < VP; ++k) acc[k] = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (J[s] < 0) continue;
        T x[VP];
#pragma unroll
        for (int k = 0; k < VP; k += 4) VecIO<T, 4>::ld(Vc + (size_t)J[s] * VP + k, x + k);
#pragma unroll
        for (int k = 0; k < VP; ++k) acc[k] += (T)w[s] * x[k];
    }
#pragma unroll
    for (int k = 0; k < VP; k += 4) VecIO<T, 4>::st(Vf + (size_t)i * VP + k, acc + k);
}

// Calls f(column, value) for the stored entries of row i in CSR order, from
// the storage EF names: EF_ELL4 the row-major 4-wide copy of the finest
// level (a row's columns and values move with one 16-byte load each),
// EF_ELL9 the column-major 9-wide copy of a coarse grid level (slot k of row
// i at k * eld + i), EF_CSR the CSR arrays.  An ELL copy's padding (i, 0) is
// visited too and adds nothing to a sum.
#define EF_CSR 0
#define EF_ELL4 4
#define EF_ELL9 9
template <int EF, typename M, typename F>
__device__ __forceinline__ void row_entries(int i, const int* __restrict__ rp, const int* __restrict__ ci,
                                            const M* __restrict__ v, const int* __restrict__ eci,
                                            const M* __restrict__ ev, int eld, F&& f) {
    if constexpr (EF == EF_ELL9) {
        int c[9];
        M w[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) { c[k] = eci[(size_t)k * eld + i]; w[k] = ev[(size_t)k * eld + i]; }
#pragma unroll
        for (int k = 0; k < 9; ++k) f(c[k], w[k]);
    } else if constexpr (EF == EF_ELL4) {
        const int4 c4 = *(const int4*)(eci + (size_t)i * 4);
        M w[4];
        Ell4Val<M>::ld(ev + (size_t)i * 4, w);
        f(c4.x, w[0]);
        f(c4.y, w[1]);
        f(c4.z, w[2]);
        f(c4.w, w[3]);
    } else {
        const int p1 = rp[i + 1];
        for (int p = rp[i]; p < p1; ++p) f(ci[p], v[p]);
    }
}

// The stored entries of an ELL row as arrays (K = 4 for ELL-4, 9 for
// ELL-9; 0: CSR, not handled here), in row_entries' order.
template <int EF>
struct RowK { static constexpr int K = EF == EF_ELL4 ? 4 : EF == EF_ELL9 ? 9 : 0; };
template <int EF, typename M, int K>
__device__ __forceinline__ void row_load(int i, const int* __restrict__ eci, const M* __restrict__ ev, int eld,
                                         int (&c)[K], M (&w)[K]) {
    if constexpr (EF == EF_ELL4) {
        const int4 c4 = *(const int4*)(eci + (size_t)i * 4);
        c[0] = c4.x; c[1] = c4.y; c[2] = c4.z; c[3] = c4.w;
        Ell4Val<M>::ld(ev + (size_t)i * 4, w);
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) { c[k] = eci[(size_t)k * eld + i]; w[k] = ev[(size_t)k * eld + i]; }
    }
}

// The columns only (for passes that need the pattern): f(column) for the
// entries row_entries visits, in the same order.
template <int EF, typename F>
__device__ __forceinline__ void row_cols(int i, const int* __restrict__ rp, const int* __restrict__ ci,
                                         const int* __restrict__ eci, int eld, F&& f) {
    if constexpr (EF == EF_ELL9) {
        int c[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) c[k] = eci[(size_t)k * eld + i];
#pragma unroll
        for (int k = 0; k < 9; ++k) f(c[k]);
    } else if constexpr (EF == EF_ELL4) {
        const int4 c4 = *(const int4*)(eci + (size_t)i * 4);
        f(c4.x);
        f(c4.y);
        f(c4.z);
        f(c4.w);
    } else {
        const int p1 = rp[i + 1];
        for (int p = rp[i]; p < p1; ++p) f(ci[p]);
    }
}

// ---------------------------------------------------------------- TV weights
// Stage 1, per chain (blockIdx.y) and row chunk of seg_rows (blockIdx.x):
// partial sums of (B x_k)_i^2 and (x_k)_i^2 for the chain's columns k of
// X = [U | V] (U: Ru columns, ld Ru; V: ld VS, a multiple of 4, unused when
// use_v == 0).  A thread takes VW adjacent columns of one row (VW divides Ru
// and VS; G groups per row, BAMG_BLK / G rows per pass), walks the row's
// entries once and moves its columns with one vector load per neighbour;
// then, per column, one thread adds the per-thread sums in row order.
// part[((c 2 WS) + k) P + chunk] = sum of (B x_k)^2, [.. + WS + k ..] = sum
// of x_k^2 (P = chunks per chain slot), for the chain's used columns only.
template <typename T, typename M, int VW, int EF>
__global__ void __launch_bounds__(BAMG_BLK)
k_colnorm_partial(const ChainGeo* __restrict__ geo, int seg_rows, int Ru, int use_v, const int* __restrict__ nvc,
                  int VS, const int* __restrict__ rp, const int* __restrict__ ci, const M* __restrict__ v,
                  const int* __restrict__ eci, const M* __restrict__ ev, int eld,
                  const T* __restrict__ U, const T* __restrict__ V, int WS, double* __restrict__ part) {
    __shared__ double sr[BAMG_BLK * VW], sx[BAMG_BLK * VW];
    const int c = blockIdx.y;
    const ChainGeo g = geo[c];
    const int GU = Ru / VW, G = GU + (use_v ? VS / VW : 0);
    const int r0 = g.off + blockIdx.x * seg_rows, r1 = min(g.off + g.n, r0 + seg_rows);
    if (r0 >= r1) return;                 // beyond this chain's own chunks
    const int t = threadIdx.x, rpp = BAMG_BLK / G, dr = t / G, kg = t - dr * G;
    const bool inU = kg < GU;
    const T* __restrict__ X = inU ? U : V;
    const int ld = inU ? Ru : VS, kx = (inU ? kg : kg - GU) * VW;
    double ar[VW], ax[VW];
#pragma unroll
    for (int q = 0; q < VW; ++q) { ar[q] = 0.0; ax[q] = 0.0; }
    if (dr < rpp) {
        if constexpr (EF == EF_ELL4) {
            // UR rows per round (i, i + rpp, ...): their entries, then every
            // neighbour's and their own values, all loads of a stage in
            // flight together; sums in the same row and entry order (on
            // ELL-9 rows this was measured slower than row by row)
            constexpr int K = RowK<EF>::K, UR = 4;
            for (int i = r0 + dr; i < r1; i += UR * rpp) {
                int cj[UR][K], ii[UR];
                M wj[UR][K];
#pragma unroll
                for (int u = 0; u < UR; ++u) {
                    ii[u] = i + u * rpp < r1 ? i + u * rpp : i;
                    row_load<EF, M, K>(ii[u], eci, ev, eld, cj[u], wj[u]);
                }
                T xj[UR][K][VW], xi[UR][VW];
#pragma unroll
                for (int u = 0; u < UR; ++u) {
#pragma unroll
                    for (int k = 0; k < K; ++k) VecIO<T, VW>::ld(X + (size_t)cj[u][k] * ld + kx, xj[u][k]);
                    VecIO<T, VW>::ld(X + (size_t)ii[u] * ld + kx, xi[u]);
                }
#pragma unroll
                for (int u = 0; u < UR; ++u) {
                    if (i + u * rpp >= r1) continue;
                    double acc[VW];
#pragma unroll
                    for (int q = 0; q < VW; ++q) acc[q] = 0.0;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const double b = (double)wj[u][k];
#pragma unroll
                        for (int q = 0; q < VW; ++q) acc[q] += b * (double)xj[u][k][q];
                    }
#pragma unroll
                    for (int q = 0; q < VW; ++q) {
                        ar[q] += acc[q] * acc[q];
                        ax[q] += (double)xi[u][q] * (double)xi[u][q];
                    }
                }
            }
        } else {
            for (int i = r0 + dr; i < r1; i += rpp) {
                double acc[VW];
#pragma unroll
                for (int q = 0; q < VW; ++q) acc[q] = 0.0;
                row_entries<EF, M>(i, rp, ci, v, eci, ev, eld, [&](int j, M bvj) {
                    const double b = (double)bvj;
                    T x[VW];
                    VecIO<T, VW>::ld(X + (size_t)j * ld + kx, x);
#pragma unroll
                    for (int q = 0; q < VW; ++q) acc[q] += b * (double)x[q];
                });
                T xi[VW];
                VecIO<T, VW>::ld(X + (size_t)i * ld + kx, xi);
#pragma unroll
                for (int q = 0; q < VW; ++q) {
                    ar[q] += acc[q] * acc[q];
                    ax[q] += (double)xi[q] * (double)xi[q];
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < VW; ++q) { sr[t * VW + q] = ar[q]; sx[t * VW + q] = ax[q]; }
    __syncthreads();
    if (t < G * VW) {
        const int kgt = t / VW, q = t - kgt * VW;
        double a = 0, b = 0;
        for (int d2 = 0; d2 < rpp; ++d2) {
            a += sr[(d2 * G + kgt) * VW + q];
            b += sx[(d2 * G + kgt) * VW + q];
        }
        const int k = kgt < GU ? t : Ru + (t - GU * VW);
        const int Rc = Ru + (use_v ? nvc[c] : 0);
        if (k < Rc) {
            part[((size_t)c * 2 * WS + k) * gridDim.x + blockIdx.x] = a;
            part[((size_t)c * 2 * WS + WS + k) * gridDim.x + blockIdx.x] = b;
        }
    }
}

// Stage 2: block (column k, chain c) adds the chunk partials in order;
// w_k = 1 / max(||B x_k||^2, (1e-14 ||x_k||)^2) (Section 3.2).
__global__ void k_colnorm_final(const ChainGeo* __restrict__ geo, int seg_rows, int P, int Ru, int use_v,
                                const int* __restrict__ nvc, int WS, const double* __restrict__ part,
                                double* __restrict__ w) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    const int c = blockIdx.y, k = blockIdx.x;
    const int R = Ru + (use_v ? nvc[c] : 0);
    if (k >= R) return;
    const int nchunks = (geo[c].n + seg_rows - 1) / seg_rows;
    const double* pa = part + ((size_t)c * 2 * WS + k) * P;
    const double* pb = part + ((size_t)c * 2 * WS + WS + k) * P;
    double a = 0, b = 0;
    for (int j = threadIdx.x; j < nchunks; j += BAMG_BLK) {
        a += pa[j];
        b += pb[j];
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
        double den = a > 1e-28 * b ? a : 1e-28 * b;
        w[(size_t)c * WS + k] = 1.0 / den;
    }
}

// ---------------------------------------------------------------- LS fit
// Masked Cholesky of the 4x4 Gram G on the slot set S (bit mask), slot order.
// Fills lower factor L (entries outside S untouched / zero), the reciprocals
// il of its diagonal, z = L^-1 b on S and the determinant product, and
// returns false if a pivot is not positive.  Divisions by a pivot are
// products with its reciprocal (v_rcp_f64 refined by two Newton steps).
__device__ __forceinline__ bool chol4(const double G[4][4], const double b[4], int S, double L[4][4],
                                      double il[4], double z[4], double& det) {
    det = 1.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) L[i][j] = 0.0;
        z[i] = 0.0;
        il[i] = 0.0;
    }
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!((S >> j) & 1)) continue;
        double d = G[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        if (!(d > 0.0)) { ok = false; d = 1.0; }
        det *= d;
        const double lj = sqrt(d), r = cz_recip(lj);
        L[j][j] = lj;
        il[j] = r;
        double zz = b[j];
#pragma unroll
        for (int k = 0; k < j; ++k) zz -= L[j][k] * z[k];
        z[j] = zz * r;
#pragma unroll
        for (int i = j + 1; i < 4; ++i) {
            if (!((S >> i) & 1)) continue;
            double s = G[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            L[i][j] = s * r;
        }
    }
    return ok;
}

// Least-squares interpolation, Algorithm 2 with the functional of eq.
// LSfuncrowi, one thread per fine point of level l.  X = [U | V]
// (Ru + Rv columns), weights w (device, R).  C point (a, b even): unit row at
// its coarse index, and with inject != nullptr its U row is copied to the
// coarse test vectors (injection, Algorithm 3).  F point: slots N_i = coarse
// points within Chebyshev distance 1, in lexicographic order of (da, db);
// G_st = sum_k w_k x_s^k x_t^k, b_s = sum_k w_k x_s^k x_i^k, sigma; greedy:
// add the admissible candidate with the smallest sigma - b_S^T G_SS^-1 b_S
// (strict minimum, ties to the lower slot) until |J| >= caliber; a candidate
// g is admissible when det(G_{J+g}) / det(G_J) > 1e-10 G_gg (its Schur
// complement pivot).  Gram and solves in FP64 whatever the storage type.
struct LsPoint {
    double G[4][4], b[4], sigma;
    double p[4];          // fitted weights in slot order (zero outside J)
    double Lls;           // the functional at the fit
    int sf[4], sc[4];     // fine / coarse index of each slot
    int valid, J;         // slot masks: non-empty, selected
};

// Weighted Gram G (lower triangle), right-hand side b and sigma of an F point
// over its first NS slots (the others contribute zero), test vectors in the
// order k = 0 .. R-1 (U columns, then V).
template <typename T, int NS>
__device__ __forceinline__ void ls_gram(int i, LsPoint& P, int valid, int Ru, int Rv, int VS, const T* __restrict__ U,
                                        const T* __restrict__ V, const double* __restrict__ w, double& sigma) {
    for (int part = 0; part < 2; ++part) {
        const T* Xp = part == 0 ? U : V;
        const int ld = part == 0 ? Ru : VS;
        const int nk = part == 0 ? Ru : Rv;
        const double* wp = w + (part == 0 ? 0 : Ru);
        auto accumulate = [&](double wk, double xi, const double (&xs)[NS]) {
            sigma += wk * xi * xi;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                double ws = wk * xs[s];
                P.b[s] += ws * xi;
#pragma unroll
                for (int t = 0; t <= s; ++t) P.G[s][t] += ws * xs[t];
            }
        };
        if (ld % 4 == 0) {
            // four columns per 16-byte load (rows are 4-aligned), CH columns
            // of the point's and its slots' rows loaded together before their
            // sums; same order.  Eight columns keep the kernel within 168
            // registers (three wavefronts per SIMD; twelve needed 196, two)
            constexpr int CH = 8;
            for (int k0 = 0; k0 < nk; k0 += CH) {
                T xi[CH], xs4[NS][CH];
                double wk[CH];
#pragma unroll
                for (int q = 0; q < CH; ++q) wk[q] = k0 + q < nk ? wp[k0 + q] : 0.0;
                // every slot's row is loaded (an empty slot points at the
                // point's own row, and columns past nk at the row's first
                // four) and masked afterwards, so that no load waits behind a
                // branch
#pragma unroll
                for (int q4 = 0; q4 < CH; q4 += 4) {
                    const int kc = k0 + q4 < nk ? k0 + q4 : 0;
                    T t4[4];
                    VecIO<T, 4>::ld(Xp + (size_t)i * ld + kc, t4);
#pragma unroll
                    for (int q = 0; q < 4; ++q) xi[q4 + q] = t4[q];
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        VecIO<T, 4>::ld(Xp + (size_t)P.sf[s] * ld + kc, t4);
#pragma unroll
                        for (int q = 0; q < 4; ++q) xs4[s][q4 + q] = t4[q];
                    }
                }
                __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the sums
#pragma unroll
                for (int q = 0; q < CH; ++q) {
                    if (k0 + q < nk) {
                        double xs[NS];
#pragma unroll
                        for (int s = 0; s < NS; ++s) xs[s] = ((valid >> s) & 1) ? (double)xs4[s][q] : 0.0;
                        accumulate(wk[q], (double)xi[q], xs);
                    }
                }
            }
        } else {
#pragma unroll 2
            for (int kk = 0; kk < nk; ++kk) {
                double xs[NS];
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const double v = (double)Xp[(size_t)P.sf[s] * ld + kk];
                    xs[s] = ((valid >> s) & 1) ? v : 0.0;
                }
                accumulate(wp[kk], (double)Xp[(size_t)i * ld + kk], xs);
            }
        }
    }
}

template <typename T>
__device__ __forceinline__ void ls_point(int i, const ChainGeo& g, int ia, int ib, int Ru, int Rv, int VS,
                                         const T* __restrict__ U, const T* __restrict__ V,
                                         const double* __restrict__ w, int caliber, LsPoint& P) {
    const int ncy = g.ncy;
    int ns = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) { P.sf[s] = i; P.sc[s] = -1; }
    // per direction: a coarse position takes offset 0 only, a fine one -1
    // and +1 (both coarse); the slots are the product, lexicographic in
    // (da, db), without (0, 0)
    const bool ca = grid_cpos(ia, g.nx, g.periodic), cb = grid_cpos(ib, g.ny, g.periodic);
#pragma unroll
    for (int da = -1; da <= 1; ++da)
#pragma unroll
        for (int db = -1; db <= 1; ++db) {
            if (da == 0 && db == 0) continue;
            if ((da == 0) != ca || (db == 0) != cb) continue;
            int na = ia + da, nb = ib + db;
            if (g.periodic) {
                na = na < 0 ? na + g.nx : (na >= g.nx ? na - g.nx : na);
                nb = nb < 0 ? nb + g.ny : (nb >= g.ny ? nb - g.ny : nb);
            } else if (na < 0 || na >= g.nx || nb < 0 || nb >= g.ny) {
                continue;
            }
            // at most 4 coarse points; ns < 4 always holds here
#pragma unroll
            for (int s = 0; s < 4; ++s)
                if (s == ns) {
                    P.sf[s] = g.off + na * g.ny + nb;
                    P.sc[s] = g.coff + ((na + 1) >> 1) * ncy + ((nb + 1) >> 1);
                }
            ++ns;
        }
    const int valid = (1 << ns) - 1;
    P.valid = valid;
    // weighted Gram, right-hand side and sigma over all test vectors
    double sigma = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        P.b[s] = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) P.G[s][t] = 0;
    }
    // U columns, then V columns (test vectors in a fixed order k = 0..R-1);
    // points with at most two slots (slots 0 and 1) take a narrower copy of
    // the same sums (the others' entries stay zero, as they would be)
    if (ns <= 2) ls_gram<T, 2>(i, P, valid, Ru, Rv, VS, U, V, w, sigma);
    else ls_gram<T, 4>(i, P, valid, Ru, Rv, VS, U, V, w, sigma);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = s + 1; t < 4; ++t) P.G[s][t] = P.G[t][s];
    P.sigma = sigma;
    // greedy selection (Algorithm 2).  When every slot stays admissible
    // whatever else is selected, the selection is all slots: the pivot a
    // candidate g gets after J, s(g | J), is at least s(g | all other slots)
    // = 1 / (G^-1)_gg.  That case is decided from one Cholesky of the full
    // set with a factor 100 over the admissibility bound, so rounding cannot
    // pass a slot the greedy steps would reject; the slots are a prefix.
    int J = 0, nsel = 0;
    double L[4][4], il[4], z[4], detJ = 1.0;
    bool all = ns > 0 && ns <= caliber;
    if (all) {
        double det;
        all = chol4(P.G, P.b, valid, L, il, z, det);
        double W[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            W[j][j] = j < ns ? il[j] : 0.0;
#pragma unroll
            for (int i = j + 1; i < 4; ++i) {
                double t = 0.0;
#pragma unroll
                for (int k = j; k < i; ++k) t += L[i][k] * W[k][j];
                W[i][j] = i < ns ? -t * il[i] : 0.0;
            }
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            if (g >= ns) continue;
            double gi = 0.0;
#pragma unroll
            for (int k = g; k < 4; ++k) gi += W[k][g] * W[k][g];
            // the pivot 1 / gi of slot g against all the others must pass
            // 100 times the admissibility bound
            all = all && (1.0 > 1e-8 * P.G[g][g] * gi);
        }
    }
    if (all) { J = valid; nsel = ns; }
    bool fresh = all;        // L, il, z hold the factor of G_JJ
#pragma unroll
    for (int step = 0; step < 4; ++step) {
        if (all || nsel >= caliber) break;
        int best = -1;
        double bestL = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (!((valid >> c) & 1) || ((J >> c) & 1)) continue;
            int S = J | (1 << c);
            double det;
            fresh = false;
            bool ok = chol4(P.G, P.b, S, L, il, z, det);
            if (!ok || !(det > 1e-10 * P.G[c][c] * detJ)) continue;
            double Lv = sigma;
#pragma unroll
            for (int s = 0; s < 4; ++s) Lv -= z[s] * z[s];
            if (best < 0 || Lv < bestL) { best = c; bestL = Lv; }
        }
        if (best < 0) break;
        J |= 1 << best;
        ++nsel;
        double det;
        chol4(P.G, P.b, J, L, il, z, det);
        detJ = det;
        fresh = true;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) P.p[s] = 0.0;
    if (J == 0) {
        J = 1;
        P.p[0] = 1.0;
        P.Lls = sigma - 2.0 * P.b[0] + P.G[0][0];
    } else {
        // the factor of G_JJ is still in L, il, z unless candidates were
        // tried after the last selection
        if (!fresh) {
            double det;
            chol4(P.G, P.b, J, L, il, z, det);
        }
        double Lv = sigma;
#pragma unroll
        for (int s = 0; s < 4; ++s) Lv -= z[s] * z[s];
        P.Lls = Lv;
        // back substitution L^T p = z on J
#pragma unroll
        for (int j = 3; j >= 0; --j) {
            if (!((J >> j) & 1)) continue;
            double s = z[j];
#pragma unroll
            for (int k = j + 1; k < 4; ++k) s -= L[k][j] * P.p[k];
            P.p[j] = s * il[j];
        }
    }
    P.J = J;
}

// Row i of P from weights p on the slots in mask J, in ascending coarse column;
// returns the number of entries.  The row is assembled in registers and
// stored as one 16-byte column vector and one value vector.
template <typename MP>
__device__ __forceinline__ int write_prow(int i, int J, const int sc[4], const double p[4], int* __restrict__ pc,
                                          MP* __restrict__ pv) {
    int cnt = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) cnt += (J >> s) & 1;
    int col[4] = {-1, -1, -1, -1};
    MP val[4] = {(MP)0, (MP)0, (MP)0, (MP)0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (!((J >> s) & 1)) continue;
        int rank = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (((J >> t) & 1) && (sc[t] < sc[s])) ++rank;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q == rank) { col[q] = sc[s]; val[q] = (MP)p[s]; }
    }
    *(int4*)(pc + (size_t)i * 4) = make_int4(col[0], col[1], col[2], col[3]);
    VecIO<MP, 4>::st(pv + (size_t)i * 4, val);
    return cnt;
}

// The 24 scale-free features of an F point (learned form):
//   [valid slot mask (4) | -b_ij / b_ii at the 8 neighbour offsets in
//    lexicographic (da, db) order (8) | b_s / G_ss (4) |
//    b_s / sqrt(sigma G_ss) (4) | sqrt(G_ss / sigma) (4)], zero for empty slots.
template <typename M>
__device__ __forceinline__ void point_features(const LsPoint& P, int i, const ChainGeo& g, int ia, int ib,
                                               const int* __restrict__ rp, const int* __restrict__ ci,
                                               const M* __restrict__ bv, float f[24]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) f[s] = ((P.valid >> s) & 1) ? 1.0f : 0.0f;
    double st[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) st[k] = 0.0;
    double diag = 1.0;
    const int p0 = rp[i], p1 = rp[i + 1];
    for (int p = p0; p < p1; ++p)
        if (ci[p] == i) diag = (double)bv[p];
    for (int p = p0; p < p1; ++p) {
        const int j = ci[p];
        if (j == i) continue;
        const int lj = j - g.off;
        const int ja = (int)g.dy.div((uint32_t)lj), jb = lj - ja * g.ny;
        const int da = grid_delta(ia, ja, g.nx, g.periodic), db = grid_delta(ib, jb, g.ny, g.periodic);
        int k = (da + 1) * 3 + (db + 1);
        k = k > 4 ? k - 1 : k;
        const double val = -(double)bv[p] / diag;
#pragma unroll
        for (int t = 0; t < 8; ++t) st[t] += (t == k) ? val : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) f[4 + k] = (float)st[k];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const double Gss = P.G[s][s];
        const bool ok = ((P.valid >> s) & 1) && Gss > 0.0 && P.sigma > 0.0;
        f[12 + s] = ok ? (float)(P.b[s] / Gss) : 0.0f;
        f[16 + s] = ok ? (float)(P.b[s] / sqrt(P.sigma * Gss)) : 0.0f;
        f[20 + s] = ok ? (float)sqrt(Gss / P.sigma) : 0.0f;
    }
}

// jcnt (optional): |J_i| per fine point, for the restriction of the cycle.
// feat_out (optional, n x 24 FP32): the features of every F point (zero rows
// for C points); slotw_out (optional, n x 4 FP32): the fitted weights in slot
// order.  Both only serve to collect training data for the learned form.
template <typename T, typename MP, typename M>
__global__ void __launch_bounds__(BAMG_BLK)
k_ls_fit(int n, const ChainGeo* __restrict__ geo, int nch, int Ru, int use_v, const int* __restrict__ nvc,
         int VS, const T* __restrict__ U, const T* __restrict__ V, const double* __restrict__ wall, int WS,
         int caliber, int* __restrict__ pc, MP* __restrict__ pv, T* __restrict__ inject,
         unsigned char* __restrict__ jcnt, const int* __restrict__ brp, const int* __restrict__ bci,
         const M* __restrict__ bv, float* __restrict__ feat_out, float* __restrict__ slotw_out) {
    const int b0 = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK, t = b0 + threadIdx.x;
    if (t >= n) return;
    const ChainGeo g = with_chain(geo, nch, b0, min(b0 + BAMG_BLK - 1, n - 1), t, [&](int c) { return geo[c]; });
    // Thread t takes a point of its own grid row: the fine columns first,
    // then the coarse ones, so a wavefront's lanes mostly take the same
    // branch (rows with C points: F points, then C points; the other rows:
    // F points with four slots, then those with two).
    const int lt = t - g.off;
    const int ia = (int)g.dy.div((uint32_t)lt), kk = lt - ia * g.ny;
    const bool rowc = grid_cpos(ia, g.nx, g.periodic);
    const int nf = grid_fine_count(g.ny, g.periodic);
    const int ib = kk < nf ? 2 * kk + 1 : grid_fine_pos(kk - nf, g.ny, g.periodic);
    const int li = ia * g.ny + ib;
    const int i = g.off + li;
    if (rowc && grid_cpos(ib, g.ny, g.periodic)) {
        int I = g.coff + ((ia + 1) >> 1) * g.ncy + ((ib + 1) >> 1);
        *(int4*)(pc + (size_t)i * 4) = make_int4(I, -1, -1, -1);
        const MP one[4] = {(MP)1, (MP)0, (MP)0, (MP)0};
        VecIO<MP, 4>::st(pv + (size_t)i * 4, one);
        if (inject) {
            if (Ru % 4 == 0) {
                for (int k = 0; k < Ru; k += 4) {
                    T x4[4];
                    VecIO<T, 4>::ld(U + (size_t)i * Ru + k, x4);
                    VecIO<T, 4>::st(inject + (size_t)I * Ru + k, x4);
                }
            } else {
                for (int k = 0; k < Ru; ++k) inject[(size_t)I * Ru + k] = U[(size_t)i * Ru + k];
            }
        }
        if (jcnt) jcnt[i] = 1;
        if (feat_out)
            for (int k = 0; k < 24; ++k) feat_out[(size_t)i * 24 + k] = 0.0f;
        if (slotw_out)
            for (int k = 0; k < 4; ++k) slotw_out[(size_t)i * 4 + k] = 0.0f;
        return;
    }
    LsPoint P;
    // the chain's weights as workgroup-uniform loads where the rows allow
    with_chain(geo, nch, b0, min(b0 + BAMG_BLK - 1, n - 1), t, [&](int c) {
        ls_point<T>(i, g, ia, ib, Ru, use_v ? nvc[c] : 0, VS, U, V, wall + (size_t)c * WS, caliber, P);
        return 0;
    });
    const int cnt = write_prow<MP>(i, P.J, P.sc, P.p, pc, pv);
    if (jcnt) jcnt[i] = (unsigned char)cnt;
    if (feat_out) {
        float f[24];
        point_features<M>(P, i, g, ia, ib, brp, bci, bv, f);
        for (int k = 0; k < 24; ++k) feat_out[(size_t)i * 24 + k] = f[k];
    }
    if (slotw_out)
        for (int k = 0; k < 4; ++k) slotw_out[(size_t)i * 4 + k] = (float)P.p[k];
}

// ---------------------------------------------------------------- Q
// Averaging restriction (Section 4): Q[I, i] = 1/|J_i| for every fine i with
// I in J_i.  Such i lie in the 3x3 fine box around I's fine position; they
// are written in ascending fine index (ELL-9, for the Galerkin products), and
// qmask[I] marks which box slots (da, db) = (s / 3 - 1, s % 3 - 1) they are.
template <typename MQ>
__global__ void k_build_q(int nc, const ChainGeo* __restrict__ geoc, const ChainGeo* __restrict__ geof, int nch,
                          const int* __restrict__ pc, int* __restrict__ qc, MQ* __restrict__ qv,
                          unsigned short* __restrict__ qmask) {
    const int b0 = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK;
    int I = b0 + threadIdx.x;
    if (I >= nc) return;
    struct G2 { ChainGeo c, f; };
    const G2 gg = with_chain(geoc, nch, b0, min(b0 + BAMG_BLK - 1, nc - 1), I,
                             [&](int c) { return G2{geoc[c], geof[c]}; });
    const ChainGeo& gc = gg.c;
    const ChainGeo& g = gg.f;
    const int lI = I - gc.off;
    int A = (int)gc.dy.div((uint32_t)lI), Bq = lI - A * gc.ny;
    int fa = grid_fine_pos(A, g.nx, g.periodic), fb = grid_fine_pos(Bq, g.ny, g.periodic);
    // the 3x3 fine box around I's fine position (empty entries: -1), then
    // every box point's P columns as one 16-byte load each (an empty entry
    // reloads the centre), all in flight together
    int fb9[9];
#pragma unroll
    for (int s = 0; s < 9; ++s) {
        int da = s / 3 - 1, db = s % 3 - 1;
        int na = fa + da, nb = fb + db;
        fb9[s] = -1;
        if (g.periodic) {
            na = na < 0 ? na + g.nx : (na >= g.nx ? na - g.nx : na);
            nb = nb < 0 ? nb + g.ny : (nb >= g.ny ? nb - g.ny : nb);
        } else if (na < 0 || na >= g.nx || nb < 0 || nb >= g.ny) {
            continue;
        }
        fb9[s] = g.off + na * g.ny + nb;
    }
    int4 jc[9];
#pragma unroll
    for (int s = 0; s < 9; ++s) jc[s] = *(const int4*)(pc + (size_t)(fb9[s] >= 0 ? fb9[s] : fb9[4]) * 4);
    int fi[9];
    double fv[9];
#pragma unroll
    for (int s = 0; s < 9; ++s) {
        fi[s] = -1; fv[s] = 0.0;
        if (fb9[s] < 0) continue;
        const int Js[4] = {jc[s].x, jc[s].y, jc[s].z, jc[s].w};
        int c = 0;
        bool hit = false;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int J = Js[t];
            c += J >= 0;
            hit |= J == I;
        }
        if (hit) { fi[s] = fb9[s]; fv[s] = 1.0 / c; }
    }
    int cnt = 0;
#pragma unroll
    for (int s = 0; s < 9; ++s) cnt += fi[s] >= 0;
#pragma unroll
    for (int s = 0; s < 9; ++s) {
        if (fi[s] < 0) continue;
        int rank = 0;
#pragma unroll
        for (int t = 0; t < 9; ++t) rank += (fi[t] >= 0) && (fi[t] < fi[s]);
        qc[(size_t)I * 9 + rank] = fi[s];
        qv[(size_t)I * 9 + rank] = (MQ)fv[s];
    }
    for (int s = cnt; s < 9; ++s) { qc[(size_t)I * 9 + s] = -1; qv[(size_t)I * 9 + s] = (MQ)0; }
    unsigned m = 0;
#pragma unroll
    for (int s = 0; s < 9; ++s) m |= (fi[s] >= 0 ? 1u : 0u) << s;
    qmask[I] = (unsigned short)m;
}

// ---------------------------------------------------------------- Galerkin
// Slot (0..8) of coarse column J in the 3x3 coarse box around coarse row I.
__device__ __forceinline__ int box_slot(int I_a, int I_b, int J, const FastDiv& dcy, int ncx, int ncy, int periodic) {
    // J: coarse column relative to the chain's first coarse row
    int Ja = (int)dcy.div((uint32_t)J), Jb = J - Ja * ncy;
    int da = grid_delta(I_a, Ja, ncx, periodic), db = grid_delta(I_b, Jb, ncy, periodic);
    return (da + 1) * 3 + (db + 1);
}

// The Galerkin passes give each coarse row I nine threads, one per slot s of
// Q row I (fine point i = qc[9I + s]); a block holds GAL_ROWS coarse rows.
#define GAL_ROWS 28
#define GAL_THREADS (9 * GAL_ROWS)

// Contribution of Q slot s of coarse row I: the box slots reached through
// i = qc[9I+s] (mask) and, with vals, tmp[u] = sum_j m_ij p_jJ (M-row order,
// then P-row order) for J in box slot u.  Row i of M comes from the storage
// EF names (row_entries; mrp null: M = I).  An ELL copy's padding (i, 0)
// adds zeros and reaches the slots of P row i, which the stored diagonal
// of M reaches anyway.
template <typename MV, bool VALS, int EF>
__device__ __forceinline__ unsigned gal_slot(int coff, int Ia, int Ib, int i, const FastDiv& dcy, int ncx, int ncy,
                                             int periodic, const int* __restrict__ mrp, const int* __restrict__ mci,
                                             const MV* __restrict__ mv, const int* __restrict__ eci,
                                             const MV* __restrict__ ev, int eld, const int* __restrict__ pc,
                                             const MV* __restrict__ pv, MV* tmp) {
    unsigned mask = 0;
    // P row j: its columns and values as two 16-byte loads
    auto load_p = [&](int j, int (&Js)[4], MV (&ps)[4]) {
        const int4 jc = *(const int4*)(pc + (size_t)j * 4);
        Js[0] = jc.x; Js[1] = jc.y; Js[2] = jc.z; Js[3] = jc.w;
        if (VALS) VecIO<MV, 4>::ld(pv + (size_t)j * 4, ps);
    };
    // without wrap-around (and ncy >= 3) the box slot of coarse column J
    // follows from J - (I - ncy - 1) = (da + 1) ncy + (db + 1), da, db in
    // {-1, 0, 1}
    const int sbase = coff + Ia * ncy + Ib - ncy - 1;
    const bool general = periodic || ncy < 3;
    auto apply = [&](MV mraw, const int (&Js)[4], const MV (&ps)[4]) {
        const MV m = VALS ? mraw : (MV)1;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (Js[t] < 0) continue;
            int sl;
            if (general) {
                sl = box_slot(Ia, Ib, Js[t] - coff, dcy, ncx, ncy, periodic);
            } else {
                const int q = Js[t] - sbase;
                const int dap = (q >= ncy ? 1 : 0) + (q >= 2 * ncy ? 1 : 0);
                sl = dap * 3 + (q - dap * ncy);
            }
            mask |= 1u << sl;
            if (VALS) {
                MV c = m * ps[t];
#pragma unroll
                for (int u = 0; u < 9; ++u) tmp[u] += (u == sl) ? c : (MV)0;
            }
        }
    };
    if (!mrp) {
        int Js[4];
        MV ps[4];
        load_p(i, Js, ps);
        apply((MV)1, Js, ps);
    } else if constexpr (EF == EF_ELL4) {
        // the row's four entries, then their P rows, all loads of a stage in
        // flight together, then the sums in entry order (on ELL-9 rows the
        // nine P rows at once were measured slower than one after another)
        constexpr int K = 4;
        int c[K];
        MV w[K];
        const int4 c4 = *(const int4*)(eci + (size_t)i * 4);
        c[0] = c4.x; c[1] = c4.y; c[2] = c4.z; c[3] = c4.w;
        if (VALS) Ell4Val<MV>::ld(ev + (size_t)i * 4, w);
        int Js[K][4];
        MV ps[K][4];
#pragma unroll
        for (int k = 0; k < K; ++k) load_p(c[k], Js[k], ps[k]);
#pragma unroll
        for (int k = 0; k < K; ++k) apply(VALS ? w[k] : (MV)1, Js[k], ps[k]);
    } else {
        auto entry = [&](int j, MV mraw) {
            int Js[4];
            MV ps[4];
            load_p(j, Js, ps);
            apply(mraw, Js, ps);
        };
        if constexpr (VALS) row_entries<EF, MV>(i, mrp, mci, mv, eci, ev, eld, entry);
        else row_cols<EF>(i, mrp, mci, eci, eld, [&](int j) { entry(j, (MV)1); });
    }
    return mask;
}

// The output stage of the Galerkin kernels (all threads of the block call
// it): thread (lr, s) of coarse row I (valid when I < nc) brings its
// slot sums tb / tt and box masks mb / mt; the nine threads of a row add the
// sums per box slot in order s = 0..8 through LDS (sv, sm) and thread u writes
// box slot u at its rank among the row's structural slots into the
// column-major ELL-9 arrays of each product, the free slots padded with
// (I, 0); *cnt[I] = structural slots of the row.
template <typename MV>
__device__ __forceinline__ void gal_write(int I, int nc, int lr, int s, int Ia, int Ib, int ncx, int ncy, int periodic,
                                          int goff, const MV (&tb)[9], const MV (&tt)[9], unsigned mb, unsigned mt,
                                          MV (*sv)[9], unsigned* sm, int* __restrict__ bcc, MV* __restrict__ bcv,
                                          int* __restrict__ bcnt, int* __restrict__ tcc, MV* __restrict__ tcv,
                                          int* __restrict__ tcnt) {
    // the row's coarse columns of the nine box slots
    int col[9];
#pragma unroll
    for (int w = 0; w < 9; ++w) {
        int a = Ia + w / 3 - 1, b = Ib + w % 3 - 1;
        if (periodic) {
            a = a < 0 ? a + ncx : (a >= ncx ? a - ncx : a);
            b = b < 0 ? b + ncy : (b >= ncy ? b - ncy : b);
        }
        col[w] = goff + a * ncy + b;
    }
    for (int prod = 0; prod < 2; ++prod) {
        if (prod) __syncthreads();
#pragma unroll
        for (int u = 0; u < 9; ++u) sv[threadIdx.x][u] = prod ? tt[u] : tb[u];
        sm[threadIdx.x] = prod ? mt : mb;
        __syncthreads();
        if (I < nc) {
            int* cc = prod ? tcc : bcc;
            MV* cv = prod ? tcv : bcv;
            unsigned mask = 0;
            for (int t = 0; t < 9; ++t) mask |= sm[lr * 9 + t];
            const int u = s;
            const int cnt = __popc(mask);
            if ((mask >> u) & 1) {
                MV acc = 0;
                for (int t = 0; t < 9; ++t) acc += sv[lr * 9 + t][u];
                int rank = 0;
#pragma unroll
                for (int t = 0; t < 9; ++t) rank += ((mask >> t) & 1) && (col[t] < col[u]);
                cc[(size_t)rank * nc + I] = col[u];
                cv[(size_t)rank * nc + I] = acc;
            }
            if (u >= cnt) { cc[(size_t)u * nc + I] = I; cv[(size_t)u * nc + I] = (MV)0; }
            if (u == 0) (prod ? tcnt : bcnt)[I] = cnt;
        }
    }
}

// Both products of a grid level in one pass: B_{l+1} = Q (B_l P) and
// T_{l+1} = Q (T_l P) (Algorithm 3), nine threads per coarse row I (GR rows
// per block, a launch shape the autotuner picks), thread (I, s) taking slot s
// of Q row I (fine point
// i = qc[9I + s]) for both products, so Q and P are read once.  B_l's rows
// come from the storage EFB names, T_l's from EFT (EFT < 0: T_l = I).  The
// sums are those of the separate numeric pass: q_Is (sum_j m_ij p_jJ) in
// row-entry and then P-slot order, the nine slots added in order s = 0..8.
// The pattern is the symbolic one (the box slots reached by any product of
// stored entries, structural zeros kept).  Thread u writes box slot u of row
// I at its rank among the row's structural slots (ascending column) into the
// column-major ELL-9 arrays of each product (slot k of row I at k nc + I),
// the free slots padded with (I, 0); *cnt[I] = structural slots of the row.
template <typename MV, int EFB, int EFT, int GR = GAL_ROWS>
__global__ void __launch_bounds__(9 * GR)
k_galerkin_bt(int nc, const ChainGeo* __restrict__ geoc, int nch, const int* __restrict__ qc,
              const MV* __restrict__ qv, const int* __restrict__ brp, const int* __restrict__ bci,
              const MV* __restrict__ bv, const int* __restrict__ beci, const MV* __restrict__ bev, int beld,
              const int* __restrict__ trp, const int* __restrict__ tci, const MV* __restrict__ tv,
              const int* __restrict__ teci, const MV* __restrict__ tev, int teld, const int* __restrict__ pc,
              const MV* __restrict__ pv, int* __restrict__ bcc, MV* __restrict__ bcv, int* __restrict__ bcnt,
              int* __restrict__ tcc, MV* __restrict__ tcv, int* __restrict__ tcnt) {
    __shared__ MV sv[9 * GR][9];
    __shared__ unsigned sm[9 * GR];
    const int lr = threadIdx.x / 9, s = threadIdx.x % 9;
    const int I = xcd_tile(blockIdx.x, gridDim.x) * GR + lr;
    MV tb[9], tt[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) { tb[u] = 0; tt[u] = 0; }
    unsigned mb = 0, mt = 0;
    int Ia = 0, Ib = 0, ncx = 1, ncy = 1, periodic = 0, goff = 0;
    const int b0 = xcd_tile(blockIdx.x, gridDim.x) * GR;
    const ChainGeo g = with_chain(geoc, nch, b0, min(b0 + GR - 1, nc - 1), min(I, nc - 1),
                                  [&](int c) { return geoc[c]; });
    if (I < nc) {
        ncx = g.nx; ncy = g.ny; periodic = g.periodic; goff = g.off;
        const int lI = I - g.off;
        Ia = (int)g.dy.div((uint32_t)lI); Ib = lI - Ia * ncy;
        const int i = qc[(size_t)I * 9 + s];
        if (i >= 0) {
            const MV q = qv[(size_t)I * 9 + s];
            mb = gal_slot<MV, true, EFB>(g.off, Ia, Ib, i, g.dy, ncx, ncy, periodic, brp, bci, bv, beci, bev, beld,
                                         pc, pv, tb);
            if constexpr (EFT < 0)
                mt = gal_slot<MV, true, EF_CSR>(g.off, Ia, Ib, i, g.dy, ncx, ncy, periodic, (const int*)nullptr,
                                                (const int*)nullptr, (const MV*)nullptr, (const int*)nullptr,
                                                (const MV*)nullptr, 0, pc, pv, tt);
            else
                mt = gal_slot<MV, true, EFT>(g.off, Ia, Ib, i, g.dy, ncx, ncy, periodic, trp, tci, tv, teci, tev,
                                             teld, pc, pv, tt);
#pragma unroll
            for (int u = 0; u < 9; ++u) { tb[u] = q * tb[u]; tt[u] = q * tt[u]; }
        }
    }
    gal_write<MV>(I, nc, lr, s, Ia, Ib, ncx, ncy, periodic, goff, tb, tt, mb, mt, sv, sm, bcc, bcv, bcnt, tcc, tcv,
                  tcnt);
}

// CSR rows of both products from their ELL-9 copies (blockIdx.y: 0 = B,
// 1 = T): row I's first rp[I + 1] - rp[I] slots, in order.  A workgroup
// takes BAMG_BLK consecutive rows: it reads their nine slots column by
// column (coalesced) into LDS, then writes the rows' contiguous CSR range
// entry by entry (coalesced), each entry finding its row by binary search
// over the rows' pointers in LDS.
template <typename MV>
__global__ void __launch_bounds__(BAMG_BLK)
k_ell9c_to_csr2(int nc, const int* __restrict__ bcc, const MV* __restrict__ bcv, const int* __restrict__ brp,
                int* __restrict__ bci, MV* __restrict__ bv, const int* __restrict__ tcc, const MV* __restrict__ tcv,
                const int* __restrict__ trp, int* __restrict__ tci, MV* __restrict__ tv) {
    __shared__ int sc[9][BAMG_BLK];
    __shared__ MV sv[9][BAMG_BLK];
    __shared__ int sp[BAMG_BLK + 1];
    const bool tt = blockIdx.y == 1;
    const int* cc = tt ? tcc : bcc;
    const MV* cv = tt ? tcv : bcv;
    const int* rp = tt ? trp : brp;
    int* ci = tt ? tci : bci;
    MV* v = tt ? tv : bv;
    const int I0 = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK;
    const int rows = min(BAMG_BLK, nc - I0);
    const int t = threadIdx.x;
    if (t < rows) {
#pragma unroll
        for (int k = 0; k < 9; ++k) { sc[k][t] = cc[(size_t)k * nc + I0 + t]; sv[k][t] = cv[(size_t)k * nc + I0 + t]; }
    }
    if (t < rows) sp[t] = rp[I0 + t];
    if (t == 0) sp[rows] = rp[I0 + rows];
    __syncthreads();
    const int base = sp[0], len = sp[rows] - base;
    for (int e = t; e < len; e += BAMG_BLK) {
        const int pe = base + e;
        int lo = 0, hi = rows - 1;          // the row r with sp[r] <= pe < sp[r + 1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sp[mid] <= pe) lo = mid; else hi = mid - 1;
        }
        const int k = pe - sp[lo];
        ci[pe] = sc[k][lo];
        v[pe] = sv[k][lo];
    }
}

// ---------------------------------------------------------------- up-leg
// One omega-Jacobi sweep on (B - lam_c T) x_c = 0 for every column c of the
// eigenvector block V (row stride VP, a multiple of 4), one thread per row
// with all VP columns: every stored entry of the row is read once and its
// neighbour's VP values are moved with 16-byte loads; the chain's first nvc
// columns are relaxed and the others copied.  kind[c]: 0 real column with
// real lam, 1 / 2 real / imaginary part of a complex pair x = V_c + i V_{c+1}
// (lam complex; both columns of a pair form (B - lam T) x, each keeps its own
// part); D_lam = diag(B) - lam diag(T).  T == identity when trp and teci
// are null; T's rows come from the storage EFT names (its ELL-9 copy on the
// coarse grid levels).  Column 0 (the null-vector approximation) has lam = 0.
// Products are added in CSR order in FP64 (an ELL copy adds its padding
// (i, 0) as zeros).  colour >= 0: one colour of a multicolour Gauss-Seidel
// sweep (k_mcgs.h), in place (Y == X), other rows untouched.  Row i of
// chain ch here; k_eig_relax below is the launch.
template <typename T, typename M, int VP, int EF, int EFT>
__device__ __forceinline__ void eig_relax_row(int i, int ch, const ChainGeo* __restrict__ geo,
                                              const int* __restrict__ nvc, int KV, const int* __restrict__ brp,
                                              const int* __restrict__ bci, const M* __restrict__ bv,
                                              const int* __restrict__ beci, const M* __restrict__ bev, int beld,
                                              const int* __restrict__ trp, const int* __restrict__ tci,
                                              const M* __restrict__ tv, const int* __restrict__ teci,
                                              const M* __restrict__ tev, int teld, const double* __restrict__ lamall,
                                              const int* __restrict__ kindall, double omega, int colour, const T* X,
                                              T* Y) {
    if (colour >= 0 && point_colour(geo[ch], i - geo[ch].off) != colour) return;
    const int nv = nvc[ch];
    auto load = [&](int row, T (&x)[VP]) {
#pragma unroll
        for (int k = 0; k < VP; k += 4) VecIO<T, 4>::ld(X + (size_t)row * VP + k, x + k);
    };
    double bs[VP], ts[VP];
#pragma unroll
    for (int c = 0; c < VP; ++c) { bs[c] = 0.0; ts[c] = 0.0; }
    double bd = 0, td = (trp || teci) ? 0.0 : 1.0;
    row_entries<EF, M>(i, brp, bci, bv, beci, bev, beld, [&](int j, M bvj) {
        const double b = (double)bvj;
        if (j == i && b != 0.0) bd = b;        // not the ELL padding (i, 0)
        T x[VP];
        load(j, x);
#pragma unroll
        for (int c = 0; c < VP; ++c) bs[c] += b * (double)x[c];
    });
    T xo[VP];
    load(i, xo);
    if (trp || teci) {
        row_entries<EFT, M>(i, trp, tci, tv, teci, tev, teld, [&](int j, M tvj) {
            const double t = (double)tvj;
            if (j == i && t != 0.0) td = t;    // not an ELL padding (i, 0)
            T x[VP];
            load(j, x);
#pragma unroll
            for (int c = 0; c < VP; ++c) ts[c] += t * (double)x[c];
        });
    } else {
#pragma unroll
        for (int c = 0; c < VP; ++c) ts[c] = (double)xo[c];
    }
    const int* kind = kindall + (size_t)ch * KV;
    const double* lam = lamall + (size_t)ch * 2 * KV;
    T out[VP];
#pragma unroll
    for (int c = 0; c < VP; ++c) {
        out[c] = xo[c];
        if (c >= nv) continue;
        const int k = kind[c];
        const double lr = lam[2 * c], li = lam[2 * c + 1];
        if (k == 0) {
            out[c] = (T)((double)xo[c] - omega * (bs[c] - lr * ts[c]) / (bd - lr * td));
        } else {
            // the pair's real and imaginary columns ca, ca + 1
            const double b0 = k == 2 ? (c > 0 ? bs[c - 1] : 0.0) : bs[c];
            const double b1 = k == 2 ? bs[c] : (c + 1 < VP ? bs[c + 1] : 0.0);
            const double t0 = k == 2 ? (c > 0 ? ts[c - 1] : 0.0) : ts[c];
            const double t1 = k == 2 ? ts[c] : (c + 1 < VP ? ts[c + 1] : 0.0);
            // r = (B - lam T) x, D = bd - lam td, correction r / D; the
            // fused multiply-adds are written out and no other contraction is
            // allowed, so that every instantiation (every storage form of B
            // and T) rounds the same way
            double q;
            {
#pragma clang fp contract(off)
                const double rr = fma(li, t1, fma(-lr, t0, b0));
                const double ri = fma(-li, t0, fma(-lr, t1, b1));
                const double dr = fma(-lr, td, bd), di = -li * td;
                const double den = fma(dr, dr, di * di);
                q = k == 1 ? fma(rr, dr, ri * di) / den : fma(ri, dr, -(rr * di)) / den;
            }
            out[c] = (T)((double)xo[c] - omega * q);
        }
    }
    T* y = Y + (size_t)i * VP;
#pragma unroll
    for (int k = 0; k < VP; k += 4) VecIO<T, 4>::st(y + k, out + k);
}

// One thread per row; a workgroup whose rows lie in one chain passes the
// chain as a workgroup-uniform value, so its kinds and eigenvalues are
// scalar loads.
template <typename T, typename M, int VP, int EF, int EFT = EF_CSR>
__global__ void __launch_bounds__(BAMG_BLK)
k_eig_relax(int n, const ChainGeo* __restrict__ geo, int nch, const int* __restrict__ nvc, int KV,
            const int* __restrict__ brp, const int* __restrict__ bci, const M* __restrict__ bv,
            const int* __restrict__ beci, const M* __restrict__ bev, int beld,
            const int* __restrict__ trp, const int* __restrict__ tci, const M* __restrict__ tv,
            const int* __restrict__ teci, const M* __restrict__ tev, int teld,
            const double* __restrict__ lamall, const int* __restrict__ kindall, double omega, int colour,
            const T* X, T* Y) {
    static_assert(VP % 4 == 0, "row stride must be a multiple of 4");
    const int b0 = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK;
    const int i = b0 + threadIdx.x;
    if (i >= n) return;
    const int cf = find_chain(geo, nch, b0), cl = nch == 1 ? cf : find_chain(geo, nch, min(b0 + BAMG_BLK - 1, n - 1));
    if (cf == cl)                                // the whole workgroup in one chain
        eig_relax_row<T, M, VP, EF, EFT>(i, __builtin_amdgcn_readfirstlane(cf), geo, nvc, KV, brp, bci, bv, beci, bev,
                                         beld, trp, tci, tv, teci, tev, teld, lamall, kindall, omega, colour, X, Y);
    else
        eig_relax_row<T, M, VP, EF, EFT>(i, find_chain(geo, nch, i), geo, nvc, KV, brp, bci, bv, beci, bev, beld,
                                         trp, tci, tv, teci, tev, teld, lamall, kindall, omega, colour, X, Y);
}

// Rayleigh quotient partials, per chain (blockIdx.y) and row chunk of
// seg_rows (blockIdx.x): for entry e (first column ent_col[e]; a pair uses
// two) the sums x^H B x and x^H T x (re, im).  Thread layout: nent slots per
// row (thread t: row t / nent, entry t % nent), then one thread per entry adds
// the per-thread sums in thread order -> part[chain][chunk][entry][4].  T's
// rows come from the storage EFT names (identity when trp and teci are null).
template <typename T, typename M, int EF, int EFT = EF_CSR>
__global__ void __launch_bounds__(BAMG_BLK)
k_rayleigh_partial(const ChainGeo* __restrict__ geo, int R, int KV, const int* __restrict__ nentc,
                   const int* __restrict__ ent_colall, const int* __restrict__ kindall,
                   const int* __restrict__ brp, const int* __restrict__ bci, const M* __restrict__ bv,
                   const int* __restrict__ beci, const M* __restrict__ bev, int beld,
                   const int* __restrict__ trp, const int* __restrict__ tci, const M* __restrict__ tv,
                   const int* __restrict__ teci, const M* __restrict__ tev, int teld,
                   const T* __restrict__ X, int seg_rows, double* __restrict__ part) {
    __shared__ double sh[4][BAMG_BLK];
    const int chn = blockIdx.y;
    const ChainGeo g = geo[chn];
    const int nent = nentc[chn];
    const int r0 = g.off + blockIdx.x * seg_rows, r1 = min(g.off + g.n, r0 + seg_rows);
    if (r0 >= r1) return;
    const int t = threadIdx.x, rpp = BAMG_BLK / nent, dr = t / nent, e = t - dr * nent;
    const int c = ent_colall[(size_t)chn * KV + e];
    const bool pair = kindall[(size_t)chn * KV + c] == 1;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    if (dr < rpp) {
        for (int i = r0 + dr; i < r1; i += rpp) {
            const double xr = (double)X[(size_t)i * R + c], xi = pair ? (double)X[(size_t)i * R + c + 1] : 0.0;
            double br = 0, bi = 0, tr = 0, ti = 0;
            row_entries<EF, M>(i, brp, bci, bv, beci, bev, beld, [&](int j, M bvj) {
                const double b = (double)bvj;
                br += b * (double)X[(size_t)j * R + c];
                if (pair) bi += b * (double)X[(size_t)j * R + c + 1];
            });
            if (trp || teci) {
                row_entries<EFT, M>(i, trp, tci, tv, teci, tev, teld, [&](int j, M tvj) {
                    const double tq = (double)tvj;
                    tr += tq * (double)X[(size_t)j * R + c];
                    if (pair) ti += tq * (double)X[(size_t)j * R + c + 1];
                });
            } else {
                tr = xr; ti = xi;
            }
            // conj(x) * y = (xr - i xi)(yr + i yi), the fused multiply-adds
            // written out (the same roundings in every instantiation)
            {
#pragma clang fp contract(off)
                s0 += fma(xr, br, xi * bi); s1 += fma(xr, bi, -(xi * br));
                s2 += fma(xr, tr, xi * ti); s3 += fma(xr, ti, -(xi * tr));
            }
        }
    }
    sh[0][t] = s0; sh[1][t] = s1; sh[2][t] = s2; sh[3][t] = s3;
    __syncthreads();
    if (t < nent) {
        double a[4] = {0, 0, 0, 0};
        for (int q = t; q < rpp * nent; q += nent)
            for (int z = 0; z < 4; ++z) a[z] += sh[z][q];
        double* o = part + (((size_t)chn * gridDim.x + blockIdx.x) * KV + t) * 4;
        for (int z = 0; z < 4; ++z) o[z] = a[z];
    }
}

// lam_e = (x^H B x) / (x^H T x) for every entry except the null vector
// (entry 0 keeps lam = 0); real columns keep a real lam.  Block (e, chain).
__global__ void k_rayleigh_final(const ChainGeo* __restrict__ geo, int seg_rows, int P, int KV,
                                 const int* __restrict__ nentc, const int* __restrict__ ent_colall,
                                 const int* __restrict__ kindall, const double* __restrict__ part,
                                 double* __restrict__ lamall) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    const int e = blockIdx.x, chn = blockIdx.y;
    if (e >= nentc[chn] || e == 0) return;
    const int nchunks = (geo[chn].n + seg_rows - 1) / seg_rows;
    double s[4] = {0, 0, 0, 0};
    for (int j = threadIdx.x; j < nchunks; j += BAMG_BLK)
        for (int q = 0; q < 4; ++q) s[q] += part[(((size_t)chn * P + j) * KV + e) * 4 + q];
    for (int q = 0; q < 4; ++q) s[q] = block_sum(s[q], sh);
    if (threadIdx.x == 0) {
        const int* ent_col = ent_colall + (size_t)chn * KV;
        const int* kind = kindall + (size_t)chn * KV;
        double* lam = lamall + (size_t)chn * 2 * KV;
        int c = ent_col[e];
        double den = s[2] * s[2] + s[3] * s[3];
        double lr = (s[0] * s[2] + s[1] * s[3]) / den, li = (s[1] * s[2] - s[0] * s[3]) / den;
        if (kind[c] == 0) li = 0.0;
        lam[2 * c] = lr; lam[2 * c + 1] = li;
        if (kind[c] == 1) { lam[2 * c + 2] = lr; lam[2 * c + 3] = li; }
    }
}

// ---------------------------------------------------------------- casts
template <typename A, typename B>
__global__ void k_cast(long long n, const A* __restrict__ a, B* __restrict__ b) {
    long long i = (long long)blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i < n) b[i] = (B)a[i];
}

// Initial test vectors: entry (i, k) of a chain's block is u(seed, stream 1,
// i_local * r + k), the same numbers a single-chain setup draws.
template <typename T>
__global__ void k_tv_init(long long total, int r, FastDiv divr, const ChainGeo* __restrict__ geo, int nch,
                          uint64_t seed, T* __restrict__ U) {
    long long t = (long long)blockIdx.x * BAMG_BLK + threadIdx.x;
    if (t >= total) return;
    int i = (int)divr.div((uint32_t)t), k = (int)(t - (long long)i * r);
    const ChainGeo g = geo[find_chain(geo, nch, i)];
    U[t] = (T)splitmix_u01(seed, 1ull, (uint64_t)(i - g.off) * r + k);
}
