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

// ---------------------------------------------------------------------------
// Arnoldi orthogonalisation of the flexible GMRES: classical Gram-Schmidt with
// one reorthogonalisation, the second pass delayed into the next step so that
// every Arnoldi step reads the basis twice (one pass of dots, one of updates).
// At step j the basis holds q_0 .. q_{j-1} (finished) and v_j (one pass of
// Gram-Schmidt, norm only estimated).  The dots pass takes w = B z_j; the
// update pass finishes q_j = (v_j - sum a_b q_b) / alpha and writes the next
// provisional vector v_{j+1} = (w - sum d_b q_b - h q_j) / nu, whose dots with
// q_0 .. q_j and itself it also returns.  In flexible GMRES z_j may be any
// vector, so preconditioning v_j before it is finished only changes the search
// direction, and the Arnoldi relation B z_{j-1} = Q h + nu v_j becomes exact
// once column j-1 is corrected with v_j = Q a + alpha q_j.
//
// Both passes return, for nb finished vectors, nb + 2 dots per chain:
//   d < nb: <q_d, x>,  d = nb: <y, x>,  d = nb + 1: <x, x>
// (dots pass: x = w, y = v_nb; update pass: x = v_{nb+1}, y = q_nb), as one
// value per chunk of seg_rows rows in part[((c NDM) + d) P + chunk].
#define GS_MAXB 64
#define GS_CS (2 * GS_MAXB + 4)

// Dots pass: <q_b, w> (b < nb), <v_nb, w>, <w, w> on a chunk of one chain.
// K >= nb accumulators per thread (1, 2, 4 or a multiple of 8); grid
// (chunks, chains).  V_b starts at V + b ldv.  Every thread issues all K
// loads of a row unconditionally (b >= nb re-reads v_nb, a cache hit) so that
// they are in flight together; the sums b >= nb are never stored.  With
// K <= 4 a thread loads GsRows<K>::U of its rows (i, i + BAMG_BLK, ...) before
// the products, which it adds in row order as one row at a time would.
template <int K>
struct GsRows { static constexpr int U = K <= 2 ? 4 : K <= 4 ? 2 : 1; };

//
// SPMV: w is not read but formed here as w = alpha B z from the ELL-4 copy of
// B_0 (eci, ev; the sums of k_spmv_e in its order, so the same bits) and
// stored to wout for the update pass: the outer product and the dots pass in
// one launch.
template <int K, bool SPMV = false>
__global__ void __launch_bounds__(BAMG_BLK)
k_gs_dots(const ChainGeo* __restrict__ geo, int seg_rows, int ldv, int nb, const int* __restrict__ act,
          const double* __restrict__ V, const double* __restrict__ w, double* __restrict__ part, int NDM,
          const int* __restrict__ eci, const double* __restrict__ ev, const double* __restrict__ z, double alpha,
          double* __restrict__ wout) {
    __shared__ double red[(BAMG_BLK / BAMG_WAVE) * (GsRed<K>::KR + 2)];
    constexpr int U = GsRows<K>::U;
    const ChainGeo g = geo[blockIdx.y];
    if (!act[blockIdx.y]) return;
    const int i0 = g.off + blockIdx.x * seg_rows, i1 = min(g.off + g.n, i0 + seg_rows);
    if (i0 >= i1) return;
    const double* y = V + (size_t)nb * ldv;
    double acc[K];
#pragma unroll
    for (int b = 0; b < K; ++b) acc[b] = 0.0;
    double ey = 0.0, ex = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += U * BAMG_BLK) {
        double x[U], q[U][K], yi[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = i + u * BAMG_BLK < i1 ? i + u * BAMG_BLK : i;
            if constexpr (SPMV) {
                const int4 c4 = *(const int4*)(eci + (size_t)r * 4);
                const double2 wa = ((const double2*)(ev + (size_t)r * 4))[0];
                const double2 wb = ((const double2*)(ev + (size_t)r * 4))[1];
                const double z0 = z[c4.x], z1 = z[c4.y], z2 = z[c4.z], z3 = z[c4.w];
                double acc = 0;
                acc += wa.x * z0;
                acc += wa.y * z1;
                acc += wb.x * z2;
                acc += wb.y * z3;
                x[u] = alpha * acc;
            } else {
                x[u] = w[r];
            }
#pragma unroll
            for (int b = 0; b < K; ++b) q[u][b] = (b < nb ? V + (size_t)b * ldv : y)[r];
            yi[u] = y[r];
        }
        __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the products
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i + u * BAMG_BLK >= i1) break;
            if constexpr (SPMV) wout[i + u * BAMG_BLK] = x[u];
#pragma unroll
            for (int b = 0; b < K; ++b) acc[b] += q[u][b] * x[u];
            ey += yi[u] * x[u];
            ex += x[u] * x[u];
        }
    }
    gs_store_partials<K>(acc, ey, ex, nb, part, NDM, red);
}

// Update pass on a chunk of one chain, with the coefficients of k_gs_step
// (cf = coef + c GS_CS: [b] a_b, [GS_MAXB + b] d_b, [2 GS_MAXB] 1/alpha,
// [+1] h, [+2] 1/nu):  q_nb = (v_nb - sum a_b q_b) / alpha over V_nb (not
// rewritten for nb = 0, where v_0 is exact), v_{nb+1} = (w - sum d_b q_b -
// h q_nb) / nu into V_{nb+1}, then the dots of v_{nb+1}.  The q_b of a row
// are loaded once into registers (K >= nb, all K loads issued together; b >=
// nb re-reads v_nb with a zero coefficient, which leaves the sums unchanged)
// for the updates and the dots, GsRows<K>::U rows at a time as in the dots
// pass; the coefficients sit in LDS.
template <int K>
__global__ void __launch_bounds__(BAMG_BLK)
k_gs_update(const ChainGeo* __restrict__ geo, int seg_rows, int ldv, int nb, const int* __restrict__ act,
            double* __restrict__ V, const double* __restrict__ w, const double* __restrict__ coef,
            double* __restrict__ part, int NDM) {
    __shared__ double red[(BAMG_BLK / BAMG_WAVE) * (GsRed<K>::KR + 2)];
    __shared__ double sa[K], sd[K];
    const ChainGeo g = geo[blockIdx.y];
    if (!act[blockIdx.y]) return;
    const int i0 = g.off + blockIdx.x * seg_rows, i1 = min(g.off + g.n, i0 + seg_rows);
    if (i0 >= i1) return;
    const double* cf = coef + (size_t)blockIdx.y * GS_CS;
    for (int t = threadIdx.x; t < K; t += BAMG_BLK) {
        sa[t] = t < nb ? cf[t] : 0.0;
        sd[t] = t < nb ? cf[GS_MAXB + t] : 0.0;
    }
    const double ia = cf[2 * GS_MAXB], hh = cf[2 * GS_MAXB + 1], inu = cf[2 * GS_MAXB + 2];
    __syncthreads();
    double* y = V + (size_t)nb * ldv;
    double* xn = V + (size_t)(nb + 1) * ldv;
    double acc[K];
#pragma unroll
    for (int b = 0; b < K; ++b) acc[b] = 0.0;
    double ey = 0.0, ex = 0.0;
    constexpr int U = GsRows<K>::U;
    for (int i = i0 + threadIdx.x; i < i1; i += U * BAMG_BLK) {
        double q[U][K], tv[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = i + u * BAMG_BLK < i1 ? i + u * BAMG_BLK : i;
#pragma unroll
            for (int b = 0; b < K; ++b) q[u][b] = (b < nb ? V + (size_t)b * ldv : y)[r];
            tv[u] = y[r];
            xv[u] = w[r];
        }
        __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the products
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = i + u * BAMG_BLK;
            if (r >= i1) break;
            double t = tv[u], x = xv[u];
#pragma unroll
            for (int b = 0; b < K; ++b) t -= sa[b] * q[u][b];
            t *= ia;
            if (nb > 0) y[r] = t;
#pragma unroll
            for (int b = 0; b < K; ++b) x -= sd[b] * q[u][b];
            x = (x - hh * t) * inu;
            xn[r] = x;
#pragma unroll
            for (int b = 0; b < K; ++b) acc[b] += q[u][b] * x;
            ey += t * x;
            ex += x * x;
        }
    }
    gs_store_partials<K>(acc, ey, ex, nb, part, NDM, red);
}

// out[c OS + d] = sum of chain c's chunk values of dot d, in chunk order.
// Grid (dots, chains); P = chunks per chain slot (the passes' grid x).
__global__ void k_gs_final(const ChainGeo* __restrict__ geo, int seg_rows, int P, const int* __restrict__ act,
                           const double* __restrict__ part, int NDM, double* __restrict__ out, int OS) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    const int d = blockIdx.x, c = blockIdx.y;
    if (!act[c]) return;
    const int np = (geo[c].n + seg_rows - 1) / seg_rows;
    const double* pp = part + ((size_t)c * NDM + d) * P;
    double s = 0;
    for (int k = threadIdx.x; k < np; k += BAMG_BLK) s += pp[k];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[(size_t)c * OS + d] = s;
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

// Step j of the Arnoldi process for every active chain (one thread each).
// dv = dots of the update pass that made v_j (a_b = dv[b], b < j; beta =
// dv[j]; unused for j = 0, where v_0 is exact), dw = dots of w (d_b, b < j;
// <v_j, w> = dw[j]; <w, w> = dw[j + 1]).  Per chain, aux holds nu_k (the norm
// estimate that made v_{k+1}), then xr_k and gr_k (row k of column k and g_k
// before Givens rotation k), GS entries each.
//  1. alpha = sqrt(beta - |a|^2) finishes v_j; column j-1 of H becomes
//     h + nu_{j-1} a with subdiagonal nu_{j-1} alpha: the change is rotated by
//     the rotations 0 .. j-2, and rotation j-1 and g_{j-1}, g_j are redone.
//  2. Column j: d_b (b < j), h_j = (<v_j, w> - a.d) / alpha, and the norm
//     estimate nu_j^2 = <w, w> - |d|^2 - h_j^2 (Pythagoras: one pass of
//     classical Gram-Schmidt against orthonormal q), rotated as usual;
//     est[c] = |g_{j+1}|.
//  3. The update pass's coefficients go to coef + c GS_CS.
// alpha = 0 (v_j inside the span: a breakdown) empties column j and ends the
// chain's inner iteration (est = 0, g_j = 0).
//  4. kd[c] = j + 1 (the columns the solution update takes), and act[c] = 0
//     once est[c] <= itol[c] or est[c] = 0: the chain's inner iteration ends
//     here and every later kernel of it skips the chain.
__global__ void k_gs_step(int nch, int j, int ld, int* __restrict__ act, const double* __restrict__ dvall,
                          const double* __restrict__ dwall, int DS, double* __restrict__ Hall, int HS,
                          double* __restrict__ csall, double* __restrict__ snall, double* __restrict__ gall,
                          double* __restrict__ auxall, int GS, double* __restrict__ coefall, double* __restrict__ est,
                          const double* __restrict__ itol, int* __restrict__ kd) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nch || !act[c]) return;
    const double* a = dvall + (size_t)c * DS;
    const double* d = dwall + (size_t)c * DS;
    double* H = Hall + (size_t)c * HS;
    double* cs = csall + (size_t)c * GS;
    double* sn = snall + (size_t)c * GS;
    double* g = gall + (size_t)c * GS;
    double* nu = auxall + (size_t)c * 3 * GS;
    double* xr = nu + GS;
    double* gr = xr + GS;
    double* cf = coefall + (size_t)c * GS_CS;
    double alpha = 1.0, hj, ad = 0.0;
    bool broke = false;
    if (j > 0) {
        double s2 = 0.0;
        for (int b = 0; b < j; ++b) { s2 += a[b] * a[b]; ad += a[b] * d[b]; }
        const double al2 = a[j] - s2;
        alpha = al2 > 0.0 ? sqrt(al2) : 0.0;
        broke = !(alpha > 0.0);
        double* cp = H + (size_t)(j - 1) * ld;
        const double np = nu[j - 1];
        double carry = np * a[0];
        for (int i = 0; i + 1 < j; ++i) {
            const double nx = np * a[i + 1];
            cp[i] += cs[i] * carry + sn[i] * nx;
            carry = -sn[i] * carry + cs[i] * nx;
        }
        const double x = xr[j - 1] + carry, yv = np * alpha;
        const double r = sqrt(x * x + yv * yv);
        const double cc = r > 0.0 ? x / r : 1.0, ss = r > 0.0 ? yv / r : 0.0;
        cp[j - 1] = r > 0.0 ? r : 1.0;
        cp[j] = 0.0;
        cs[j - 1] = cc; sn[j - 1] = ss;
        g[j - 1] = cc * gr[j - 1];
        g[j] = -ss * gr[j - 1];
        hj = broke ? 0.0 : (d[j] - ad) / alpha;
    } else {
        hj = d[0];
    }
    double* col = H + (size_t)j * ld;
    double nu2 = d[j + 1] - hj * hj;
    for (int b = 0; b < j; ++b) {
        col[b] = broke ? 0.0 : d[b];
        nu2 -= d[b] * d[b];
    }
    col[j] = hj;
    const double nuj = (!broke && nu2 > 0.0) ? sqrt(nu2) : 0.0;
    for (int i = 0; i < j; ++i) {
        const double u = col[i], v = col[i + 1];
        col[i] = cs[i] * u + sn[i] * v;
        col[i + 1] = -sn[i] * u + cs[i] * v;
    }
    xr[j] = col[j];
    gr[j] = g[j];
    nu[j] = nuj;
    const double x = col[j];
    const double r = sqrt(x * x + nuj * nuj);
    const double cc = r > 0.0 ? x / r : 1.0, ss = r > 0.0 ? nuj / r : 0.0;
    col[j] = r > 0.0 ? r : 1.0;
    col[j + 1] = 0.0;
    cs[j] = cc; sn[j] = ss;
    g[j + 1] = -ss * g[j];
    g[j] = cc * g[j];
    const double e = broke ? 0.0 : fabs(g[j + 1]);
    est[c] = e;
    for (int b = 0; b < j; ++b) { cf[b] = a[b]; cf[GS_MAXB + b] = d[b]; }
    cf[2 * GS_MAXB] = 1.0 / alpha;
    cf[2 * GS_MAXB + 1] = hj;
    cf[2 * GS_MAXB + 2] = nuj > 0.0 ? 1.0 / nuj : 0.0;
    kd[c] = j + 1;
    if (e <= itol[c] || e == 0.0) act[c] = 0;
}

// The same step for the multigrid-preconditioned Arnoldi method (Section
// 4.3): H is kept as it is (no Givens rotations) because its eigenpairs are
// wanted.  Column j-1 becomes h + nu_{j-1} a with subdiagonal nu_{j-1} alpha,
// column j is (d_b, h_j, nu_j); the update pass's coefficients as in
// k_gs_step; sc[c * SS] = nu_j (0 at a breakdown).
__global__ void k_arn_step(int nch, int j, int ld, const int* __restrict__ act, const double* __restrict__ dvall,
                           const double* __restrict__ dwall, int DS, double* __restrict__ Hall, int HS,
                           double* __restrict__ auxall, int GS, double* __restrict__ coefall,
                           double* __restrict__ sc, int SS) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nch || !act[c]) return;
    const double* a = dvall + (size_t)c * DS;
    const double* d = dwall + (size_t)c * DS;
    double* H = Hall + (size_t)c * HS;
    double* nu = auxall + (size_t)c * 3 * GS;
    double* cf = coefall + (size_t)c * GS_CS;
    double alpha = 1.0, hj, ad = 0.0;
    bool broke = false;
    if (j > 0) {
        double s2 = 0.0;
        for (int b = 0; b < j; ++b) { s2 += a[b] * a[b]; ad += a[b] * d[b]; }
        const double al2 = a[j] - s2;
        alpha = al2 > 0.0 ? sqrt(al2) : 0.0;
        broke = !(alpha > 0.0);
        double* cp = H + (size_t)(j - 1) * ld;
        const double np = nu[j - 1];
        for (int b = 0; b < j; ++b) cp[b] += np * a[b];
        cp[j] = np * alpha;
        hj = broke ? 0.0 : (d[j] - ad) / alpha;
    } else {
        hj = d[0];
    }
    double* col = H + (size_t)j * ld;
    double nu2 = d[j + 1] - hj * hj;
    for (int b = 0; b < j; ++b) {
        col[b] = broke ? 0.0 : d[b];
        nu2 -= d[b] * d[b];
    }
    col[j] = hj;
    const double nuj = (!broke && nu2 > 0.0) ? sqrt(nu2) : 0.0;
    col[j + 1] = nuj;
    nu[j] = nuj;
    sc[(size_t)c * SS] = nuj;
    for (int b = 0; b < j; ++b) { cf[b] = a[b]; cf[GS_MAXB + b] = d[b]; }
    cf[2 * GS_MAXB] = 1.0 / alpha;
    cf[2 * GS_MAXB + 1] = hj;
    cf[2 * GS_MAXB + 2] = nuj > 0.0 ? 1.0 / nuj : 0.0;
}

// x_i = sum_{b < kd[c]} eta_b V_b[i] on the rows of chains with act[c].
// (V_b starts at V + b ldv.)
__global__ void k_seg_ritz(int N, int ldv, const ChainGeo* __restrict__ geo, int nch, const int* __restrict__ act,
                           const int* __restrict__ kd, const double* __restrict__ V, const double* __restrict__ etaall,
                           int ES, double* __restrict__ x) {
    const int i = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK + threadIdx.x;
    if (i >= N) return;
    const int c = find_chain(geo, nch, i);
    if (!act[c]) return;
    const int k = kd[c];
    const double* eta = etaall + (size_t)c * ES;
    double s = 0.0;
    for (int b = 0; b < k; ++b) s += eta[b] * V[(size_t)b * ldv + i];
    x[i] = s;
}

// g = [beta_c, 0, ...] for every chain (beta2 per chain at stride).
__global__ void k_seg_gmres_init(int nch, int m, const double* __restrict__ beta2, int stride, double* __restrict__ gall,
                                 int GS) {
    int c = blockIdx.x;
    if (c >= nch) return;
    for (int k = threadIdx.x; k <= m; k += blockDim.x) gall[(size_t)c * GS + k] = 0.0;
    if (threadIdx.x == 0) gall[(size_t)c * GS] = sqrt(beta2[(size_t)c * stride]);
}

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

// x += sum_{j < kd[c]} y_cj Z_j (Z_j at Z + j ldv).
__global__ void k_seg_xupdate(int N, int ldv, const ChainGeo* __restrict__ geo, int nch, const int* __restrict__ kd,
                              const double* __restrict__ Z, const double* __restrict__ yall, int GS,
                              double* __restrict__ x) {
    int i = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK + threadIdx.x;
    if (i >= N) return;
    const int c = find_chain(geo, nch, i);
    const int k = kd[c];
    const double* y = yall + (size_t)c * GS;
    double s = x[i];
    for (int j = 0; j < k; ++j) s += y[j] * Z[(size_t)j * ldv + i];
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
