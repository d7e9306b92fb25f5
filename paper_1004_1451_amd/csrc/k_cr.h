// Coarsening without a grid and the operators built on it (Section 3.1,
// Algorithm 1; eq. neighbor_def; Algorithm 2 on candidate lists; Section 4:
// averaging Q and the Petrov-Galerkin products).
//
// Layouts (device), single chain, level l with n rows:
//   st      : int[n] independent-set state (MIS_UND, MIS_IN, MIS_OUT).
//   isC     : int[n] 1 for a coarse point.
//   cmap    : int[n] coarse index of a C point (rank among the C points in
//             ascending row order), -1 for an F point.
//   Q_l     : CSR (nc rows), fine columns ascending, values 1/|J_i|.
//   P_l     : ELL-4 as on grids.
#pragma once
#include "common.h"
#include "k_sparse.h"

enum : int {
    ERR_UNSYM = 32,       // pattern of B not symmetric
    ERR_NOCOARSE = 64,    // an F point without a coarse neighbour
    ERR_WIDEN = 128,      // more candidates than LSU_K
    ERR_GALCAP = 256,     // a product row needs more than RP_CAP terms
};

enum : int { MIS_UND = 0, MIS_IN = 1, MIS_OUT = 2 };

// Stream of the compatible-relaxation start vectors: STREAM_CR + level.
#define STREAM_CR 16ull
#define CR_RED_BLOCKS 64      // blocks of the fixed-partition norm reduction

// ---------------------------------------------------------------- pattern
// Every stored (i, j), j != i, has a stored (j, i): binary search in row j.
__global__ void k_check_sym(int n, const int* __restrict__ rp, const int* __restrict__ ci, int* __restrict__ err) {
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    bool ok = true;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        if (j == i) continue;
        int lo = rp[j], hi = rp[j + 1] - 1;
        bool found = false;
        while (lo <= hi) {
            const int mid = (lo + hi) >> 1;
            const int c = ci[mid];
            if (c == i) { found = true; break; }
            if (c < i) lo = mid + 1; else hi = mid - 1;
        }
        ok = ok && found;
    }
    if (!ok) atomicOr(err, ERR_UNSYM);
}

// ---------------------------------------------------------------- MIS
// The standard independent set of the candidates (cand == nullptr: all
// points), taken greedily in increasing index: a candidate joins when no
// neighbour has joined.  Computed in rounds that decide a point once its
// lower-index neighbours are decided (joined points make their neighbours
// MIS_OUT, and a point joins when every lower-index neighbour is MIS_OUT),
// which reproduces the sequential greedy exactly.  Decisions read only final
// states, so a round may run in place.
__global__ void k_mis_init(int n, const int* __restrict__ cand, int* __restrict__ st) {
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    st[i] = (cand == nullptr || cand[i]) ? MIS_UND : MIS_OUT;
}

__global__ void k_mis_round(int n, const int* __restrict__ rp, const int* __restrict__ ci, int* st,
                            int* __restrict__ open) {
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    if (__atomic_load_n(&st[i], __ATOMIC_RELAXED) != MIS_UND) return;
    bool nb_in = false, lower_und = false;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        if (j == i) continue;
        const int sj = __atomic_load_n(&st[j], __ATOMIC_RELAXED);
        nb_in = nb_in || sj == MIS_IN;
        lower_und = lower_und || (sj == MIS_UND && j < i);
    }
    if (nb_in) __atomic_store_n(&st[i], (int)MIS_OUT, __ATOMIC_RELAXED);
    else if (!lower_und) __atomic_store_n(&st[i], (int)MIS_IN, __ATOMIC_RELAXED);
    else *open = 1;
}

// isC |= (st == MIS_IN); with first != 0, isC = (st == MIS_IN).
__global__ void k_mis_take(int n, const int* __restrict__ st, int first, int* __restrict__ isC) {
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const int in = st[i] == MIS_IN;
    isC[i] = first ? in : (isC[i] | in);
}

// ---------------------------------------------------------------- CR
// u^0_i = 1 + u(seed, STREAM_CR + level, base + i) on F, 0 on C.
__global__ void k_cr_start(int n, const int* __restrict__ isC, uint64_t seed, uint64_t stream, uint64_t base,
                           double* __restrict__ u0, double* __restrict__ u) {
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const double v = isC[i] ? 0.0 : 1.0 + splitmix_u01(seed, stream, base + (uint64_t)i);
    u0[i] = v;
    u[i] = v;
}

// One F-relaxation sweep of eq. frelax with omega-Jacobi on B u = 0:
// u_i <- u_i - (omega / b_ii) sum_j b_ij u_j on F (u = 0 on C).  The row sum
// runs in stored order with separate roundings (contraction into fused
// multiply-adds is off), so the iterates, and the decisions taken on them,
// are reproducible.
template <typename M>
__global__ void k_cr_sweep(int n, const int* __restrict__ rp, const int* __restrict__ ci, const M* __restrict__ v,
                           double omega, const int* __restrict__ isC, const double* __restrict__ uin,
                           double* __restrict__ uout) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    if (isC[i]) { uout[i] = 0.0; return; }
    double s = 0.0, d = 1.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        const double b = (double)v[p];
        if (j == i) d = b;
        s = s + b * uin[j];
    }
    const double w = omega / d;
    uout[i] = uin[i] - w * s;
}

// Per-block partial sums of u0^2 and u^2 (fixed partition).
__global__ void k_cr_ssq_partial(int n, const double* __restrict__ u0, const double* __restrict__ u,
                                 double* __restrict__ part) {
    __shared__ double sh[2][BAMG_BLK / BAMG_WAVE];
    double a = 0.0, b = 0.0;
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < n; i += gridDim.x * BAMG_BLK) {
        a += u0[i] * u0[i];
        b += u[i] * u[i];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x / BAMG_WAVE, lane = threadIdx.x % BAMG_WAVE;
    if (lane == 0) { sh[0][w] = a; sh[1][w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int k = 0; k < BAMG_BLK / BAMG_WAVE; ++k) { x += sh[0][k]; y += sh[1][k]; }
        part[2 * blockIdx.x] = x;
        part[2 * blockIdx.x + 1] = y;
    }
}

__global__ void k_cr_ssq_final(int nb, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double x = 0.0, y = 0.0;
    for (int k = 0; k < nb; ++k) { x += part[2 * k]; y += part[2 * k + 1]; }
    out[0] = x;
    out[1] = y;
}

// Candidate set of Algorithm 1: F points with |u_i^nu| > theta |u_i^(nu-1)|
// (the ratio test as a product, in the same roundings as the oracle);
// any[0] = 1 when there is one.
__global__ void k_cr_cand(int n, const int* __restrict__ isC, const double* __restrict__ prev,
                          const double* __restrict__ last, double theta, int* __restrict__ cand,
                          int* __restrict__ any) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    const double bound = theta * fabs(prev[i]);
    const int c = !isC[i] && fabs(last[i]) > bound;
    cand[i] = c;
    if (c) *any = 1;
}

// cmap[i] = rank of a C point (from the exclusive scan of isC), -1 on F.
__global__ void k_cr_cmap(int n, const int* __restrict__ isC, const int* __restrict__ pos, int* __restrict__ cmap) {
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
    cmap[i] = isC[i] ? pos[i] : -1;
}

// ---------------------------------------------------------------- LS fit
// Algorithm 2 on candidate lists: N_i = the C points j != i with b_ij stored
// (graph distance 1 in G(B), eq. neighbor_def), in ascending coarse index.
// One thread per row; the weighted Gram of the candidates lives in LDS
// (lane-minor, so that the lanes of a wavefront hit distinct banks).  The
// greedy, the admissibility test and the solves are those of the grid form:
// starting from J = {}, add the admissible candidate with the smallest
// sigma - b_S^T G_SS^-1 b_S (strict minimum, ties to the lower slot) until
// |J| >= caliber; a candidate g is admissible when det(G_{J+g}) / det(G_J)
// exceeds 1e-10 G_gg.  No admissible candidate: the first one gets weight 1.
#define LSU_K 16
#define LSU_BLK 64
#define LSU_G (LSU_K * (LSU_K + 1) / 2)

__device__ __forceinline__ int lsu_gi(int s, int t) { return s >= t ? s * (s + 1) / 2 + t : t * (t + 1) / 2 + s; }

template <typename T, typename MP>
__global__ void __launch_bounds__(LSU_BLK)
k_ls_fit_u(int n, int Ru, int Rv, int VS, const T* __restrict__ U, const T* __restrict__ V,
           const double* __restrict__ w, int caliber, const int* __restrict__ cmap, const int* __restrict__ brp,
           const int* __restrict__ bci, int* __restrict__ pc, MP* __restrict__ pv, T* __restrict__ inject,
           unsigned char* __restrict__ jcnt, int* __restrict__ err) {
    __shared__ double sG[LSU_G][LSU_BLK];
    __shared__ double sb[LSU_K][LSU_BLK];
    __shared__ int sf[LSU_K][LSU_BLK];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * LSU_BLK + tid;
    if (i >= n) return;
    const int ci_ = cmap[i];
    if (ci_ >= 0) {
        pc[(size_t)i * 4] = ci_; pv[(size_t)i * 4] = (MP)1;
#pragma unroll
        for (int s = 1; s < 4; ++s) { pc[(size_t)i * 4 + s] = -1; pv[(size_t)i * 4 + s] = (MP)0; }
        if (inject)
            for (int k = 0; k < Ru; ++k) inject[(size_t)ci_ * Ru + k] = U[(size_t)i * Ru + k];
        if (jcnt) jcnt[i] = 1;
        return;
    }
    // candidates
    int K = 0;
    for (int p = brp[i]; p < brp[i + 1]; ++p) {
        const int j = bci[p];
        if (j == i || cmap[j] < 0) continue;
        if (K == LSU_K) { atomicOr(err, ERR_WIDEN); break; }
        sf[K][tid] = j;
        ++K;
    }
    if (K == 0) {
        atomicOr(err, ERR_NOCOARSE);
#pragma unroll
        for (int s = 0; s < 4; ++s) { pc[(size_t)i * 4 + s] = -1; pv[(size_t)i * 4 + s] = (MP)0; }
        if (jcnt) jcnt[i] = 0;
        return;
    }
    // weighted Gram, right-hand side and sigma: U columns, then V columns
    double sigma = 0.0;
    for (int part = 0; part < 2; ++part) {
        const T* Xp = part == 0 ? U : V;
        const int ld = part == 0 ? Ru : VS;
        const int nk = part == 0 ? Ru : Rv;
        const double* wp = w + (part == 0 ? 0 : Ru);
        for (int k = 0; k < nk; ++k) {
            const double xi = (double)Xp[(size_t)i * ld + k];
            sigma += wp[k] * xi * xi;
        }
        for (int s = 0; s < K; ++s) {
            const int fs = sf[s][tid];
            double bs = 0.0;
            for (int k = 0; k < nk; ++k)
                bs += wp[k] * (double)Xp[(size_t)fs * ld + k] * (double)Xp[(size_t)i * ld + k];
            sb[s][tid] = (part == 0 ? 0.0 : sb[s][tid]) + bs;
            for (int t = 0; t <= s; ++t) {
                const int ft = sf[t][tid];
                double g = 0.0;
                for (int k = 0; k < nk; ++k)
                    g += wp[k] * (double)Xp[(size_t)fs * ld + k] * (double)Xp[(size_t)ft * ld + k];
                double& G = sG[s * (s + 1) / 2 + t][tid];
                G = (part == 0 ? 0.0 : G) + g;
            }
        }
    }
    // greedy selection
    int jl[4] = {0, 0, 0, 0};
    int nsel = 0;
    double detJ = 1.0;
    double G4[4][4], b4[4], L[4][4], il[4], z[4];
    auto load_set = [&](const int (&idx)[4], int m) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            b4[a] = a < m ? sb[idx[a]][tid] : 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) G4[a][c] = (a < m && c < m) ? sG[lsu_gi(idx[a], idx[c])][tid] : 0.0;
        }
    };
    const int steps = K < caliber ? K : caliber;
    for (int step = 0; step < steps; ++step) {
        int best = -1;
        double bestL = 0.0;
        for (int c = 0; c < K; ++c) {
            bool in = false;
#pragma unroll
            for (int a = 0; a < 4; ++a) in = in || (a < nsel && jl[a] == c);
            if (in) continue;
            // S = J u {c} in ascending slot order
            int idx[4] = {0, 0, 0, 0};
            int m = 0;
            bool put = false;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                if (a < nsel) {
                    if (!put && c < jl[a]) { idx[m++] = c; put = true; }
                    if (m < 4) idx[m++] = jl[a];
                }
            }
            if (!put && m < 4) idx[m++] = c;
            load_set(idx, m);
            double det;
            const bool ok = chol4(G4, b4, (1 << m) - 1, L, il, z, det);
            const double gcc = sG[lsu_gi(c, c)][tid];
            if (!ok || !(det > 1e-10 * gcc * detJ)) continue;
            double Lv = sigma;
#pragma unroll
            for (int a = 0; a < 4; ++a) Lv -= z[a] * z[a];
            if (best < 0 || Lv < bestL) { best = c; bestL = Lv; }
        }
        if (best < 0) break;
        // insert best keeping jl ascending
        int pos = nsel;
        while (pos > 0 && jl[pos - 1] > best) { jl[pos] = jl[pos - 1]; --pos; }
        jl[pos] = best;
        ++nsel;
        load_set(jl, nsel);
        double det;
        chol4(G4, b4, (1 << nsel) - 1, L, il, z, det);
        detJ = det;
    }
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    if (nsel == 0) {
        nsel = 1;
        jl[0] = 0;
        p[0] = 1.0;
    } else {
        load_set(jl, nsel);
        double det;
        chol4(G4, b4, (1 << nsel) - 1, L, il, z, det);
#pragma unroll
        for (int a = 3; a >= 0; --a) {
            if (a >= nsel) continue;
            double s = z[a];
#pragma unroll
            for (int c = a + 1; c < 4; ++c)
                if (c < nsel) s -= L[c][a] * p[c];
            p[a] = s * il[a];
        }
    }
    // the slots are in ascending coarse index, so the row is already sorted
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (a < nsel) {
            pc[(size_t)i * 4 + a] = cmap[sf[jl[a]][tid]];
            pv[(size_t)i * 4 + a] = (MP)p[a];
        } else {
            pc[(size_t)i * 4 + a] = -1;
            pv[(size_t)i * 4 + a] = (MP)0;
        }
    }
    if (jcnt) jcnt[i] = (unsigned char)nsel;
}

// ---------------------------------------------------------------- Q
// Averaging restriction: Q[I, i] = 1/|J_i| for every fine i with I in J_i.
// Counts per coarse row, then (after the scan) a fill at atomic cursors and a
// per-row sort by fine index, so that the result does not depend on timing.
__global__ void k_qu_count(int n, const int* __restrict__ pc, int* __restrict__ cnt) {
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int I = pc[(size_t)i * 4 + s];
        if (I >= 0) atomicAdd(&cnt[I], 1);
    }
}

__global__ void k_qu_fill(int n, const int* __restrict__ pc, const int* __restrict__ qrp, int* __restrict__ cur,
                          int* __restrict__ qci) {
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int I = pc[(size_t)i * 4 + s];
        if (I >= 0) qci[qrp[I] + atomicAdd(&cur[I], 1)] = i;
    }
}

template <typename MQ>
__global__ void k_qu_finish(int nc, const int* __restrict__ qrp, int* __restrict__ qci,
                            const unsigned char* __restrict__ jcnt, MQ* __restrict__ qv) {
    const int I = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (I >= nc) return;
    const int p0 = qrp[I], p1 = qrp[I + 1];
    for (int p = p0 + 1; p < p1; ++p) {
        const int v = qci[p];
        int q = p - 1;
        while (q >= p0 && qci[q] > v) { qci[q + 1] = qci[q]; --q; }
        qci[q + 1] = v;
    }
    for (int p = p0; p < p1; ++p) qv[p] = (MQ)(1.0 / (double)jcnt[qci[p]]);
}

// ---------------------------------------------------------------- Galerkin
// Row-wise sparse product C = L R, one wavefront per row I of L (CSR, values
// lv; lv = nullptr: all ones).  R is ELL-4 (RCSR = false: rci/rv are the
// 4-slot columns/values of P, -1 = empty) or CSR (rrp, rci, rv).  The
// products l_Ia r_{i_a J} are enumerated in loop order (entry a of row I,
// then the entries of row i_a of R) and tagged with their position; sorting
// the keys (J << RP_POSB) | position groups equal columns with the positions
// in loop order, so each value is summed over a in the order of L's row, as
// a sequential row-times-matrix product does.  The Galerkin products are
// B_{l+1} = Q (B P) and T_{l+1} = Q (T P), each as W = M P, then Q W (the
// order of the plain definition; M = I needs only Q P).  Pass 0 counts the
// columns of each row into cnt; pass 1 writes the row at rp[I].
#define RP_CAP 4096
#define RP_POSB 12
#define RP_MAXL 1024

template <typename MV, bool RCSR>
__global__ void __launch_bounds__(BAMG_WAVE)
k_rowprod(int nrows, int ncols, int pass, const int* __restrict__ lrp, const int* __restrict__ lci,
          const MV* __restrict__ lv, const int* __restrict__ rrp, const int* __restrict__ rci,
          const MV* __restrict__ rv, int* __restrict__ cnt, const int* __restrict__ rp, int* __restrict__ ci,
          MV* __restrict__ cv, int* __restrict__ err) {
    __shared__ unsigned key[RP_CAP];
    __shared__ int tix[RP_CAP];
    __shared__ unsigned short la[RP_CAP];
    __shared__ int off[RP_MAXL + 1];
    __shared__ int ustart[RP_CAP + 1];
    const int I = blockIdx.x;
    const int lane = threadIdx.x;
    if (I >= nrows) return;
    const int q0 = lrp[I], nq = lrp[I + 1] - q0;
    if (nq > RP_MAXL || ncols >= (1 << (32 - RP_POSB))) {
        if (lane == 0) { atomicOr(err, ERR_GALCAP); if (pass == 0) cnt[I] = 0; }
        return;
    }
    // products per entry of L's row, then their offsets
    for (int a = lane; a < nq; a += BAMG_WAVE) {
        const int i = lci[q0 + a];
        int c = 0;
        if (RCSR) {
            c = rrp[i + 1] - rrp[i];
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) c += rci[(size_t)i * 4 + s] >= 0;
        }
        off[a + 1] = c;
    }
    __syncthreads();
    if (lane == 0) {
        off[0] = 0;
        for (int a = 0; a < nq; ++a) off[a + 1] += off[a];
    }
    __syncthreads();
    const int tot = off[nq];
    if (tot > RP_CAP) {
        if (lane == 0) { atomicOr(err, ERR_GALCAP); if (pass == 0) cnt[I] = 0; }
        return;
    }
    for (int a = lane; a < nq; a += BAMG_WAVE) {
        const int i = lci[q0 + a];
        int pos = off[a];
        const int t0 = RCSR ? rrp[i] : i * 4, t1 = RCSR ? rrp[i + 1] : i * 4 + 4;
        for (int t = t0; t < t1; ++t) {
            const int J = rci[t];
            if (J < 0) continue;
            key[pos] = ((unsigned)J << RP_POSB) | (unsigned)pos;
            tix[pos] = t;
            la[pos] = (unsigned short)a;
            ++pos;
        }
    }
    // bitonic sort of the keys, padded to a power of two
    int len = 1;
    while (len < tot) len <<= 1;
    for (int t = tot + lane; t < len; t += BAMG_WAVE) key[t] = 0xFFFFFFFFu;
    __syncthreads();
    for (int kk = 2; kk <= len; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < len; t += BAMG_WAVE) {
                const int u = t ^ j;
                if (u > t) {
                    const unsigned a = key[t], b = key[u];
                    const bool up = (t & kk) == 0;
                    if ((a > b) == up) { key[t] = b; key[u] = a; }
                }
            }
            __syncthreads();
        }
    }
    // segment starts of equal columns
    int nu = 0;
    for (int base = 0; base < tot; base += BAMG_WAVE) {
        const int t = base + lane;
        bool first = false;
        if (t < tot) first = t == 0 || (key[t] >> RP_POSB) != (key[t - 1] >> RP_POSB);
        const unsigned long long mask = __ballot(first);
        const int rank = nu + __popcll(mask & ((1ull << lane) - 1ull));
        if (first) ustart[rank] = t;
        nu += __popcll(mask);
    }
    __syncthreads();
    if (pass == 0) {
        if (lane == 0) cnt[I] = nu;
        return;
    }
    if (lane == 0) ustart[nu] = tot;
    __syncthreads();
    const int o = rp[I];
    for (int u = lane; u < nu; u += BAMG_WAVE) {
        const int t0 = ustart[u], t1 = ustart[u + 1];
        double sum = 0.0;
        for (int t = t0; t < t1; ++t) {
            const int pos = (int)(key[t] & ((1u << RP_POSB) - 1u));
            const double l = lv ? (double)lv[q0 + la[pos]] : 1.0;
            sum += l * (double)rv[tix[pos]];
        }
        ci[o + u] = (int)(key[t0] >> RP_POSB);
        cv[o + u] = (MV)sum;
    }
}

// ---------------------------------------------------------------- cycle
// f_c = Q r (restriction of the cycle on a level without a grid).
template <typename T>
__global__ void k_restrict_csr(int nc, const int* __restrict__ qrp, const int* __restrict__ qci,
                               const T* __restrict__ qv, const T* __restrict__ r, T* __restrict__ fc) {
    const int I = xcd_tile(blockIdx.x, gridDim.x) * BAMG_BLK + threadIdx.x;
    if (I >= nc) return;
    T s = (T)0;
    for (int p = qrp[I]; p < qrp[I + 1]; ++p) s += qv[p] * r[qci[p]];
    fc[I] = s;
}
