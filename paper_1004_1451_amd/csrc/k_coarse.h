// Coarsest level of every chain, batched: blockIdx.y (or a loop) selects the
// chain.  Each chain has exactly one coarsest level (at its own depth); the
// descriptor below locates its operator inside that level's arrays and its
// dense / vector storage inside the pools.
//
// Per chain (n = n_L, Section 4.2 and Algorithm 3 with l = L):
//   W  = B_L^+ (n x n, row-major)         formed from the inverse of the
//        padded operator [[B_11, 0], [0, 1]] (block tridiagonal in grid rows,
//        blocks of b = ny <= 64, plus the corner blocks when periodic: block
//        LU and substitution with those, divide and conquer without), then
//        W = Pi_y [[B_11^-1, 0], [0, 0]] Pi_1;
//   y  spans null(B_L); c = T_L^T 1; cy = c^T y;
//   Arnoldi on v -> u - y (c^T u)/cy, u = W T_L v, for the coarsest
//   eigenpairs.
#pragma once
#include "common.h"
#include "k_dense.h"

// Block-LU path limits: block side ny <= GJ_NB, block rows nx <= CZ_MAX_NX
// (larger coarsest grids take the dense Gauss-Jordan path).
#define CZ_MAX_NX 256

struct CoarseDesc {
    int n, nx, ny, periodic;
    long long soff;           // dense B_L the block extraction reads (W pool offset)
    int sld;                  // its row length
    int bord;                 // 1: the main part of a bordered grid (below)
    int row0;                 // first row of the chain on its coarsest level
    int voff;                 // offset of its length-n vectors in the vector pools
    long long woff;           // offset of its n x n block in the W pool
    long long boff;           // offset of its block-LU factors (5 * nx * ny^2)
    long long aoff;           // offset of its Arnoldi basis (n * (am + 1))
    long long wfoff;          // offset of its FP32 copy of W (rows of wfld)
    int wfld;                 // that copy's row length (n rounded up to 4)
    int am;                   // Arnoldi steps (0: no eigenpairs)
    FastDiv dy;
    const int* brp; const int* bci; const void* bv;   // CSR of B on that level
    const int* trp; const int* tci; const void* tv;   // CSR of T (null: T = I)
};

// ---------------------------------------------------------------- densify
// W[i, j] = B_L[i, j] (W and bcol zeroed first); column n-1 also saved in bcol.
template <typename M>
__global__ void k_cz_densify(const CoarseDesc* __restrict__ cd, double* __restrict__ Wp, double* __restrict__ bcolp) {
    const CoarseDesc d = cd[blockIdx.y];
    double* W = Wp + d.woff;
    const M* v = (const M*)d.bv;
    for (int li = blockIdx.x * BAMG_BLK + threadIdx.x; li < d.n; li += gridDim.x * BAMG_BLK) {
        const int i = d.row0 + li;
        for (int p = d.brp[i]; p < d.brp[i + 1]; ++p) {
            const int lj = d.bci[p] - d.row0;
            W[(size_t)li * d.n + lj] = (double)v[p];
            if (lj == d.n - 1) bcolp[d.voff + li] = (double)v[p];
        }
    }
}

// max |B_L| per chain (the pivot scale): block maxima over a grid-stride range
// of the chain's nonzeros (grid (P, nch)) into part[chain * P + block], then
// one block per chain -> scale[chain].  The nonzeros of the sparse B_L are
// exactly those of its dense copy.
template <typename M>
__global__ void k_cz_absmax_sparse(const CoarseDesc* __restrict__ cd, double* __restrict__ part) {
    __shared__ double sh[BAMG_BLK];
    const CoarseDesc d = cd[blockIdx.y];
    const M* v = (const M*)d.bv;
    const int p0 = d.brp[d.row0], p1 = d.brp[d.row0 + d.n];
    double m = 0;
    for (int p = p0 + blockIdx.x * BAMG_BLK + threadIdx.x; p < p1; p += gridDim.x * BAMG_BLK)
        m = fmax(m, fabs((double)v[p]));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = BAMG_BLK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = sh[0];
}

__global__ void k_cz_absmax_final(int P, const double* __restrict__ part, double* __restrict__ scale) {
    __shared__ double sh[BAMG_BLK];
    double m = 0;
    for (int j = threadIdx.x; j < P; j += BAMG_BLK) m = fmax(m, part[(size_t)blockIdx.x * P + j]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = BAMG_BLK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) scale[blockIdx.x] = sh[0];
}

// ---------------------------------------------------------------- block LU
// Block storage of chain d: Dk | Up | Lo | Cl | Rw, each nx blocks of b x b.
__device__ __forceinline__ double* cz_blk(double* base, const CoarseDesc& d, int part, int k) {
    const long long bb = (long long)d.ny * d.ny;
    return base + d.boff + ((long long)part * d.nx + k) * bb;
}

// Extract the blocks of the padded operator from the dense B_L (in W).
__global__ void k_cz_extract(const CoarseDesc* __restrict__ cd, const double* __restrict__ Wp, double* __restrict__ Fp) {
    const CoarseDesc d = cd[blockIdx.z];
    const int k = blockIdx.y;
    const int nx = d.nx, b = d.ny, K = nx - 1, n = d.n, bb = b * b;
    if (k >= nx) return;
    const bool arrow = d.periodic && nx >= 3;
    const double* A = Wp + d.soff;
    for (int kind = 0; kind < 5; ++kind) {
        int bi, bj;
        if (kind == 0) { bi = k; bj = k; }
        else if (kind == 1) { if (k >= K) continue; bi = k; bj = k + 1; }
        else if (kind == 2) { if (k < 1) continue; bi = k; bj = k - 1; }
        else if (kind == 3) { if (!arrow || k >= K - 1) continue; bi = k; bj = K; }
        else { if (!arrow || k >= K - 1) continue; bi = K; bj = k; }
        double* dst = cz_blk(Fp, d, kind, k);
        for (int e = blockIdx.x * BAMG_BLK + threadIdx.x; e < bb; e += gridDim.x * BAMG_BLK) {
            int r = e / b, c = e % b;
            int gi = bi * b + r, gj = bj * b + c;
            // the main part of a bordered grid: grid rows of b + 1 points in
            // the source, no padded unknown
            const int si = d.bord ? bi * (b + 1) + r : gi, sj = d.bord ? bj * (b + 1) + c : gj;
            double v = A[(size_t)si * d.sld + sj];
            if (!d.bord && (gi == n - 1 || gj == n - 1)) v = (gi == gj) ? 1.0 : 0.0;
            dst[e] = v;
        }
    }
}

// Inversion of one diagonal block: Gauss-Jordan elimination without
// pivoting on the block padded to 64 x 64 with the identity.  Thread (w, c)
// of CZ_GJ_THREADS keeps column c of rows CZ_GJ_ROWS w .. + CZ_GJ_ROWS - 1 in
// registers.  Before each step's barrier the owner wave puts the pivot rows
// into LDS (two buffers, alternating).  1/p is v_rcp_f64 refined by two
// Newton steps (cz_recip).
#define CZ_GJ_THREADS 256
#define CZ_GJ_ROWS (GJ_NB * BAMG_WAVE / CZ_GJ_THREADS)

// Gauss-Jordan on the 64 x 64 block held in S by the CZ_GJ_THREADS threads
// (w = wave, c = lane), two pivots per step: with the pivot block
// P = A[J, J], J = {s, s+1}, and its closed-form inverse Q,
//   A[J, c] <- Q A[J, c],  A[r, J] <- -A[r, J] Q,  A[J, J] <- Q,
//   A[r, c] <- A[r, c] - A[r, J] Q A[J, c]  (r, c outside J),
// the same Schur complements as two scalar steps.  Each entry takes two
// fused multiply-adds; the pivot columns use m = e_j + Q[:, j] so the same
// update leaves -A[r, J] Q there.  A wave's rows of the pivot columns sit in
// its own lanes s and s+1 (read with v_readlane); only the two pivot rows go
// through LDS, from the wave that holds them.  mp (thread 0) takes the
// smallest |scalar pivot| / sc of the first nb (a and det / a per block):
// thread t keeps step t's pair and the quotients and their minimum are
// formed once at the end, off the chain of dependent steps.
__device__ __forceinline__ void cz_gj(double (&S)[CZ_GJ_ROWS], int w, int c, int nb, double sc, double& mp,
                                      double (*prow)[2][GJ_NB]) {
    static_assert(CZ_GJ_ROWS % 2 == 0, "pivot pairs stay inside one wave");
    static_assert(GJ_NB == BAMG_WAVE, "lane = column of the block");
    double my_a = 1.0, my_det = 1.0;
    for (int blk = 0; blk < GJ_NB / CZ_GJ_ROWS; ++blk) {
#pragma unroll
        for (int ss = 0; ss < CZ_GJ_ROWS / 2; ++ss) {
            const int s0 = CZ_GJ_ROWS * blk + 2 * ss, buf = ss & 1;
            const int j = c - s0;
            const bool cj = j == 0 || j == 1;
            if (w == blk) { prow[buf][0][c] = S[2 * ss]; prow[buf][1][c] = S[2 * ss + 1]; }
            double fx[CZ_GJ_ROWS], fy[CZ_GJ_ROWS];
#pragma unroll
            for (int i = 0; i < CZ_GJ_ROWS; ++i) {
                fx[i] = readlane_f64(S[i], s0);
                fy[i] = readlane_f64(S[i], s0 + 1);
            }
            __syncthreads();
            const double a = prow[buf][0][s0], b = prow[buf][0][s0 + 1];
            const double cc = prow[buf][1][s0], d = prow[buf][1][s0 + 1];
            const double r0 = prow[buf][0][c], r1 = prow[buf][1][c];
            const double det = fma(a, d, -b * cc);
            const double id = cz_recip(det);
            const double q00 = d * id, q01 = -b * id, q10 = -cc * id, q11 = a * id;
            if (threadIdx.x == s0 / 2) { my_a = a; my_det = det; }
            const double g0 = fma(q00, r0, q01 * r1), g1 = fma(q10, r0, q11 * r1);
            const double p0 = j == 0 ? q00 : q01, p1 = j == 0 ? q10 : q11;     // column j of Q
            const double m0 = cj ? (j == 0 ? 1.0 : 0.0) + p0 : g0;
            const double m1 = cj ? (j == 1 ? 1.0 : 0.0) + p1 : g1;
#pragma unroll
            for (int i = 0; i < CZ_GJ_ROWS; ++i) S[i] = fma(-fx[i], m0, fma(-fy[i], m1, S[i]));
            if (w == blk) { S[2 * ss] = cj ? p0 : g0; S[2 * ss + 1] = cj ? p1 : g1; }
        }
    }
    if (threadIdx.x < BAMG_WAVE) {
        const int s0 = 2 * threadIdx.x;
        double v = 1e300;
        if (s0 < GJ_NB && s0 < nb) v = fmin(v, fabs(my_a) / sc);
        if (s0 < GJ_NB && s0 + 1 < nb) v = fmin(v, fabs(my_det / my_a) / sc);
#pragma unroll
        for (int o = BAMG_WAVE / 2; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, BAMG_WAVE));
        if (threadIdx.x == 0) mp = fmin(mp, v);
    }
}

// In-place inverse of the diagonal block A[k0:k0+nb, k0:k0+nb] (ld) of the
// dense Gauss-Jordan inverse: the block (padded to 64 x 64 with the identity)
// in registers as cz_gj keeps it, two pivots per step.  Records min |pivot| /
// scale in *minpiv (scale = max |B_L| entry; one workgroup runs this kernel).
__global__ void __launch_bounds__(CZ_GJ_THREADS)
k_gj_diag(int ld, int k0, int nb, double* __restrict__ A, const double* __restrict__ scale,
          double* __restrict__ minpiv) {
    __shared__ double prow[2][2][GJ_NB];
    const int w = threadIdx.x / BAMG_WAVE, c = threadIdx.x % BAMG_WAVE;
    double S[CZ_GJ_ROWS];
#pragma unroll
    for (int i = 0; i < CZ_GJ_ROWS; ++i) {
        const int r = CZ_GJ_ROWS * w + i;
        S[i] = (r < nb && c < nb) ? A[(size_t)(k0 + r) * ld + k0 + c] : (r == c ? 1.0 : 0.0);
    }
    double mp = 1e300;
    cz_gj(S, w, c, nb, *scale, mp, prow);
#pragma unroll
    for (int i = 0; i < CZ_GJ_ROWS; ++i) {
        const int r = CZ_GJ_ROWS * w + i;
        if (r < nb && c < nb) A[(size_t)(k0 + r) * ld + k0 + c] = S[i];
    }
    if (threadIdx.x == 0) *minpiv = fmin(*minpiv, mp);
}

// One b x b product C = A B (mode 0, C may alias A) or C -= A B (mode 1):
// A staged transposed and B as is in LDS (zero-padded to 64 x 64), each
// thread a 4 x 4 tile of C at rows tr.., columns tc.., summed over t in
// ascending order.
__device__ __forceinline__ void cz_stage(int b, const double* A, double (*AsT)[GJ_NB + 2], const double* Bm,
                                         double (*Bs)[GJ_NB + 2]) {
    for (int e = threadIdx.x; e < GJ_NB * GJ_NB; e += BAMG_BLK) {
        const int r = e / GJ_NB, c = e % GJ_NB;
        const bool ok = r < b && c < b;
        AsT[c][r] = ok ? A[r * b + c] : 0.0;
        if (Bm) Bs[r][c] = ok ? Bm[r * b + c] : 0.0;
    }
}

__device__ __forceinline__ void cz_tile(int b, const double (*AsT)[GJ_NB + 2], const double (*Bs)[GJ_NB + 2], int tr,
                                        int tc, double (&acc)[4][4]) {
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
}

__device__ void cz_gemm(int b, const double* A, const double* Bm, double* C, int mode, double (*AsT)[GJ_NB + 2],
                        double (*Bs)[GJ_NB + 2]) {
    cz_stage(b, A, AsT, Bm, Bs);
    __syncthreads();
    const int tid = threadIdx.x, tr = (tid / 16) * 4, tc = (tid % 16) * 4;
    double acc[4][4];
    cz_tile(b, AsT, Bs, tr, tc, acc);
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

// Elimination of block column k for every chain with k < K = nx - 1.
// phase 0: multipliers  Lo[k+1] = Lo[k+1] Dinv_k  (and Rw[k] = Rw[k] Dinv_k);
// phase 1: updates of the blocks in rows {k+1, K} x columns {k+1, K}.
// q = product (0..3); one workgroup.
__device__ void cz_elim_part(const CoarseDesc& d, int k, int phase, int q, double* __restrict__ Fp,
                             double (*AsT)[GJ_NB + 2], double (*Bs)[GJ_NB + 2]) {
    const int K = d.nx - 1;
    if (k >= K || d.n < 2) return;
    const bool arrow = d.periodic && d.nx >= 3;
    const int b = d.ny;
    const double *A = nullptr, *Bm = nullptr;
    double* C = nullptr;
    int mode = 1;
    if (k + 1 < K) {
        if (phase == 0) {
            if (q == 0) { A = cz_blk(Fp, d, 2, k + 1); Bm = cz_blk(Fp, d, 0, k); C = cz_blk(Fp, d, 2, k + 1); mode = 0; }
            else if (q == 1 && arrow) { A = cz_blk(Fp, d, 4, k); Bm = cz_blk(Fp, d, 0, k); C = cz_blk(Fp, d, 4, k); mode = 0; }
        } else {
            if (q == 0) { A = cz_blk(Fp, d, 2, k + 1); Bm = cz_blk(Fp, d, 1, k); C = cz_blk(Fp, d, 0, k + 1); }
            else if (arrow && q == 1) {
                A = cz_blk(Fp, d, 2, k + 1); Bm = cz_blk(Fp, d, 3, k);
                C = (k + 1 < K - 1) ? cz_blk(Fp, d, 3, k + 1) : cz_blk(Fp, d, 1, k + 1);
            } else if (arrow && q == 2) {
                A = cz_blk(Fp, d, 4, k); Bm = cz_blk(Fp, d, 1, k);
                C = (k + 1 < K - 1) ? cz_blk(Fp, d, 4, k + 1) : cz_blk(Fp, d, 2, K);
            } else if (arrow && q == 3) {
                A = cz_blk(Fp, d, 4, k); Bm = cz_blk(Fp, d, 3, k); C = cz_blk(Fp, d, 0, K);
            }
        }
    } else {   // k + 1 == K: row K is row k + 1
        if (phase == 0 && q == 0) { A = cz_blk(Fp, d, 2, K); Bm = cz_blk(Fp, d, 0, k); C = cz_blk(Fp, d, 2, K); mode = 0; }
        if (phase == 1 && q == 0) { A = cz_blk(Fp, d, 2, K); Bm = cz_blk(Fp, d, 1, k); C = cz_blk(Fp, d, 0, K); }
    }
    if (!C) return;
    cz_gemm(b, A, Bm, C, mode, AsT, Bs);
}

// Multipliers of step k for the periodic (arrow) chains only (grid (2, nch)):
// Lo_{k+1} = Lo_{k+1} Dinv_k and Rw_k = Rw_k Dinv_k.  The other chains get
// theirs inside k_cz_lu_step.
__global__ void __launch_bounds__(BAMG_BLK)
k_cz_elim_arrow(const CoarseDesc* __restrict__ cd, int k, double* __restrict__ Fp) {
    __shared__ double AsT[GJ_NB][GJ_NB + 2];
    __shared__ double Bs[GJ_NB][GJ_NB + 2];
    const CoarseDesc d = cd[blockIdx.y];
    if (!(d.periodic && d.nx >= 3)) return;
    cz_elim_part(d, k, 0, blockIdx.x, Fp, AsT, Bs);
}

// Step k of the block LU for every chain with the periodic arrow (k < 0:
// the chain's last block K), grid (4, nch); the other chains take the
// twisted factorisation.  Workgroup 0 forms D_k - Lo_k Up_{k-1} (the update
// of step k-1, summed as cz_gemm does) in the Gauss-Jordan registers,
// inverts it and stores Dinv_k; workgroups 1..3 do the other updates of step
// k-1, which touch none of the blocks workgroup 0 reads or writes, and the
// multipliers follow in k_cz_elim_arrow.  One launch per block row instead
// of three.
// Columns t of row j of a block that couples two grid rows of the coarsest
// level (3 x 3 box: |t - j| <= 1, wrapping on periodic grids), in ascending
// order, -1 for none.  Such blocks (Lo, Up) are banded, so a product with
// them takes 3 terms per entry.
__device__ __forceinline__ void cz_band(int j, int b, int periodic, int (&t)[3]) {
    int a0 = j - 1, a1 = j, a2 = j + 1;
    if (periodic && b >= 3) {
        if (a0 < 0) a0 += b;
        if (a2 >= b) a2 -= b;
        // ascending: the wrapped neighbour moves to the other end
        if (j == 0) { t[0] = a1; t[1] = a2; t[2] = a0; return; }
        if (j == b - 1) { t[0] = a2; t[1] = a0; t[2] = a1; return; }
    } else {
        if (a0 < 0) a0 = -1;
        if (a2 >= b) a2 = -1;
    }
    t[0] = a0; t[1] = a1; t[2] = a2;
}

__global__ void __launch_bounds__(BAMG_BLK)
k_cz_lu_step(const CoarseDesc* __restrict__ cd, int k, double* __restrict__ Fp, const double* __restrict__ scale,
             double* __restrict__ minpiv) {
    static_assert(CZ_GJ_THREADS == BAMG_BLK, "one workgroup size for both parts");
    __shared__ double lds[2 * GJ_NB * (GJ_NB + 2)];
    __shared__ __align__(16) double prow[2][2][GJ_NB];
    const CoarseDesc d = cd[blockIdx.y];
    const int K = d.nx - 1, q = blockIdx.x;
    const int kk = k < 0 ? K : k;
    if (d.n < 2 || (k >= 0 && k >= K)) return;
    if (!(d.periodic && d.nx >= 3)) return;  // inverted by divide and conquer (k_dc_*)
    if (q > 0) {
        if (kk >= 1)
            cz_elim_part(d, kk - 1, 1, q, Fp, (double(*)[GJ_NB + 2])lds, (double(*)[GJ_NB + 2])(lds + GJ_NB * (GJ_NB + 2)));
        return;
    }
    double (*Bs)[GJ_NB + 2] = (double(*)[GJ_NB + 2])(lds + GJ_NB * (GJ_NB + 2));
    const int b = d.ny, tid = threadIdx.x;
    const int c = tid % BAMG_WAVE, w = tid / BAMG_WAVE;
    double* D = cz_blk(Fp, d, 0, kk);
    double Dv[CZ_GJ_ROWS];
#pragma unroll
    for (int i = 0; i < CZ_GJ_ROWS; ++i) {
        const int r = CZ_GJ_ROWS * w + i;
        Dv[i] = (r < b && c < b) ? D[r * b + c] : 0.0;
    }
    double S[CZ_GJ_ROWS];
    if (kk >= 1) {
        // the arrow elimination fills the block that couples the last two
        // grid rows, so the product stays dense (4 x 4 tiles, then through
        // LDS into this thread's column strip)
        double (*AsT)[GJ_NB + 2] = (double(*)[GJ_NB + 2])lds;
        const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
        cz_stage(b, cz_blk(Fp, d, 2, kk), AsT, cz_blk(Fp, d, 1, kk - 1), Bs);
        __syncthreads();
        double acc[4][4];
        cz_tile(b, AsT, Bs, tr, tc, acc);
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) AsT[tr + a][tc + q4] = acc[a][q4];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < CZ_GJ_ROWS; ++i) {
            const int r = CZ_GJ_ROWS * w + i;
            S[i] = (r < b && c < b) ? Dv[i] - AsT[r][c] : (r == c ? 1.0 : 0.0);
        }
    } else {
#pragma unroll
        for (int i = 0; i < CZ_GJ_ROWS; ++i) {
            const int r = CZ_GJ_ROWS * w + i;
            S[i] = (r < b && c < b) ? Dv[i] : (r == c ? 1.0 : 0.0);
        }
    }
    double mp = 1e300;
    cz_gj(S, w, c, b, scale[blockIdx.y], mp, prow);
#pragma unroll
    for (int i = 0; i < CZ_GJ_ROWS; ++i) {
        const int r = CZ_GJ_ROWS * w + i;
        if (r < b && c < b) D[r * b + c] = S[i];
    }
    if (tid == 0) minpiv[blockIdx.y] = fmin(minpiv[blockIdx.y], mp);
}

// All substitution steps of W = (L U)^-1 for a chain with the arrow (the
// others take the divide and conquer below), for one tile of CZ_SUB_TC columns
// of one chain per workgroup (grid (ceil(n / CZ_SUB_TC), nch)): the columns of
// W are independent right-hand sides (the identity), so a workgroup walks
// every block row on its own, with the previous block row of the solution
// kept in LDS.
//   forward:  Y_0 = I_0;  Y_s = I_s - Lo_s Y_{s-1}  (s < K);
//             Y_K = I_K - sum_{j < K-1} Rw_j Y_j - Lo_K Y_{K-1}  (the arrow
//             terms), in that order;
//   backward: X_K = Dinv_K Y_K;
//             X_k = Dinv_k (Y_k - Up_k X_{k+1} - Cl_k X_K)  (k = K-1 .. 0).
// Lo_s and Rw_j hold the multipliers (already times Dinv), Dk the inverted
// diagonal blocks of the LU; every product adds over t in ascending order.
// Block rows above the tile's first identity block s0 have Y_s = 0: they are
// stored as zeros and take no products.  Thread t keeps rows 4 (t / 16) ..
// + 3 of column t % 16 of the tile.
#define CZ_SUB_TC 16
__device__ __forceinline__ void cz_ident(int blk, int b, int c0, int w, int tr, int tc, double X[4]) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int r = tr + a;
        X[a] = (r < b && tc < w && blk * b + r == c0 + tc) ? 1.0 : 0.0;
    }
}

// acc (+)= sign Ms[rows tr.., 0:b] * Xs[0:b, column tc]
__device__ __forceinline__ void cz_mac(int b, const double (*Ms)[GJ_NB + 1], const double (*Xs)[CZ_SUB_TC + 1],
                                       int tr, int tc, double acc[4], double sign) {
    for (int t = 0; t < b; ++t) {
        const double xv = sign * Xs[t][tc];
#pragma unroll
        for (int a = 0; a < 4; ++a) acc[a] += Ms[tr + a][t] * xv;
    }
}

__device__ __forceinline__ void cz_put(const double X[4], double (*Xs)[CZ_SUB_TC + 1], int tr, int tc) {
#pragma unroll
    for (int a = 0; a < 4; ++a) Xs[tr + a][tc] = X[a];
}

// The blocks a substitution workgroup of a chain with the arrow multiplies
// by, in the order it uses them (index part * nx + k into the chain's block
// storage), for a tile whose first identity block is s0.
__device__ int cz_subst_sequence(int K, int s0, int* seq) {
    int m = 0;
    for (int s = s0; s < K; ++s) {
        if (s > s0) seq[m++] = 2 * (K + 1) + s;               // Lo_s
        if (s < K - 1) seq[m++] = 4 * (K + 1) + s;            // Rw_s
        if (s == K - 1) seq[m++] = 2 * (K + 1) + K;           // Lo_K
    }
    seq[m++] = K;                                              // Dinv_K
    for (int k = K - 1; k >= 0; --k) {
        seq[m++] = (K + 1) + k;                                // Up_k
        if (k < K - 1) seq[m++] = 3 * (K + 1) + k;            // Cl_k
        seq[m++] = k;                                          // Dinv_k
    }
    return m;
}

__global__ void __launch_bounds__(BAMG_BLK)
k_cz_subst(const CoarseDesc* __restrict__ cd, double* __restrict__ Wp, const double* __restrict__ Fp) {
    __shared__ double Ms[GJ_NB][GJ_NB + 1];
    __shared__ double Xs[GJ_NB][CZ_SUB_TC + 1];
    __shared__ double Ks[GJ_NB][CZ_SUB_TC + 1];
    __shared__ int seq[5 * CZ_MAX_NX + 8];
    __shared__ int nseq;
    const CoarseDesc d = cd[blockIdx.y];
    const int K = d.nx - 1, b = d.ny, n = d.n;
    const int c0 = blockIdx.x * CZ_SUB_TC;
    if (n < 2 || c0 >= n) return;
    const bool arrow = d.periodic && d.nx >= 3;
    if (!arrow) return;                              // k_dc_* invert those chains
    const double* F = Fp + d.boff;
    double* W = Wp + d.woff;
    const int w = min(CZ_SUB_TC, n - c0);
    const int s0 = c0 / b;
    const int tid = threadIdx.x, tr = (tid / CZ_SUB_TC) * 4, tc = tid % CZ_SUB_TC;
    const long long bb = (long long)b * b;
    if (tid == 0) nseq = cz_subst_sequence(K, s0, seq);
    __syncthreads();
    // The next block of the sequence is loaded into registers while the
    // current one is in use; next_block() moves it to Ms (the caller has
    // synchronised) and starts loading the one after.
    double pre[GJ_NB * GJ_NB / BAMG_BLK];
    int sidx = 0;
    auto fetch = [&](int i) {
        const double* M = F + (long long)seq[i] * bb;
#pragma unroll
        for (int q = 0; q < GJ_NB * GJ_NB / BAMG_BLK; ++q) {
            const int e = tid + q * BAMG_BLK, r = e / GJ_NB, c = e % GJ_NB;
            pre[q] = (r < b && c < b) ? M[r * b + c] : 0.0;
        }
    };
    auto next_block = [&]() {
#pragma unroll
        for (int q = 0; q < GJ_NB * GJ_NB / BAMG_BLK; ++q) {
            const int e = tid + q * BAMG_BLK;
            Ms[e / GJ_NB][e % GJ_NB] = pre[q];
        }
        if (++sidx < nseq) fetch(sidx);
    };
    fetch(0);
    auto store = [&](int blk, const double X[4]) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int r = tr + a;
            if (r < b && tc < w) W[(size_t)(blk * b + r) * n + c0 + tc] = X[a];
        }
    };
    double T[4], TK[4];
    cz_ident(K, b, c0, w, tr, tc, TK);
    // forward substitution (L has unit diagonal blocks)
#pragma unroll
    for (int a = 0; a < 4; ++a) T[a] = 0.0;
    for (int s = 0; s < min(s0, K); ++s) store(s, T);
    for (int s = s0; s < K; ++s) {
        cz_ident(s, b, c0, w, tr, tc, T);
        if (s > s0) {                                // Xs holds Y_{s-1}
            __syncthreads();
            next_block();                            // Lo_s
            __syncthreads();
            cz_mac(b, Ms, Xs, tr, tc, T, -1.0);
        }
        __syncthreads();
        cz_put(T, Xs, tr, tc);
        store(s, T);
        if (s < K - 1) {
            next_block();                            // Rw_s
            __syncthreads();
            cz_mac(b, Ms, Xs, tr, tc, TK, -1.0);
        }
        if (s == K - 1) {
            __syncthreads();
            next_block();                            // Lo_K
            __syncthreads();
            cz_mac(b, Ms, Xs, tr, tc, TK, -1.0);
        }
    }
    // X_K = Dinv_K Y_K, kept in Ks for the arrow terms
    __syncthreads();
    next_block();                                    // Dinv_K
    cz_put(TK, Xs, tr, tc);
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a) T[a] = 0.0;
    cz_mac(b, Ms, Xs, tr, tc, T, 1.0);
    store(K, T);
    __syncthreads();
    cz_put(T, Ks, tr, tc);
    cz_put(T, Xs, tr, tc);                           // X_{k+1} for k = K-1
    // backward substitution
    for (int k = K - 1; k >= 0; --k) {
        double U[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int r = tr + a;
            U[a] = (r < b && tc < w) ? W[(size_t)(k * b + r) * n + c0 + tc] : 0.0;
        }
        __syncthreads();
        next_block();                                // Up_k
        __syncthreads();
        cz_mac(b, Ms, Xs, tr, tc, U, -1.0);
        if (k < K - 1) {
            __syncthreads();
            next_block();                            // Cl_k
            __syncthreads();
            cz_mac(b, Ms, Ks, tr, tc, U, -1.0);
        }
        __syncthreads();
        next_block();                                // Dinv_k
        cz_put(U, Xs, tr, tc);
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 4; ++a) T[a] = 0.0;
        cz_mac(b, Ms, Xs, tr, tc, T, 1.0);
        store(k, T);
        __syncthreads();
        cz_put(T, Xs, tr, tc);
    }
}

// ---------------------------------------------------------------- divide and conquer
// Inverse of the block tridiagonal operator of a chain without the arrow by
// divide and conquer over its block rows.  The leaves are the diagonal
// blocks, W[k, k] = D_k^-1.  Level t joins the segment X = [a, m), m = a +
// 2^t (a a multiple of 2^(t+1)), with Y = [m, e), e = min(a + 2^(t+1), nx),
// whose inverses Xi and Yi are in place in W.  X and Y are coupled only by
// E = U_{m-1} (block (m-1, m)) and F = L_m (block (m, m-1)), so the Schur
// complement Y - F Xi E differs from Y in its first block alone:
//   C = L_m Xi[m-1, m-1] U_{m-1},  G = Yi[m, m],  K = (I - C G)^-1 C
// (the Woodbury formula: its inverse is Yi + Yi[:, m] K Yi[m, :]).  With the
// block column P1 = Xi[:, m-1] U_{m-1}, the block row R1 = L_m Xi[m-1, :],
// P2 = Yi[:, m] and R2 = Yi[m, :], the inverse of the joined segment is
//   [[Xi + P1 (G + G K G) R1,  -P1 (I + G K) R2],
//    [-P2 (I + K G) R1,         Yi + P2 K R2    ]].
// The chain of dependent inversions is 1 + ceil(log2 nx) long (a leaf, then
// one I - C G per level) instead of the nx block rows of an elimination.
// Three launches per level: k_dc_core (C, G, K per join, one workgroup),
// k_dc_panels (per block row: the left panels P1 (G + G K G), -P1 (I + G K),
// -P2 (I + K G), P2 K and the right panels R1, R2) and k_dc_tiles (each b x b
// tile of a joined segment: W = (W or 0) + left panel rows x right panel
// columns).  Dense 64 x 64 products run on the FP64 matrix cores; the
// banded U and L take their band terms in ascending order.  Smallest pivots:
// the leaves' relative to max |B_L| and the joins' I - C G (dimensionless)
// into dmp[chain DC_MP + k] and [chain DC_MP + nx + m].
#define DC_MP (2 * CZ_MAX_NX)

__device__ __forceinline__ bool dc_plain(const CoarseDesc& d) { return d.n >= 2 && !(d.periodic && d.nx >= 3); }

// The join q of level t: X = [a, m), Y = [m, e); false when Y is empty.
struct DcJoin { int a, m, e; };
__device__ __forceinline__ bool dc_join(int nx, int t, int q, DcJoin& g) {
    g.a = q << (t + 1);
    g.m = g.a + (1 << t);
    g.e = min(g.a + (2 << t), nx);
    return g.m < nx;
}

// acc[cb] (+)= A[16 wv + rows, 0:64] B[0:64, 16 cb + columns], cb = 0..3, by
// v_mfma_f64_16x16x4f64 in ascending k: lane l, register q of acc[cb] holds
// row 16 wv + l / 16 + 4 q, column 16 cb + l % 16 (the layout the
// instruction returns; its operands: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16] of the 16 x 4 and 4 x 16 blocks).
typedef double dc_d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void dc_mfma(const double (*A)[GJ_NB + 1], const double (*B)[GJ_NB + 1], int wv, int lane,
                                        dc_d4 (&acc)[4]) {
    const int ar = 16 * wv + lane % 16, kq = lane / 16, bc = lane % 16;
#pragma unroll
    for (int kk = 0; kk < GJ_NB / 4; ++kk) {
        const double av = A[ar][4 * kk + kq];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
            acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, B[4 * kk + kq][16 * cb + bc], acc[cb], 0, 0, 0);
    }
}
__device__ __forceinline__ void dc_zero(dc_d4 (&acc)[4]) {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = dc_d4{0.0, 0.0, 0.0, 0.0};
}
__device__ __forceinline__ int dc_row(int wv, int lane, int q) { return 16 * wv + lane / 16 + 4 * q; }
__device__ __forceinline__ int dc_col(int lane, int cb) { return 16 * cb + lane % 16; }

// Stage two 64 x 64 matrices into LDS, entry (r, c) from f1(r, c) and
// f2(r, c): every load of a thread is issued before its LDS stores.
template <typename F1, typename F2>
__device__ __forceinline__ void dc_stage2(double (*D1)[GJ_NB + 1], F1 f1, double (*D2)[GJ_NB + 1], F2 f2) {
    constexpr int Q = GJ_NB * GJ_NB / BAMG_BLK;
    double v1[Q], v2[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e = threadIdx.x + q * BAMG_BLK;
        v1[q] = f1(e / GJ_NB, e % GJ_NB);
        v2[q] = f2(e / GJ_NB, e % GJ_NB);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e = threadIdx.x + q * BAMG_BLK;
        D1[e / GJ_NB][e % GJ_NB] = v1[q];
        D2[e / GJ_NB][e % GJ_NB] = v2[q];
    }
}

// acc (dc_mfma layout) += A B for 64 x 64 operands A (entry (r, k) from
// fa(r, k)) and B (entry (k, c) from fb(k, c)), k ascending as in dc_mfma.
// The operands pass through LDS in chunks of DC_KC values of k (17 KB for
// both), each chunk's loads issued while the previous chunk's products run,
// so that several workgroups share a CU.
#define DC_KC 16
template <typename FA, typename FB>
__device__ __forceinline__ void dc_rank64(FA fa, FB fb, double (*As)[DC_KC + 1], double (*Bs)[GJ_NB + 1], int wv,
                                          int lane, dc_d4 (&acc)[4]) {
    constexpr int NQ = GJ_NB * DC_KC / BAMG_BLK;
    double ra[NQ], rb[NQ];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = threadIdx.x + q * BAMG_BLK;
            ra[q] = fa(e / DC_KC, k0 + e % DC_KC);
            rb[q] = fb(k0 + e / GJ_NB, e % GJ_NB);
        }
    };
    load(0);
    const int ar = 16 * wv + lane % 16, kq = lane / 16, bc = lane % 16;
    for (int k0 = 0; k0 < GJ_NB; k0 += DC_KC) {
        __syncthreads();                        // the previous chunk's products are done
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = threadIdx.x + q * BAMG_BLK;
            As[e / DC_KC][e % DC_KC] = ra[q];
            Bs[e / GJ_NB][e % GJ_NB] = rb[q];
        }
        __syncthreads();
        if (k0 + DC_KC < GJ_NB) load(k0 + DC_KC);
#pragma unroll
        for (int kk = 0; kk < DC_KC / 4; ++kk) {
            const double av = As[ar][4 * kk + kq];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Bs[4 * kk + kq][16 * cb + bc], acc[cb], 0, 0, 0);
        }
    }
}

// Leaves: W[k, k] = D_k^-1 (grid (block rows, chains)).
__global__ void __launch_bounds__(BAMG_BLK)
k_dc_leaf(const CoarseDesc* __restrict__ cd, double* __restrict__ Fp, double* __restrict__ Wp,
          const double* __restrict__ scale, double* __restrict__ dmp) {
    static_assert(CZ_GJ_THREADS == BAMG_BLK, "one Gauss-Jordan block per workgroup");
    __shared__ __align__(16) double prow[2][2][GJ_NB];
    const int ch = blockIdx.y, k = blockIdx.x;
    const CoarseDesc d = cd[ch];
    if (!dc_plain(d) || k >= d.nx) return;
    const int b = d.ny, n = d.n, c = threadIdx.x % BAMG_WAVE, w = threadIdx.x / BAMG_WAVE;
    const double* D = cz_blk(Fp, d, 0, k);
    double S[CZ_GJ_ROWS];
#pragma unroll
    for (int i = 0; i < CZ_GJ_ROWS; ++i) {
        const int r = CZ_GJ_ROWS * w + i;
        S[i] = (r < b && c < b) ? D[r * b + c] : (r == c ? 1.0 : 0.0);
    }
    double mp = 1e300;
    cz_gj(S, w, c, b, scale[ch], mp, prow);
    double* W = Wp + d.woff;
#pragma unroll
    for (int i = 0; i < CZ_GJ_ROWS; ++i) {
        const int r = CZ_GJ_ROWS * w + i;
        if (r < b && c < b) W[(size_t)(k * b + r) * n + k * b + c] = S[i];
    }
    if (threadIdx.x == 0) dmp[(size_t)ch * DC_MP + k] = mp;
}

// One join of level t per workgroup (grid (joins, chains)): C, G and
// K = (I - C G)^-1 C into block slots 3 and 4 of the join's index (free on
// chains without the arrow).
__global__ void __launch_bounds__(BAMG_BLK)
k_dc_core(const CoarseDesc* __restrict__ cd, int t, double* __restrict__ Fp, const double* __restrict__ Wp,
          double* __restrict__ dmp) {
    __shared__ double Xs[GJ_NB][GJ_NB + 1];     // Xi[m-1, m-1], then X U, then I - C G, then its inverse
    __shared__ double Gs[GJ_NB][GJ_NB + 1];
    __shared__ double Cs[GJ_NB][GJ_NB + 1];
    __shared__ __align__(16) double prow[2][2][GJ_NB];
    const int ch = blockIdx.y;
    const CoarseDesc d = cd[ch];
    DcJoin g;
    if (!dc_plain(d) || !dc_join(d.nx, t, blockIdx.x, g)) return;
    const int b = d.ny, n = d.n, tid = threadIdx.x, c = tid % BAMG_WAVE, w = tid / BAMG_WAVE;
    const double* W = Wp + d.woff;
    const int x0 = (g.m - 1) * b, y0 = g.m * b;
    const double* U = cz_blk(Fp, d, 1, g.m - 1);
    const double* L = cz_blk(Fp, d, 2, g.m);
    int tc[3];
    cz_band(c, b, d.periodic, tc);
    double uc[3];
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) uc[sl] = (c < b && tc[sl] >= 0) ? U[tc[sl] * b + c] : 0.0;
    dc_stage2(
        Xs, [&](int r, int cc) { return (r < b && cc < b) ? W[(size_t)(x0 + r) * n + x0 + cc] : 0.0; },
        Gs, [&](int r, int cc) { return (r < b && cc < b) ? W[(size_t)(y0 + r) * n + y0 + cc] : 0.0; });
    __syncthreads();
    // X U: column c of U holds its band rows tc
    double T[CZ_GJ_ROWS];
#pragma unroll
    for (int i = 0; i < CZ_GJ_ROWS; ++i) {
        const int r = CZ_GJ_ROWS * w + i;
        double acc = 0.0;
#pragma unroll
        for (int sl = 0; sl < 3; ++sl)
            if (tc[sl] >= 0) acc = fma(Xs[r][tc[sl]], uc[sl], acc);
        T[i] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CZ_GJ_ROWS; ++i) Xs[CZ_GJ_ROWS * w + i][c] = T[i];
    __syncthreads();
    // C = L (X U): row r of L holds its band columns
#pragma unroll
    for (int i = 0; i < CZ_GJ_ROWS; ++i) {
        const int r = CZ_GJ_ROWS * w + i;
        int tr[3];
        cz_band(r, b, d.periodic, tr);
        double acc = 0.0;
        if (r < b) {
#pragma unroll
            for (int sl = 0; sl < 3; ++sl)
                if (tr[sl] >= 0) acc = fma(L[r * b + tr[sl]], Xs[tr[sl]][c], acc);
        }
        Cs[r][c] = acc;
    }
    __syncthreads();
    // I - C G (the identity beyond b: C and G are zero there)
    dc_d4 acc[4];
    dc_zero(acc);
    dc_mfma(Cs, Gs, w, c, acc);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = dc_row(w, c, q), col = dc_col(c, cb);
            Xs[row][col] = (row == col ? 1.0 : 0.0) - acc[cb][q];
        }
    __syncthreads();
    double S[CZ_GJ_ROWS];
#pragma unroll
    for (int i = 0; i < CZ_GJ_ROWS; ++i) S[i] = Xs[CZ_GJ_ROWS * w + i][c];
    double mp = 1e300;
    cz_gj(S, w, c, b, 1.0, mp, prow);
#pragma unroll
    for (int i = 0; i < CZ_GJ_ROWS; ++i) Xs[CZ_GJ_ROWS * w + i][c] = S[i];
    __syncthreads();
    dc_zero(acc);
    dc_mfma(Xs, Cs, w, c, acc);                 // K = (I - C G)^-1 C
    double* Ko = cz_blk(Fp, d, 3, blockIdx.x);
    double* Go = cz_blk(Fp, d, 4, blockIdx.x);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = dc_row(w, c, q), col = dc_col(c, cb);
            if (row < b && col < b) Ko[row * b + col] = acc[cb][q];
        }
    for (int e = tid; e < b * b; e += BAMG_BLK) Go[e] = Gs[e / b][e % b];
    if (tid == 0) dmp[(size_t)ch * DC_MP + d.nx + g.m] = mp;
}

// The panels of level t for one block row k of a joined segment (grid
// (block rows, chains)).  Left panels, row i of the chain at
// Pp[(voff + i) 2 GJ_NB + side GJ_NB + s] for the X columns (side 0) and the
// Y columns (side 1); right panels at Rp[s rld + voff + j] for column j.
__global__ void __launch_bounds__(BAMG_BLK)
k_dc_panels(const CoarseDesc* __restrict__ cd, int t, double* __restrict__ Fp, const double* __restrict__ Wp,
            double* __restrict__ Pp, double* __restrict__ Rp, int rld) {
    __shared__ double Gs[GJ_NB][GJ_NB + 1];
    __shared__ double Ks[GJ_NB][GJ_NB + 1];
    __shared__ double As[GJ_NB][GJ_NB + 1];     // P1 or P2 rows, then P1 G K
    __shared__ double Qs[GJ_NB][GJ_NB + 1];     // P1 G or P2 K
    const int ch = blockIdx.y, k = blockIdx.x;
    const CoarseDesc d = cd[ch];
    DcJoin g;
    if (!dc_plain(d) || k >= d.nx || !dc_join(d.nx, t, k >> (t + 1), g)) return;
    const bool xside = k < g.m;
    const int b = d.ny, n = d.n, tid = threadIdx.x, c = tid % BAMG_WAVE, w = tid / BAMG_WAVE;
    const double* W = Wp + d.woff;
    const double* Kq = cz_blk(Fp, d, 3, k >> (t + 1));
    const double* Gq = cz_blk(Fp, d, 4, k >> (t + 1));
    dc_stage2(Gs, [&](int r, int cc) { return (r < b && cc < b) ? Gq[r * b + cc] : 0.0; },
              Ks, [&](int r, int cc) { return (r < b && cc < b) ? Kq[r * b + cc] : 0.0; });
    const int r0 = k * b;
    if (xside) {
        // P1 = Xi[rows, m-1] U_{m-1}; R1 = L_m Xi[m-1, columns]
        const double* U = cz_blk(Fp, d, 1, g.m - 1);
        const double* L = cz_blk(Fp, d, 2, g.m);
        const int x0 = (g.m - 1) * b;
        int tc[3];
        cz_band(c, b, d.periodic, tc);
        double uc[3];
#pragma unroll
        for (int sl = 0; sl < 3; ++sl) uc[sl] = (c < b && tc[sl] >= 0) ? U[tc[sl] * b + c] : 0.0;
        // every load of the thread first, then the band sums
        // (column r0 + c of Xi's block row m - 1 at the band rows of L's row r)
        double wr[CZ_GJ_ROWS][3], lr[CZ_GJ_ROWS][3], wl[CZ_GJ_ROWS][3];
        int ts[CZ_GJ_ROWS][3];
#pragma unroll
        for (int i = 0; i < CZ_GJ_ROWS; ++i) {
            const int r = CZ_GJ_ROWS * w + i;
            cz_band(r, b, d.periodic, ts[i]);
#pragma unroll
            for (int sl = 0; sl < 3; ++sl) {
                const bool tin = r < b && c < b && tc[sl] >= 0, sin = r < b && c < b && ts[i][sl] >= 0;
                wr[i][sl] = tin ? W[(size_t)(r0 + r) * n + x0 + tc[sl]] : 0.0;
                lr[i][sl] = sin ? L[r * b + ts[i][sl]] : 0.0;
                wl[i][sl] = sin ? W[(size_t)(x0 + ts[i][sl]) * n + r0 + c] : 0.0;
            }
        }
#pragma unroll
        for (int i = 0; i < CZ_GJ_ROWS; ++i) {
            const int r = CZ_GJ_ROWS * w + i;
            double acc = 0.0, acr = 0.0;
#pragma unroll
            for (int sl = 0; sl < 3; ++sl) {
                if (tc[sl] >= 0) acc = fma(wr[i][sl], uc[sl], acc);
                if (ts[i][sl] >= 0) acr = fma(lr[i][sl], wl[i][sl], acr);
            }
            As[r][c] = acc;
            if (c < b) Rp[(size_t)r * rld + d.voff + r0 + c] = acr;
        }
    } else {
        // P2 = Yi[rows, m]; R2 = Yi[m, columns]
        const int y0 = g.m * b;
        double pr[CZ_GJ_ROWS], rr[CZ_GJ_ROWS];
#pragma unroll
        for (int i = 0; i < CZ_GJ_ROWS; ++i) {
            const int r = CZ_GJ_ROWS * w + i;
            pr[i] = (r < b && c < b) ? W[(size_t)(r0 + r) * n + y0 + c] : 0.0;
            rr[i] = (r < b && c < b) ? W[(size_t)(y0 + r) * n + r0 + c] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < CZ_GJ_ROWS; ++i) {
            const int r = CZ_GJ_ROWS * w + i;
            As[r][c] = pr[i];
            if (c < b) Rp[(size_t)r * rld + d.voff + r0 + c] = rr[i];
        }
    }
    __syncthreads();
    double* P = Pp + (size_t)(d.voff + r0) * (2 * GJ_NB);
    dc_d4 a1[4], a2[4];
    dc_zero(a1);
    dc_zero(a2);
    if (xside) {
        dc_mfma(As, Gs, w, c, a1);              // P1 G
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) Qs[dc_row(w, c, q)][dc_col(c, cb)] = a1[cb][q];
        __syncthreads();
        dc_mfma(Qs, Ks, w, c, a2);              // P1 G K
        // -P1 (I + G K) for the Y columns
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = dc_row(w, c, q), col = dc_col(c, cb);
                if (row < b) P[(size_t)row * 2 * GJ_NB + GJ_NB + col] = -(As[row][col] + a2[cb][q]);
            }
        __syncthreads();
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) As[dc_row(w, c, q)][dc_col(c, cb)] = a2[cb][q];
        __syncthreads();
        dc_zero(a1);
        dc_mfma(As, Gs, w, c, a1);              // P1 G K G
        // P1 (G + G K G) for the X columns
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = dc_row(w, c, q), col = dc_col(c, cb);
                if (row < b) P[(size_t)row * 2 * GJ_NB + col] = Qs[row][col] + a1[cb][q];
            }
    } else {
        dc_mfma(As, Ks, w, c, a1);              // P2 K for the Y columns
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = dc_row(w, c, q), col = dc_col(c, cb);
                Qs[row][col] = a1[cb][q];
                if (row < b) P[(size_t)row * 2 * GJ_NB + GJ_NB + col] = a1[cb][q];
            }
        __syncthreads();
        dc_mfma(Qs, Gs, w, c, a2);              // P2 K G
        // -P2 (I + K G) for the X columns
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = dc_row(w, c, q), col = dc_col(c, cb);
                if (row < b) P[(size_t)row * 2 * GJ_NB + col] = -(As[row][col] + a2[cb][q]);
            }
    }
}

// The tiles of level t: grid (joins S^2, chains) with S = min(2^(t+1), nx);
// tile (I, J) of join q: W[I, J] = (W[I, J] if I and J are on the same side,
// else 0) + left panel rows of I for J's side times the right panel columns
// of J.
__global__ void __launch_bounds__(BAMG_BLK)
k_dc_tiles(const CoarseDesc* __restrict__ cd, int t, const double* __restrict__ Pp, const double* __restrict__ Rp,
           int rld, double* __restrict__ Wp) {
    __shared__ double As[GJ_NB][DC_KC + 1];
    __shared__ double Bs[DC_KC][GJ_NB + 1];
    const CoarseDesc d = cd[blockIdx.y];
    if (!dc_plain(d)) return;
    const int S = min(2 << t, d.nx);
    const int q = blockIdx.x / (S * S), loc = blockIdx.x % (S * S);
    DcJoin g;
    if (!dc_join(d.nx, t, q, g)) return;
    const int I = g.a + loc / S, J = g.a + loc % S;
    if (I >= g.e || J >= g.e) return;
    const int side = J >= g.m ? 1 : 0;
    const bool same = (I >= g.m ? 1 : 0) == side;
    const int b = d.ny, n = d.n, tid = threadIdx.x, c = tid % BAMG_WAVE, w = tid / BAMG_WAVE;
    const double* P = Pp + (size_t)(d.voff + I * b) * (2 * GJ_NB) + side * GJ_NB;
    double* W = Wp + d.woff + (size_t)(I * b) * n + J * b;
    // the accumulators start from the tile's current entries (same side)
    dc_d4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2) {
            const int row = dc_row(w, c, q2), col = dc_col(c, cb);
            acc[cb][q2] = (same && row < b && col < b) ? W[(size_t)row * n + col] : 0.0;
        }
    dc_rank64([&](int r, int k) { return r < b ? P[(size_t)r * 2 * GJ_NB + k] : 0.0; },
              [&](int k, int cc) { return (k < b && cc < b) ? Rp[(size_t)k * rld + d.voff + J * b + cc] : 0.0; },
              As, Bs, w, c, acc);
#pragma unroll
    for (int q2 = 0; q2 < 4; ++q2)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int row = dc_row(w, c, q2), col = dc_col(c, cb);
            if (row < b && col < b) W[(size_t)row * n + col] = acc[cb][q2];
        }
}

// minpiv[chain] = min(minpiv, the leaves' and joins' smallest pivots); one
// wavefront per chain.
__global__ void k_dc_minpiv(const CoarseDesc* __restrict__ cd, const double* __restrict__ dmp,
                            double* __restrict__ minpiv) {
    const CoarseDesc d = cd[blockIdx.x];
    if (!dc_plain(d)) return;
    double v = 1e300;
    for (int i = threadIdx.x; i < 2 * d.nx; i += BAMG_WAVE)
        if (i != d.nx) v = fmin(v, dmp[(size_t)blockIdx.x * DC_MP + i]);
#pragma unroll
    for (int o = BAMG_WAVE / 2; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, BAMG_WAVE));
    if (threadIdx.x == 0) minpiv[blockIdx.x] = fmin(minpiv[blockIdx.x], v);
}

// ---------------------------------------------------------------- bordered grids
// A coarsest grid (not periodic) whose rows hold GJ_NB + 1 points, with at
// most GJ_NB + 1 rows, is split into its first GJ_NB columns (the main part:
// block tridiagonal with GJ_NB x GJ_NB blocks, inverted by the block path
// above into Am) and its last column (the border: nx - 1 points; the last
// point of the grid is the padded unknown).  With the padded operator
// K = [[A, E], [F, D]] (main part first, then the border), Z = A^-1 E,
// Y = F A^-1, the Schur complement S = D - F Z and G = Z S^-1, H = S^-1 Y:
//   K^-1 = [[A^-1 + G Y, -G], [-H, S^-1]].
// S is a nonsingular M-matrix as K is (no pivoting).  In the 3x3 box a
// border point (e, GJ_NB) couples with the main part only through column
// GJ_NB - 1 of grid rows e - 1 .. e + 1, so a column of Z and a row of Y are
// sums of at most three columns / rows of A^-1 (in ascending grid row).
// Z is nm x GJ_NB and G likewise (row-major, columns e >= ne zero); Y and H
// are GJ_NB x nm (rows e >= ne zero); S is GJ_NB x GJ_NB.  One chain.
#define BD_B GJ_NB

__device__ __forceinline__ int bd_nat_main(int i) { return (i / BD_B) * (BD_B + 1) + i % BD_B; }
__device__ __forceinline__ int bd_nat_edge(int e) { return e * (BD_B + 1) + BD_B; }

__global__ void __launch_bounds__(BAMG_BLK)
k_bd_zy(const CoarseDesc* __restrict__ cd, const CoarseDesc* __restrict__ cs, const double* __restrict__ Wp,
        double* __restrict__ Z, double* __restrict__ Y) {
    const CoarseDesc d = cd[0], m = cs[0];
    const int nx = d.nx, ne = nx - 1, nm = m.n, n = d.n;
    const double* Bd = Wp + d.woff;
    const double* Am = Wp + m.woff;
    const long long tot = (long long)nm * BD_B;
    for (long long t = (long long)blockIdx.x * BAMG_BLK + threadIdx.x; t < tot; t += (long long)gridDim.x * BAMG_BLK) {
        // Z[i, e] (e fastest) and Y[e, j] (j fastest) share the index t
        {
            const int i = (int)(t / BD_B), e = (int)(t % BD_B);
            double z = 0.0;
            if (e < ne) {
                const int ce = bd_nat_edge(e);
                for (int a = max(e - 1, 0); a <= min(e + 1, nx - 1); ++a) {
                    const int cm = a * BD_B + BD_B - 1;
                    z += Am[(size_t)i * nm + cm] * Bd[(size_t)bd_nat_main(cm) * n + ce];
                }
            }
            Z[t] = z;
        }
        {
            const int e = (int)(t / nm), j = (int)(t % nm);
            double y = 0.0;
            if (e < ne) {
                const int re = bd_nat_edge(e);
                for (int a = max(e - 1, 0); a <= min(e + 1, nx - 1); ++a) {
                    const int rm = a * BD_B + BD_B - 1;
                    y += Bd[(size_t)re * n + bd_nat_main(rm)] * Am[(size_t)rm * nm + j];
                }
            }
            Y[t] = y;
        }
    }
}

// S = D - F Z on the ne x ne border block (ld GJ_NB); the entries outside are
// left alone (the Gauss-Jordan step pads with the identity).
__global__ void __launch_bounds__(BAMG_BLK)
k_bd_schur(const CoarseDesc* __restrict__ cd, const double* __restrict__ Wp, const double* __restrict__ Z,
           double* __restrict__ S) {
    const CoarseDesc d = cd[0];
    const int nx = d.nx, ne = nx - 1, n = d.n;
    const double* Bd = Wp + d.woff;
    for (int t = threadIdx.x; t < BD_B * BD_B; t += BAMG_BLK) {
        const int e = t / BD_B, e2 = t % BD_B;
        if (e >= ne || e2 >= ne) continue;
        const int re = bd_nat_edge(e);
        double v = Bd[(size_t)re * n + bd_nat_edge(e2)];
        for (int a = max(e - 1, 0); a <= min(e + 1, nx - 1); ++a) {
            const int rm = a * BD_B + BD_B - 1;
            v -= Bd[(size_t)re * n + bd_nat_main(rm)] * Z[(size_t)rm * BD_B + e2];
        }
        S[t] = v;
    }
}

// G = Z S^-1 and H = S^-1 Y (S^-1 in LDS; sums over e ascending).
__global__ void __launch_bounds__(BAMG_BLK)
k_bd_gh(const CoarseDesc* __restrict__ cd, const CoarseDesc* __restrict__ cs, const double* __restrict__ Si,
        const double* __restrict__ Z, const double* __restrict__ Y, double* __restrict__ G, double* __restrict__ H) {
    __shared__ double sS[BD_B][BD_B + 1];
    const int ne = cd[0].nx - 1, nm = cs[0].n;
    for (int t = threadIdx.x; t < BD_B * BD_B; t += BAMG_BLK) {
        const int e = t / BD_B, e2 = t % BD_B;
        sS[e][e2] = (e < ne && e2 < ne) ? Si[t] : 0.0;
    }
    __syncthreads();
    const long long tot = (long long)nm * BD_B;
    for (long long t = (long long)blockIdx.x * BAMG_BLK + threadIdx.x; t < tot; t += (long long)gridDim.x * BAMG_BLK) {
        {
            const int i = (int)(t / BD_B), e2 = (int)(t % BD_B);
            double g = 0.0;
            for (int e = 0; e < ne; ++e) g += Z[(size_t)i * BD_B + e] * sS[e][e2];
            G[t] = g;
        }
        {
            const int e = (int)(t / nm), j = (int)(t % nm);
            double h = 0.0;
            for (int e2 = 0; e2 < ne; ++e2) h += sS[e][e2] * Y[(size_t)e2 * nm + j];
            H[t] = h;
        }
    }
}

// W (natural order) from the pieces: grid (nx, nx) workgroups for the main x
// main tiles (grid rows a, a2): W = A^-1 + G Y, the rank-ne product (ne <= 64,
// zero beyond) on the FP64 matrix cores with e ascending, added to the tile
// of A^-1 held in the accumulators.
__global__ void __launch_bounds__(BAMG_BLK)
k_bd_combine_main(const CoarseDesc* __restrict__ cd, const CoarseDesc* __restrict__ cs, double* __restrict__ Wp,
                  const double* __restrict__ G, const double* __restrict__ Y) {
    static_assert(BAMG_BLK == 256 && BD_B == GJ_NB, "four wavefronts on a 64 x 64 tile");
    __shared__ double As[GJ_NB][DC_KC + 1];
    __shared__ double Bs[DC_KC][GJ_NB + 1];
    const CoarseDesc d = cd[0], m = cs[0];
    const int ne = d.nx - 1, nm = m.n, n = d.n;
    const double* Am = Wp + m.woff;
    double* W = Wp + d.woff;
    const int i0 = blockIdx.y * BD_B, j0 = blockIdx.x * BD_B;
    const int c = threadIdx.x % BAMG_WAVE, w = threadIdx.x / BAMG_WAVE;
    dc_d4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[cb][q] = Am[(size_t)(i0 + dc_row(w, c, q)) * nm + j0 + dc_col(c, cb)];
    dc_rank64([&](int r, int k) { return k < ne ? G[(size_t)(i0 + r) * BD_B + k] : 0.0; },
              [&](int k, int cc) { return k < ne ? Y[(size_t)k * nm + j0 + cc] : 0.0; }, As, Bs, w, c, acc);
    const int r0 = blockIdx.y * (BD_B + 1), c0 = blockIdx.x * (BD_B + 1);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int q = 0; q < 4; ++q) W[(size_t)(r0 + dc_row(w, c, q)) * n + c0 + dc_col(c, cb)] = acc[cb][q];
}

// The border rows and columns of W: row of border point e: -H (main
// columns), S^-1 (border columns); column of border point e: -G (main rows);
// the padded unknown's row and column are zero.
__global__ void __launch_bounds__(BAMG_BLK)
k_bd_combine_edge(const CoarseDesc* __restrict__ cd, const CoarseDesc* __restrict__ cs, double* __restrict__ Wp,
                  const double* __restrict__ G, const double* __restrict__ H, const double* __restrict__ Si) {
    const CoarseDesc d = cd[0];
    const int nx = d.nx, ne = nx - 1, nm = cs[0].n, n = d.n;
    double* W = Wp + d.woff;
    const long long tot = (long long)nx * n;
    for (long long t = (long long)blockIdx.x * BAMG_BLK + threadIdx.x; t < tot; t += (long long)gridDim.x * BAMG_BLK) {
        const int e = (int)(t / n), j = (int)(t % n);
        const int ja = j / (BD_B + 1), jc = j % (BD_B + 1);
        // row of border point e, column j
        double v = 0.0;
        if (e < ne) {
            if (jc < BD_B) v = -H[(size_t)e * nm + ja * BD_B + jc];
            else if (ja < ne) v = Si[e * BD_B + ja];
        }
        W[(size_t)bd_nat_edge(e) * n + j] = v;
        // column of border point e, row j (main rows only: border rows above)
        if (jc < BD_B) W[(size_t)j * n + bd_nat_edge(e)] = e < ne ? -G[(size_t)(ja * BD_B + jc) * BD_B + e] : 0.0;
    }
}

// ---------------------------------------------------------------- projections
// Zero the last row and column of W (the padding).
__global__ void k_cz_zero_border(const CoarseDesc* __restrict__ cd, double* __restrict__ Wp) {
    const CoarseDesc d = cd[blockIdx.y];
    double* W = Wp + d.woff;
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < d.n; i += gridDim.x * BAMG_BLK) {
        W[(size_t)(d.n - 1) * d.n + i] = 0.0;
        W[(size_t)i * d.n + d.n - 1] = 0.0;
    }
}

// sum_{j < m} a[j] x[j] by one wavefront (result in every lane): lane L takes
// the column pairs 2q, 2q + 1 (q = L, L + 64, ...) in order, then the tail
// column 2 (m / 2) + L.  One 16-byte load per pair when a and x are 16-byte
// aligned, two 8-byte loads otherwise: the same sum either way.
__device__ __forceinline__ double wave_row_dot(const double* __restrict__ a, const double* __restrict__ x, int m,
                                               int lane) {
    const int m2 = m / 2;
    double s = 0;
    if (((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(x)) & 15) == 0) {
        const double2* a2 = (const double2*)a;
        const double2* x2 = (const double2*)x;
#pragma unroll 16
        for (int q = lane; q < m2; q += BAMG_WAVE) {
            const double2 av = a2[q], xv = x2[q];
            s += av.x * xv.x;
            s += av.y * xv.y;
        }
    } else {
        for (int q = lane; q < m2; q += BAMG_WAVE) {
            s += a[2 * q] * x[2 * q];
            s += a[2 * q + 1] * x[2 * q + 1];
        }
    }
    if (2 * m2 + lane < m) s += a[2 * m2 + lane] * x[2 * m2 + lane];
    s = wave_sum(s);
    return __shfl(s, 0, BAMG_WAVE);
}

// out[voff + i] = sum_j W[i, j] x[voff + j] (i < rows(d), j < cols(d)):
// one wavefront per row.  which = 0: rows = cols = n; 1: rows = cols = n-1.
__global__ void __launch_bounds__(BAMG_BLK)
k_cz_gemv(const CoarseDesc* __restrict__ cd, int which, const double* __restrict__ Wp, const double* __restrict__ x,
          double* __restrict__ out) {
    const CoarseDesc d = cd[blockIdx.y];
    const int m = which ? d.n - 1 : d.n;
    const double* W = Wp + d.woff;
    const int lane = threadIdx.x % BAMG_WAVE;
    for (int row = blockIdx.x * (BAMG_BLK / BAMG_WAVE) + threadIdx.x / BAMG_WAVE; row < m;
         row += gridDim.x * (BAMG_BLK / BAMG_WAVE)) {
        const double s = wave_row_dot(W + (size_t)row * d.n, x + d.voff, m, lane);
        if (lane == 0) out[d.voff + row] = s;
    }
}

// FP32 copy of every chain's W for the mixed-precision cycle, rows padded
// with zeros to wfld columns (grid (blocks, chains)).
__global__ void k_cz_w_f32(const CoarseDesc* __restrict__ cd, const double* __restrict__ Wp,
                           float* __restrict__ Wf) {
    const CoarseDesc d = cd[blockIdx.y];
    const int ld = d.wfld, tot = d.n * ld;
    for (int e = blockIdx.x * BAMG_BLK + threadIdx.x; e < tot; e += gridDim.x * BAMG_BLK) {
        const int r = e / ld, c = e - r * ld;
        Wf[d.wfoff + e] = c < d.n ? (float)Wp[d.woff + (size_t)r * d.n + c] : 0.0f;
    }
}

// FP32 copy of the same product for the mixed-precision cycle (vector in
// the level's FP32 cycle buffer at row0).
__global__ void __launch_bounds__(BAMG_BLK)
k_cz_gemv_f32(const CoarseDesc* __restrict__ cd, const float* __restrict__ Wp, const float* __restrict__ x,
              float* __restrict__ out, const int* __restrict__ act) {
    if (act && !act[blockIdx.y]) return;
    const CoarseDesc d = cd[blockIdx.y];
    const float* W = Wp + d.wfoff;
    const int lane = threadIdx.x % BAMG_WAVE;
    // Lane L sums the column groups 4j .. 4j+3, j = L, L + 64, ..., in column
    // order, then tail column 4 (n / 4) + L; with 16-byte aligned rows (the
    // copy's rows are padded to a multiple of 4) and vector each group is one
    // 16-byte load, otherwise four scalar loads in the same order (so the sum
    // does not depend on the alignment).
    const int n4 = d.n / 4;
    const bool v4 = (d.wfld & 3) == 0 && (d.row0 & 3) == 0 && (d.wfoff & 3) == 0;
    for (int row = blockIdx.x * (BAMG_BLK / BAMG_WAVE) + threadIdx.x / BAMG_WAVE; row < d.n;
         row += gridDim.x * (BAMG_BLK / BAMG_WAVE)) {
        const float* a = W + (size_t)row * d.wfld;
        const float* xr = x + d.row0;
        float s = 0;
        if (v4) {
            const float4* a4 = (const float4*)a;
            const float4* x4 = (const float4*)xr;
            // 16 groups per lane cover a 4096-column row: all loads in flight
#pragma unroll 16
            for (int j = lane; j < n4; j += BAMG_WAVE) {
                const float4 av = a4[j], xv = x4[j];
                s += av.x * xv.x;
                s += av.y * xv.y;
                s += av.z * xv.z;
                s += av.w * xv.w;
            }
        } else {
            for (int j = lane; j < n4; j += BAMG_WAVE)
#pragma unroll
                for (int q = 0; q < 4; ++q) s += a[4 * j + q] * xr[4 * j + q];
        }
        if (4 * n4 + lane < d.n) s += a[4 * n4 + lane] * xr[4 * n4 + lane];
        s = wave_sum(s);
        if (lane == 0) out[d.row0 + row] = s;
    }
}

// FP64 coarse solve inside the cycle: e[row0 + i] = sum_j W[i, j] f[row0 + j].
__global__ void __launch_bounds__(BAMG_BLK)
k_cz_gemv_rows(const CoarseDesc* __restrict__ cd, const double* __restrict__ Wp, const double* __restrict__ x,
               double* __restrict__ out, const int* __restrict__ act) {
    if (act && !act[blockIdx.y]) return;
    const CoarseDesc d = cd[blockIdx.y];
    const double* W = Wp + d.woff;
    const int lane = threadIdx.x % BAMG_WAVE;
    for (int row = blockIdx.x * (BAMG_BLK / BAMG_WAVE) + threadIdx.x / BAMG_WAVE; row < d.n;
         row += gridDim.x * (BAMG_BLK / BAMG_WAVE)) {
        const double s = wave_row_dot(W + (size_t)row * d.n, x + d.row0, d.n, lane);
        if (lane == 0) out[d.row0 + row] = s;
    }
}

// u = y^T W per chain: column-chunk partials then a fixed-order final.
__global__ void k_cz_gemv_t_partial(const CoarseDesc* __restrict__ cd, const double* __restrict__ Wp,
                                    const double* __restrict__ y, double* __restrict__ part, int RCH) {
    const CoarseDesc d = cd[blockIdx.z];
    const int j = blockIdx.x * BAMG_BLK + threadIdx.x;
    const int r0 = blockIdx.y * RCH;
    if (j >= d.n || r0 >= d.n) return;
    const double* W = Wp + d.woff;
    double s = 0;
    const int r1 = min(d.n, r0 + RCH);
    for (int i = r0; i < r1; ++i) s += y[d.voff + i] * W[(size_t)i * d.n + j];
    part[(long long)gridDim.y * d.voff + (long long)blockIdx.y * d.n + j] = s;
}

__global__ void k_cz_gemv_t_final(const CoarseDesc* __restrict__ cd, int nchunk_max, int RCH,
                                  const double* __restrict__ part, double* __restrict__ out) {
    const CoarseDesc d = cd[blockIdx.y];
    const int j = blockIdx.x * BAMG_BLK + threadIdx.x;
    if (j >= d.n) return;
    const int nchunks = (d.n + RCH - 1) / RCH;
    double s = 0;
    for (int c = 0; c < nchunks; ++c) s += part[(long long)nchunk_max * d.voff + (long long)c * d.n + j];
    out[d.voff + j] = s;
}

// Per-chain dot product of two pooled vectors -> out[chain] (one block each).
__global__ void k_cz_dot(const CoarseDesc* __restrict__ cd, const double* __restrict__ a, const double* __restrict__ b,
                         double* __restrict__ out, int stride) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    const CoarseDesc d = cd[blockIdx.x];
    double s = 0;
    for (int i = threadIdx.x; i < d.n; i += BAMG_BLK) s += a[d.voff + i] * b[d.voff + i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[(size_t)blockIdx.x * stride] = s;
}

// y_1 = -g, y_n = 1 (g = Binv b_col).
__global__ void k_cz_null(const CoarseDesc* __restrict__ cd, const double* __restrict__ g, double* __restrict__ y) {
    const CoarseDesc d = cd[blockIdx.y];
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < d.n; i += gridDim.x * BAMG_BLK)
        y[d.voff + i] = (i < d.n - 1) ? -g[d.voff + i] : 1.0;
}

// W <- W - s 1^T / n - y (u - (y^T s) 1^T / n)^T / (y^T y), with
// sc[chain*SCS + 0] = y^T s, sc[chain*SCS + 1] = y^T y.
__global__ void k_cz_project(const CoarseDesc* __restrict__ cd, double* __restrict__ Wp, const double* __restrict__ s,
                             const double* __restrict__ u, const double* __restrict__ y, const double* __restrict__ sc,
                             int SCS) {
    const CoarseDesc d = cd[blockIdx.y];
    double* W = Wp + d.woff;
    const double inv_n = 1.0 / d.n;
    const double ys = sc[(size_t)blockIdx.y * SCS], yy = sc[(size_t)blockIdx.y * SCS + 1];
    const long long nn = (long long)d.n * d.n;
    for (long long e = (long long)blockIdx.x * BAMG_BLK + threadIdx.x; e < nn; e += (long long)gridDim.x * BAMG_BLK) {
        int i = (int)(e / d.n), j = (int)(e % d.n);
        W[e] = W[e] - s[d.voff + i] * inv_n - y[d.voff + i] * (u[d.voff + j] - ys * inv_n) / yy;
    }
}

// c_j = sum_i T_L[i, j] (T = I: c = 1), gathered from the 3x3 box rows in
// ascending row order.  Without a grid (nx = 0) the pattern of T_L is
// symmetric, so the rows holding column j are the columns of row j.
template <typename M>
__global__ void k_cz_colsum(const CoarseDesc* __restrict__ cd, double* __restrict__ c) {
    const CoarseDesc d = cd[blockIdx.y];
    for (int j = blockIdx.x * BAMG_BLK + threadIdx.x; j < d.n; j += gridDim.x * BAMG_BLK) {
        if (!d.trp) { c[d.voff + j] = 1.0; continue; }
        const M* tv = (const M*)d.tv;
        if (d.nx == 0) {
            double sum = 0;
            const int gj = d.row0 + j;
            for (int q = d.trp[gj]; q < d.trp[gj + 1]; ++q) {
                const int gi = d.tci[q];
                for (int p = d.trp[gi]; p < d.trp[gi + 1]; ++p)
                    if (d.tci[p] == gj) sum += (double)tv[p];
            }
            c[d.voff + j] = sum;
            continue;
        }
        int ja = (int)d.dy.div((uint32_t)j), jb = j - ja * d.ny;
        int rows[9];
#pragma unroll
        for (int s = 0; s < 9; ++s) {
            int a = ja + s / 3 - 1, b = jb + s % 3 - 1;
            rows[s] = -1;
            if (d.periodic) {
                a = a < 0 ? a + d.nx : (a >= d.nx ? a - d.nx : a);
                b = b < 0 ? b + d.ny : (b >= d.ny ? b - d.ny : b);
            } else if (a < 0 || a >= d.nx || b < 0 || b >= d.ny) {
                continue;
            }
            rows[s] = a * d.ny + b;
        }
        double sum = 0;
        for (int pass = 0; pass < 9; ++pass) {
            int best = -1;
            for (int t = 0; t < 9; ++t) {
                if (rows[t] < 0) continue;
                int rank = 0;
                for (int u = 0; u < 9; ++u) rank += rows[u] >= 0 && rows[u] < rows[t];
                if (rank == pass) best = rows[t];
            }
            if (best < 0) break;
            const int gi = d.row0 + best;
            for (int p = d.trp[gi]; p < d.trp[gi + 1]; ++p)
                if (d.tci[p] == d.row0 + j) sum += (double)tv[p];
        }
        c[d.voff + j] = sum;
    }
}

// ---------------------------------------------------------------- Arnoldi
// Basis of chain d: Vb[aoff + j*n + i], j <= am.  Steps run in lockstep over
// the chains; a chain with j >= am (or no eigenpairs) is idle.
// start vector: seeded u - 1/2, then projected onto {c^T v = 0}.
__global__ void k_cz_arn_start(const CoarseDesc* __restrict__ cd, uint64_t seed, double* __restrict__ Vb) {
    const CoarseDesc d = cd[blockIdx.y];
    if (d.am < 1) return;
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < d.n; i += gridDim.x * BAMG_BLK)
        Vb[d.aoff + i] = splitmix_u01(seed, 7ull, (uint64_t)i) - 0.5;
}

// w = T v_j (pooled vector tmp), for chains with j < am.
template <typename M>
__global__ void k_cz_tv(const CoarseDesc* __restrict__ cd, int j, const double* __restrict__ Vb, double* __restrict__ w) {
    const CoarseDesc d = cd[blockIdx.y];
    if (j >= d.am) return;
    const double* v = Vb + d.aoff + (size_t)j * d.n;
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < d.n; i += gridDim.x * BAMG_BLK) {
        double s;
        if (!d.trp) {
            s = v[i];
        } else {
            const M* tv = (const M*)d.tv;
            s = 0;
            const int gi = d.row0 + i;
            for (int p = d.trp[gi]; p < d.trp[gi + 1]; ++p) s += (double)tv[p] * v[d.tci[p] - d.row0];
        }
        w[d.voff + i] = s;
    }
}

// u = W w into basis column j+1 (a GEMV per chain).
__global__ void __launch_bounds__(BAMG_BLK)
k_cz_arn_gemv(const CoarseDesc* __restrict__ cd, int j, const double* __restrict__ Wp, const double* __restrict__ w,
              double* __restrict__ Vb) {
    const CoarseDesc d = cd[blockIdx.y];
    if (j >= d.am) return;
    const double* W = Wp + d.woff;
    double* u = Vb + d.aoff + (size_t)(j + 1) * d.n;
    const int lane = threadIdx.x % BAMG_WAVE;
    for (int row = blockIdx.x * (BAMG_BLK / BAMG_WAVE) + threadIdx.x / BAMG_WAVE; row < d.n;
         row += gridDim.x * (BAMG_BLK / BAMG_WAVE)) {
        const double s = wave_row_dot(W + (size_t)row * d.n, w + d.voff, d.n, lane);
        if (lane == 0) u[row] = s;
    }
}

// The same product from the FP32 copy of W (mixed precision): the vector
// stays FP64 and every product and sum is FP64, so the only change from
// the FP64 form is W rounded to FP32.  One workgroup per pair of rows, so
// that each load of w serves both and every wavefront has its loads of a
// quarter of the row in flight at once: thread t sums the column groups
// 4q .. 4q+3, q = t, t + BAMG_BLK, ..., in column order (thread t < n mod 4
// also tail column 4 (n / 4) + t), then each wavefront's sum, then the four
// in order.  The last row of an odd n pairs with itself (read twice, stored
// once).
__global__ void __launch_bounds__(BAMG_BLK)
k_cz_arn_gemv_f32(const CoarseDesc* __restrict__ cd, int j, const float* __restrict__ Wf,
                  const double* __restrict__ w, double* __restrict__ Vb) {
    __shared__ double red[BAMG_BLK / BAMG_WAVE][2];
    const CoarseDesc d = cd[blockIdx.y];
    if (j >= d.am) return;
    const float* W = Wf + d.wfoff;
    const double* x = w + d.voff;
    double* u = Vb + d.aoff + (size_t)(j + 1) * d.n;
    const int t = threadIdx.x, lane = t % BAMG_WAVE, wv = t / BAMG_WAVE;
    const int n4 = d.n / 4;
    const bool v4 = (d.wfld & 3) == 0 &&
                    ((reinterpret_cast<uintptr_t>(W) | reinterpret_cast<uintptr_t>(x)) & 15) == 0;
    for (int r0 = 2 * blockIdx.x; r0 < d.n; r0 += 2 * gridDim.x) {
        const int r1 = min(r0 + 1, d.n - 1);
        const float* a0 = W + (size_t)r0 * d.wfld;
        const float* a1 = W + (size_t)r1 * d.wfld;
        double s0 = 0, s1 = 0;
        if (v4) {
            const float4* p4 = (const float4*)a0;
            const float4* q4 = (const float4*)a1;
            const double2* x2 = (const double2*)x;
#pragma unroll 4
            for (int q = t; q < n4; q += BAMG_BLK) {
                const float4 p = p4[q], r = q4[q];
                const double2 xa = x2[2 * q], xb = x2[2 * q + 1];
                s0 += (double)p.x * xa.x;
                s0 += (double)p.y * xa.y;
                s0 += (double)p.z * xb.x;
                s0 += (double)p.w * xb.y;
                s1 += (double)r.x * xa.x;
                s1 += (double)r.y * xa.y;
                s1 += (double)r.z * xb.x;
                s1 += (double)r.w * xb.y;
            }
        } else {
            for (int q = t; q < n4; q += BAMG_BLK)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double xv = x[4 * q + e];
                    s0 += (double)a0[4 * q + e] * xv;
                    s1 += (double)a1[4 * q + e] * xv;
                }
        }
        if (4 * n4 + t < d.n) {
            const double xv = x[4 * n4 + t];
            s0 += (double)a0[4 * n4 + t] * xv;
            s1 += (double)a1[4 * n4 + t] * xv;
        }
        s0 = wave_sum(s0);
        s1 = wave_sum(s1);
        if (lane == 0) { red[wv][0] = s0; red[wv][1] = s1; }
        __syncthreads();
        if (t == 0) {
            double b0 = 0, b1 = 0;
#pragma unroll
            for (int k = 0; k < BAMG_BLK / BAMG_WAVE; ++k) { b0 += red[k][0]; b1 += red[k][1]; }
            u[r0] = b0;
            if (r0 + 1 < d.n) u[r0 + 1] = b1;
        }
        __syncthreads();
    }
}

// This block's sums of u^2 and u y (fixed order) into npart[(chain,
// block) * 2 ..], for k_cz_arn_normalize.
__device__ __forceinline__ void cz_norm_partials(double ss, double st, double* sh, double* sh2,
                                                 double* __restrict__ npart) {
    ss = block_sum(ss, sh);
    st = block_sum(st, sh2);
    if (threadIdx.x == 0) {
        double* o = npart + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 2;
        o[0] = ss;
        o[1] = st;
    }
}

// The projection against c and the first Gram-Schmidt pass in one pair of
// launches.  Dots pass (grid (j + 2, chains)): dots[0] = <c, u>, dots[1 + b]
// = <v_b, u> (b <= j), each by one block in a fixed order.
__global__ void k_cz_arn_dots2(const CoarseDesc* __restrict__ cd, int j, const double* __restrict__ cvec,
                               const double* __restrict__ Vb, double* __restrict__ dots, int DS) {
    __shared__ double sh[BAMG_BLK / BAMG_WAVE];
    const CoarseDesc d = cd[blockIdx.y];
    const int b = blockIdx.x;
    if (j >= d.am || b > j + 1) return;
    const double* u = Vb + d.aoff + (size_t)(j + 1) * d.n;
    const double* x = b == 0 ? cvec + d.voff : Vb + d.aoff + (size_t)(b - 1) * d.n;
    // i ascending in steps of the block, 8 rows' loads issued together
    double s = 0;
    for (int i0 = threadIdx.x; i0 < d.n; i0 += 8 * BAMG_BLK) {
        double xv[8], uv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = i0 + q * BAMG_BLK;
            xv[q] = i < d.n ? x[i] : 0.0;
            uv[q] = i < d.n ? u[i] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (i0 + q * BAMG_BLK < d.n) s += xv[q] * uv[q];
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) dots[(size_t)blockIdx.y * DS + b] = s;
}

// Update of that pair: with a = <c, u> / cy, the projected u' = u - a y has
// <v_b, u'> = <v_b, u> - a <v_b, y> (<v_b, y> = vy[b], kept from when v_b
// was normalised), so u <- u - a y - sum_{b<=j} (<v_b, u> - a vy[b]) v_b and
// H[0..j, j] += those coefficients (block 0).
__global__ void k_cz_arn_update2(const CoarseDesc* __restrict__ cd, int j, const double* __restrict__ y,
                                 const double* __restrict__ cy, const double* __restrict__ dots,
                                 const double* __restrict__ vy, int DS, double* __restrict__ Vb,
                                 double* __restrict__ H, int HS, double* __restrict__ npart) {
    __shared__ double cf[HQR_MAXM];
    __shared__ double sh[BAMG_BLK / BAMG_WAVE], sh2[BAMG_BLK / BAMG_WAVE];
    const CoarseDesc d = cd[blockIdx.y];
    if (j >= d.am) return;
    const double* dt = dots + (size_t)blockIdx.y * DS;
    const double a = dt[0] / cy[blockIdx.y];
    for (int b = threadIdx.x; b <= j; b += BAMG_BLK) cf[b] = dt[1 + b] - a * vy[(size_t)blockIdx.y * DS + b];
    __syncthreads();
    double* u = Vb + d.aoff + (size_t)(j + 1) * d.n;
    double ss = 0, st = 0;
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < d.n; i += gridDim.x * BAMG_BLK) {
        double s = u[i];
        s -= y[d.voff + i] * a;
        for (int b = 0; b <= j; ++b) s -= cf[b] * Vb[d.aoff + (size_t)b * d.n + i];
        u[i] = s;
        ss += s * s;
        st += s * y[d.voff + i];
    }
    if (blockIdx.x == 0 && (int)threadIdx.x <= j)
        H[(size_t)blockIdx.y * HS + (size_t)j * (d.am + 1) + threadIdx.x] += cf[threadIdx.x];
    if (j < 0) cz_norm_partials(ss, st, sh, sh2, npart);    // the start vector goes to the norm next
}

// Steps j >= 0 after the dots pass k_cz_arn_dots2, with K >= j + 1 (a
// multiple of 8) accumulators: every thread loads v_0 .. v_{K-1} of its row
// together (b > j re-reads v_j with a zero coefficient).
//   k_cz_arn_update2p: the update of k_cz_arn_update2 (u <- u - a y -
//     sum cf_b v_b in place, H[0..j, j] += cf) and this block's sums of the
//     second Gram-Schmidt pass <v_b, u> (b <= j) into
//     apart[((chain DS) + b) G + block] (G blocks per chain);
//   k_cz_arn_updatep: dt_b = the G sums of b in block order, u - sum dt_b v_b
//     into ub (the vector pool), H[0..j, j] += dt, the norm partials;
//   k_cz_arn_normtv: v_{j+1} = u / ||u|| into the basis, H[j+1, j], vy, and
//     w = T v_{j+1} for the next step (the neighbours' entries divided the same
//     way; reading ub keeps them stable while the basis column is written).
template <int K>
__global__ void __launch_bounds__(BAMG_BLK)
k_cz_arn_update2p(const CoarseDesc* __restrict__ cd, int j, const double* __restrict__ y,
                  const double* __restrict__ cy, const double* __restrict__ dots, const double* __restrict__ vy,
                  int DS, double* __restrict__ Vb, double* __restrict__ H, int HS, double* __restrict__ apart) {
    __shared__ double cf[K];
    __shared__ double red[(BAMG_BLK / BAMG_WAVE) * (GsRed<K>::KR + 2)];
    const CoarseDesc d = cd[blockIdx.y];
    if (j >= d.am) return;
    const double* dt = dots + (size_t)blockIdx.y * DS;
    const double a = dt[0] / cy[blockIdx.y];
    for (int b = threadIdx.x; b < K; b += BAMG_BLK) cf[b] = b <= j ? dt[1 + b] - a * vy[(size_t)blockIdx.y * DS + b] : 0.0;
    __syncthreads();
    const double* V = Vb + d.aoff;
    double* u = Vb + d.aoff + (size_t)(j + 1) * d.n;
    double acc[K];
#pragma unroll
    for (int b = 0; b < K; ++b) acc[b] = 0.0;
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < d.n; i += gridDim.x * BAMG_BLK) {
        double q[K];
#pragma unroll
        for (int b = 0; b < K; ++b) q[b] = V[(size_t)min(b, j) * d.n + i];
        const double yi = y[d.voff + i];
        double s = u[i];
        __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the products
        s -= yi * a;
#pragma unroll
        for (int b = 0; b < K; ++b) s -= cf[b] * q[b];
        u[i] = s;
#pragma unroll
        for (int b = 0; b < K; ++b) acc[b] += q[b] * s;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x <= j)
        H[(size_t)blockIdx.y * HS + (size_t)j * (d.am + 1) + threadIdx.x] += cf[threadIdx.x];
    gs_store_partials<K>(acc, 0.0, 0.0, j + 1, apart, DS, red);
}

template <int K>
__global__ void __launch_bounds__(BAMG_BLK)
k_cz_arn_updatep(const CoarseDesc* __restrict__ cd, int j, const double* __restrict__ y,
                 const double* __restrict__ apart, int DS, const double* __restrict__ Vb, double* __restrict__ H,
                 int HS, double* __restrict__ ub, double* __restrict__ npart) {
    __shared__ double dt[K];
    __shared__ double sh[BAMG_BLK / BAMG_WAVE], sh2[BAMG_BLK / BAMG_WAVE];
    const CoarseDesc d = cd[blockIdx.y];
    if (j >= d.am) return;
    const int G = gridDim.x;
    for (int b = threadIdx.x; b < K; b += BAMG_BLK) {
        double s = 0;
        if (b <= j) {
            const double* pb = apart + ((size_t)blockIdx.y * DS + b) * G;
            for (int g0 = 0; g0 < G; g0 += 8) {     // in block order, 8 loads in flight
                double v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) v[q] = g0 + q < G ? pb[g0 + q] : 0.0;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (g0 + q < G) s += v[q];
            }
        }
        dt[b] = s;
    }
    __syncthreads();
    const double* V = Vb + d.aoff;
    const double* u = Vb + d.aoff + (size_t)(j + 1) * d.n;
    double ss = 0, st = 0;
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < d.n; i += gridDim.x * BAMG_BLK) {
        double q[K];
#pragma unroll
        for (int b = 0; b < K; ++b) q[b] = V[(size_t)min(b, j) * d.n + i];
        const double yi = y[d.voff + i];
        double s = u[i];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < K; ++b) s -= dt[b] * q[b];
        ub[d.voff + i] = s;
        ss += s * s;
        st += s * yi;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x <= j)
        H[(size_t)blockIdx.y * HS + (size_t)j * (d.am + 1) + threadIdx.x] += dt[threadIdx.x];
    cz_norm_partials(ss, st, sh, sh2, npart);
}

template <typename M>
__global__ void k_cz_arn_normtv(const CoarseDesc* __restrict__ cd, int j, const double* __restrict__ ub,
                                double* __restrict__ Vb, double* __restrict__ H, int HS, double* __restrict__ vy,
                                int DS, const double* __restrict__ npart, double* __restrict__ w) {
    const CoarseDesc d = cd[blockIdx.y];
    if (j >= d.am) return;
    const double* u = ub + d.voff;
    double* v = Vb + d.aoff + (size_t)(j + 1) * d.n;
    const M* tv = (const M*)d.tv;
    // this thread's row of T first: its entries and the neighbours' u are
    // loaded while the norm's partials are summed
    constexpr int TR = 9;
    const int i = blockIdx.x * BAMG_BLK + threadIdx.x;
    int p0 = 0, p1 = 0;
    if (d.trp && i < d.n) { p0 = d.trp[d.row0 + i]; p1 = d.trp[d.row0 + i + 1]; }
    const double* pp = npart + (size_t)blockIdx.y * gridDim.x * 2;
    double s = 0, t = 0;
    for (int q0 = 0; q0 < (int)gridDim.x; q0 += 8) {   // in block order, 8 pairs in flight
        double a[8], c[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bool ok = q0 + q < (int)gridDim.x;
            a[q] = ok ? pp[2 * (q0 + q)] : 0.0;
            c[q] = ok ? pp[2 * (q0 + q) + 1] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q0 + q < (int)gridDim.x) { s += a[q]; t += c[q]; }
    }
    double tw[TR], uc[TR];
#pragma unroll
    for (int k = 0; k < TR; ++k) {
        const int p = p0 + k;
        const bool ok = p < p1;
        tw[k] = ok ? (double)tv[p] : 0.0;
        uc[k] = ok ? u[d.tci[p] - d.row0] : 0.0;
    }
    const double nrm = sqrt(s);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        H[(size_t)blockIdx.y * HS + (size_t)j * (d.am + 1) + j + 1] = nrm;
        vy[(size_t)blockIdx.y * DS + j + 1] = nrm > 0 ? t / nrm : 0.0;
    }
    for (int r = i; r < d.n; r += gridDim.x * BAMG_BLK) {
        const double vi = nrm > 0 ? u[r] / nrm : 0.0;
        v[r] = vi;
        double tvs;
        if (!d.trp) {
            tvs = vi;
        } else {
            // the neighbours' entries divided the same way as the basis column
            tvs = 0;
            const int q0 = r == i ? p0 : d.trp[d.row0 + r], q1 = r == i ? p1 : d.trp[d.row0 + r + 1];
#pragma unroll
            for (int k = 0; k < TR; ++k)
                if (r == i && p0 + k < p1) tvs += tw[k] * (nrm > 0 ? uc[k] / nrm : 0.0);
            for (int p = r == i ? q0 + TR : q0; p < q1; ++p)
                tvs += (double)tv[p] * (nrm > 0 ? u[d.tci[p] - d.row0] / nrm : 0.0);
        }
        w[d.voff + r] = tvs;
    }
}

// Normalise basis column j+1 (or column 0 with j = -1): v = u / ||u||,
// H[j+1, j] = ||u||, and vy[j+1] = <v, y> = <u, y> / ||u|| for the
// projections of later steps.  The sums come from the partials of the
// update kernel that formed u (one pair per block, added in block order);
// grid (blocks, chains) as that kernel's.
__global__ void k_cz_arn_normalize(const CoarseDesc* __restrict__ cd, int j, double* __restrict__ Vb,
                                   double* __restrict__ H, int HS, double* __restrict__ vy, int DS,
                                   const double* __restrict__ npart) {
    const CoarseDesc d = cd[blockIdx.y];
    if (j >= d.am || d.am < 1) return;
    const double* pp = npart + (size_t)blockIdx.y * gridDim.x * 2;
    double s = 0, t = 0;
    for (int q = 0; q < (int)gridDim.x; ++q) { s += pp[2 * q]; t += pp[2 * q + 1]; }
    const double nrm = sqrt(s);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (j >= 0) H[(size_t)blockIdx.y * HS + (size_t)j * (d.am + 1) + j + 1] = nrm;
        vy[(size_t)blockIdx.y * DS + j + 1] = nrm > 0 ? t / nrm : 0.0;
    }
    double* u = Vb + d.aoff + (size_t)(j + 1) * d.n;
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < d.n; i += gridDim.x * BAMG_BLK)
        u[i] = nrm > 0 ? u[i] / nrm : 0.0;
}

// Ritz vector of entry e of chain (blockIdx.y): v = Vb[:, 0:m] s_e, m =
// min(am, mcap) Arnoldi steps.
__global__ void k_cz_ritz(const CoarseDesc* __restrict__ cd, int e, int mcap, const int* __restrict__ nsel, int NS,
                          const double* __restrict__ Vb, const double* __restrict__ sel_s, int SS,
                          double* __restrict__ rre, double* __restrict__ rim) {
    const CoarseDesc d = cd[blockIdx.y];
    if (e >= nsel[(size_t)blockIdx.y * NS]) return;
    const double* s = sel_s + (size_t)blockIdx.y * SS + (size_t)e * 2 * d.am;
    const int m = min(d.am, mcap);
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < d.n; i += gridDim.x * BAMG_BLK) {
        double a = 0, b = 0;
        for (int j = 0; j < m; ++j) {
            double v = Vb[d.aoff + (size_t)j * d.n + i];
            a += v * s[2 * j]; b += v * s[2 * j + 1];
        }
        rre[d.voff + i] = a; rim[d.voff + i] = b;
    }
}

// Normalise entry e's Ritz vector (||v|| = 1, largest-modulus entry real
// positive, lowest index on ties) into its column(s) of the chain's V rows
// (row0 .. on its coarsest level, row stride VS).  One block per chain.
template <typename T>
__global__ void k_cz_eigvec(const CoarseDesc* __restrict__ cd, int e, const int* __restrict__ nsel, int NS,
                            const double* __restrict__ sel_lam, int LS, const double* __restrict__ rre,
                            const double* __restrict__ rim, const int* __restrict__ ent_col, int KV,
                            T* __restrict__ V, int VS) {
    __shared__ double sh[BAMG_BLK];
    __shared__ int shi[BAMG_BLK];
    __shared__ double shs[BAMG_BLK / BAMG_WAVE];
    __shared__ double fac[2];
    const CoarseDesc d = cd[blockIdx.x];
    if (e >= nsel[(size_t)blockIdx.x * NS]) return;
    const bool pair = sel_lam[(size_t)blockIdx.x * LS + 2 * e + 1] != 0.0;
    const int c = ent_col[(size_t)blockIdx.x * KV + e + 1];
    const double* vr = rre + d.voff;
    const double* vi = rim + d.voff;
    double s = 0, best = -1;
    int bi = 0;
    for (int i = threadIdx.x; i < d.n; i += BAMG_BLK) {
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
    if (threadIdx.x == 0) {
        int im = shi[0];
        double ar = vr[im], ai = pair ? vi[im] : 0.0;
        double mod = sqrt(ar * ar + ai * ai);
        double nrm = sqrt(s);
        fac[0] = ar / mod / nrm; fac[1] = -ai / mod / nrm;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < d.n; i += BAMG_BLK) {
        double a = vr[i], b = pair ? vi[i] : 0.0;
        double nr = a * fac[0] - b * fac[1], ni = a * fac[1] + b * fac[0];
        V[(size_t)(d.row0 + i) * VS + c] = (T)nr;
        if (pair) V[(size_t)(d.row0 + i) * VS + c + 1] = (T)ni;
    }
}

// Column 0 of V: y / (c^T y).
template <typename T>
__global__ void k_cz_ycol(const CoarseDesc* __restrict__ cd, const double* __restrict__ y, const double* __restrict__ cy,
                          T* __restrict__ V, int VS) {
    const CoarseDesc d = cd[blockIdx.y];
    for (int i = blockIdx.x * BAMG_BLK + threadIdx.x; i < d.n; i += gridDim.x * BAMG_BLK)
        V[(size_t)(d.row0 + i) * VS] = (T)(y[d.voff + i] / cy[blockIdx.y]);
}

// Eigenvalue / column tables of every chain from its selection (one thread
// per chain): lam[chain][2*KV], kind[chain][KV], ent_col[chain][KV],
// nvc[chain], nentc[chain].
__global__ void k_cz_tables(int nch, const int* __restrict__ nsel, int NS, const double* __restrict__ sel_lam, int LS,
                            double* __restrict__ lamall, int* __restrict__ kindall, int* __restrict__ ent_colall,
                            int KV, int* __restrict__ nvc, int* __restrict__ nentc) {
    int ch = blockIdx.x * blockDim.x + threadIdx.x;
    if (ch >= nch) return;
    double* lam = lamall + (size_t)ch * 2 * KV;
    int* kind = kindall + (size_t)ch * KV;
    int* ent_col = ent_colall + (size_t)ch * KV;
    for (int q = 0; q < 2 * KV; ++q) lam[q] = 0.0;
    for (int q = 0; q < KV; ++q) { kind[q] = 0; ent_col[q] = 0; }
    int ne = nsel[(size_t)ch * NS];
    int c = 1;
    for (int e = 0; e < ne; ++e) {
        double lr = sel_lam[(size_t)ch * LS + 2 * e], li = sel_lam[(size_t)ch * LS + 2 * e + 1];
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
    nvc[ch] = c;
    nentc[ch] = ne + 1;
}

// One wavefront per chain with act[c]: the nearest-to-zero eigenvector of
// the leading k x k block of its Arnoldi matrix (hessenberg_near_zero_body).
__global__ void __launch_bounds__(BAMG_WAVE)
k_hess_near0(int k, const int* __restrict__ act, const double* __restrict__ Hall, int HS, int ld,
             double* __restrict__ eta, int ES, int* __restrict__ fail) {
    const int c = blockIdx.x;
    if (!act[c]) return;
    hessenberg_near_zero_body(k, Hall + (size_t)c * HS, ld, eta + (size_t)c * ES, fail + c);
}

// One wavefront per chain: eigenvalues of the leading min(am, mcap) steps of
// its Arnoldi Hessenberg matrix (stride HS), selection and eigenvectors (see
// hessenberg_select_body).  Chains without eigenpairs report no selection.
__global__ void __launch_bounds__(BAMG_WAVE)
k_cz_hess(const CoarseDesc* __restrict__ cd, int want, int mcap, const double* __restrict__ Hh, int HS,
          int* __restrict__ nsel, int NS, double* __restrict__ sel_lam, int LS) {
    const int c = blockIdx.x;
    const CoarseDesc d = cd[c];
    if (d.am < 1 || want < 1) {
        if (threadIdx.x == 0) { nsel[(size_t)c * NS] = 0; nsel[(size_t)c * NS + 1] = 0; nsel[(size_t)c * NS + 2] = 0; }
        return;
    }
    hessenberg_select_body(min(d.am, mcap), d.am + 1, want, Hh + (size_t)c * HS, nsel + (size_t)c * NS,
                           sel_lam + (size_t)c * LS);
}

// The eigenvectors of the selected eigenvalues, one wavefront per entry e
// (blockIdx.x) and chain (blockIdx.y), all at once.
__global__ void __launch_bounds__(BAMG_WAVE)
k_cz_hess_vec(const CoarseDesc* __restrict__ cd, int mcap, const double* __restrict__ Hh, int HS,
              const int* __restrict__ nsel, int NS, const double* __restrict__ sel_lam, int LS,
              double* __restrict__ sel_s, int SS) {
    const int c = blockIdx.y, e = blockIdx.x;
    const CoarseDesc d = cd[c];
    if (d.am < 1 || e >= nsel[(size_t)c * NS] || nsel[(size_t)c * NS + 2]) return;
    const double* th = sel_lam + (size_t)c * LS + HSEL_THETA + 2 * e;
    hessenberg_vec_body(min(d.am, mcap), d.am + 1, Hh + (size_t)c * HS, th[0], th[1],
                        sel_s + (size_t)c * SS + (size_t)e * 2 * d.am);
}

// Whether the Ritz pairs selected from the first m = min(am, mcap) Arnoldi
// steps are converged (one thread per chain): the residual of a Ritz pair
// (theta, V_m s) with ||s||_2 = 1 is |h_{m+1,m}| |s_m| (the Arnoldi
// relation), taken relative to |theta|; ok[c] = 1 when every selected
// entry's is at most tol, or when the chain ran all its steps (m = am).
__global__ void k_cz_ritz_check(int nch, const CoarseDesc* __restrict__ cd, int mcap, const double* __restrict__ Hh,
                                int HS, const int* __restrict__ nsel, int NS, const double* __restrict__ sel_lam,
                                int LS, const double* __restrict__ sel_s, int SS, double tol, int* __restrict__ ok) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nch) return;
    const CoarseDesc d = cd[c];
    const int m = min(d.am, mcap);
    if (d.am < 1 || m >= d.am) { ok[c] = 1; return; }
    const int* ns = nsel + (size_t)c * NS;
    if (ns[2]) { ok[c] = 0; return; }
    const double h = fabs(Hh[(size_t)c * HS + (size_t)(m - 1) * (d.am + 1) + m]);
    int good = 1;
    for (int e = 0; e < ns[0]; ++e) {
        const double* th = sel_lam + (size_t)c * LS + HSEL_THETA + 2 * e;
        const double* sv = sel_s + (size_t)c * SS + (size_t)e * 2 * d.am + 2 * (m - 1);
        const double res = h * sqrt(sv[0] * sv[0] + sv[1] * sv[1]);
        if (!(res <= tol * sqrt(th[0] * th[0] + th[1] * th[1]))) good = 0;
    }
    ok[c] = good;
}
