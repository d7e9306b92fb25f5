// Shared device helpers of the Bootstrap AMG library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define BAMG_BLK 256
#define BAMG_WAVE 64
#define BAMG_NXCD 8        // MI355X: 8 accelerator complex dies, 32 CUs each

// Workgroups are dispatched round-robin over the XCDs (block b runs on XCD
// b % 8).  Renumber them so that each XCD owns one contiguous range of tiles:
// stencil neighbours of a tile (rows +-ny) then sit in the same XCD's L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
    const int per = nblocks / BAMG_NXCD, rem = nblocks % BAMG_NXCD;
    const int x = bid % BAMG_NXCD, k = bid / BAMG_NXCD;
    return x * per + (x < rem ? x : rem) + k;
}

// Division of non-negative 31-bit integers by a runtime constant d >= 1:
// q = (mulhi(x, m) + x) >> l with l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1
// (round-up multiplier method; exact for x < 2^31).
struct FastDiv {
    uint32_t d, m, l;
    FastDiv() : d(1), m(1), l(0) {}
    explicit FastDiv(uint32_t dd) : d(dd) {
        l = 0;
        while ((1ull << l) < dd) ++l;
        m = (uint32_t)((((1ull << l) - dd) << 32) / dd + 1);
    }
    __host__ __device__ __forceinline__ uint32_t div(uint32_t x) const {
#ifdef __HIP_DEVICE_COMPILE__
        uint32_t hi = __umulhi(x, m);
#else
        uint32_t hi = (uint32_t)(((uint64_t)x * m) >> 32);
#endif
        return (hi + x) >> l;
    }
};

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) used as a counter-based
// generator: h = mix(key + GAMMA), key = (seed ^ stream*GAMMA) + idx,
// u = (h >> 11) * 2^-53 in [0, 1).
__host__ __device__ __forceinline__ double splitmix_u01(uint64_t seed, uint64_t stream, uint64_t idx) {
    const uint64_t G = 0x9E3779B97F4A7C15ull;
    uint64_t z = ((seed ^ (stream * G)) + idx) + G;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * 0x1.0p-53;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = BAMG_WAVE / 2; off > 0; off >>= 1) v += __shfl_down(v, off, BAMG_WAVE);
    return v;   // valid in lane 0
}

// Sums of K per-lane values a[0..K-1] over the wavefront at once (K = 8, 16,
// 32 or 64): on each of the top log2 K lane bits every lane keeps one half of
// its values and adds the partner lane's copy of that half (K - 1 exchanges
// in all, instead of 6 K for K separate sums), then the lanes that share an
// index add up over the remaining bits.  On return a[0] of lane l is the
// total of value l >> (6 - log2 K); the order of the additions is fixed.
template <int K, int H, int O>
__device__ __forceinline__ void wave_sum_halve(double (&a)[K], int lane) {
    if constexpr (H >= 1) {
        const bool up = (lane & O) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const double keep = up ? a[i + H] : a[i];
            const double send = up ? a[i] : a[i + H];
            a[i] = keep + __shfl_xor(send, O, BAMG_WAVE);
        }
        wave_sum_halve<K, H / 2, O / 2>(a, lane);
    } else {
#pragma unroll
        for (int o = O; o >= 1; o >>= 1) a[0] += __shfl_xor(a[0], o, BAMG_WAVE);
    }
}

template <int K>
__device__ __forceinline__ void wave_sum_many(double (&a)[K]) {
    wave_sum_halve<K, K / 2, BAMG_WAVE / 2>(a, threadIdx.x % BAMG_WAVE);
}

// Reduction scratch of the passes (per wave: the KR + 2 sums of a row block).
template <int K>
struct GsRed { static constexpr int KR = K <= 8 ? 8 : K <= 16 ? 16 : K <= 32 ? 32 : 64; };

// Partial sums of a block for several dots at once: K accumulators per
// thread (K <= 64) reduced per wavefront by butterfly exchanges on the next
// power of two KR of K (so a dot's summation order depends only on KR), then
// the four wave totals in order.  Writes nb + 2 values, d < nb: acc[d],
// d = nb: ey, d = nb + 1: ex, to part[((blockIdx.y NDM) + d) gridDim.x +
// blockIdx.x].  red: (BAMG_BLK / BAMG_WAVE) (KR + 2) doubles of LDS.
template <int K>
__device__ __forceinline__ void gs_store_partials(double (&acc_k)[K], double ey, double ex, int nb,
                                                  double* __restrict__ part, int NDM, double* red) {
    // the lane reduction runs on the next power of two (8 .. 64) of K, so a
    // dot's summation order depends only on that power, not on K itself
    constexpr int KR = K <= 8 ? 8 : K <= 16 ? 16 : K <= 32 ? 32 : 64;
    constexpr int SH = KR >= 64 ? 0 : KR >= 32 ? 1 : KR >= 16 ? 2 : 3;
    static_assert((BAMG_WAVE >> SH) == KR && K <= KR, "K must be at most 64");
    double acc[KR];
#pragma unroll
    for (int b = 0; b < KR; ++b) acc[b] = b < K ? acc_k[b] : 0.0;
    const int lane = threadIdx.x % BAMG_WAVE, wv = threadIdx.x / BAMG_WAVE;
    wave_sum_many<KR>(acc);
    ey = wave_sum(ey);
    ex = wave_sum(ex);
    if ((lane & ((1 << SH) - 1)) == 0) red[wv * (KR + 2) + (lane >> SH)] = acc[0];
    if (lane == 0) { red[wv * (KR + 2) + KR] = ey; red[wv * (KR + 2) + KR + 1] = ex; }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < nb + 2) {
        const int src = t < nb ? t : KR + (t - nb);
        double v = 0;
#pragma unroll
        for (int q = 0; q < BAMG_BLK / BAMG_WAVE; ++q) v += red[q * (KR + 2) + src];
        part[((size_t)blockIdx.y * NDM + t) * gridDim.x + blockIdx.x] = v;
    }
}

// Sum over a block of BAMG_BLK threads in a fixed order (lane tree, then the
// four wave totals in order).  Result valid in thread 0.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x % BAMG_WAVE, w = threadIdx.x / BAMG_WAVE;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    T s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < BAMG_BLK / BAMG_WAVE; ++i) s += sh[i];
    return s;
}

// 1/p from v_rcp_f64 refined by two Newton steps (within an ulp or so of the
// rounded quotient, without the full division sequence).
__device__ __forceinline__ double cz_recip(double p) {
    double r = __builtin_amdgcn_rcp(p);
    double e = fma(-p, r, 1.0);
    r = fma(r, e, r);
    e = fma(-p, r, 1.0);
    return fma(r, e, r);
}

// Lane l's value of v (l uniform across the wave), without LDS.
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)u, l), hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__host__ __device__ __forceinline__ int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Full coarsening along one grid direction of length m: the coarse
// positions are the even ones and, on a side that is not periodic, also the
// last position m - 1 (both ends of every side stay coarse, as "every other
// point" does on the sides 2^k + 1 of Section 5).  A coarse position y has
// rank (y + 1) >> 1 among the coarse positions of its side; coarse position
// A sits at fine position 2A, or m - 1 for the last one of a non-periodic
// side.  A fine position is odd and interpolates from y - 1 and y + 1, both
// coarse (periodic sides wrap).
__host__ __device__ __forceinline__ bool grid_cpos(int y, int m, int periodic) {
    return !(y & 1) || (!periodic && y == m - 1);
}
__host__ __device__ __forceinline__ int grid_coarse_side(int m, int periodic) {
    return periodic ? (m + 1) / 2 : m / 2 + 1;
}
__host__ __device__ __forceinline__ int grid_fine_pos(int A, int m, int periodic) {
    return (periodic || 2 * A < m) ? 2 * A : m - 1;
}
// Number of fine positions (odd ones, the last of a non-periodic side
// excepted) along a side of length m.
__host__ __device__ __forceinline__ int grid_fine_count(int m, int periodic) {
    return m / 2 - ((!periodic && m > 1 && !(m & 1)) ? 1 : 0);
}

// Several chains are handled as one block-diagonal system: on every level the
// rows of chain c form the range [off, off + n).  Chains are ordered by depth
// (deepest first), so the chains that continue to the next level always form
// a prefix of the rows.  One record per chain and level:
struct ChainGeo {
    int off, n;             // rows of this chain on this level
    int nx, ny, periodic;   // its grid (state s = a*ny + b, local numbering);
                            // nx = 0 (ny = 1): no grid
    FastDiv dy;             // division by ny
    int coff, cn;           // its rows on the next level (cn = 0: coarsest here)
    int ncx, ncy;           // next-level grid
    FastDiv dcy;            // division by ncy
};

// Chain owning row i (the records are sorted by off; nch >= 1).
__device__ __forceinline__ int find_chain(const ChainGeo* __restrict__ g, int nch, int i) {
    int lo = 0, hi = nch - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (g[mid].off <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// f(chain of row i) for a row i of a workgroup whose rows are b0 .. b1
// (b0 <= i <= b1).  When those rows lie in one chain (the usual case) the
// chain is passed as a workgroup-uniform value, so the per-chain records f
// reads are scalar loads rather than one vector load per lane.
template <typename F>
__device__ __forceinline__ auto with_chain(const ChainGeo* __restrict__ g, int nch, int b0, int b1, int i, F&& f) {
    const int cf = find_chain(g, nch, b0);
    const int cl = nch == 1 ? cf : find_chain(g, nch, b1);
    if (cf == cl) return f(__builtin_amdgcn_readfirstlane(cf));
    return f(find_chain(g, nch, i));
}

// Colours of the multicolour Gauss-Seidel relaxation: along one grid
// direction of length m the positions alternate between colours 0 and 1, and
// a periodic direction of odd length gives its last position colour 2, so
// neighbours always differ; a point's colour is ca * (colours along b) + cb.
// Two distinct points within Chebyshev distance 1 (the stencil reach of every
// operator of the hierarchy) therefore never share a colour.
__host__ __device__ __forceinline__ int dir_colours(int m, int periodic) {
    return (periodic && (m & 1) && m > 1) ? 3 : 2;
}
__host__ __device__ __forceinline__ int dir_colour(int a, int m, int periodic) {
    return (periodic && (m & 1) && m > 1 && a == m - 1) ? 2 : (a & 1);
}
__device__ __forceinline__ int point_colour(const ChainGeo& g, int li) {
    const int ia = (int)g.dy.div((uint32_t)li), ib = li - ia * g.ny;
    return dir_colour(ia, g.nx, g.periodic) * dir_colours(g.ny, g.periodic) + dir_colour(ib, g.ny, g.periodic);
}

// Chain mask of the batched cycle: a workgroup whose rows [r0, r1] belong only
// to chains with act[c] == 0 has nothing to do (act == nullptr: every chain is
// active).  The result is the same for every thread of the workgroup.
struct RowMask {
    const ChainGeo* geo;
    int nch;
    const int* act;
};

__device__ __forceinline__ bool rows_active(const RowMask& m, int r0, int r1) {
    if (!m.act) return true;
    const int c0 = find_chain(m.geo, m.nch, r0), c1 = find_chain(m.geo, m.nch, r1);
    for (int c = c0; c <= c1; ++c)
        if (m.act[c]) return true;
    return false;
}

// Rows [tile * blk / R, ((tile + 1) * blk - 1) / R] of an n-row operator
// handled by workgroup `tile` of a thread-per-(row, column) kernel.
__device__ __forceinline__ bool tile_active(const RowMask& m, int tile, int blk, int R, int n) {
    if (!m.act) return true;
    const long long t0 = (long long)tile * blk;
    const int r0 = (int)(t0 / R);
    const int r1 = (int)min((long long)n - 1, (t0 + blk - 1) / R);
    return r0 < n && rows_active(m, r0, r1);
}
