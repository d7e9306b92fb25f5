// Relaxation sweeps on interleaved test vectors (Section 3, eq. amg_relax):
// the row product used by every sweep and the vector forms of the multi-vector
// sweep the autotuner chooses from.  Kept in a header of its own so that its
// measured HBM traffic is tied to exactly this source.
#pragma once
#include "common.h"

template <typename T, typename M>
__device__ __forceinline__ T row_dot(int p0, int p1, const int* __restrict__ ci, const M* __restrict__ v,
                                     const T* __restrict__ X, int R, int k, int self) {
    T acc = 0;
    for (int p = p0; p < p1; p += 4) {
        int c[4];
        M w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            bool ok = p + u < p1;
            c[u] = ok ? ci[p + u] : self;
            w[u] = ok ? v[p + u] : (M)0;
        }
        T x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = X[(size_t)c[u] * R + k];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += (T)w[u] * x[u];
    }
    return acc;
}

// Vector forms of the sweep for the autotuner: a thread owns VW adjacent
// columns of one row (G = R / VW threads per row) and moves them with 8- or
// 16-byte loads; blocks of BS threads.  Same arithmetic per entry as k_sweep
// (products added in CSR order), so every variant gives the same bits.
template <typename T, int VW>
struct VecIO;
template <> struct VecIO<double, 1> {
    static __device__ __forceinline__ void ld(const double* p, double* x) { x[0] = *p; }
    static __device__ __forceinline__ void st(double* p, const double* x) { *p = x[0]; }
};
template <> struct VecIO<double, 2> {
    static __device__ __forceinline__ void ld(const double* p, double* x) {
        const double2 v = *(const double2*)p; x[0] = v.x; x[1] = v.y;
    }
    static __device__ __forceinline__ void st(double* p, const double* x) { *(double2*)p = make_double2(x[0], x[1]); }
};
template <> struct VecIO<double, 4> {
    static __device__ __forceinline__ void ld(const double* p, double* x) {
        const double2 a = ((const double2*)p)[0], b = ((const double2*)p)[1];
        x[0] = a.x; x[1] = a.y; x[2] = b.x; x[3] = b.y;
    }
    static __device__ __forceinline__ void st(double* p, const double* x) {
        ((double2*)p)[0] = make_double2(x[0], x[1]);
        ((double2*)p)[1] = make_double2(x[2], x[3]);
    }
};
template <> struct VecIO<float, 1> {
    static __device__ __forceinline__ void ld(const float* p, float* x) { x[0] = *p; }
    static __device__ __forceinline__ void st(float* p, const float* x) { *p = x[0]; }
};
template <> struct VecIO<float, 2> {
    static __device__ __forceinline__ void ld(const float* p, float* x) {
        const float2 v = *(const float2*)p; x[0] = v.x; x[1] = v.y;
    }
    static __device__ __forceinline__ void st(float* p, const float* x) { *(float2*)p = make_float2(x[0], x[1]); }
};
template <> struct VecIO<float, 4> {
    static __device__ __forceinline__ void ld(const float* p, float* x) {
        const float4 v = *(const float4*)p; x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    }
    static __device__ __forceinline__ void st(float* p, const float* x) {
        *(float4*)p = make_float4(x[0], x[1], x[2], x[3]);
    }
};

// Wider groups: 3, 6 or 12 adjacent columns.  For doubles, VW even -> 16-byte
// pieces (row bases are 16-byte aligned when R is even); otherwise 8-byte.
// For floats, 4-float pieces when VW % 4 == 0, else 2-float or single.
template <typename T, int VW>
struct VecIOn {
    static constexpr int P = sizeof(T) == 8 ? (VW % 2 == 0 ? 2 : 1) : (VW % 4 == 0 ? 4 : (VW % 2 == 0 ? 2 : 1));
    static __device__ __forceinline__ void ld(const T* p, T* x) {
#pragma unroll
        for (int k = 0; k < VW; k += P) VecIO<T, P>::ld(p + k, x + k);
    }
    static __device__ __forceinline__ void st(T* p, const T* x) {
#pragma unroll
        for (int k = 0; k < VW; k += P) VecIO<T, P>::st(p + k, x + k);
    }
};
template <> struct VecIO<double, 3> : VecIOn<double, 3> {};
template <> struct VecIO<double, 6> : VecIOn<double, 6> {};
template <> struct VecIO<double, 12> : VecIOn<double, 12> {};
template <> struct VecIO<float, 3> : VecIOn<float, 3> {};
template <> struct VecIO<float, 6> : VecIOn<float, 6> {};
template <> struct VecIO<float, 12> : VecIOn<float, 12> {};

template <typename T, typename M, int VW, int BS>
__global__ void __launch_bounds__(BS)
k_sweep_v(int n, int G, FastDiv divG, const int* __restrict__ rp, const int* __restrict__ ci,
          const M* __restrict__ v, const M* __restrict__ dinv, const T* __restrict__ X,
          const T* __restrict__ F, T* __restrict__ Y) {
    const int t = xcd_tile(blockIdx.x, gridDim.x) * BS + threadIdx.x;
    if (t >= n * G) return;
    const int i = (int)divG.div((uint32_t)t), kg = t - i * G;
    const int R = G * VW;
    const size_t base = (size_t)i * R + (size_t)kg * VW;
    T xt[VW], f[VW], acc[VW];
    VecIO<T, VW>::ld(X + base, xt);
    if (F) VecIO<T, VW>::ld(F + base, f);
    else
#pragma unroll
        for (int q = 0; q < VW; ++q) f[q] = (T)0;
#pragma unroll
    for (int q = 0; q < VW; ++q) acc[q] = (T)0;
    const T d = (T)dinv[i];
    const int p0 = rp[i], p1 = rp[i + 1];
    for (int p = p0; p < p1; p += 4) {
        int c[4];
        M w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool ok = p + u < p1;
            c[u] = ok ? ci[p + u] : i;
            w[u] = ok ? v[p + u] : (M)0;
        }
        T x[4][VW];
#pragma unroll
        for (int u = 0; u < 4; ++u) VecIO<T, VW>::ld(X + (size_t)c[u] * R + (size_t)kg * VW, x[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < VW; ++q) acc[q] += (T)w[u] * x[u][q];
    }
    T y[VW];
#pragma unroll
    for (int q = 0; q < VW; ++q) y[q] = xt[q] + d * (f[q] - acc[q]);
    VecIO<T, VW>::st(Y + base, y);
}


// The same sweep on a 4-wide ELL copy of B (row i's entries at 4i .. 4i+3 in
// CSR order, padded with (i, 0)): the columns and values of a row arrive in
// one 16-byte load each and no row pointer is read first.  Rows of B with at
// most 4 entries only; the sums are those of k_sweep_v bit for bit.
template <typename M>
struct Ell4Val;
template <> struct Ell4Val<float> {
    static __device__ __forceinline__ void ld(const float* p, float* w) {
        const float4 a = *(const float4*)p; w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
    }
    // the four FP64 values rounded to FP32, one 16-byte store
    static __device__ __forceinline__ void st(float* p, const double* w) {
        *(float4*)p = make_float4((float)w[0], (float)w[1], (float)w[2], (float)w[3]);
    }
};
template <> struct Ell4Val<double> {
    static __device__ __forceinline__ void ld(const double* p, double* w) {
        const double2 a = ((const double2*)p)[0], b = ((const double2*)p)[1];
        w[0] = a.x; w[1] = a.y; w[2] = b.x; w[3] = b.y;
    }
    static __device__ __forceinline__ void st(double* p, const double* w) {
        ((double2*)p)[0] = make_double2(w[0], w[1]);
        ((double2*)p)[1] = make_double2(w[2], w[3]);
    }
};

// Streaming forms of the accesses that touch each byte once (the ELL arrays,
// D^-1 and the output): non-temporal, so that they do not displace the
// neighbour rows of X from the caches.  Used where a row piece is 8 or 16
// bytes; otherwise the plain forms.
template <typename T, int VW>
struct StreamIO {
    static constexpr bool vec = (sizeof(T) * VW == 16 || sizeof(T) * VW == 8) && VW > 1;
    static __device__ __forceinline__ void st(T* p, const T* x) {
        if constexpr (vec) {
            typedef T V __attribute__((ext_vector_type(VW)));
            V v;
#pragma unroll
            for (int q = 0; q < VW; ++q) v[q] = x[q];
            __builtin_nontemporal_store(v, (V*)p);
        } else if constexpr (VW == 1) {
            __builtin_nontemporal_store(x[0], p);
        } else {
            VecIO<T, VW>::st(p, x);
        }
    }
};
__device__ __forceinline__ int4 ld_nt_i4(const int* p) {
    typedef int V __attribute__((ext_vector_type(4)));
    const V v = __builtin_nontemporal_load((const V*)p);
    return make_int4(v[0], v[1], v[2], v[3]);
}
template <typename M>
__device__ __forceinline__ void ld_nt_w4(const M* p, M* w) {
    typedef M V __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(M) == 4) {
        typedef M V4 __attribute__((ext_vector_type(4)));
        const V4 v = __builtin_nontemporal_load((const V4*)p);
        w[0] = v[0]; w[1] = v[1]; w[2] = v[2]; w[3] = v[3];
    } else {
        const V a = __builtin_nontemporal_load((const V*)p), b = __builtin_nontemporal_load((const V*)p + 1);
        w[0] = a[0]; w[1] = a[1]; w[2] = b[0]; w[3] = b[1];
    }
}

// A thread takes RP row pieces spaced ceil(n G / RP) pieces apart: with two,
// each wavefront has twice the loads in flight at the same occupancy.  The
// index loads of all its pieces are issued first, then all gathers.
template <typename T, typename M, int VW, int BS, int RP = 1>
__global__ void __launch_bounds__(BS)
k_sweep_ve(int n, int G, FastDiv divG, const int* __restrict__ eci, const M* __restrict__ ev,
           const M* __restrict__ dinv, const T* __restrict__ X, const T* __restrict__ F, T* __restrict__ Y) {
    const int tot = n * G, span = RP == 1 ? tot : (tot + RP - 1) / RP;
    const int t0 = xcd_tile(blockIdx.x, gridDim.x) * BS + threadIdx.x;
    if (t0 >= span) return;
    const int R = G * VW;
    int i[RP], kg[RP];
    bool ok[RP];
    int4 c4[RP];
    M w[RP][4];
    T xt[RP][VW], f[RP][VW], d[RP];
#pragma unroll
    for (int h = 0; h < RP; ++h) {
        const int t = t0 + h * span;
        ok[h] = h == 0 || t < tot;
        const int tt = ok[h] ? t : t0;            // a piece past the end redoes the first one
        i[h] = (int)divG.div((uint32_t)tt);
        kg[h] = tt - i[h] * G;
        c4[h] = ld_nt_i4(eci + (size_t)i[h] * 4);
        ld_nt_w4<M>(ev + (size_t)i[h] * 4, w[h]);
        const size_t base = (size_t)i[h] * R + (size_t)kg[h] * VW;
        VecIO<T, VW>::ld(X + base, xt[h]);
        if (F) VecIO<T, VW>::ld(F + base, f[h]);
        else
#pragma unroll
            for (int q = 0; q < VW; ++q) f[h][q] = (T)0;
        d[h] = (T)__builtin_nontemporal_load(dinv + i[h]);
    }
    T x[RP][4][VW];
#pragma unroll
    for (int h = 0; h < RP; ++h) {
        const int c[4] = {c4[h].x, c4[h].y, c4[h].z, c4[h].w};
#pragma unroll
        for (int u = 0; u < 4; ++u) VecIO<T, VW>::ld(X + (size_t)c[u] * R + (size_t)kg[h] * VW, x[h][u]);
    }
#pragma unroll
    for (int h = 0; h < RP; ++h) {
        T acc[VW];
#pragma unroll
        for (int q = 0; q < VW; ++q) acc[q] = (T)0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < VW; ++q) acc[q] += (T)w[h][u] * x[h][u][q];
        T y[VW];
#pragma unroll
        for (int q = 0; q < VW; ++q) y[q] = xt[h][q] + d[h] * (f[h][q] - acc[q]);
        if (ok[h]) StreamIO<T, VW>::st(Y + (size_t)i[h] * R + (size_t)kg[h] * VW, y);
    }
}

