// Learned interpolation weights: a 24-64-64-4 ReLU network on the matrix
// cores (v_mfma_f32_16x16x16_bf16: bfloat16 operands, FP32 accumulation).
//
// The network maps 24 scale-free features of a fine point's least-squares
// problem (Section 3.2) to its 4 slot weights.  Parameters are FP32 master
// copies (flat, row-major): W1 [64][24], b1 [64], W2 [64][64], b2 [64],
// W3 [4][64], b3 [4]; every product rounds its operands to bfloat16 (nearest,
// ties to even) and accumulates in FP32.
//
// MFMA 16x16x16 operand layout (wave64, lane l, q = l / 16, r = l % 16):
//   A (16 x 16, M x K): lane holds A[r][4q .. 4q+3]
//   B (16 x 16, K x N): lane holds B[4q .. 4q+3][r]
//   D (16 x 16, M x N): lane holds D[4q .. 4q+3][r]
// So a D tile of X is, read lane by lane, the A operand of X^T and the B
// operand of X: the weight gradients (sums over points) take activations and
// output gradients straight from the registers; only the products with the
// points as rows need a transpose through LDS.
#pragma once
#include "common.h"

#define MLP_IN 24
#define MLP_INP 32
#define MLP_H 64
#define MLP_OUT 4
#define MLP_NPARAM 6020
#define MLP_OW1 0
#define MLP_OB1 1536
#define MLP_OW2 1600
#define MLP_OB2 5696
#define MLP_OW3 5760
#define MLP_OB3 6016

typedef short mlp_bf4 __attribute__((ext_vector_type(4)));
typedef float mlp_f4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest, ties to even (NaN kept quiet).
__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ mlp_f4 mfma16(mlp_bf4 a, mlp_bf4 b, mlp_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ mlp_bf4 pack4(float a, float b, float c, float d) {
    mlp_bf4 v;
    v[0] = (short)f2bf(a); v[1] = (short)f2bf(b); v[2] = (short)f2bf(c); v[3] = (short)f2bf(d);
    return v;
}
__device__ __forceinline__ mlp_bf4 pack4(mlp_f4 x) { return pack4(x[0], x[1], x[2], x[3]); }

// Four consecutive bfloat16 values (8-byte aligned) from LDS or global memory.
__device__ __forceinline__ mlp_bf4 ld4(const unsigned short* p) { return *(const mlp_bf4*)p; }

// The weights as bfloat16 in the layouts the B operands read (each lane reads
// four consecutive values), plus FP32 biases.  Built once per parameter
// vector (k_mlp_pack) and copied into LDS by every workgroup that uses it.
struct MlpPack {
    unsigned short w1[MLP_H][MLP_INP];     // W1, inputs padded to 32 with zeros
    unsigned short w2[MLP_H][MLP_H];       // W2 [out][in]
    unsigned short w2t[MLP_H][MLP_H];      // W2^T [in][out]
    unsigned short w3[16][MLP_H];          // W3, outputs padded to 16
    unsigned short w3t[MLP_H][16];         // W3^T, outputs padded to 16
    float b1[MLP_H], b2[MLP_H], b3[16];
};

__global__ void k_mlp_pack(const float* __restrict__ th, MlpPack* __restrict__ pk) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < MLP_H * MLP_H; e += gridDim.x * blockDim.x) {
        const int o = e / MLP_H, i = e % MLP_H;
        const unsigned short w2 = f2bf(th[MLP_OW2 + o * MLP_H + i]);
        pk->w2[o][i] = w2;
        pk->w2t[i][o] = w2;
        if (i < MLP_INP) pk->w1[o][i] = i < MLP_IN ? f2bf(th[MLP_OW1 + o * MLP_IN + i]) : (unsigned short)0;
        if (o < 16) {
            const unsigned short w3 = o < MLP_OUT ? f2bf(th[MLP_OW3 + o * MLP_H + i]) : (unsigned short)0;
            pk->w3[o][i] = w3;
            pk->w3t[i][o] = w3;
        }
        if (e < MLP_H) { pk->b1[e] = th[MLP_OB1 + e]; pk->b2[e] = th[MLP_OB2 + e]; }
        if (e < 16) pk->b3[e] = e < MLP_OUT ? th[MLP_OB3 + e] : 0.0f;
    }
}

// Copy the packed weights into LDS (16-byte pieces), all threads of a block.
__device__ __forceinline__ void mlp_stage(const MlpPack* __restrict__ g, MlpPack* s) {
    const uint4* src = (const uint4*)g;
    uint4* dst = (uint4*)s;
    for (int e = threadIdx.x; e < (int)(sizeof(MlpPack) / 16); e += blockDim.x) dst[e] = src[e];
}

// He-uniform initial weights, U(-sqrt(6 / fan_in), sqrt(6 / fan_in)) from the
// counter generator (seed, stream 5, flat index); biases zero.
__global__ void k_mlp_init(uint64_t seed, float* __restrict__ th) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= MLP_NPARAM) return;
    double lim = 0.0;
    if (k < MLP_OB1) lim = sqrt(6.0 / MLP_IN);
    else if (k >= MLP_OW2 && k < MLP_OB2) lim = sqrt(6.0 / MLP_H);
    else if (k >= MLP_OW3 && k < MLP_OB3) lim = sqrt(6.0 / MLP_H);
    th[k] = lim > 0 ? (float)((2.0 * splitmix_u01(seed, 5ull, (uint64_t)k) - 1.0) * lim) : 0.0f;
}

// Input rows as bfloat16, padded to 32 (for training and standalone use).
__global__ void k_mlp_prep(long long n, const float* __restrict__ feat, unsigned short* __restrict__ xb) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * MLP_INP) return;
    const long long p = e / MLP_INP;
    const int k = (int)(e - p * MLP_INP);
    xb[e] = k < MLP_IN ? f2bf(feat[p * MLP_IN + k]) : (unsigned short)0;
}

// Forward pass of one 16-point tile of a wave.  xt: the tile's inputs in LDS
// ([16][32] bfloat16, row stride MLP_INP); ht: wave scratch [16][MLP_H + 8];
// returns the output tile (D layout, outputs 0..3 in lanes r < 4) and keeps
// the pre-activations and activations the backward pass needs.
struct MlpTile {
    mlp_f4 z1[4], z2[4];        // pre-activations, D layout, N-tile t = features 16 t ..
    mlp_bf4 h1[4], h2[4];       // activations as bfloat16, D layout
    mlp_f4 y;                   // outputs, D layout (r < 4)
};

#define MLP_HLD (MLP_H + 8)

__device__ __forceinline__ void mlp_tile_forward(const MlpPack& W, const unsigned short* xt, unsigned short* ht,
                                                 MlpTile& T) {
    const int l = threadIdx.x % BAMG_WAVE, q = l / 16, r = l % 16;
    mlp_bf4 ax[2];
    ax[0] = ld4(xt + r * MLP_INP + 4 * q);
    ax[1] = ld4(xt + r * MLP_INP + 16 + 4 * q);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        mlp_f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) acc = mfma16(ax[ks], ld4(&W.w1[16 * t + r][16 * ks + 4 * q]), acc);
        const float bias = W.b1[16 * t + r];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += bias;
        T.z1[t] = acc;
        T.h1[t] = pack4(fmaxf(acc[0], 0.f), fmaxf(acc[1], 0.f), fmaxf(acc[2], 0.f), fmaxf(acc[3], 0.f));
#pragma unroll
        for (int i = 0; i < 4; ++i) ht[(4 * q + i) * MLP_HLD + 16 * t + r] = (unsigned short)T.h1[t][i];
    }
    __syncthreads();
    mlp_bf4 ah[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) ah[ks] = ld4(ht + r * MLP_HLD + 16 * ks + 4 * q);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        mlp_f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) acc = mfma16(ah[ks], ld4(&W.w2[16 * t + r][16 * ks + 4 * q]), acc);
        const float bias = W.b2[16 * t + r];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += bias;
        T.z2[t] = acc;
        T.h2[t] = pack4(fmaxf(acc[0], 0.f), fmaxf(acc[1], 0.f), fmaxf(acc[2], 0.f), fmaxf(acc[3], 0.f));
#pragma unroll
        for (int i = 0; i < 4; ++i) ht[(4 * q + i) * MLP_HLD + 16 * t + r] = (unsigned short)T.h2[t][i];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) ah[ks] = ld4(ht + r * MLP_HLD + 16 * ks + 4 * q);
    __syncthreads();
    mlp_f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) acc = mfma16(ah[ks], ld4(&W.w3[r][16 * ks + 4 * q]), acc);
    const float bias = W.b3[r];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += bias;
    T.y = acc;
}

// Standalone inference: Y[p][0..3] for n input rows (bfloat16, stride 32).
// Blocks of 256 threads; each wave takes 64 consecutive points per pass.
struct MlpInferSmem {
    MlpPack w;
    unsigned short x[4][64][MLP_INP];
    unsigned short h[4][16][MLP_HLD];
};

__global__ void __launch_bounds__(BAMG_BLK)
k_mlp_infer(long long n, const unsigned short* __restrict__ xb, const MlpPack* __restrict__ pk, float* __restrict__ Y) {
    __shared__ MlpInferSmem S;
    mlp_stage(pk, &S.w);
    const int w = threadIdx.x / BAMG_WAVE, l = threadIdx.x % BAMG_WAVE, q = l / 16, r = l % 16;
    __syncthreads();
    for (long long base = (long long)blockIdx.x * 256; base < n; base += (long long)gridDim.x * 256) {
        const long long p0 = base + 64 * w;
        // this wave's 64 rows (row l), zero past the end
        {
            const long long p = p0 + l;
            const uint4* src = (const uint4*)(xb + p * MLP_INP);
            uint4* dst = (uint4*)&S.x[w][l][0];
#pragma unroll
            for (int k = 0; k < MLP_INP / 8; ++k) dst[k] = p < n ? src[k] : make_uint4(0, 0, 0, 0);
        }
        __syncthreads();
        for (int m = 0; m < 4; ++m) {
            MlpTile T;
            mlp_tile_forward(S.w, &S.x[w][16 * m][0], &S.h[w][0][0], T);
            if (r < MLP_OUT) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const long long p = p0 + 16 * m + 4 * q + i;
                    if (p < n) Y[p * MLP_OUT + r] = T.y[i];
                }
            }
        }
        __syncthreads();
    }
}

// Sample index of batch element e of training step `step`: contiguous
// (seed == 0: first + e) or drawn with replacement from the counter
// generator (stream 6).
__device__ __forceinline__ long long mlp_sample(long long n, long long first, uint64_t seed, long long step, int bsz,
                                                int e) {
    if (seed == 0) return first + e;
    const double u = splitmix_u01(seed, 6ull, (uint64_t)(step * bsz + e));
    long long p = (long long)(u * (double)n);
    return p < n ? p : n - 1;
}

// Number of fitted outputs (valid slots, the first 4 inputs) of a batch,
// per block -> part[block]; k_mlp_sum adds them in order.
__global__ void k_mlp_count(long long n, int bsz, long long first, uint64_t seed, long long step,
                            const unsigned short* __restrict__ xb, float* __restrict__ part) {
    __shared__ float sh[BAMG_BLK / BAMG_WAVE];
    const int e = blockIdx.x * BAMG_BLK + threadIdx.x;
    float c = 0.f;
    if (e < bsz) {
        const long long p = mlp_sample(n, first, seed, step, bsz, e);
#pragma unroll
        for (int s = 0; s < MLP_OUT; ++s) c += bf2f(xb[p * MLP_INP + s]);
    }
    c = block_sum(c, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = c;
}

// Forward and backward of one batch: each wave takes 64 batch elements (four
// tiles of 16) and writes its partial gradient (MLP_NPARAM floats) and its
// partial loss sum M (Y - T)^2 / cnt to wpart[wave].  cnt: device scalar.
struct MlpTrainSmem {
    MlpPack w;
    unsigned short x[4][64][MLP_INP];
    unsigned short h[4][16][MLP_HLD];
    unsigned short dy[4][16][16];
};

__global__ void __launch_bounds__(BAMG_BLK)
k_mlp_fwdbwd(long long n, int bsz, long long first, uint64_t seed, long long step, const unsigned short* __restrict__ xb,
             const float* __restrict__ tgt, const MlpPack* __restrict__ pk, const float* __restrict__ cntp,
             float* __restrict__ wpart, float* __restrict__ lpart) {
    __shared__ MlpTrainSmem S;
    mlp_stage(pk, &S.w);
    const int w = threadIdx.x / BAMG_WAVE, l = threadIdx.x % BAMG_WAVE, q = l / 16, r = l % 16;
    const int e0 = (blockIdx.x * 4 + w) * 64;          // first batch element of this wave
    {
        const int e = e0 + l;
        uint4* dst = (uint4*)&S.x[w][l][0];
        if (e < bsz) {
            const long long p = mlp_sample(n, first, seed, step, bsz, e);
            const uint4* src = (const uint4*)(xb + p * MLP_INP);
#pragma unroll
            for (int k = 0; k < MLP_INP / 8; ++k) dst[k] = src[k];
        } else {
#pragma unroll
            for (int k = 0; k < MLP_INP / 8; ++k) dst[k] = make_uint4(0, 0, 0, 0);
        }
    }
    __syncthreads();
    const float inv_cnt = 1.0f / fmaxf(1.0f, *cntp);
    mlp_f4 gw1[4][2], gw2[4][4], gw3[4];
    mlp_f4 gb1[4], gb2[4];
    float gb3 = 0.f, lsum = 0.f;
    const mlp_f4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gw3[a] = zero; gb1[a] = zero; gb2[a] = zero;
#pragma unroll
        for (int b = 0; b < 2; ++b) gw1[a][b] = zero;
#pragma unroll
        for (int b = 0; b < 4; ++b) gw2[a][b] = zero;
    }
    unsigned short* ht = &S.h[w][0][0];
    for (int m = 0; m < 4; ++m) {
        MlpTile T;
        const unsigned short* xt = &S.x[w][16 * m][0];
        mlp_tile_forward(S.w, xt, ht, T);
        // dY = 2 M (Y - T) / cnt in lanes r < 4 (output r of points 4q + i)
        float dy[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int pt = 4 * q + i, e = e0 + 16 * m + pt;
            float d = 0.f;
            if (r < MLP_OUT && e < bsz) {
                const long long p = mlp_sample(n, first, seed, step, bsz, e);
                const float mk = bf2f(xt[pt * MLP_INP + r]);
                d = mk * (T.y[i] - tgt[p * MLP_OUT + r]);
            }
            lsum += d * d;
            dy[i] = 2.0f * d * inv_cnt;
            gb3 += dy[i];
        }
        const mlp_bf4 dyb = pack4(dy[0], dy[1], dy[2], dy[3]);
        // dW3 += dY^T H2
#pragma unroll
        for (int t = 0; t < 4; ++t) gw3[t] = mfma16(dyb, T.h2[t], gw3[t]);
        // dH2 = dY W3 (dY as the A operand: points as rows, through LDS)
#pragma unroll
        for (int i = 0; i < 4; ++i) S.dy[w][4 * q + i][r] = (unsigned short)dyb[i];
        __syncthreads();
        const mlp_bf4 ady = ld4(&S.dy[w][r][4 * q]);
        __syncthreads();
        mlp_f4 dz2[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            mlp_f4 acc = mfma16(ady, ld4(&S.w.w3t[16 * t + r][4 * q]), zero);
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = T.z2[t][i] > 0.f ? acc[i] : 0.f;
            dz2[t] = acc;
#pragma unroll
            for (int i = 0; i < 4; ++i) gb2[t][i] += acc[i];
        }
        mlp_bf4 dz2b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) dz2b[t] = pack4(dz2[t]);
        // dW2 += dZ2^T H1
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) gw2[a][b] = mfma16(dz2b[a], T.h1[b], gw2[a][b]);
        // dH1 = dZ2 W2 (dZ2 transposed through LDS)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) ht[(4 * q + i) * MLP_HLD + 16 * t + r] = (unsigned short)dz2b[t][i];
        __syncthreads();
        mlp_bf4 adz[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) adz[ks] = ld4(ht + r * MLP_HLD + 16 * ks + 4 * q);
        __syncthreads();
        mlp_bf4 dz1b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            mlp_f4 acc = zero;
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) acc = mfma16(adz[ks], ld4(&S.w.w2t[16 * t + r][16 * ks + 4 * q]), acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = T.z1[t][i] > 0.f ? acc[i] : 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) gb1[t][i] += acc[i];
            dz1b[t] = pack4(acc);
        }
        // dW1 += dZ1^T X: X as the B operand (points as K) read from LDS
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            mlp_bf4 xbk;
#pragma unroll
            for (int j = 0; j < 4; ++j) xbk[j] = (short)xt[(4 * q + j) * MLP_INP + 16 * b + r];
#pragma unroll
            for (int a = 0; a < 4; ++a) gw1[a][b] = mfma16(dz1b[a], xbk, gw1[a][b]);
        }
    }
    // write this wave's partial gradient
    float* g = wpart + (size_t)(blockIdx.x * 4 + w) * MLP_NPARAM;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int in = 16 * b + r;
            if (in < MLP_IN)
#pragma unroll
                for (int i = 0; i < 4; ++i) g[MLP_OW1 + (16 * a + 4 * q + i) * MLP_IN + in] = gw1[a][b][i];
        }
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) g[MLP_OW2 + (16 * a + 4 * q + i) * MLP_H + 16 * b + r] = gw2[a][b][i];
        if (q == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i) g[MLP_OW3 + i * MLP_H + 16 * a + r] = gw3[a][i];
    }
    // bias gradients: sum the four point groups (lanes r, r+16, r+32, r+48)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float s1 = gb1[t][0] + gb1[t][1] + gb1[t][2] + gb1[t][3];
        float s2 = gb2[t][0] + gb2[t][1] + gb2[t][2] + gb2[t][3];
        s1 += __shfl_xor(s1, 16, BAMG_WAVE);
        s1 += __shfl_xor(s1, 32, BAMG_WAVE);
        s2 += __shfl_xor(s2, 16, BAMG_WAVE);
        s2 += __shfl_xor(s2, 32, BAMG_WAVE);
        if (q == 0) { g[MLP_OB1 + 16 * t + r] = s1; g[MLP_OB2 + 16 * t + r] = s2; }
    }
    gb3 += __shfl_xor(gb3, 16, BAMG_WAVE);
    gb3 += __shfl_xor(gb3, 32, BAMG_WAVE);
    if (q == 0 && r < MLP_OUT) g[MLP_OB3 + r] = gb3;
    lsum = wave_sum(lsum);
    if (l == 0) lpart[blockIdx.x * 4 + w] = lsum * inv_cnt;
}

// grad[k] = sum over waves w < nw of wpart[w][k] (in wave order).
__global__ void k_mlp_reduce(int nw, const float* __restrict__ wpart, float* __restrict__ grad) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= MLP_NPARAM) return;
    float s = 0.f;
    for (int w = 0; w < nw; ++w) s += wpart[(size_t)w * MLP_NPARAM + k];
    grad[k] = s;
}

// out[0] = sum of part[0 .. np) in order (one block).
__global__ void k_mlp_sum(int np, const float* __restrict__ part, float* __restrict__ out) {
    __shared__ float sh[BAMG_BLK / BAMG_WAVE];
    float s = 0.f;
    for (int j = threadIdx.x; j < np; j += BAMG_BLK) s += part[j];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[0] = s;
}

// Adam (Kingma and Ba, 2015) on the FP32 master weights; c1, c2: the bias
// corrections 1 / (1 - beta^t) of this step.
__global__ void k_mlp_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, float lr, float beta1, float beta2, float eps, float c1,
                           float c2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= MLP_NPARAM) return;
    const float gk = g[k];
    const float mk = beta1 * m[k] + (1.f - beta1) * gk;
    const float vk = beta2 * v[k] + (1.f - beta2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    th[k] -= lr * (mk * c1) / (sqrtf(vk * c2) + eps);
}
