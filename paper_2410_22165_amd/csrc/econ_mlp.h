// econ_mlp.h -- internal device code shared by the policy forward and the
// PPO backward kernels: MLP dimensions, weight layouts, bf16 MFMA tiles.
//
// The network is d_in -> H -> H -> (A logits, 1 value) with ReLU.  fp32
// parameters live in one flat vector (row-major W[in][out], then bias).  The
// kernels read bf16 copies arranged as K-chunks of 32: for a matrix used as
// the B operand of C = A B, element (k, n) sits at [k / 32][n][k % 32], so a
// 32-deep chunk of all N columns is one contiguous block (N x 64 bytes) that
// a workgroup stages into LDS with 16-byte loads.
#pragma once
#include "econ_common.h"

namespace econ {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

struct MlpDims {
    int32_t D, Ds, H, A, A1, K1p, A1p, NC;
    // fp32 parameter offsets (elements)
    int64_t oW1, ob1, oW2, ob2, oW3, ob3, n_params;
    // bf16 work offsets (elements): forward chunks W1f, W2f, W3f; backward chunks W3b, W2b
    int64_t oW1f, oW2f, oW3f, oW3b, oW2b, n_work;
};

__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

__host__ inline int mlp_dims(int D, int Ds, int H, int A, MlpDims* d)
{
    if (D <= 0 || D > 64 || Ds < D || (Ds & 7) != 0 || Ds > 64) return EJ_EUNSUPPORTED;
    if (!(H == 64 || H == 128 || H == 256 || H == 512)) return EJ_EUNSUPPORTED;
    if (A <= 0 || A + 1 > 1024) return EJ_EUNSUPPORTED;
    d->D = D;
    d->Ds = Ds;
    d->H = H;
    d->A = A;
    d->A1 = A + 1;
    d->K1p = 64;  // first-layer input padded to 64 (one layout for every D <= 64)
    d->A1p = round_up(A + 1, 128);
    d->NC = d->A1p / 128;
    int64_t o = 0;
    d->oW1 = o; o += (int64_t)D * H;
    d->ob1 = o; o += H;
    d->oW2 = o; o += (int64_t)H * H;
    d->ob2 = o; o += H;
    d->oW3 = o; o += (int64_t)H * (A + 1);
    d->ob3 = o; o += A + 1;
    d->n_params = o;
    int64_t w = 0;
    d->oW1f = w; w += (int64_t)d->K1p * H;
    d->oW2f = w; w += (int64_t)H * H;
    d->oW3f = w; w += (int64_t)H * d->A1p;
    d->oW3b = w; w += (int64_t)d->A1p * H;
    d->oW2b = w; w += (int64_t)H * H;
    d->n_work = w;
    return EJ_OK;
}

// ---------------------------------------------------------------------------
// LDS-staged weight chunks: [n][40] bf16 (32 k + 8 pad: 80-byte rows keep the
// 16 lanes of a fragment read on distinct banks)
// ---------------------------------------------------------------------------
constexpr int WSTRIDE = 40;

__device__ inline bf16x8 lds_frag(const uint16_t* p) { return *(const bf16x8*)p; }

__device__ inline f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// C[RT*16 rows][N] += A[rows][k-chunk kt] * Wchunk: A rows from LDS (row
// stride `as`, own rows starting at `arow0`), weight chunk staged in wbuf.
template <int RT, int CT>
__device__ inline void mfma_chunk(f32x4 (&acc)[RT][CT], const uint16_t* abuf, int as, int arow0, int kcol,
                                  const uint16_t* wbuf)
{
    const int l = lane_id();
    bf16x8 a[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) a[rt] = lds_frag(abuf + (arow0 + rt * 16 + (l & 15)) * as + kcol + 8 * (l >> 4));
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        bf16x8 b = lds_frag(wbuf + (ct * 16 + (l & 15)) * WSTRIDE + 8 * (l >> 4));
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = mfma16(a[rt], b, acc[rt][ct]);
    }
}

template <int RT, int CT>
__device__ inline void zero_acc(f32x4 (&acc)[RT][CT])
{
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// One dense layer for the workgroup's row tile: every wave multiplies its own
// rows of `abuf` by a weight matrix streamed chunk by chunk through `wbuf`
// (single LDS buffer; the next chunk is prefetched into registers while the
// current one is consumed).  All 256 threads must call it.
// `kstride`: elements between the global chunks of consecutive k-steps.
template <int RT, int N>
__device__ inline void dense_layer(f32x4 (&acc)[RT][N / 16], const uint16_t* abuf, int as, int arow0, int K,
                                   const uint16_t* __restrict__ wglob, int64_t kstride, uint16_t* wbuf,
                                   bool zero = true, int acol0 = 0)
{
    if (zero) zero_acc(acc);
    // register prefetch of the next chunk: plain scalars (an aggregate here
    // ends up in scratch memory)
    constexpr int NP = N / 64;
    uint4 q0, q1, q2, q3, q4, q5, q6, q7;
    auto gload = [&](const uint16_t* src) {
        const uint4* g = (const uint4*)src + threadIdx.x;
        q0 = g[0];
        if constexpr (NP > 1) q1 = g[256];
        if constexpr (NP > 2) { q2 = g[512]; q3 = g[768]; }
        if constexpr (NP > 4) { q4 = g[1024]; q5 = g[1280]; q6 = g[1536]; q7 = g[1792]; }
    };
    auto sput = [&](int j, uint4 v) {
        const int piece = threadIdx.x + 256 * j;
        *(uint4*)(wbuf + (piece >> 2) * WSTRIDE + (piece & 3) * 8) = v;
    };
    gload(wglob);
    const int nk = K / 32;
    for (int kt = 0; kt < nk; ++kt) {
        __syncthreads();  // everyone is done with the previous chunk
        sput(0, q0);
        if constexpr (NP > 1) sput(1, q1);
        if constexpr (NP > 2) { sput(2, q2); sput(3, q3); }
        if constexpr (NP > 4) { sput(4, q4); sput(5, q5); sput(6, q6); sput(7, q7); }
        __syncthreads();
        // the last step re-reads its own chunk: no branch around the loads
        gload(wglob + (int64_t)(kt + 1 < nk ? kt + 1 : kt) * kstride);
        mfma_chunk<RT, N / 16>(acc, abuf, as, arow0, acol0 + kt * 32, wbuf);
    }
}

// bias + ReLU, rounded to bf16, written to the wave's own rows of hbuf
template <int RT, int CT>
__device__ inline void epilogue_relu(const f32x4 (&acc)[RT][CT], const float* __restrict__ bias, uint16_t* hbuf,
                                     int hs, int arow0)
{
    const int l = lane_id();
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const int col = ct * 16 + (l & 15);
        const float b = bias[col];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = acc[rt][ct][i] + b;
                v = v > 0.f ? v : 0.f;
                hbuf[(arow0 + rt * 16 + 4 * (l >> 4) + i) * hs + col] = f32_to_bf16(v);
            }
    }
}

__device__ inline void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// uniform in (0, 1) from the top 24 bits of a word: (top + 1/2) / 2^24
__device__ inline float unif24(uint64_t w) { return ((float)(uint32_t)(w >> 40) + 0.5f) * (1.0f / 16777216.0f); }

template <int H>
struct MlpTile {
    static constexpr int RPW = H <= 256 ? 32 : 16;  // rows per wave
    static constexpr int RT = RPW / 16;
    static constexpr int TILE = 4 * RPW;             // rows per workgroup
    static constexpr int HS = H + 8;                 // LDS row stride of activations
    static constexpr int WREG = (H > 128 ? H : 128) * WSTRIDE;  // weight chunk elements
};

}  // namespace econ
