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

constexpr int K1P = 64;  // first-layer input padded to 64 (one layout for every D <= 64)

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
    d->K1p = K1P;
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
    const uint16_t* bp = wbuf + (l & 15) * WSTRIDE + 8 * (l >> 4);
    bf16x8 a[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) a[rt] = lds_frag(abuf + (arow0 + rt * 16 + (l & 15)) * as + kcol + 8 * (l >> 4));
    // B fragments run four column tiles ahead of the MFMAs that consume them
    constexpr int PD = CT < 4 ? CT : 4;
    bf16x8 b[PD];
#pragma unroll
    for (int j = 0; j < PD; ++j) b[j] = lds_frag(bp + j * 16 * WSTRIDE);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const bf16x8 cur = b[ct % PD];
        if (ct + PD < CT) b[ct % PD] = lds_frag(bp + (ct + PD) * 16 * WSTRIDE);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = mfma16(a[rt], cur, acc[rt][ct]);
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

// Weight-chunk prefetch registers: eight 16-byte pieces per thread at most
// (N / 64 used).  Plain scalars passed by reference: an aggregate here ends up
// in scratch memory.
#define ECON_Q8_PARAMS uint4 &q0, uint4 &q1, uint4 &q2, uint4 &q3, uint4 &q4, uint4 &q5, uint4 &q6, uint4 &q7
#define ECON_Q8_ARGS q0, q1, q2, q3, q4, q5, q6, q7
#define ECON_Q8_DECL uint4 q0, q1, q2, q3, q4, q5, q6, q7

template <int N>
__device__ __forceinline__ void chunk_gload(const uint16_t* __restrict__ src, ECON_Q8_PARAMS)
{
    constexpr int NP = N / 64;
    const uint4* g = (const uint4*)src + threadIdx.x;
    q0 = g[0];
    if constexpr (NP > 1) q1 = g[256];
    if constexpr (NP > 2) { q2 = g[512]; q3 = g[768]; }
    if constexpr (NP > 4) { q4 = g[1024]; q5 = g[1280]; q6 = g[1536]; q7 = g[1792]; }
}

__device__ __forceinline__ void chunk_sput(uint16_t* wbuf, int j, const uint4& v)
{
    const int piece = threadIdx.x + 256 * j;  // row n = piece / 4, k-quarter piece % 4
    *(uint4*)(wbuf + (piece >> 2) * WSTRIDE + (piece & 3) * 8) = v;
}

template <int N>
__device__ __forceinline__ void chunk_lds_store(uint16_t* wbuf, ECON_Q8_PARAMS)
{
    constexpr int NP = N / 64;
    chunk_sput(wbuf, 0, q0);
    if constexpr (NP > 1) chunk_sput(wbuf, 1, q1);
    if constexpr (NP > 2) { chunk_sput(wbuf, 2, q2); chunk_sput(wbuf, 3, q3); }
    if constexpr (NP > 4) { chunk_sput(wbuf, 4, q4); chunk_sput(wbuf, 5, q5); chunk_sput(wbuf, 6, q6); chunk_sput(wbuf, 7, q7); }
}

// One dense layer for the workgroup's row tile: every wave multiplies its own
// rows of `abuf` (row stride `as`, rows from `arow0`, columns from `acol0`)
// by a weight matrix streamed 32 k-rows at a time through LDS.  With DB the
// chunks alternate between two LDS buffers (one barrier per k-step); without
// it one buffer is refilled between two barriers.  The next chunk is
// prefetched into registers while the current one is consumed; after the
// last chunk the first chunk of the next layer (`next`, N2 columns) is
// prefetched instead, so that the next call can start with `preloaded`.
// `kstride`: elements between the global chunks of consecutive k-steps.
// All 256 threads must call it.
template <int RT, int N, int N2 = N, bool DB = false>
__device__ inline void dense_layer_pf(f32x4 (&acc)[RT][N / 16], const uint16_t* abuf, int as, int arow0, int K,
                                      const uint16_t* __restrict__ wglob, int64_t kstride, uint16_t* wbuf,
                                      bool preloaded, const uint16_t* __restrict__ next, ECON_Q8_PARAMS,
                                      bool zero = true, int acol0 = 0)
{
    if (zero) zero_acc(acc);
    if (!preloaded) chunk_gload<N>(wglob, ECON_Q8_ARGS);
    const int nk = K / 32;
    if constexpr (DB) {
        constexpr int WB = N * WSTRIDE;  // elements per buffer
        __syncthreads();                 // the previous layer is done with both buffers
        chunk_lds_store<N>(wbuf, ECON_Q8_ARGS);
        if (nk > 1) chunk_gload<N>(wglob + kstride, ECON_Q8_ARGS);
        else if (next) chunk_gload<N2>(next, ECON_Q8_ARGS);
        for (int kt = 0; kt < nk; ++kt) {
            __syncthreads();  // chunk kt is in LDS; the other buffer is free
            if (kt + 1 < nk) {
                chunk_lds_store<N>(wbuf + ((kt + 1) & 1) * WB, ECON_Q8_ARGS);
                if (kt + 2 < nk) chunk_gload<N>(wglob + (int64_t)(kt + 2) * kstride, ECON_Q8_ARGS);
                else if (next) chunk_gload<N2>(next, ECON_Q8_ARGS);
            }
            mfma_chunk<RT, N / 16>(acc, abuf, as, arow0, acol0 + kt * 32, wbuf + (kt & 1) * WB);
        }
    } else {
        for (int kt = 0; kt < nk; ++kt) {
            __syncthreads();  // everyone is done with the previous chunk
            chunk_lds_store<N>(wbuf, ECON_Q8_ARGS);
            __syncthreads();
            if (kt + 1 < nk) chunk_gload<N>(wglob + (int64_t)(kt + 1) * kstride, ECON_Q8_ARGS);
            else if (next) chunk_gload<N2>(next, ECON_Q8_ARGS);
            mfma_chunk<RT, N / 16>(acc, abuf, as, arow0, acol0 + kt * 32, wbuf);
        }
    }
}

template <int RT, int N, bool DB = false>
__device__ inline void dense_layer(f32x4 (&acc)[RT][N / 16], const uint16_t* abuf, int as, int arow0, int K,
                                   const uint16_t* __restrict__ wglob, int64_t kstride, uint16_t* wbuf,
                                   bool zero = true, int acol0 = 0)
{
    ECON_Q8_DECL;
    dense_layer_pf<RT, N, N, DB>(acc, abuf, as, arow0, K, wglob, kstride, wbuf, false, nullptr, ECON_Q8_ARGS, zero,
                                 acol0);
}

// One dense layer split by columns: the wave multiplies ALL TR x 16 rows of
// `abuf` (row stride `as`) by its own CTW x 16 columns of the weights,
// starting at column `col0`.  B fragments come straight from global memory
// (L2-resident weights in the K-chunk layout: lane l reads the 16 bytes of
// column l % 16, k = 8 (l / 16) .. + 7), PF k-steps ahead of the MFMAs;
// A fragments come from LDS one k-step ahead.  Every A fragment feeds CTW
// MFMAs and every B fragment TR, and no weight passes through LDS.  The
// caller synchronises before (abuf complete) and after (before abuf is
// overwritten).  ZERO = false accumulates onto acc.  TRANS swaps the MFMA
// operands, which transposes each accumulator tile: lane l then holds row
// l % 16 and the four adjacent columns 4 (l / 16) .. + 3 (instead of column
// l % 16 of rows 4 (l / 16) .. + 3), so an epilogue stores 4 columns at once.
template <int TR, int CTW, int NK, bool ZERO = true, int PF = 2, bool PIN = false, bool TRANS = false>
__device__ inline void dense_cs(f32x4 (&acc)[TR][CTW], const uint16_t* abuf, int as,
                                const uint16_t* __restrict__ wglob, int64_t kstride, int col0)
{
    if constexpr (ZERO) zero_acc(acc);
    const int l = lane_id();
    const uint16_t* bp = wglob + (int64_t)(col0 + (l & 15)) * 32 + 8 * (l >> 4);
    const uint16_t* ap = abuf + (l & 15) * as + 8 * (l >> 4);
    bf16x8 bq[NK][CTW];
    bf16x8 aq[NK][TR];
#pragma unroll
    for (int p = 0; p < PF && p < NK; ++p)
#pragma unroll
        for (int ct = 0; ct < CTW; ++ct) bq[p][ct] = *(const bf16x8*)(bp + (int64_t)p * kstride + ct * 16 * 32);
#pragma unroll
    for (int rt = 0; rt < TR; ++rt) aq[0][rt] = lds_frag(ap + rt * 16 * as);
#pragma unroll
    for (int kt = 0; kt < NK; ++kt) {
        if (kt + PF < NK)
#pragma unroll
            for (int ct = 0; ct < CTW; ++ct)
                bq[kt + PF][ct] = *(const bf16x8*)(bp + (int64_t)(kt + PF) * kstride + ct * 16 * 32);
        if (kt + 1 < NK)
#pragma unroll
            for (int rt = 0; rt < TR; ++rt) aq[kt + 1][rt] = lds_frag(ap + rt * 16 * as + (kt + 1) * 32);
        // PIN keeps the loads here (the scheduler otherwise sinks each one next
        // to its first MFMA, trading latency hiding for registers)
        if constexpr (PIN) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ct = 0; ct < CTW; ++ct)
#pragma unroll
            for (int rt = 0; rt < TR; ++rt)
                acc[rt][ct] = TRANS ? mfma16(bq[kt][ct], aq[kt][rt], acc[rt][ct])
                                    : mfma16(aq[kt][rt], bq[kt][ct], acc[rt][ct]);
    }
}

// bias + ReLU of a column-split layer, rounded to bf16, written to hbuf
template <int TR, int CTW>
__device__ inline void epilogue_relu_cs(const f32x4 (&acc)[TR][CTW], const float* __restrict__ bias,
                                        uint16_t* hbuf, int hs, int col0)
{
    const int l = lane_id();
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) {
        const int col = col0 + ct * 16 + (l & 15);
        const float b = bias[col];
#pragma unroll
        for (int rt = 0; rt < TR; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = acc[rt][ct][i] + b;
                v = v > 0.f ? v : 0.f;
                hbuf[(rt * 16 + 4 * (l >> 4) + i) * hs + col] = f32_to_bf16(v);
            }
    }
}

// Transposed accumulators (dense_cs with TRANS) started at the bias: lane
// l's four columns col0 + 16 ct + 4 (l / 16) .. + 3 of every row tile.  The
// loads go out with the layer's first weight fragments (fp32 bias, 16-byte
// aligned), so the epilogue has no bias to wait for.
template <int TR, int CTW>
__device__ inline void bias_init_t(f32x4 (&acc)[TR][CTW], const float* __restrict__ bias, int col0)
{
    const int l = lane_id();
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) {
        const float4 b = *(const float4*)(bias + col0 + ct * 16 + 4 * (l >> 4));
#pragma unroll
        for (int rt = 0; rt < TR; ++rt) acc[rt][ct] = f32x4{b.x, b.y, b.z, b.w};
    }
}

// ReLU of transposed accumulators (bias included), rounded to bf16: one
// 8-byte store of 4 adjacent columns per tile
template <int TR, int CTW>
__device__ inline void relu_store_t(const f32x4 (&acc)[TR][CTW], uint16_t* hbuf, int hs, int col0)
{
    const int l = lane_id();
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) {
        const int col = col0 + ct * 16 + 4 * (l >> 4);
#pragma unroll
        for (int rt = 0; rt < TR; ++rt) {
            const float v0 = fmaxf(acc[rt][ct][0], 0.f), v1 = fmaxf(acc[rt][ct][1], 0.f);
            const float v2 = fmaxf(acc[rt][ct][2], 0.f), v3 = fmaxf(acc[rt][ct][3], 0.f);
            const uint2 pk = {(uint32_t)f32_to_bf16(v0) | ((uint32_t)f32_to_bf16(v1) << 16),
                              (uint32_t)f32_to_bf16(v2) | ((uint32_t)f32_to_bf16(v3) << 16)};
            *(uint2*)(hbuf + (rt * 16 + (l & 15)) * hs + col) = pk;
        }
    }
}

// fp32 logit chunk in LDS: a row's 128 columns as four 32-column quarters,
// each padded to ZQ words, so that the four lanes reading one row's quarters
// (and the rows a wave reads together) fall on distinct banks
constexpr int ZQ = 36, ZS = 4 * ZQ;
__device__ inline int zcol(int cc) { return (cc >> 5) * ZQ + (cc & 31); }

// b1 [H], b2 [H], b3 [A1p] (zero beyond A1) -> sbias, by a 256-thread
// workgroup; all loads are issued before the first store (A1p <= 1024)
template <int H>
__device__ inline void load_biases(const MlpDims& d, const float* __restrict__ params, float* sbias)
{
    constexpr int NI = (2 * H + 1024 + 255) / 256;
    const int n = 2 * H + d.A1p;
    float v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int p = threadIdx.x + 256 * i;
        v[i] = p >= n ? 0.f
                      : p < H ? params[d.ob1 + p]
                              : p < 2 * H ? params[d.ob2 + p - H] : (p - 2 * H < d.A1 ? params[d.ob3 + p - 2 * H] : 0.f);
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int p = threadIdx.x + 256 * i;
        if (p < n) sbias[p] = v[i];
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

// Row tile of the MLP kernels: RPW_ rows per wave, four waves.  128-row tiles
// (H <= 256) reuse every weight fragment for two 16-row MFMA tiles and
// double-buffer the weight chunks (one workgroup per CU); 64-row tiles halve
// the LDS footprint so that two workgroups share a CU.
template <int H, int RPW_ = (H <= 256 ? 32 : 16)>
struct MlpTile {
    static constexpr int RPW = RPW_;                 // rows per wave
    static constexpr int RT = RPW / 16;
    static constexpr int TILE = 4 * RPW;             // rows per workgroup
    static constexpr int HS = H + 8;                 // LDS row stride of activations
    static constexpr int WREG = (H > 128 ? H : 128) * WSTRIDE;  // weight chunk elements
    static constexpr bool DB = H <= 256 && RPW == 32;  // double-buffered weight chunks fit in LDS
    static constexpr int WBUF = DB ? 2 * WREG : WREG;
};

}  // namespace econ
