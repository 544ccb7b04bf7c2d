// econ_mlp.h -- internal device code shared by the policy forward and the
// PPO backward kernels: MLP dimensions, weight layouts, bf16 MFMA tiles.
//
// The network is d_in -> H -> H -> (A logits, 1 value) with ReLU.  fp32
// parameters live in one flat vector (row-major W[in][out], then bias).  The
// kernels read bf16 copies arranged as K-chunks of 32: for a matrix used as
// the B operand of C = A B, element (k, n) sits at [k / 32][n][k % 32], so one
// lane's MFMA fragment (column n, 8 consecutive k) is 16 contiguous bytes and a
// 16-column fragment is 1 KB, read straight from L2 into registers.
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

// First-layer input padded to K1p = 64 columns for rows of at most 64
// features (D_stride <= 64), else to 128 (wide rows, H >= 128: the LDS row of
// activations, H + 8 columns, must hold them).  The LDS tile and the K-chunk
// layout of W1 take K1p columns; the product runs K1p / 32 k-steps.
constexpr int K1P = 64;
constexpr int K1P_WIDE = 128;

__host__ inline int mlp_dims(int D, int Ds, int H, int A, MlpDims* d)
{
    if (D <= 0 || Ds < D || (Ds & 7) != 0 || Ds > K1P_WIDE) return EJ_EUNSUPPORTED;
    if (!(H == 64 || H == 128 || H == 256 || H == 512)) return EJ_EUNSUPPORTED;
    if (Ds > K1P && H < 128) return EJ_EUNSUPPORTED;
    if (A <= 0 || A + 1 > 1024) return EJ_EUNSUPPORTED;
    d->D = D;
    d->Ds = Ds;
    d->H = H;
    d->A = A;
    d->A1 = A + 1;
    d->K1p = Ds <= K1P ? K1P : K1P_WIDE;
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

// LDS-staged K-chunks (the weight-gradient kernel): [n][40] bf16 (32 k + 8
// pad: 80-byte rows keep the 16 lanes of a fragment read on distinct banks)
constexpr int WSTRIDE = 40;

__device__ inline bf16x8 lds_frag(const uint16_t* p) { return *(const bf16x8*)p; }

__device__ inline f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Weight fragments are read through a buffer resource over the (uniform)
// weight base: every lane keeps one 32-bit byte offset (its column l % 16
// and k group l / 16) and the k-step and column-tile offsets are uniform
// scalar offsets, so a fragment load costs no vector address arithmetic.
// Raw buffer resource words for gfx9: no stride, 2^31 - 1 bytes of range,
// 32-bit data format.
__device__ inline __amdgpu_buffer_rsrc_t weight_rsrc(const uint16_t* base)
{
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, 0x7fffffff, 0x00020000);
}

__device__ inline bf16x8 buf_frag(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    typedef __attribute__((ext_vector_type(4))) unsigned int u32x4_t;
    const u32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    return __builtin_bit_cast(bf16x8, v);
}

// One dense layer split by columns: the wave multiplies ALL TR x 16 rows of
// `abuf` (row stride `as`) by its own CTW x 16 columns of the weights,
// starting at column `col0` (the same on every lane of the wave).  B
// fragments come straight from global memory (L2-resident weights in the
// K-chunk layout: lane l reads the 16 bytes of column l % 16, k = 8 (l / 16)
// .. + 7), PF k-steps ahead of the MFMAs; A fragments come from LDS one
// k-step ahead.  Every A fragment feeds CTW MFMAs and every B fragment TR,
// and no weight passes through LDS.  The caller synchronises before (abuf
// complete) and after (before abuf is overwritten).  The first k-step's
// accumulator input is, by CM: 0 acc itself (accumulate), 1 zero, 2 cb[ct]
// (the same vector for every row tile: a bias).  TRANS swaps the MFMA
// operands, which transposes each accumulator tile: lane l then holds row
// l % 16 and the four adjacent columns 4 (l / 16) .. + 3 (instead of column
// l % 16 of rows 4 (l / 16) .. + 3), so an epilogue stores 4 columns at once.
template <int TR, int CTW, int NK, int CM, int PF, bool PIN, bool TRANS>
__device__ inline void dense_core(f32x4 (&acc)[TR][CTW], const f32x4* cb, const uint16_t* abuf, int as,
                                  const uint16_t* __restrict__ wglob, int64_t kstride, int col0)
{
    const int l = lane_id();
    const __amdgpu_buffer_rsrc_t wr = weight_rsrc(wglob);
    const int voff = ((l & 15) * 32 + 8 * (l >> 4)) * 2;
    const int c0 = __builtin_amdgcn_readfirstlane(col0), ks = (int)kstride;
    auto soff = [&](int kt, int ct) { return (kt * ks + (c0 + ct * 16) * 32) * 2; };
    const uint16_t* ap = abuf + (l & 15) * as + 8 * (l >> 4);
    bf16x8 bq[NK][CTW];
    bf16x8 aq[NK][TR];
#pragma unroll
    for (int p = 0; p < PF && p < NK; ++p)
#pragma unroll
        for (int ct = 0; ct < CTW; ++ct) bq[p][ct] = buf_frag(wr, voff, soff(p, ct));
#pragma unroll
    for (int rt = 0; rt < TR; ++rt) aq[0][rt] = lds_frag(ap + rt * 16 * as);
#pragma unroll
    for (int kt = 0; kt < NK; ++kt) {
        if (kt + PF < NK)
#pragma unroll
            for (int ct = 0; ct < CTW; ++ct) bq[kt + PF][ct] = buf_frag(wr, voff, soff(kt + PF, ct));
        if (kt + 1 < NK)
#pragma unroll
            for (int rt = 0; rt < TR; ++rt) aq[kt + 1][rt] = lds_frag(ap + rt * 16 * as + (kt + 1) * 32);
        // PIN keeps the loads here (the scheduler otherwise sinks each one next
        // to its first MFMA, trading latency hiding for registers)
        if constexpr (PIN) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ct = 0; ct < CTW; ++ct)
#pragma unroll
            for (int rt = 0; rt < TR; ++rt) {
                const f32x4 c = (kt > 0 || CM == 0) ? acc[rt][ct] : (CM == 1 ? f32x4{0.f, 0.f, 0.f, 0.f} : cb[ct]);
                acc[rt][ct] = TRANS ? mfma16(bq[kt][ct], aq[kt][rt], c) : mfma16(aq[kt][rt], bq[kt][ct], c);
            }
    }
}

// ZERO = false accumulates onto acc, ZERO = true starts from zero
template <int TR, int CTW, int NK, bool ZERO = true, int PF = 2, bool PIN = false, bool TRANS = false>
__device__ inline void dense_cs(f32x4 (&acc)[TR][CTW], const uint16_t* abuf, int as,
                                const uint16_t* __restrict__ wglob, int64_t kstride, int col0)
{
    dense_core<TR, CTW, NK, ZERO ? 1 : 0, PF, PIN, TRANS>(acc, nullptr, abuf, as, wglob, kstride, col0);
}

// started at the bias: cb[ct] is the accumulator input of the first k-step
// (16 more live registers than dense_cs during that step)
template <int TR, int CTW, int NK, int PF = 2, bool PIN = false, bool TRANS = false>
__device__ inline void dense_cs_bias(f32x4 (&acc)[TR][CTW], const f32x4 (&cb)[CTW], const uint16_t* abuf, int as,
                                     const uint16_t* __restrict__ wglob, int64_t kstride, int col0)
{
    dense_core<TR, CTW, NK, 2, PF, PIN, TRANS>(acc, cb, abuf, as, wglob, kstride, col0);
}

// The first layer (K1p = 64 or 128 input columns: two or four k-steps),
// started at the bias (dense_cs_bias)
template <int TR, int CTW, int PF, bool PIN, bool TRANS>
__device__ inline void dense_first_bias(f32x4 (&acc)[TR][CTW], const f32x4 (&cb)[CTW], const uint16_t* abuf, int as,
                                        const uint16_t* __restrict__ wglob, int64_t kstride, int col0, int K1p)
{
    if (K1p == K1P)
        dense_cs_bias<TR, CTW, K1P / 32, PF, PIN, TRANS>(acc, cb, abuf, as, wglob, kstride, col0);
    else
        dense_cs_bias<TR, CTW, K1P_WIDE / 32, PF, PIN, TRANS>(acc, cb, abuf, as, wglob, kstride, col0);
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

// two fp32 values rounded to a packed bf16 pair (a in the low half) by one
// packed round-to-nearest-even conversion
__device__ inline uint32_t bf16x2_bits(float a, float b)
{
    typedef __attribute__((ext_vector_type(2))) float f32x2;
    typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}

// ReLU of two fp32 values rounded to a packed bf16 pair: a bf16 with its sign
// bit set is a negative 16-bit integer, so a signed 16-bit max with 0 clears
// exactly the negative values (and -0).  Rounding keeps the sign, so this
// equals rounding the ReLU of the fp32 values.
__device__ inline uint32_t relu_bf16x2(float a, float b)
{
    typedef short __attribute__((ext_vector_type(2))) i16x2;
    const i16x2 v = __builtin_elementwise_max(__builtin_bit_cast(i16x2, bf16x2_bits(a, b)), i16x2{0, 0});
    return __builtin_bit_cast(uint32_t, v);
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
            *(uint2*)(hbuf + (rt * 16 + (l & 15)) * hs + col) =
                uint2{relu_bf16x2(acc[rt][ct][0], acc[rt][ct][1]), relu_bf16x2(acc[rt][ct][2], acc[rt][ct][3])};
        }
    }
}

// fp32 logit chunk in LDS: a row's 128 columns as four 32-column quarters,
// each padded to ZQ words, so that the four lanes reading one row's quarters
// (and the rows a wave reads together) fall on distinct banks.
constexpr int ZQ = 36, ZS = 4 * ZQ;
// The 16 rows of a transposed MFMA tile store the same four columns at once:
// with a row stride of ZS = 144 words rows r and r + 4 would share banks, so
// the 4-column group g (0..7) inside a quarter sits at g ^ zsw(row).  The
// four consecutive rows that a wave's quad reads together share zsw, so
// their reads stay conflict-free too.
__device__ inline int zsw(int row) { return (row >> 2) & 3; }
__device__ inline int zcol(int row, int cc) { return (cc >> 5) * ZQ + ((((cc >> 2) & 7) ^ zsw(row)) << 2) + (cc & 3); }

// b1 [H], b2 [H], b3 [A1p] (zero beyond A1) -> sbias, by a workgroup of NT
// threads; all loads are issued before the first store (A1p <= 1024)
template <int H, int NT = 256>
__device__ inline void load_biases(const MlpDims& d, const float* __restrict__ params, float* sbias)
{
    constexpr int NI = (2 * H + 1024 + NT - 1) / NT;
    const int n = 2 * H + d.A1p;
    float v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int p = threadIdx.x + NT * i;
        v[i] = p >= n ? 0.f
                      : p < H ? params[d.ob1 + p]
                              : p < 2 * H ? params[d.ob2 + p - H] : (p - 2 * H < d.A1 ? params[d.ob3 + p - 2 * H] : 0.f);
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int p = threadIdx.x + NT * i;
        if (p < n) sbias[p] = v[i];
    }
}

// uniform in (0, 1) from the top 24 bits of a word: (top + 1/2) / 2^24
__device__ inline float unif24(uint64_t w) { return ((float)(uint32_t)(w >> 40) + 0.5f) * (1.0f / 16777216.0f); }

// Row tile of the policy kernel: RPW_ rows per wave, four waves (64-row
// tiles by default; 128-row tiles for H <= 256 on request)
template <int H, int RPW_ = 16>
struct MlpTile {
    static constexpr int RPW = RPW_;      // rows per wave
    static constexpr int TILE = 4 * RPW;  // rows per workgroup
    static constexpr int HS = H + 8;      // LDS row stride of activations
};

}  // namespace econ
