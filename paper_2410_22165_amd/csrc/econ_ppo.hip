// econ_ppo.hip -- the PPO learner on gfx950: generalised advantage
// estimation, the fused minibatch backward of the shared policy network, the
// weight-gradient GEMMs with a deterministic split-M reduction, and Adam.
//
// PPO as configured in the paper's Table 2 (clipped surrogate, clipped value
// loss with coefficient c_v, entropy bonus c_e, GAE(gamma, lambda)); the
// network and its masked softmax are those of econ_policy.hip.
//
// Backward data flow for a minibatch of `rows` samples (row j of the epoch
// maps to sample (a j + c) mod M):
//   ppo_rows_kernel  per 64-row tile: gathers the samples, recomputes
//     h1, h2 and the logits (never stored per rollout: activations are
//     recomputed here), forms the loss gradient dY = dL/d[logits | value]
//     from the row statistics of the masked softmax, and back-propagates
//     dh2 = (dY W3^T) * [h2 > 0] and dh1 = (dh2 W2^T) * [h1 > 0].  The GEMM
//     operands of the weight gradients h2, dY, dh2, dh1 are written in bf16
//     "m-block" layout [rows / 32][column][32 rows]; the gathered
//     observations leave as plain rows [rows][K1p].
//   dw_kernel        dW = X^T Y as bf16 MFMA with the 32-row m-block as the
//     k-step; every workgroup owns a C tile and a contiguous range of
//     m-blocks and writes an fp32 partial; column sums of Y give the bias
//     gradients.  dW1 transposes the observation rows into its LDS tile; dW2
//     recomputes h1 from them (a quarter of dW2's products), so neither the
//     observations' m-blocks nor h1 pass through HBM.
//   dw_reduce_kernel sums the partials in a fixed order (deterministic).
#include "econ_mlp.h"

#include <mutex>

namespace econ {

struct PpoBatchDev {
    const uint16_t* obs;
    const uint32_t* mask;
    const int32_t* act;
    const float* logp_old;
    const float* val_old;
    const float* adv;
    const float* ret;
    int64_t Mtot, a, c, begin, rows;
    uint64_t mu;  // floor((2^64 - 1) / Mtot): Barrett reciprocal of the permutation modulus
    int64_t rstride, roff;  // sample s sits at storage index s * rstride + roff
    const unsigned char* rec;  // nullable: packed records (record s = sample s)
    int64_t rb;                // record bytes
    int rmask, rsc;            // byte offsets of the mask words and of the five scalars in a record
};

// Record of one sample (ej_ppo_pack): the observation row (Ds bf16, padded to
// 16 bytes), the W mask words, then act, logp_old, val_old, adv, ret; the
// whole rounded up to 128 bytes
__host__ __device__ inline void record_layout(int Ds, int W, int* rmask, int* rsc, int64_t* rb)
{
    *rmask = (2 * Ds + 15) / 16 * 16;
    *rsc = *rmask + 4 * W;
    *rb = (int64_t)(*rsc + 20 + 127) / 128 * 128;
}

struct PpoHp {
    float clip, vclip, vf_coef, ent_coef;
};

// sample behind minibatch row j: (a (begin + j) + c) mod Mtot.  With a, c,
// begin + j < Mtot <= 2^31 - 1 the argument is below 2^63, and the Barrett
// quotient umulhi(x, mu) undershoots floor(x / Mtot) by at most 2.
__device__ inline int64_t perm_of(const PpoBatchDev& B, int64_t j)
{
    const uint64_t M = (uint64_t)B.Mtot;
    const uint64_t x = (uint64_t)B.a * (uint64_t)(B.begin + j) + (uint64_t)B.c;
    uint64_t r = x - __umul64hi(x, B.mu) * M;
    r = r >= M ? r - M : r;
    r = r >= M ? r - M : r;
    return (int64_t)r;
}

// its storage index in the arrays
__device__ inline int64_t sample_of(const PpoBatchDev& B, int64_t j) { return perm_of(B, j) * B.rstride + B.roff; }

// ---------------------------------------------------------------------------
// GAE: one thread per row, reverse over time; coalesced over rows
// ---------------------------------------------------------------------------
__global__ void gae_kernel(const float* __restrict__ rew, const float* __restrict__ val,
                           const uint8_t* __restrict__ done, const float* __restrict__ last_val, int T, int64_t M,
                           float gamma, float lam, float* __restrict__ adv, float* __restrict__ ret)
{
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < M; m += (int64_t)gridDim.x * blockDim.x) {
        float next_val = last_val[m], next_adv = 0.f;
        for (int t = T - 1; t >= 0; --t) {
            const int64_t i = (int64_t)t * M + m;
            const float nonterm = done[i] ? 0.f : 1.f;
            const float v = val[i];
            const float delta = rew[i] + gamma * next_val * nonterm - v;
            next_adv = delta + gamma * lam * nonterm * next_adv;
            adv[i] = next_adv;
            ret[i] = next_adv + v;
            next_val = v;
        }
    }
}

// ---------------------------------------------------------------------------
// advantage statistics of the minibatch (two deterministic stages)
// ---------------------------------------------------------------------------
__global__ void adv_stats_partial(const PpoBatchDev B, double* __restrict__ part)
{
    __shared__ double red[2][16];
    double s1 = 0.0, s2 = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < B.rows; j += (int64_t)gridDim.x * blockDim.x) {
        const double a = B.adv[sample_of(B, j)];
        s1 += a;
        s2 += a * a;
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        red[0][w] = s1;
        red[1][w] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            a += red[0][k];
            b += red[1][k];
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// The same sums by one streaming pass over the whole batch, for minibatches
// of at least 1/32 of it (a gathered row costs a whole cache line, a
// streamed sample 4 bytes): sample s is epoch row j = ainv (s - c) mod Mtot
// (ainv the inverse of a modulo Mtot) and belongs to the minibatch when
// begin <= j < begin + rows.  Thread t visits s = t, t + T, ... (T threads
// in the grid), so its row advances by the constant step = ainv T mod Mtot;
// kc = ainv c mod Mtot.  Mtot < 2^31.  Fixed order per thread and per block.
__global__ void adv_stats_stream(const PpoBatchDev B, uint32_t ainv, uint32_t kc, uint32_t step,
                                 double* __restrict__ part)
{
    __shared__ double red[2][16];
    const uint32_t M = (uint32_t)B.Mtot;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x, T = gridDim.x * blockDim.x;
    const uint32_t at = (uint32_t)(((uint64_t)t * ainv) % M);
    uint32_t jr = at >= kc ? at - kc : at + (M - kc);
    const uint32_t begin = (uint32_t)B.begin, rows = (uint32_t)B.rows;
    double s1 = 0.0, s2 = 0.0;
    // sixteen loads in flight per thread (1024 workgroups hold about 16 MB in
    // flight); every sample is loaded: at 1/32 of the batch or more nearly
    // every cache line holds a row of the minibatch
    for (uint32_t base = t; base < M; base += 16 * T) {
        float v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t sm = min(base + k * T, M - 1);  // clamped: the loads stay unconditional
            v[k] = B.adv[(int64_t)sm * B.rstride + B.roff];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (jr - begin < rows && base + k * T < M) {
                const double a = v[k];
                s1 += a;
                s2 += a * a;
            }
            jr += step;
            jr = jr >= M ? jr - M : jr;
        }
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        red[0][w] = s1;
        red[1][w] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            a += red[0][k];
            b += red[1][k];
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// sums of n records of C doubles-or-floats by one 256-thread workgroup: thread
// t takes records t, t + 256, ...; then a fixed wave and LDS tree (the same
// order on every call, so the result is deterministic)
template <int C, typename T>
__device__ inline void block_sum_records(const T* __restrict__ rec, int64_t n, double (&out)[C])
{
    __shared__ double red[C][4];
    double s[C];
#pragma unroll
    for (int c = 0; c < C; ++c) s[c] = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += 256) {
#pragma unroll
        for (int c = 0; c < C; ++c) s[c] += (double)rec[k * C + c];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        s[c] = wave_sum(s[c]);
        if (lane_id() == 0) red[c][threadIdx.x >> 6] = s[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) out[c] = (red[c][0] + red[c][1]) + (red[c][2] + red[c][3]);
}

// stats[0] = mean, stats[1] = 1 / (population std + 1e-8); one 256-thread workgroup
__global__ void __launch_bounds__(256) adv_stats_final(const double* __restrict__ part, int nb, int64_t rows,
                                                       float* __restrict__ stats)
{
    double t[2];
    block_sum_records<2>(part, nb, t);
    if (threadIdx.x != 0) return;
    const double mean = t[0] / (double)rows;
    double var = t[1] / (double)rows - mean * mean;
    if (var < 0.0) var = 0.0;
    stats[0] = (float)mean;
    stats[1] = (float)(1.0 / (sqrt(var) + 1e-8));
}

// ---------------------------------------------------------------------------
// the fused row kernel
// ---------------------------------------------------------------------------

// bias + ReLU of a column-split hidden layer with transposed accumulators
// (dense_cs with TRANS: lane l holds row 16 rt + l % 16, columns col0 +
// 16 ct + 4 (l / 16) .. + 3): bf16 activations -> hbuf (A operand of the next
// layer and source of the m-block copy), one 8-byte store per tile, and the
// ReLU pattern of the lane's columns (bit 4 ct + i of bits[rt]) for the
// backward, whose products use the same layout
template <int TR, int CTW, bool ADD_BIAS = true>
__device__ inline void ppo_hidden_epilogue_cs(const f32x4 (&acc)[TR][CTW], const float* __restrict__ bias,
                                              uint16_t* hbuf, int hs, int col0, uint32_t (&bits)[TR])
{
    const int l = lane_id();
#pragma unroll
    for (int rt = 0; rt < TR; ++rt) bits[rt] = 0u;
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) {
        const int col = col0 + ct * 16 + 4 * (l >> 4);
        const float4 b = ADD_BIAS ? *(const float4*)(bias + col) : float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int rt = 0; rt < TR; ++rt) {
            const float x0 = ADD_BIAS ? acc[rt][ct][0] + b.x : acc[rt][ct][0];
            const float x1 = ADD_BIAS ? acc[rt][ct][1] + b.y : acc[rt][ct][1];
            const float x2 = ADD_BIAS ? acc[rt][ct][2] + b.z : acc[rt][ct][2];
            const float x3 = ADD_BIAS ? acc[rt][ct][3] + b.w : acc[rt][ct][3];
            bits[rt] |= ((x0 > 0.f ? 1u : 0u) | (x1 > 0.f ? 2u : 0u) | (x2 > 0.f ? 4u : 0u) | (x3 > 0.f ? 8u : 0u))
                        << (ct * 4);
            *(uint2*)(hbuf + (rt * 16 + (l & 15)) * hs + col) = uint2{relu_bf16x2(x0, x1), relu_bf16x2(x2, x3)};
        }
    }
    // The words go through an identity lane move, which the compiler cannot
    // see through: otherwise it keeps every comparison as a 64-bit lane mask
    // in scalar registers until the backward's use and spills them.
#pragma unroll
    for (int rt = 0; rt < TR; ++rt) bits[rt] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)bits[rt], 0xE4, 0xF, 0xF, false);
}

// masked input gradient of a column-split layer (transposed accumulators, as
// above) -> bf16 rows in hbuf
template <int TR, int CTW>
__device__ inline void ppo_masked_grad_cs(const f32x4 (&dh)[TR][CTW], const uint32_t (&bits)[TR], uint16_t* hbuf,
                                          int hs, int col0)
{
    const int l = lane_id();
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) {
        const int col = col0 + ct * 16 + 4 * (l >> 4);
#pragma unroll
        for (int rt = 0; rt < TR; ++rt) {
            // bit 4 ct + i spread to a whole word keeps or clears the value
            float v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                v[i] = __int_as_float(__float_as_int(dh[rt][ct][i]) & __builtin_amdgcn_sbfe((int)bits[rt], ct * 4 + i, 1));
            *(uint2*)(hbuf + (rt * 16 + (l & 15)) * hs + col) = uint2{bf16x2_bits(v[0], v[1]), bf16x2_bits(v[2], v[3])};
        }
    }
}

// masked input gradient of a column-split layer in the plain accumulator
// layout (dense_cs without TRANS: lane l holds column col0 + 16 ct + l % 16,
// rows 16 rt + 4 (l / 16) .. + 3) -> its bf16 m-blocks directly: a lane's four
// rows are 8 contiguous bytes of T[(mb0 + rt / 2) ncol + column][32].  The
// ReLU pattern comes in the transposed layout (bits[rt] bit 4 ct + i: row
// 16 rt + l % 16, column col0 + 16 ct + 4 (l / 16) + i); the bit of (row
// 16 rt + 4 g + i, column col0 + 16 ct + c) sits in lane 4 g + i + 16 (c / 4),
// bit 4 ct + c % 4.
template <int TR, int CTW>
__device__ inline void ppo_grad_to_mblocks(const f32x4 (&dh)[TR][CTW], const uint32_t (&bits)[TR], uint16_t* T,
                                           int64_t mb0, int ncol, int col0)
{
    const int l = lane_id(), c = l & 15, g = l >> 4;
#pragma unroll
    for (int rt = 0; rt < TR; ++rt) {
        uint32_t mk[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) mk[i] = (uint32_t)__shfl((int)bits[rt], 4 * g + i + 16 * (c >> 2), 64);
#pragma unroll
        for (int ct = 0; ct < CTW; ++ct) {
            const int sh = 4 * ct + (c & 3);
            float v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                v[i] = __int_as_float(__float_as_int(dh[rt][ct][i]) & __builtin_amdgcn_sbfe((int)mk[i], sh, 1));
            *(uint2*)(T + ((mb0 + (rt >> 1)) * ncol + col0 + 16 * ct + c) * 32 + 16 * (rt & 1) + 4 * g) =
                uint2{bf16x2_bits(v[0], v[1]), bf16x2_bits(v[2], v[3])};
        }
    }
}

// m-block copy of an LDS tile: rows [0, rows) x columns [0, ncol) of a bf16
// tile (row stride hs, a multiple of 4) -> T[(mb0 + row / 32) ncol_total +
// col_off + col][32].  A work item is (32-row block, group of four columns,
// quarter of 8 rows): eight 8-byte LDS reads give the quarter of all four
// columns, which leave as four 16-byte stores (each column's 64 bytes of a
// block come from four consecutive lanes).  ncol is a multiple of 4.  All
// threads call it.
__device__ inline void tile_to_mblocks(const uint16_t* tile, int hs, int rows, int ncol, uint16_t* T, int64_t mb0,
                                       int ncol_total, int col_off)
{
    const int ng = ncol >> 2;
    const int np = (rows / 32) * ng * 4;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        const int qq = p & 3, g = (p >> 2) % ng, blk = (p >> 2) / ng;
        uint2 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = *(const uint2*)(tile + (blk * 32 + qq * 8 + k) * hs + 4 * g);
        uint16_t* dst = T + ((mb0 + blk) * ncol_total + col_off + 4 * g) * 32 + qq * 8;
        // column 4 g + j of rows 2 k, 2 k + 1: the (j & 1) half of word j / 2
        // of each, packed by one byte permute (low halves 0x05040100, high
        // halves 0x07060302; bytes 0-3 of the selection come from the second
        // operand)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t sel = (j & 1) ? 0x07060302u : 0x05040100u;
            uint32_t w[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t lo = j < 2 ? v[2 * k].x : v[2 * k].y;
                const uint32_t hi = j < 2 ? v[2 * k + 1].x : v[2 * k + 1].y;
                w[k] = __builtin_amdgcn_perm(hi, lo, sel);
            }
            *(uint4*)(dst + j * 32) = uint4{w[0], w[1], w[2], w[3]};
        }
    }
}

// Row tile of the PPO kernel: 64 rows, four waves; every H-wide product is
// split by columns (wave w: all rows x columns [w H / 4, (w + 1) H / 4)).
template <int H>
struct PpoTile {
    // H = 512: eight waves, so that a wave's share of every product (four
    // 16-column tiles) fits its registers; below, four waves
    static constexpr int NW = H >= 512 ? 8 : 4, NTH = 64 * NW;
    static constexpr int TILE = 64, TR = 4, HS = H + 8, CTW = H / (16 * NW);
    static constexpr int LCT = 128 / (16 * NW);  // 16-column tiles of a logit chunk per wave
    static constexpr int YS = 136;  // bf16 row stride of the dY chunk (aliases the logit chunk)
};

template <int H>
size_t ppo_rows_lds_bytes(int W, int A1p)
{
    using P = PpoTile<H>;
    return (size_t)P::TILE * P::HS * 2 + (size_t)P::TILE * ZS * 4 + (size_t)P::TILE * 6 * 4 +
           (size_t)P::TILE * W * 4 + 64 * 4 + (size_t)(2 * H + A1p) * 4;
}

// One fused pass over a tile of minibatch rows: recompute the forward (bf16
// MFMA), the masked-softmax statistics and the loss terms, then dY = dL/d
// [logits | value], dh2 = (dY W3^T) * [h2 > 0] and dh1 = (dh2 W2^T) *
// [h1 > 0].  The weight-gradient GEMMs read the m-block copies and the
// observation rows written here.  The workgroup's threads talk through LDS
// only.
//
// The rows of a minibatch are scattered samples (the permutation), so their
// gather is latency-bound: every load of the tile's inputs (observation, mask
// words, the five per-sample scalars, the biases) is issued before the first
// of them is stored to LDS, one round trip for all; with packed records
// (ej_ppo_pack) a row's inputs are one aligned block.  MWP mask words per
// thread cover the tile's TILE x W words (TILE W <= NTH MWP).
template <int H, int MWP>
__global__ void __launch_bounds__(PpoTile<H>::NTH, H <= 256 ? 2 : 1)  // H <= 256: 73 KB of LDS, two workgroups per CU
ppo_rows_kernel(const MlpDims d, const float* __restrict__ params, const uint16_t* __restrict__ work,
                const PpoBatchDev B, const PpoHp hp, const float* __restrict__ stats, int W,
                uint16_t* __restrict__ Orows, uint16_t* __restrict__ Th2, uint16_t* __restrict__ TdY,
                uint16_t* __restrict__ Tdh2, uint16_t* __restrict__ Tdh1, float* __restrict__ loss_parts)
{
    using P = PpoTile<H>;
    constexpr int TILE = P::TILE, TR = P::TR, HS = P::HS, CTW = P::CTW, YS = P::YS, NW = P::NW, NTH = P::NTH;
    constexpr int LCT = P::LCT;
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t* hbuf = (uint16_t*)smem;                 // [TILE][HS] obs -> h1 -> h2 -> dh2
    float* zbuf = (float*)(hbuf + TILE * HS);         // [TILE][ZS] logit chunk
    uint16_t* ybuf = (uint16_t*)zbuf;                 // [TILE][YS] dY chunk once the logits are consumed
    float* rinfo = zbuf + TILE * ZS;                  // [6][TILE]: act, logp_old, val_old, adv_hat, ret, valid
    uint32_t* smask = (uint32_t*)(rinfo + 6 * TILE);  // [TILE][W]
    float* lred = (float*)(smask + TILE * W);         // [NW waves][4] (64 floats)
    float* sbias = lred + 64;                         // b1 [H], b2 [H], b3 [A1p] (zero padded)

    const int wave = threadIdx.x >> 6, l = lane_id(), q = l & 3;
    const float inv_n = 1.0f / (float)B.rows;
    const int col0 = wave * (H / NW);
    // the masked softmax works on rows: four waves own 16 rows each (eight
    // waves: the last four only join the products)
    const bool rowner = NW == 4 || wave < 4;

    // gather registers (the tile's inputs)
    constexpr int NPC = TILE * (K1P / 8) / NTH;  // 16-byte observation pieces per thread and 64 columns
    uint4 pv[NPC];
    float gs[5] = {0.f, 0.f, 0.f, 0.f, 0.f};  // act (bits), logp_old, val_old, adv, ret of row threadIdx.x
    uint32_t gm[MWP];
    float mean = 0.f, istd = 0.f;  // advantage normalisation of the minibatch
    auto obs_half = [&](int64_t tile, int h) {  // observation columns [64 h, 64 h + 64)
        const int64_t row0 = tile * TILE;
#pragma unroll
        for (int i = 0; i < NPC; ++i) {
            const int p = threadIdx.x + NTH * i, r = p >> 3, cc = h * 8 + (p & 7);
            const int64_t j = row0 + r;
            const uint16_t* src = B.rec ? (const uint16_t*)(B.rec + perm_of(B, j) * B.rb) : B.obs + sample_of(B, j) * d.Ds;
            pv[i] = (j < B.rows && cc * 8 < d.Ds) ? *(const uint4*)(src + cc * 8) : uint4{0u, 0u, 0u, 0u};
        }
    };
    auto store_half = [&](int64_t tile, int h) {  // -> the LDS tile and the minibatch's observation rows
#pragma unroll
        for (int i = 0; i < NPC; ++i) {
            const int p = threadIdx.x + NTH * i, cc = h * 8 + (p & 7);
            *(uint4*)(hbuf + (p >> 3) * HS + cc * 8) = pv[i];
            *(uint4*)(Orows + (tile * TILE + (p >> 3)) * d.K1p + cc * 8) = pv[i];
        }
    };
    auto gather = [&](int64_t tile) {
        const int64_t row0 = tile * TILE;
        mean = stats[0];
        istd = stats[1];
        if ((int)threadIdx.x < TILE && row0 + (int)threadIdx.x < B.rows) {
            if (B.rec) {  // one record: five consecutive words
                const float* sc = (const float*)(B.rec + perm_of(B, row0 + threadIdx.x) * B.rb + B.rsc);
#pragma unroll
                for (int k = 0; k < 5; ++k) gs[k] = sc[k];
            } else {
                const int64_t sidx = sample_of(B, row0 + threadIdx.x);
                gs[0] = __int_as_float(B.act[sidx]);
                gs[1] = B.logp_old[sidx];
                gs[2] = B.val_old[sidx];
                gs[3] = B.adv[sidx];
                gs[4] = B.ret[sidx];
            }
        }
#pragma unroll
        for (int i = 0; i < MWP; ++i) {
            const int p = threadIdx.x + NTH * i;
            const int r = p / W;
            const int64_t j = row0 + r;
            const uint32_t* src = B.rec ? (const uint32_t*)(B.rec + perm_of(B, j) * B.rb + B.rmask)
                                        : B.mask + sample_of(B, j) * W;
            gm[i] = (r < TILE && j < B.rows) ? src[p - r * W] : 0u;
        }
        obs_half(tile, 0);
    };
    auto commit = [&](int64_t tile) {
        const int64_t row0 = tile * TILE;
        if ((int)threadIdx.x < TILE) {
            const int r = threadIdx.x;
            const bool v = row0 + r < B.rows;
            rinfo[0 * TILE + r] = v ? gs[0] : 0.f;
            rinfo[1 * TILE + r] = v ? gs[1] : 0.f;
            rinfo[2 * TILE + r] = v ? gs[2] : 0.f;
            rinfo[3 * TILE + r] = v ? (gs[3] - mean) * istd : 0.f;
            rinfo[4 * TILE + r] = v ? gs[4] : 0.f;
            rinfo[5 * TILE + r] = v ? 1.f : 0.f;
        }
#pragma unroll
        for (int i = 0; i < MWP; ++i) {
            const int p = threadIdx.x + NTH * i;
            if (p < TILE * W) smask[p] = gm[i];
        }
        store_half(tile, 0);
        if (d.K1p > K1P) {  // wide rows: the second 64 columns, one more round trip
            obs_half(tile, 1);
            store_half(tile, 1);
        }
    };

    const int64_t tile = blockIdx.x;
    gather(tile);
    load_biases<H, NTH>(d, params, sbias);
    commit(tile);
    lds_barrier();
    const int64_t tile_row0 = tile * TILE;
    const int64_t mb0 = tile_row0 >> 5;

    // ---- forward of the hidden layers (column split); every layer's bf16
    // output also leaves as m-blocks for the weight gradients
    // (the first k-step of each layer takes the bias as its accumulator input)
    f32x4 acc[TR][CTW], cb[CTW];
    uint32_t m1[TR], m2[TR];
    auto bias_frags = [&](const float* bias) {
#pragma unroll
        for (int ct = 0; ct < CTW; ++ct) {
            const float4 b = *(const float4*)(bias + col0 + ct * 16 + 4 * (l >> 4));
            cb[ct] = f32x4{b.x, b.y, b.z, b.w};
        }
    };
    bias_frags(sbias);
    dense_first_bias<TR, CTW, 2, true, true>(acc, cb, hbuf, HS, work + d.oW1f, (int64_t)H * 32, col0, d.K1p);
    lds_barrier();  // every wave is done reading the observations
    ppo_hidden_epilogue_cs<TR, CTW, false>(acc, nullptr, hbuf, HS, col0, m1);
    bias_frags(sbias + H);
    lds_barrier();
    dense_cs_bias<TR, CTW, H / 32, 3, true, true>(acc, cb, hbuf, HS, work + d.oW2f, (int64_t)H * 32, col0);
    lds_barrier();
    ppo_hidden_epilogue_cs<TR, CTW, false>(acc, nullptr, hbuf, HS, col0, m2);
    lds_barrier();
    tile_to_mblocks(hbuf, HS, TILE, H, Th2, mb0, H, 0);

    // Logit chunks: wave w computes columns [16 LCT w, 16 LCT (w + 1)) of the
    // chunk for every row into LDS (fp32); then a quad of lanes of a row-owning
    // wave owns a row (q = lane % 4 takes the chunk's columns 32 q .. 32 q + 31).
    const float NEG = -__builtin_huge_valf();
    const int srow = (wave & 3) * 16 + (l >> 2);
    const int a_taken = __float_as_int(rinfo[srow]);
    // Masked logits become MASKED, a finite stand-in for -inf (the network's
    // logits are finite): exp(MASKED - shift) is exactly 0 for any finite
    // shift, and so is its product with any finite factor, so the sums and
    // gradients below need no per-action select.  Bit j of the quarter's
    // mask word, spread to a whole word, keeps the logit (extract + insert).
    constexpr float MASKED = -1e30f;
    auto mask_logit = [&](float zj, uint32_t mw, int j) {
        const int keep = __builtin_amdgcn_sbfe((int)mw, j, 1);
        return __int_as_float((__float_as_int(zj) & keep) | (__float_as_int(MASKED) & ~keep));
    };
    // allowed actions of this lane's quarter of chunk c (bits past the last action cleared)
    auto quarter_mask = [&](int c) {
        const int wi = c * 4 + q, nact = d.A - (c * 128 + 32 * q);
        const uint32_t mw = wi < W ? smask[srow * W + wi] : 0u;
        return nact >= 32 ? mw : (nact <= 0 ? 0u : mw & ((1u << nact) - 1u));
    };
    auto logit_chunk = [&](int c) {
        f32x4 acc3[TR][LCT];
        dense_cs<TR, LCT, H / 32, true, 3, true, true>(acc3, hbuf, HS, work + d.oW3f + (int64_t)c * 128 * 32,
                                                        (int64_t)d.A1p * 32, 16 * LCT * wave);
#pragma unroll
        for (int ct = 0; ct < LCT; ++ct) {
            const int cc = 16 * LCT * wave + ct * 16 + 4 * (l >> 4);  // 4 adjacent columns of row l % 16
            const float4 b = *(const float4*)(sbias + 2 * H + c * 128 + cc);
#pragma unroll
            for (int rt = 0; rt < TR; ++rt)
                *(float4*)(zbuf + (rt * 16 + (l & 15)) * ZS + zcol(l & 15, cc)) =
                    float4{acc3[rt][ct][0] + b.x, acc3[rt][ct][1] + b.y, acc3[rt][ct][2] + b.z, acc3[rt][ct][3] + b.w};
        }
    };
    auto load_row = [&](float (&z)[32]) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float4 v = *(const float4*)(zbuf + srow * ZS + q * ZQ + 4 * (j ^ zsw(srow)));
            z[4 * j] = v.x;
            z[4 * j + 1] = v.y;
            z[4 * j + 2] = v.z;
            z[4 * j + 3] = v.w;
        }
    };

    // ---- pass 1: masked-softmax statistics, logit of the taken action, value
    float sm = NEG, sS = 0.f, sT = 0.f, za = 0.f, zv = 0.f;
    for (int c = 0; c < d.NC; ++c) {
        logit_chunk(c);
        lds_barrier();
        if (rowner) {
        float z[32];
        load_row(z);
        const uint32_t mw = quarter_mask(c);
        // the taken action's logit and the value head: one read each (the
        // quad's four lanes read the same word)
        const int ta = a_taken - c * 128, va = d.A - c * 128;
        if (ta >= 0 && ta < 128) za += zbuf[srow * ZS + zcol(srow, ta)];
        if (va >= 0 && va < 128) zv += zbuf[srow * ZS + zcol(srow, va)];
        float zmax = MASKED;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            z[j] = mask_logit(z[j], mw, j);
            zmax = fmaxf(zmax, z[j]);
        }
        zmax = quad_max(zmax);
        const bool any = zmax > MASKED;
        const float zs = any ? zmax : 0.f;  // a finite shift: masked weights are exactly 0
        float se = 0.f, te = 0.f;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const float dz = z[j] - zs;
            const float e = __expf(dz);
            se += e;
            te = __builtin_fmaf(e, dz, te);
        }
        se = quad_sum(se);
        te = quad_sum(te);
        const float mn = any ? fmaxf(sm, zmax) : sm;
        const float fo = sm == NEG ? 0.f : __expf(sm - mn), fc = any ? __expf(zmax - mn) : 0.f;
        sT = (sm == NEG ? 0.f : fo * (sT + (sm - mn) * sS)) + (any ? fc * (te + (zmax - mn) * se) : 0.f);
        sS = sS * fo + se * fc;
        sm = mn;
        }  // rowner
        if (c + 1 < d.NC) lds_barrier();  // before the next chunk overwrites the logits
    }

    // ---- per-row loss terms and gradient coefficients
    const bool valid = rinfo[5 * TILE + srow] != 0.f && sS > 0.f;
    const float lS = valid ? __logf(sS) : 0.f;
    const float lse = sm + lS;
    const float ent = valid ? lS - sT / sS : 0.f;
    const float lpn = za - lse;
    const float ratio = __expf(lpn - rinfo[1 * TILE + srow]);
    const float ah = rinfo[3 * TILE + srow];
    const float s1 = ratio * ah;
    const float rc = fminf(fmaxf(ratio, 1.f - hp.clip), 1.f + hp.clip);
    const float s2 = rc * ah;
    const bool active = !(s1 > s2);
    const float cpg = valid ? (active ? -ah * ratio : 0.f) * inv_n : 0.f;
    const float V = zv, vo = rinfo[2 * TILE + srow], R = rinfo[4 * TILE + srow];
    const float dvv = V - vo;
    const float vc = vo + fminf(fmaxf(dvv, -hp.vclip), hp.vclip);
    const float l1 = (V - R) * (V - R), l2 = (vc - R) * (vc - R);
    const float gv = l1 >= l2 ? (V - R) : ((dvv >= -hp.vclip && dvv <= hp.vclip) ? (vc - R) : 0.f);
    const float dzv = valid ? hp.vf_coef * gv * inv_n : 0.f;
    {
        const bool cnt = valid && q == 0;
        float part_pg = cnt ? -fminf(s1, s2) : 0.f;
        float part_vf = cnt ? 0.5f * fmaxf(l1, l2) : 0.f;
        float part_ent = cnt ? ent : 0.f;
        float part_clip = cnt && fabsf(ratio - 1.f) > hp.clip ? 1.f : 0.f;
        part_pg = wave_sum(part_pg);
        part_vf = wave_sum(part_vf);
        part_ent = wave_sum(part_ent);
        part_clip = wave_sum(part_clip);
        if (l == 0) {
            lred[wave * 4 + 0] = part_pg;
            lred[wave * 4 + 1] = part_vf;
            lred[wave * 4 + 2] = part_ent;
            lred[wave * 4 + 3] = part_clip;
        }
    }

    // ---- pass 2: dY = dL/d[logits | value] per chunk, dh2 += dY W3^T
    const float cent = hp.ent_coef * inv_n;
    const float kq = cent * ent - cpg;
    const float lse2 = valid ? lse : 0.f;  // rows without an allowed action: every weight exactly 0
    // the taken action, when allowed: its gradient takes cpg more
    const bool taken_ok = valid && a_taken >= 0 && a_taken < d.A &&
                          ((smask[srow * W + (a_taken >> 5)] >> (a_taken & 31)) & 1u);
    const float lp_taken = za - lse2;
    const float g_taken = __expf(lp_taken) * __builtin_fmaf(cent, lp_taken, kq) + cpg;
    f32x4 dh[TR][CTW];
    for (int c = 0; c < d.NC; ++c) {
        if (d.NC > 1) {  // with one chunk its logits are still in LDS
            lds_barrier();  // everyone is done with the previous chunk's dY
            logit_chunk(c);
            lds_barrier();
        }
        uint32_t gp[16];
        if (rowner) {
        float z[32];
        load_row(z);
        const uint32_t mw = quarter_mask(c);
        // allowed action a: dL/dz_a = cpg ([a taken] - p_a) + cent p_a (lp_a + ent)
        //                            = p_a (cent lp_a + kq) + cpg [a taken];
        // the taken action's term and the value head are set below
#pragma unroll
        for (int j = 0; j < 32; j += 2) {
            float g2[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float lp = mask_logit(z[j + h], mw, j + h) - lse2;
                const float p = __expf(lp);
                g2[h] = p * __builtin_fmaf(cent, lp, kq);
            }
            gp[j >> 1] = bf16x2_bits(g2[0], g2[1]);
        }
        }  // rowner
        lds_barrier();  // every lane has read its logits: the chunk's space takes dY
        if (rowner) {
            uint4* yrow = (uint4*)(ybuf + srow * YS + 32 * q);  // 16-byte stores: no bank conflicts
#pragma unroll
            for (int j = 0; j < 4; ++j) yrow[j] = uint4{gp[4 * j], gp[4 * j + 1], gp[4 * j + 2], gp[4 * j + 3]};
            // after the row's stores (LDS keeps a wave's order): the taken
            // action's gradient and the value head's
            const int ta = a_taken - c * 128, va = d.A - c * 128;
            if (q == 0 && taken_ok && ta >= 0 && ta < 128) ybuf[srow * YS + ta] = f32_to_bf16(g_taken);
            if (q == 0 && va >= 0 && va < 128) ybuf[srow * YS + va] = f32_to_bf16(dzv);
        }
        lds_barrier();
        tile_to_mblocks(ybuf, YS, TILE, 128, TdY, mb0, d.A1p, c * 128);  // dY for dW3
        if (c == 0)
            dense_cs<TR, CTW, 4, true, 3, true, true>(dh, ybuf, YS, work + d.oW3b, (int64_t)H * 32, col0);
        else
            dense_cs<TR, CTW, 4, false, 3, true, true>(dh, ybuf, YS, work + d.oW3b + (int64_t)c * 4 * H * 32,
                                                       (int64_t)H * 32, col0);
    }

    // ---- dh2 = (dY W3^T) * [h2 > 0] -> LDS (A operand of the next product) and m-blocks
    lds_barrier();  // the activations h2 are no longer read
    ppo_masked_grad_cs<TR, CTW>(dh, m2, hbuf, HS, col0);
    lds_barrier();
    tile_to_mblocks(hbuf, HS, TILE, H, Tdh2, mb0, H, 0);
    // ---- dh1 = (dh2 W2^T) * [h1 > 0] -> m-blocks, straight from the
    // accumulators (plain layout: a lane's four rows of one column are 8
    // contiguous bytes of the m-block)
    dense_cs<TR, CTW, H / 32, true, 3, true, false>(dh, hbuf, HS, work + d.oW2b, (int64_t)H * 32, col0);
    ppo_grad_to_mblocks<TR, CTW>(dh, m1, Tdh1, mb0, H, col0);
    if (threadIdx.x < 4) {
        float sum = 0.f;
        for (int w = 0; w < 4; ++w) sum += lred[w * 4 + threadIdx.x];
        loss_parts[tile * 4 + threadIdx.x] = sum;
    }
}

// ---------------------------------------------------------------------------
// weight gradients: C[j][n] = sum_m X[m][j] Y[m][n] over m-blocks
// ---------------------------------------------------------------------------
// Where X comes from.  XM_BLOCKS: X's own m-blocks.  XM_OBS: X is the
// observation tile, read as minibatch rows [rows][K1p] and transposed into
// the LDS tile (dW1).  XM_H1: X = h1 = relu(obs W1 + b1), recomputed for the
// tile's columns from the observation rows with the same bf16 MFMA products
// and rounding as the row kernel (dW2), so that h1 never passes through HBM.
enum { XM_BLOCKS = 0, XM_OBS = 1, XM_H1 = 2 };

struct DwX {
    const uint16_t* obs;  // [rows][K1p] bf16 observation rows, minibatch order (XM_OBS, XM_H1)
    const uint16_t* w1f;  // W1 K-chunks [K1p / 32][H][32] (XM_H1)
    const float* b1;      // [H] (XM_H1)
    int K1p;
};

template <int WJ, int WN, int TJ, int TN, int XM, int NK1 = 2>
__global__ void __launch_bounds__(WJ* WN * 64)
dw_kernel(const uint16_t* __restrict__ Tx, int J, const uint16_t* __restrict__ Ty, int N, int64_t nmb, int G,
          float* __restrict__ part, float* __restrict__ colsum, const DwX xsrc)
{
    constexpr int CJ = WJ * TJ * 16, CN = WN * TN * 16, NTH = WJ * WN * 64, NW = NTH / 64;
    // two LDS stages of [X tile | Y tile]: the products of an m-block read one
    // stage while the next m-block is written to the other (one barrier per
    // m-block)
    extern __shared__ __align__(16) unsigned char dw_smem[];
    constexpr int STAGE = (CJ + CN) * WSTRIDE;  // bf16 elements per stage
    uint16_t* const lds0 = (uint16_t*)dw_smem;
    const int njt = J / CJ;
    const int jt = blockIdx.x % njt, nt = blockIdx.x / njt;
    const int j0 = jt * CJ, n0 = nt * CN;
    const int g = blockIdx.y;
    const int64_t mb0 = nmb * g / G, mb1 = nmb * (g + 1) / G;
    const int wave = threadIdx.x >> 6, l = lane_id();
    const int wj = wave % WJ, wn = wave / WJ;
    f32x4 acc[TJ][TN];
#pragma unroll
    for (int a = 0; a < TJ; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    float cs = 0.f;
    constexpr int PX = CJ * 4, PY = CN * 4;  // 16-byte pieces per tile (at most two per thread)
    static_assert(PX <= 2 * NTH && PY <= 2 * NTH, "two prefetch registers per operand");

    // XM_H1: the X tile is CJ / 16 column tiles x 2 row tiles of 16 x 16; wave
    // w computes XT of them (tiles t = w XT + i: column tile t / 2, row tile
    // t % 2) from its W1 fragments (held for the whole launch) and the
    // observation fragments of the m-block
    constexpr int XT = XM == XM_H1 ? CJ / 8 / NW : 1;
    constexpr int XJ = XT >= 2 ? XT / 2 : 1;  // distinct column tiles per wave
    constexpr int XR = XT >= 2 ? 2 : 1;       // row tiles per wave
    static_assert(XM != XM_H1 || (XT >= 1 && (XT == 1 || XT % 2 == 0)), "X tiles per wave");
    bf16x8 w1q[XM == XM_H1 ? XJ : 1][NK1];
    float b1v[XM == XM_H1 ? XJ : 1];
    const int xt0 = wave * XT;
    if constexpr (XM == XM_H1) {
#pragma unroll
        for (int a = 0; a < XJ; ++a) {
            const int j = j0 + ((xt0 >> 1) + a) * 16 + (l & 15);
            b1v[a] = xsrc.b1[j];
#pragma unroll
            for (int kt = 0; kt < NK1; ++kt)  // (X = h1 has J = H columns: W1f is [K1p / 32][J][32])
                w1q[a][kt] = *(const bf16x8*)(xsrc.w1f + ((int64_t)kt * J + j) * 32 + 8 * (l >> 4));
        }
    }

    // the next m-block's global data (plain scalars: arrays indexed at run
    // time would land in scratch memory)
    uint4 rx0, rx1, ry0, ry1;
    bf16x8 oq[XM == XM_H1 ? XR : 1][NK1];
    auto load = [&](int64_t mb) {
        const int p0 = threadIdx.x, p1 = threadIdx.x + NTH;
        if constexpr (XM == XM_BLOCKS) {
            if (p0 < PX) rx0 = *(const uint4*)(Tx + (mb * J + j0 + (p0 >> 2)) * 32 + (p0 & 3) * 8);
            if (p1 < PX) rx1 = *(const uint4*)(Tx + (mb * J + j0 + (p1 >> 2)) * 32 + (p1 & 3) * 8);
        } else if constexpr (XM == XM_OBS) {  // piece p: row p / (CJ / 8), columns 8 (p % (CJ / 8)) .. + 7
            constexpr int PR = CJ / 8;
            if (p0 < PX) rx0 = *(const uint4*)(xsrc.obs + (mb * 32 + p0 / PR) * xsrc.K1p + j0 + (p0 % PR) * 8);
            if (p1 < PX) rx1 = *(const uint4*)(xsrc.obs + (mb * 32 + p1 / PR) * xsrc.K1p + j0 + (p1 % PR) * 8);
        } else {  // A operand of obs W1: row m = 16 mt + lane % 16, k = 32 kt + 8 (lane / 16) .. + 7
#pragma unroll
            for (int r = 0; r < XR; ++r) {
                const int mt = XT >= 2 ? r : (xt0 & 1);
#pragma unroll
                for (int kt = 0; kt < NK1; ++kt)
                    oq[r][kt] = *(const bf16x8*)(xsrc.obs + (mb * 32 + mt * 16 + (l & 15)) * xsrc.K1p + kt * 32 +
                                                   8 * (l >> 4));
            }
        }
        if (p0 < PY) ry0 = *(const uint4*)(Ty + (mb * N + n0 + (p0 >> 2)) * 32 + (p0 & 3) * 8);
        if (p1 < PY) ry1 = *(const uint4*)(Ty + (mb * N + n0 + (p1 >> 2)) * 32 + (p1 & 3) * 8);
    };
    // observation piece -> eight transposed bf16 entries of the X tile
    auto put_obs = [&](uint16_t* xs, int p, const uint4& v) {
        constexpr int PR = CJ / 8;
        const int m = p / PR, jj = (p % PR) * 8;
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 8; ++i) xs[(jj + i) * WSTRIDE + m] = (uint16_t)(w[i >> 1] >> (16 * (i & 1)));
    };
    // registers -> LDS stage s (the X tile computed in XM_H1)
    auto produce = [&](int s) {
        uint16_t* xs = lds0 + s * STAGE;
        uint16_t* ys = xs + CJ * WSTRIDE;
        const int p0 = threadIdx.x, p1 = threadIdx.x + NTH;
        if constexpr (XM == XM_BLOCKS) {
            if (p0 < PX) *(uint4*)(xs + (p0 >> 2) * WSTRIDE + (p0 & 3) * 8) = rx0;
            if (p1 < PX) *(uint4*)(xs + (p1 >> 2) * WSTRIDE + (p1 & 3) * 8) = rx1;
        } else if constexpr (XM == XM_OBS) {
            if (p0 < PX) put_obs(xs, p0, rx0);
            if (p1 < PX) put_obs(xs, p1, rx1);
        } else {  // h1 = relu(obs W1 + b1) -> bf16, lane: column j, rows 4 (lane / 16) .. + 3
#pragma unroll
            for (int i = 0; i < XT; ++i) {
                const int t = xt0 + i, a = XT >= 2 ? i >> 1 : 0, r = XT >= 2 ? (i & 1) : 0;
                f32x4 h = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kt = 0; kt < NK1; ++kt) h = mfma16(oq[r][kt], w1q[a][kt], h);
                *(uint2*)(xs + ((t >> 1) * 16 + (l & 15)) * WSTRIDE + (t & 1) * 16 + 4 * (l >> 4)) =
                    uint2{relu_bf16x2(h[0] + b1v[a], h[1] + b1v[a]), relu_bf16x2(h[2] + b1v[a], h[3] + b1v[a])};
            }
        }
        if (p0 < PY) *(uint4*)(ys + (p0 >> 2) * WSTRIDE + (p0 & 3) * 8) = ry0;
        if (p1 < PY) *(uint4*)(ys + (p1 >> 2) * WSTRIDE + (p1 & 3) * 8) = ry1;
    };
    // the products of the m-block in LDS stage s
    auto consume = [&](int s) {
        const uint16_t* xs = lds0 + s * STAGE;
        const uint16_t* ys = xs + CJ * WSTRIDE;
        bf16x8 af[TJ];
#pragma unroll
        for (int a = 0; a < TJ; ++a) af[a] = lds_frag(xs + (wj * TJ * 16 + a * 16 + (l & 15)) * WSTRIDE + 8 * (l >> 4));
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const bf16x8 bf = lds_frag(ys + (wn * TN * 16 + b * 16 + (l & 15)) * WSTRIDE + 8 * (l >> 4));
#pragma unroll
            for (int a = 0; a < TJ; ++a) acc[a][b] = mfma16(af[a], bf, acc[a][b]);
        }
        if (jt == 0 && (int)threadIdx.x < CN) {  // column sums of Y (the bias gradient): 16-byte reads
            const uint4* yrow = (const uint4*)(ys + threadIdx.x * WSTRIDE);
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
                const uint4 v = yrow[q4];
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    cs += __uint_as_float(w[e] << 16);
                    cs += __uint_as_float(w[e] & 0xffff0000u);
                }
            }
        }
    };
    // m-block mb sits in stage s and the registers hold m-block mb + 1: run
    // the products of mb, write mb + 1 to the other stage, load mb + 2 (a
    // whole m-block of products ahead of its use), one barrier
    if (mb0 < mb1) {
        load(mb0);
        produce(0);
        if (mb0 + 1 < mb1) load(mb0 + 1);
        __syncthreads();
    }
    for (int64_t mb = mb0; mb < mb1; ++mb) {
        const int s = (int)((mb - mb0) & 1);
        consume(s);
        if (mb + 1 < mb1) produce(s ^ 1);
        if (mb + 2 < mb1) load(mb + 2);
        __syncthreads();
    }
    float* out = part + (int64_t)g * J * N;
#pragma unroll
    for (int a = 0; a < TJ; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int n = n0 + wn * TN * 16 + b * 16 + (l & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = j0 + wj * TJ * 16 + a * 16 + 4 * (l >> 4) + i;
                out[(int64_t)j * N + n] = acc[a][b][i];
            }
        }
    if (jt == 0 && (int)threadIdx.x < CN) colsum[(int64_t)g * N + n0 + threadIdx.x] = cs;
}

// grad[woff + j ldw + n] = sum_g part[g][j][n] (j < Jv, n < Nv); bias from the
// column sums.  A workgroup takes 32 consecutive elements: eight slices of
// its threads sum the partials g = s, s + 8, ... (coalesced 128-byte rows,
// many loads in flight), and slice sums are added in the order s = 0 .. 7,
// a fixed order for every call.
__global__ void __launch_bounds__(256) dw_reduce_kernel(const float* __restrict__ part, const float* __restrict__ colsum,
                                                        int J, int N, int G, int Jv, int Nv, float* __restrict__ grad,
                                                        int64_t woff, int ldw, int64_t boff)
{
    __shared__ float red[8][32];
    const int i = threadIdx.x & 31, sl = threadIdx.x >> 5;
    const int64_t total = (int64_t)J * N;
    const int64_t idx = (int64_t)blockIdx.x * 32 + i;
    const bool in = idx < total + N;
    const float* src = idx < total ? part + idx : colsum + (idx - total);
    const int64_t stride = idx < total ? total : N;
    float acc = 0.f;
    if (in) {
        int g = sl;
        for (; g + 24 < G; g += 32) {  // four loads in flight per thread
            const float v0 = src[(int64_t)g * stride], v1 = src[(int64_t)(g + 8) * stride];
            const float v2 = src[(int64_t)(g + 16) * stride], v3 = src[(int64_t)(g + 24) * stride];
            acc += v0;
            acc += v1;
            acc += v2;
            acc += v3;
        }
        for (; g < G; g += 8) acc += src[(int64_t)g * stride];
    }
    red[sl][i] = acc;
    __syncthreads();
    if (sl == 0 && in) {
        float sum = 0.f;
#pragma unroll
        for (int k = 0; k < 8; ++k) sum += red[k][i];
        if (idx < total) {
            const int j = (int)(idx / N), n = (int)(idx % N);
            if (j < Jv && n < Nv) grad[woff + (int64_t)j * ldw + n] = sum;
        } else {
            const int n = (int)(idx - total);
            if (n < Nv) grad[boff + n] = sum;
        }
    }
}

// minibatch means of the four loss terms from the per-tile partial sums: the
// tiles are cut into fixed slices (one workgroup each, partial sums in
// double), then one workgroup adds the slices in order
__global__ void __launch_bounds__(256) loss_slices_kernel(const float* __restrict__ parts, int nparts, int nslices,
                                                          double* __restrict__ slice_sums)
{
    const int64_t b0 = (int64_t)nparts * blockIdx.x / nslices, b1 = (int64_t)nparts * (blockIdx.x + 1) / nslices;
    double t[4];
    block_sum_records<4>(parts + 4 * b0, b1 - b0, t);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) slice_sums[4 * blockIdx.x + c] = t[c];
    }
}

// out[0..3] = means of the surrogate, value and entropy terms and the clipped
// fraction; out[4] = surrogate + c_v value - c_e entropy (the minibatch loss)
__global__ void __launch_bounds__(256) loss_final_kernel(const double* __restrict__ slice_sums, int nslices,
                                                         int64_t rows, float vf_coef, float ent_coef,
                                                         float* __restrict__ out)
{
    double t[4];
    block_sum_records<4>(slice_sums, nslices, t);
    if (threadIdx.x == 0) {
        double m[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            m[c] = t[c] / (double)rows;
            out[c] = (float)m[c];
        }
        out[4] = (float)(m[0] + (double)vf_coef * m[1] - (double)ent_coef * m[2]);
    }
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// rows_mode (the population's row kernel): o_obs holds the observation rows
// [rows][K1p] (the same bytes as their m-blocks) and there is no h1 buffer.
// G1 row splits for dW1 (a narrow tile: two workgroups per CU), G for dW2
// and dW3.
struct PpoWorkspace {
    int64_t nmb, ntiles, G, G1;
    bool rows_mode;
    size_t o_obs, o_h1, o_h2, o_dy, o_dh2, o_dh1, o_p1, o_p2, o_p3, o_c1, o_c2, o_c3, o_adv, o_stats, o_loss, o_lslices,
        bytes;
};

static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

static int ppo_tile_rows(int) { return 64; }

static int ppo_workspace(const MlpDims& d, int64_t rows, PpoWorkspace* w, bool rows_mode = true)
{
    const int TILE = ppo_tile_rows(d.H);
    w->rows_mode = rows_mode;
    w->ntiles = (rows + TILE - 1) / TILE;
    w->nmb = w->ntiles * TILE / 32;
    w->G = w->nmb < 256 ? w->nmb : 256;
    if (w->G < 1) w->G = 1;
    w->G1 = w->nmb < 512 ? w->nmb : 512;
    if (w->G1 < 1) w->G1 = 1;
    size_t o = 0;
    const size_t mbrow = (size_t)w->nmb * 32 * 2;  // bytes per column of an m-block buffer
    w->o_obs = o; o = al256(o + mbrow * d.K1p);
    w->o_h1 = o; o = al256(o + (rows_mode ? 0 : mbrow * d.H));
    w->o_h2 = o; o = al256(o + mbrow * d.H);
    w->o_dy = o; o = al256(o + mbrow * d.A1p);
    w->o_dh2 = o; o = al256(o + mbrow * d.H);
    w->o_dh1 = o; o = al256(o + mbrow * d.H);
    w->o_p1 = o; o = al256(o + (size_t)w->G1 * d.K1p * d.H * 4);
    w->o_p2 = o; o = al256(o + (size_t)w->G * d.H * d.H * 4);
    w->o_p3 = o; o = al256(o + (size_t)w->G * d.H * d.A1p * 4);
    w->o_c1 = o; o = al256(o + (size_t)w->G1 * d.H * 4);
    w->o_c2 = o; o = al256(o + (size_t)w->G * d.H * 4);
    w->o_c3 = o; o = al256(o + (size_t)w->G * d.A1p * 4);
    w->o_adv = o; o = al256(o + 2 * 1024 * 8);
    w->o_stats = o; o = al256(o + 16);
    w->o_loss = o; o = al256(o + (size_t)w->ntiles * 16);
    w->o_lslices = o; o = al256(o + 256 * 4 * 8);
    w->bytes = o;
    return EJ_OK;
}

// Workspace of ej_ppo_backward_static: one array per device, which each
// device holds until the process ends.  Host code never passes `scratch`
// itself to a kernel or a copy (in host code the name is a stand-in, not a
// device address): it uses the address hipGetSymbolAddress returns for the
// current device, taken once per device on its first call.  Nothing in it
// needs to start at zero: every kernel of the backward writes what it
// later reads within the same call.
static __device__ __align__(256) unsigned char scratch[EJ_PPO_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static void* g_scratch_addr[kMaxDevices];
static std::mutex g_scratch_mu;

static int static_scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_last_hip_error(e);
        return EJ_EHIP;
    }
    if (dev < 0 || dev >= kMaxDevices) return EJ_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_last_hip_error(e);
            return EJ_EHIP;
        }
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return EJ_OK;
}

template <int XM, int NK1 = 2>
static int launch_dw(const uint16_t* Tx, int J, const uint16_t* Ty, int N, int64_t nmb, int G, float* part,
                     float* colsum, const DwX& xs, hipStream_t st)
{
    auto grid = [&](int CJ, int CN) { return dim3((unsigned)((J / CJ) * (N / CN)), (unsigned)G); };
#define EJ_DW(WJ, WN, TJ, TN)                                                                                   \
    dw_kernel<WJ, WN, TJ, TN, XM, NK1><<<grid(WJ * TJ * 16, WN * TN * 16), WJ * WN * 64,                        \
                                         (size_t)2 * (WJ * TJ * 16 + WN * TN * 16) * WSTRIDE * 2, st>>>(            \
        Tx, J, Ty, N, nmb, G, part, colsum, xs)
    if (J % 256 == 0 && N % 256 == 0)
        EJ_DW(4, 2, 4, 8);
    else if (J % 256 == 0 && N % 128 == 0)
        EJ_DW(4, 2, 4, 4);
    else if (J % 128 == 0 && N % 128 == 0)
        EJ_DW(2, 2, 4, 4);
    else if (J % 64 == 0 && N % 256 == 0)
        EJ_DW(1, 8, 4, 2);
    else if (J % 64 == 0 && N % 128 == 0)
        EJ_DW(1, 4, 4, 2);
    else if (J % 64 == 0 && N % 64 == 0)
        EJ_DW(1, 4, 4, 1);
    else
        return EJ_EUNSUPPORTED;
#undef EJ_DW
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

template <int H>
static int launch_rows(const MlpDims& d, const float* params, const uint16_t* work, const PpoBatchDev& B,
                       const PpoHp& hp, const float* stats, int W, uint16_t* const* T, float* loss_parts, int64_t ntiles,
                       hipStream_t st)
{
    const size_t lds = ppo_rows_lds_bytes<H>(W, d.A1p);
    const unsigned grid = (unsigned)ntiles;
    constexpr int NTH = PpoTile<H>::NTH;
    if (PpoTile<H>::TILE * W <= NTH)
        ppo_rows_kernel<H, 1><<<grid, NTH, lds, st>>>(d, params, work, B, hp, stats, W, T[0], T[2], T[3], T[4], T[5],
                                                      loss_parts);
    else
        ppo_rows_kernel<H, 8><<<grid, NTH, lds, st>>>(d, params, work, B, hp, stats, W, T[0], T[2], T[3], T[4], T[5],
                                                      loss_parts);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}


// record s <- sample s of the batch (storage index s * rstride + roff): the
// threads of a block row (threadIdx.y) write one record, one 4-byte word each
// (coalesced reads of the arrays, coalesced writes of the records)
__global__ void ppo_pack_kernel(const PpoBatchDev B, int Ds, int W, uint32_t* __restrict__ rec)
{
    const int wpr = (int)(B.rb / 4), w = threadIdx.x, byte = 4 * w;
    for (int64_t sm = (int64_t)blockIdx.x * blockDim.y + threadIdx.y; sm < B.Mtot; sm += (int64_t)gridDim.x * blockDim.y) {
        const int64_t g = sm * B.rstride + B.roff;
        uint32_t v = 0u;
        if (byte < 2 * Ds) {
            v = ((const uint32_t*)(B.obs + g * Ds))[w];
        } else if (byte >= B.rmask && byte < B.rsc) {
            v = B.mask[g * W + (byte - B.rmask) / 4];
        } else if (byte >= B.rsc && byte < B.rsc + 20) {
            switch ((byte - B.rsc) / 4) {
            case 0: v = (uint32_t)B.act[g]; break;
            case 1: v = __float_as_uint(B.logp_old[g]); break;
            case 2: v = __float_as_uint(B.val_old[g]); break;
            case 3: v = __float_as_uint(B.adv[g]); break;
            default: v = __float_as_uint(B.ret[g]); break;
            }
        }
        rec[sm * wpr + w] = v;
    }
}

// ===========================================================================
// The government's policy (Sec. 3 "Government Agent", "Setting tax rates"):
// the same two-hidden-layer network on the economy's government
// observation, with K independent categorical heads of 21 tax levels (a
// multi-discrete action, the logits of bracket k at columns 21 k .. 21 k +
// 20) and the value at column 21 K.  log pi(levels) is the sum of the K heads'
// log-probabilities and the entropy the sum of theirs.  One row per economy;
// at most 12 brackets (21 K + 1 <= 256) and H <= 256.
// ===========================================================================
constexpr int GOV_LEVELS = EJ_GOV_LEVELS;
constexpr int GOV_MAXK = 12;
constexpr int GOV_A1P = 256;  // logits + value, padded (two 128-column chunks)
constexpr int GOV_LS = GOV_A1P + 4;  // fp32 row stride of the full logit tile
constexpr int GOV_YS = GOV_A1P + 8;  // bf16 row stride of the dY tile

// government observation rows: fp32 features times their scale, rounded to
// bf16, zero beyond D -> LDS tile [64][hs] (columns < K1P) and, when `out`
// is given, the bf16 rows [rows][Ds] the learner stores
__device__ inline void gov_load_obs(const float* __restrict__ gobs, const float* __restrict__ scale, int64_t row0,
                                    int64_t E, int D, int Ds, uint16_t* hbuf, int hs, uint16_t* __restrict__ out)
{
    for (int p = threadIdx.x; p < 64 * K1P; p += blockDim.x) {
        const int r = p / K1P, c = p - r * K1P;
        const int64_t e = row0 + r;
        uint16_t v = 0;
        if (e < E && c < D) v = f32_to_bf16(gobs[e * D + c] * scale[c]);
        hbuf[r * hs + c] = v;
        if (out && e < E && c < Ds) out[e * Ds + c] = v;
    }
}

// the K heads of one row: max, sum of exp(z - m) and sum of exp(z - m)(z - m)
// over the 21 levels of head k (fp32, level order)
__device__ inline void gov_head_stats(const float* z, float& m, float& S, float& T)
{
    m = z[0];
#pragma unroll
    for (int j = 1; j < GOV_LEVELS; ++j) m = fmaxf(m, z[j]);
    S = 0.f;
    T = 0.f;
#pragma unroll
    for (int j = 0; j < GOV_LEVELS; ++j) {
        const float dz = z[j] - m;
        const float e = __expf(dz);
        S += e;
        T += e * dz;
    }
}

// Forward and sampling for 64 economies per workgroup: the network as in the
// population policy (column-split bf16 MFMA layers), the full logit row in
// LDS (fp32), then one thread per (economy, bracket): the head's softmax and
// an inverse-CDF draw in level order with the uniform of word k % 4 of
// Philox(GOV_SAMPLE; seed; economy, ctr, k / 4).
template <int H>
__global__ void __launch_bounds__(256)
gov_forward_kernel(const MlpDims d, int K, const float* __restrict__ params, const uint16_t* __restrict__ work,
                   const float* __restrict__ gobs, const float* __restrict__ scale, int64_t E, uint64_t seed,
                   uint64_t ctr_arg, const uint64_t* __restrict__ ctr_base, int32_t* __restrict__ levels,
                   float* __restrict__ logp, float* __restrict__ val, float* __restrict__ ent,
                   uint16_t* __restrict__ obs_out, float* __restrict__ logits)
{
    constexpr int TILE = 64, TR = 4, HS = H + 8, CTW = H / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t* hbuf = (uint16_t*)smem;                  // [64][HS]
    float* lbuf = (float*)(hbuf + TILE * HS);          // [64][GOV_LS]
    float* hl = lbuf + TILE * GOV_LS;                  // [64][GOV_MAXK] log-probabilities of the draws
    float* he = hl + TILE * GOV_MAXK;                  // [64][GOV_MAXK] head entropies
    float* sb3 = he + TILE * GOV_MAXK;                 // [GOV_A1P]
    const uint64_t ctr = ctr_arg + (ctr_base ? *ctr_base : 0ull);
    const int wave = threadIdx.x >> 6, l = lane_id();
    const int64_t row0 = (int64_t)blockIdx.x * TILE;
    gov_load_obs(gobs, scale, row0, E, d.D, d.Ds, hbuf, HS, obs_out);
    for (int p = threadIdx.x; p < GOV_A1P; p += 256) sb3[p] = p < d.A1 ? params[d.ob3 + p] : 0.f;
    {
        const int col0 = wave * (H / 4);
        f32x4 acc[TR][CTW];
        bias_init_t<TR, CTW>(acc, params + d.ob1, col0);
        lds_barrier();
        dense_cs<TR, CTW, 2, false, 2, false, true>(acc, hbuf, HS, work + d.oW1f, (int64_t)H * 32, col0);
        lds_barrier();
        relu_store_t<TR, CTW>(acc, hbuf, HS, col0);
        bias_init_t<TR, CTW>(acc, params + d.ob2, col0);
        lds_barrier();
        dense_cs<TR, CTW, H / 32, false, 2, false, true>(acc, hbuf, HS, work + d.oW2f, (int64_t)H * 32, col0);
        lds_barrier();
        relu_store_t<TR, CTW>(acc, hbuf, HS, col0);
        lds_barrier();
    }
    for (int c = 0; c < d.NC; ++c) {
        f32x4 acc3[TR][2];
        dense_cs<TR, 2, H / 32, true, 2, false, true>(acc3, hbuf, HS, work + d.oW3f + (int64_t)c * 128 * 32,
                                                      (int64_t)d.A1p * 32, 32 * wave);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const int cc = c * 128 + 32 * wave + ct * 16 + 4 * (l >> 4);
#pragma unroll
            for (int rt = 0; rt < TR; ++rt)
                *(float4*)(lbuf + (rt * 16 + (l & 15)) * GOV_LS + cc) =
                    float4{acc3[rt][ct][0] + sb3[cc], acc3[rt][ct][1] + sb3[cc + 1], acc3[rt][ct][2] + sb3[cc + 2],
                           acc3[rt][ct][3] + sb3[cc + 3]};
        }
    }
    lds_barrier();
    if (logits) {
        const int A = d.A;
        for (int p = threadIdx.x; p < TILE * A; p += 256) {
            const int r = p / A, c = p - r * A;
            if (row0 + r < E) logits[(row0 + r) * A + c] = lbuf[r * GOV_LS + c];
        }
    }
    for (int idx = threadIdx.x; idx < TILE * K; idx += 256) {
        const int r = idx / K, k = idx - r * K;
        const int64_t e = row0 + r;
        if (e >= E) continue;
        const float* z = lbuf + r * GOV_LS + k * GOV_LEVELS;
        float m, S, T;
        gov_head_stats(z, m, S, T);
        const u64x4 w = philox(seed, PURPOSE_GOV_SAMPLE, (uint64_t)e, ctr, (uint64_t)(k >> 2), 0);
        const float u = unif24(word_of(w, k & 3));
        const float target = u * S;
        float cum = 0.f;
        int j = GOV_LEVELS - 1;
#pragma unroll
        for (int q = 0; q < GOV_LEVELS; ++q) {
            cum += __expf(z[q] - m);
            if (cum > target) {
                j = q;
                break;
            }
        }
        const float lS = __logf(S);
        levels[e * K + k] = j;
        hl[r * GOV_MAXK + k] = z[j] - m - lS;
        he[r * GOV_MAXK + k] = lS - T / S;
    }
    lds_barrier();
    if (threadIdx.x < TILE) {
        const int r = threadIdx.x;
        const int64_t e = row0 + r;
        if (e < E) {
            float a = 0.f, b = 0.f;
            for (int k = 0; k < K; ++k) {  // bracket order
                a += hl[r * GOV_MAXK + k];
                b += he[r * GOV_MAXK + k];
            }
            logp[e] = a;
            ent[e] = b;
            val[e] = lbuf[r * GOV_LS + d.A];
        }
    }
}

// One fused pass over 64 minibatch rows of the government's PPO loss: the
// forward recomputed (its bf16 products and ReLU patterns kept), the full
// logit row in LDS, the K heads' softmax statistics, the per-row loss terms
// (ratio of the summed log-probabilities), dY = dL/d[logits | value] with
// dL/dz_kj = c_pg (1[j = a_k] - p_kj) + c_e/n p_kj (log p_kj + H_k), then
// dh2 and dh1 as in the population's kernel; every GEMM operand of the
// weight gradients leaves as bf16 m-blocks for dw_kernel.
template <int H>
__global__ void __launch_bounds__(256, 1)
gov_rows_kernel(const MlpDims d, int K, const float* __restrict__ params, const uint16_t* __restrict__ work,
                const PpoBatchDev B, const PpoHp hp, const float* __restrict__ stats, uint16_t* __restrict__ Tobs,
                uint16_t* __restrict__ Th1, uint16_t* __restrict__ Th2, uint16_t* __restrict__ TdY,
                uint16_t* __restrict__ Tdh2, uint16_t* __restrict__ Tdh1, float* __restrict__ loss_parts)
{
    constexpr int TILE = 64, TR = 4, HS = H + 8, CTW = H / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t* hbuf = (uint16_t*)smem;                      // [64][HS] obs -> h1 -> h2 -> dh2
    uint16_t* ybuf = hbuf + TILE * HS;                     // [64][GOV_YS] dY (bf16)
    float* lbuf = (float*)(ybuf + TILE * GOV_YS);          // [64][GOV_LS] logits
    float* rinfo = lbuf + TILE * GOV_LS;                   // [5][64] logp_old, val_old, adv_hat, ret, valid
    float* hm = rinfo + 5 * TILE;                          // [64][GOV_MAXK] head max
    float* hls = hm + TILE * GOV_MAXK;                     // [64][GOV_MAXK] log sum exp(z - max)
    float* hH = hls + TILE * GOV_MAXK;                     // [64][GOV_MAXK] head entropy
    float* hlp = hH + TILE * GOV_MAXK;                     // [64][GOV_MAXK] log-probability of the taken level
    int32_t* lvl = (int32_t*)(hlp + TILE * GOV_MAXK);      // [64][GOV_MAXK] taken levels
    float* coef = (float*)(lvl + TILE * GOV_MAXK);         // [64][3] c_pg, dL/dV, entropy of the row
    float* lred = coef + TILE * 3;                         // [4 waves][4]
    float* sbias = lred + 64;                              // b1 [H], b2 [H], b3 [GOV_A1P]

    const int wave = threadIdx.x >> 6, l = lane_id();
    const int64_t tile_row0 = (int64_t)blockIdx.x * TILE;
    const float inv_n = 1.0f / (float)B.rows;
    const int col0 = wave * (H / 4);

    for (int r = threadIdx.x; r < TILE; r += 256) {
        const int64_t j = tile_row0 + r;
        float lpo = 0.f, vo = 0.f, ah = 0.f, rt = 0.f, valid = 0.f;
        if (j < B.rows) {
            const int64_t sidx = sample_of(B, j);
            lpo = B.logp_old[sidx];
            vo = B.val_old[sidx];
            ah = (B.adv[sidx] - stats[0]) * stats[1];
            rt = B.ret[sidx];
            valid = 1.f;
        }
        rinfo[0 * TILE + r] = lpo;
        rinfo[1 * TILE + r] = vo;
        rinfo[2 * TILE + r] = ah;
        rinfo[3 * TILE + r] = rt;
        rinfo[4 * TILE + r] = valid;
    }
    for (int p = threadIdx.x; p < TILE * K; p += 256) {
        const int r = p / K, k = p - r * K;
        const int64_t j = tile_row0 + r;
        lvl[r * GOV_MAXK + k] = j < B.rows ? B.act[sample_of(B, j) * K + k] : 0;
    }
    for (int p = threadIdx.x; p < 2 * H + GOV_A1P; p += 256)
        sbias[p] = p < H ? params[d.ob1 + p]
                         : p < 2 * H ? params[d.ob2 + p - H] : (p - 2 * H < d.A1 ? params[d.ob3 + p - 2 * H] : 0.f);
    for (int p = threadIdx.x; p < TILE * (K1P / 8); p += 256) {
        const int r = p >> 3, cc = p & 7;
        const int64_t j = tile_row0 + r;
        const uint4 v = (j < B.rows && cc * 8 < d.Ds) ? *(const uint4*)(B.obs + sample_of(B, j) * d.Ds + cc * 8)
                                                       : uint4{0u, 0u, 0u, 0u};
        *(uint4*)(hbuf + r * HS + cc * 8) = v;
    }
    lds_barrier();
    const int64_t mb0 = tile_row0 >> 5;
    tile_to_mblocks(hbuf, HS, TILE, d.K1p, Tobs, mb0, d.K1p, 0);

    f32x4 acc[TR][CTW];
    uint32_t m1[TR], m2[TR];
    dense_cs<TR, CTW, 2, true, 2, true, true>(acc, hbuf, HS, work + d.oW1f, (int64_t)H * 32, col0);
    lds_barrier();
    ppo_hidden_epilogue_cs<TR, CTW>(acc, sbias, hbuf, HS, col0, m1);
    lds_barrier();
    tile_to_mblocks(hbuf, HS, TILE, H, Th1, mb0, H, 0);
    dense_cs<TR, CTW, H / 32, true, 3, true, true>(acc, hbuf, HS, work + d.oW2f, (int64_t)H * 32, col0);
    lds_barrier();
    ppo_hidden_epilogue_cs<TR, CTW>(acc, sbias + H, hbuf, HS, col0, m2);
    lds_barrier();
    tile_to_mblocks(hbuf, HS, TILE, H, Th2, mb0, H, 0);

    for (int c = 0; c < d.NC; ++c) {
        f32x4 acc3[TR][2];
        dense_cs<TR, 2, H / 32, true, 3, true, true>(acc3, hbuf, HS, work + d.oW3f + (int64_t)c * 128 * 32,
                                                      (int64_t)d.A1p * 32, 32 * wave);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const int cc = c * 128 + 32 * wave + ct * 16 + 4 * (l >> 4);
            const float* b3 = sbias + 2 * H + cc;
#pragma unroll
            for (int rt = 0; rt < TR; ++rt)
                *(float4*)(lbuf + (rt * 16 + (l & 15)) * GOV_LS + cc) =
                    float4{acc3[rt][ct][0] + b3[0], acc3[rt][ct][1] + b3[1], acc3[rt][ct][2] + b3[2],
                           acc3[rt][ct][3] + b3[3]};
        }
    }
    lds_barrier();
    // heads: softmax statistics and the taken level's log-probability
    for (int idx = threadIdx.x; idx < TILE * K; idx += 256) {
        const int r = idx / K, k = idx - r * K;
        const float* z = lbuf + r * GOV_LS + k * GOV_LEVELS;
        float m, S, T;
        gov_head_stats(z, m, S, T);
        const float lS = __logf(S);
        int a = lvl[r * GOV_MAXK + k];
        a = a < 0 ? 0 : (a >= GOV_LEVELS ? GOV_LEVELS - 1 : a);
        hm[r * GOV_MAXK + k] = m;
        hls[r * GOV_MAXK + k] = lS;
        hH[r * GOV_MAXK + k] = lS - T / S;
        hlp[r * GOV_MAXK + k] = z[a] - m - lS;
    }
    lds_barrier();
    // rows: ratio, loss terms and the coefficients of dY
    {
        float part_pg = 0.f, part_vf = 0.f, part_ent = 0.f, part_clip = 0.f;
        if (threadIdx.x < TILE) {
            const int r = threadIdx.x;
            const bool valid = rinfo[4 * TILE + r] != 0.f;
            float lp = 0.f, H_ = 0.f;
            for (int k = 0; k < K; ++k) {
                lp += hlp[r * GOV_MAXK + k];
                H_ += hH[r * GOV_MAXK + k];
            }
            const float ratio = __expf(lp - rinfo[0 * TILE + r]);
            const float ah = rinfo[2 * TILE + r];
            const float s1 = ratio * ah;
            const float rc = fminf(fmaxf(ratio, 1.f - hp.clip), 1.f + hp.clip);
            const float s2 = rc * ah;
            const bool active = !(s1 > s2);
            const float V = lbuf[r * GOV_LS + d.A], vo = rinfo[1 * TILE + r], R = rinfo[3 * TILE + r];
            const float dvv = V - vo;
            const float vc = vo + fminf(fmaxf(dvv, -hp.vclip), hp.vclip);
            const float l1 = (V - R) * (V - R), l2 = (vc - R) * (vc - R);
            const float gv = l1 >= l2 ? (V - R) : ((dvv >= -hp.vclip && dvv <= hp.vclip) ? (vc - R) : 0.f);
            coef[r * 3 + 0] = valid ? (active ? -ah * ratio : 0.f) * inv_n : 0.f;
            coef[r * 3 + 1] = valid ? hp.vf_coef * gv * inv_n : 0.f;
            coef[r * 3 + 2] = valid ? 1.f : 0.f;
            if (valid) {
                part_pg = -fminf(s1, s2);
                part_vf = 0.5f * fmaxf(l1, l2);
                part_ent = H_;
                part_clip = fabsf(ratio - 1.f) > hp.clip ? 1.f : 0.f;
            }
        }
        part_pg = wave_sum(part_pg);
        part_vf = wave_sum(part_vf);
        part_ent = wave_sum(part_ent);
        part_clip = wave_sum(part_clip);
        if (l == 0) {
            lred[wave * 4 + 0] = part_pg;
            lred[wave * 4 + 1] = part_vf;
            lred[wave * 4 + 2] = part_ent;
            lred[wave * 4 + 3] = part_clip;
        }
    }
    lds_barrier();
    // dY (bf16): the heads' columns, the value column, zero padding
    const float cent = hp.ent_coef * inv_n;
    const int KL = K * GOV_LEVELS;
    for (int p = threadIdx.x; p < TILE * (GOV_A1P / 2); p += 256) {
        const int r = p / (GOV_A1P / 2), c0 = 2 * (p - r * (GOV_A1P / 2));
        uint32_t pk = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int col = c0 + h;
            float g = 0.f;
            if (coef[r * 3 + 2] != 0.f) {
                if (col < KL) {
                    const int k = col / GOV_LEVELS, j = col - k * GOV_LEVELS;
                    const float lp = lbuf[r * GOV_LS + col] - hm[r * GOV_MAXK + k] - hls[r * GOV_MAXK + k];
                    const float pj = __expf(lp);
                    const float taken = j == lvl[r * GOV_MAXK + k] ? 1.f : 0.f;
                    g = coef[r * 3 + 0] * (taken - pj) + cent * pj * (lp + hH[r * GOV_MAXK + k]);
                } else if (col == KL) {
                    g = coef[r * 3 + 1];
                }
            }
            pk |= (uint32_t)f32_to_bf16(g) << (16 * h);
        }
        *(uint32_t*)(ybuf + r * GOV_YS + c0) = pk;
    }
    lds_barrier();
    tile_to_mblocks(ybuf, GOV_YS, TILE, d.A1p, TdY, mb0, d.A1p, 0);
    // dh2 = (dY W3^T) * [h2 > 0], chunk by chunk of 128 logit columns
    f32x4 dh[TR][CTW];
    for (int c = 0; c < d.NC; ++c) {
        if (c == 0)
            dense_cs<TR, CTW, 4, true, 3, true, true>(dh, ybuf, GOV_YS, work + d.oW3b, (int64_t)H * 32, col0);
        else
            dense_cs<TR, CTW, 4, false, 3, true, true>(dh, ybuf + c * 128, GOV_YS, work + d.oW3b + (int64_t)c * 4 * H * 32,
                                                       (int64_t)H * 32, col0);
    }
    lds_barrier();  // the activations h2 are no longer read
    ppo_masked_grad_cs<TR, CTW>(dh, m2, hbuf, HS, col0);
    lds_barrier();
    tile_to_mblocks(hbuf, HS, TILE, H, Tdh2, mb0, H, 0);
    dense_cs<TR, CTW, H / 32, true, 3, true, true>(dh, hbuf, HS, work + d.oW2b, (int64_t)H * 32, col0);
    lds_barrier();
    ppo_masked_grad_cs<TR, CTW>(dh, m1, hbuf, HS, col0);
    lds_barrier();
    tile_to_mblocks(hbuf, HS, TILE, H, Tdh1, mb0, H, 0);
    if (threadIdx.x < 4) {
        float sum = 0.f;
        for (int w = 0; w < 4; ++w) sum += lred[w * 4 + threadIdx.x];
        loss_parts[(int64_t)blockIdx.x * 4 + threadIdx.x] = sum;
    }
}

template <int H>
size_t gov_forward_lds_bytes()
{
    return (size_t)64 * (H + 8) * 2 + (size_t)64 * GOV_LS * 4 + 2 * (size_t)64 * GOV_MAXK * 4 + GOV_A1P * 4;
}

template <int H>
size_t gov_rows_lds_bytes()
{
    return (size_t)64 * (H + 8) * 2 + (size_t)64 * GOV_YS * 2 + (size_t)64 * GOV_LS * 4 + 5 * 64 * 4 +
           5 * (size_t)64 * GOV_MAXK * 4 + 64 * 3 * 4 + 64 * 4 + (size_t)(2 * H + GOV_A1P) * 4;
}

__global__ void sum_steps_kernel(const float* __restrict__ x, int t0, int t1, int64_t E, float* __restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int t = t0; t < t1; ++t) s += x[(int64_t)t * E + e];
        out[e] = s;
    }
}

static int gov_dims(const ej_mlp_desc* m, int32_t K, MlpDims* d)
{
    if (!m || K < 1 || K > GOV_MAXK || m->A != K * GOV_LEVELS) return EJ_EINVAL;
    if (m->H > 256 || m->D_stride > K1P) return EJ_EUNSUPPORTED;  // (its kernels take 64 input columns)
    return mlp_dims(m->D, m->D_stride, m->H, m->A, d);
}
}  // namespace econ

using namespace econ;

extern "C" {

int ej_gae(const float* d_rew, const float* d_val, const uint8_t* d_done, const float* d_last_val, int32_t T,
           int64_t M, float gamma, float lam, float* d_adv, float* d_ret, void* stream)
{
    if (!d_rew || !d_val || !d_done || !d_last_val || !d_adv || !d_ret || T <= 0 || M < 0) return EJ_EINVAL;
    if (M == 0) return EJ_OK;
    int64_t blocks = (M + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    gae_kernel<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(d_rew, d_val, d_done, d_last_val, T, M, gamma, lam,
                                                                 d_adv, d_ret);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

int ej_ppo_workspace_size(const ej_mlp_desc* m, int64_t rows, int64_t* bytes)
{
    if (!m || !bytes || rows <= 0) return EJ_EINVAL;
    MlpDims d;
    int rc = mlp_dims(m->D, m->D_stride, m->H, m->A, &d);
    if (rc != EJ_OK) return rc;
    PpoWorkspace w;
    ppo_workspace(d, rows, &w);
    *bytes = (int64_t)w.bytes;
    return EJ_OK;
}

int ej_ppo_record_bytes(const ej_mlp_desc* m, int64_t* bytes)
{
    if (!m || !bytes) return EJ_EINVAL;
    MlpDims d;
    int rc = mlp_dims(m->D, m->D_stride, m->H, m->A, &d);
    if (rc != EJ_OK) return rc;
    int rmask = 0, rsc = 0;
    record_layout(d.Ds, (d.A + 31) / 32, &rmask, &rsc, bytes);
    return EJ_OK;
}

int ej_ppo_pack(const ej_mlp_desc* m, const ej_ppo_batch* b, void* d_records, void* stream)
{
    if (!m || !b || !d_records) return EJ_EINVAL;
    if (!b->obs || !b->mask || !b->act || !b->logp_old || !b->val_old || !b->adv || !b->ret) return EJ_EINVAL;
    if (!aligned16(b->obs) || !aligned16(d_records)) return EJ_EINVAL;
    if (b->M_total <= 0 || b->M_total > INT32_MAX || b->row_offset < 0 ||
        (b->row_stride > 0 && b->row_offset >= b->row_stride))
        return EJ_EINVAL;
    MlpDims d;
    int rc = mlp_dims(m->D, m->D_stride, m->H, m->A, &d);
    if (rc != EJ_OK) return rc;
    const int W = (d.A + 31) / 32;
    PpoBatchDev B{b->obs, b->mask, b->act, b->logp_old, b->val_old, b->adv, b->ret, b->M_total, 1, 0, 0, 0, 0,
                  b->row_stride > 0 ? b->row_stride : 1, b->row_offset, nullptr, 0, 0, 0};
    record_layout(d.Ds, W, &B.rmask, &B.rsc, &B.rb);
    const int wpr = (int)(B.rb / 4);  // 32 .. 128 words (Ds <= 128, W <= 32)
    const int spb = wpr >= 256 ? 1 : 256 / wpr;
    int64_t blocks = (b->M_total + spb - 1) / spb;
    if (blocks > 65536) blocks = 65536;
    ppo_pack_kernel<<<(unsigned)blocks, dim3((unsigned)wpr, (unsigned)spb), 0, (hipStream_t)stream>>>(B, d.Ds, W,
                                                                                                     (uint32_t*)d_records);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

static int ppo_weight_grads_and_loss(const MlpDims& d, const PpoWorkspace& w, unsigned char* ws, int64_t rows,
                                     const ej_ppo_hparams& hp, const float* d_params, const uint16_t* d_work,
                                     float* d_grads, float* d_loss, hipStream_t st);

// a^-1 mod M by the extended Euclidean algorithm (0 < a < M); 0 when
// gcd(a, M) > 1 (then j -> a j + c is no permutation and has no inverse)
static uint64_t inverse_mod(int64_t a, int64_t M)
{
    int64_t r0 = M, r1 = a, t0 = 0, t1 = 1;
    while (r1 != 0) {
        const int64_t q = r0 / r1, r2 = r0 - q * r1, t2 = t0 - q * t1;
        r0 = r1;
        r1 = r2;
        t0 = t1;
        t1 = t2;
    }
    if (r0 != 1) return 0;
    if (t0 < 0) t0 += M;
    return (uint64_t)t0;
}

// the minibatch's advantage mean and 1 / (std + 1e-8) -> stats[0..1]:
// gathered per row for small minibatches, streamed otherwise
static void launch_adv_stats(const PpoBatchDev& B, double* part, float* stats, hipStream_t st)
{
    int nb;
    const uint64_t ainv = B.Mtot > 1 ? inverse_mod(B.a, B.Mtot) : 0;
    if (B.rows * 32 >= B.Mtot && ainv != 0 && B.Mtot < ((int64_t)1 << 31)) {
        nb = (int)((B.Mtot + 4095) / 4096);
        if (nb > 1024) nb = 1024;
        const uint64_t M = (uint64_t)B.Mtot;
        const uint32_t kc = (uint32_t)(ainv * (uint64_t)B.c % M);
        const uint32_t step = (uint32_t)(ainv * ((uint64_t)nb * 256u) % M);
        adv_stats_stream<<<nb, 256, 0, st>>>(B, (uint32_t)ainv, kc, step, part);
    } else {
        nb = (int)((B.rows + 255) / 256);
        if (nb > 1024) nb = 1024;
        adv_stats_partial<<<nb, 256, 0, st>>>(B, part);
    }
    adv_stats_final<<<1, 256, 0, st>>>(part, nb, B.rows, stats);
}

static int ppo_backward_impl(const ej_mlp_desc* m, const float* d_params, const uint16_t* d_work,
                             const ej_ppo_batch* b, const ej_ppo_hparams* hp, void* d_workspace,
                             int64_t workspace_bytes, float* d_grads, float* d_loss, void* stream)
{
    if (!m || !d_params || !d_work || !b || !hp || !d_workspace || !d_grads || !d_loss) return EJ_EINVAL;
    if (!b->obs || !b->mask || !b->act || !b->logp_old || !b->val_old || !b->adv || !b->ret) return EJ_EINVAL;
    if (!aligned16(d_params) || !aligned16(d_work) || !aligned16(b->obs) || !aligned16(d_workspace) ||
        !aligned16(d_grads) || !aligned16(b->records))
        return EJ_EINVAL;
    if (b->M_total <= 0 || b->M_total > INT32_MAX || b->rows <= 0 || b->perm_a <= 0 || b->perm_c < 0 ||
        b->row_begin < 0 || b->row_begin + b->rows > INT32_MAX || b->row_offset < 0 ||
        (b->row_stride > 0 && b->row_offset >= b->row_stride))
        return EJ_EINVAL;
    MlpDims d;
    int rc = mlp_dims(m->D, m->D_stride, m->H, m->A, &d);
    if (rc != EJ_OK) return rc;
    PpoWorkspace w;
    ppo_workspace(d, b->rows, &w);
    if (workspace_bytes < (int64_t)w.bytes) return EJ_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    unsigned char* ws = (unsigned char*)d_workspace;
    const int64_t a = b->M_total == 1 ? 1 : b->perm_a % b->M_total;
    if (a == 0) return EJ_EINVAL;
    PpoBatchDev B{b->obs, b->mask, b->act, b->logp_old, b->val_old, b->adv, b->ret, b->M_total, a,
                  b->perm_c % b->M_total, b->row_begin, b->rows, UINT64_MAX / (uint64_t)b->M_total,
                  b->row_stride > 0 ? b->row_stride : 1, b->row_offset, (const unsigned char*)b->records, 0, 0, 0};
    if (B.rec) record_layout(m->D_stride, (m->A + 31) / 32, &B.rmask, &B.rsc, &B.rb);
    PpoHp h{hp->clip, hp->vclip, hp->vf_coef, hp->ent_coef};
    const int W = (m->A + 31) / 32;
    double* advp = (double*)(ws + w.o_adv);
    float* stats = (float*)(ws + w.o_stats);
    launch_adv_stats(B, advp, stats, st);
    EJ_LAUNCH_CHECK();
    uint16_t* T[6] = {(uint16_t*)(ws + w.o_obs), (uint16_t*)(ws + w.o_h1), (uint16_t*)(ws + w.o_h2),
                      (uint16_t*)(ws + w.o_dy), (uint16_t*)(ws + w.o_dh2), (uint16_t*)(ws + w.o_dh1)};
    float* lparts = (float*)(ws + w.o_loss);
    switch (m->H) {
    case 64: rc = launch_rows<64>(d, d_params, d_work, B, h, stats, W, T, lparts, w.ntiles, st); break;
    case 128: rc = launch_rows<128>(d, d_params, d_work, B, h, stats, W, T, lparts, w.ntiles, st); break;
    case 256: rc = launch_rows<256>(d, d_params, d_work, B, h, stats, W, T, lparts, w.ntiles, st); break;
    default: rc = launch_rows<512>(d, d_params, d_work, B, h, stats, W, T, lparts, w.ntiles, st); break;
    }
    if (rc != EJ_OK) return rc;
    return ppo_weight_grads_and_loss(d, w, ws, b->rows, *hp, d_params, d_work, d_grads, d_loss, st);
}

// weight gradients from the m-blocks (dW GEMMs, fixed-order reduction) and
// the minibatch means of the loss terms from the per-tile partial sums
static int ppo_weight_grads_and_loss(const MlpDims& d, const PpoWorkspace& w, unsigned char* ws, int64_t rows,
                                     const ej_ppo_hparams& hp, const float* d_params, const uint16_t* d_work,
                                     float* d_grads, float* d_loss, hipStream_t st)
{
    int rc = EJ_OK;
    uint16_t* T[6] = {(uint16_t*)(ws + w.o_obs), (uint16_t*)(ws + w.o_h1), (uint16_t*)(ws + w.o_h2),
                      (uint16_t*)(ws + w.o_dy), (uint16_t*)(ws + w.o_dh2), (uint16_t*)(ws + w.o_dh1)};
    float* lparts = (float*)(ws + w.o_loss);
    float *p1 = (float*)(ws + w.o_p1), *p2 = (float*)(ws + w.o_p2), *p3 = (float*)(ws + w.o_p3);
    float *c1 = (float*)(ws + w.o_c1), *c2 = (float*)(ws + w.o_c2), *c3 = (float*)(ws + w.o_c3);
    const int G = (int)w.G, G1 = (int)w.G1;
    const DwX xs{T[0], d_work + d.oW1f, d_params + d.ob1, d.K1p};
    if (w.rows_mode) {  // dW1 from the observation rows, dW2 with h1 recomputed from them
        if ((rc = launch_dw<XM_OBS>(nullptr, d.K1p, T[5], d.H, w.nmb, G1, p1, c1, xs, st)) != EJ_OK) return rc;
        rc = d.K1p == K1P ? launch_dw<XM_H1, K1P / 32>(nullptr, d.H, T[4], d.H, w.nmb, G, p2, c2, xs, st)
                          : launch_dw<XM_H1, K1P_WIDE / 32>(nullptr, d.H, T[4], d.H, w.nmb, G, p2, c2, xs, st);
        if (rc != EJ_OK) return rc;
    } else {
        if ((rc = launch_dw<XM_BLOCKS>(T[0], d.K1p, T[5], d.H, w.nmb, G1, p1, c1, xs, st)) != EJ_OK) return rc;
        if ((rc = launch_dw<XM_BLOCKS>(T[1], d.H, T[4], d.H, w.nmb, G, p2, c2, xs, st)) != EJ_OK) return rc;
    }
    if ((rc = launch_dw<XM_BLOCKS>(T[2], d.H, T[3], d.A1p, w.nmb, G, p3, c3, xs, st)) != EJ_OK) return rc;
    auto red_blocks = [](int64_t n) { return (unsigned)((n + 31) / 32); };
    dw_reduce_kernel<<<red_blocks((int64_t)d.K1p * d.H + d.H), 256, 0, st>>>(p1, c1, d.K1p, d.H, G1, d.D, d.H, d_grads,
                                                                            d.oW1, d.H, d.ob1);
    EJ_LAUNCH_CHECK();
    dw_reduce_kernel<<<red_blocks((int64_t)d.H * d.H + d.H), 256, 0, st>>>(p2, c2, d.H, d.H, G, d.H, d.H, d_grads,
                                                                          d.oW2, d.H, d.ob2);
    EJ_LAUNCH_CHECK();
    dw_reduce_kernel<<<red_blocks((int64_t)d.H * d.A1p + d.A1p), 256, 0, st>>>(p3, c3, d.H, d.A1p, G, d.H, d.A1,
                                                                              d_grads, d.oW3, d.A1, d.ob3);
    EJ_LAUNCH_CHECK();
    const int nslices = (int)(w.ntiles < 256 ? w.ntiles : 256);
    double* lslices = (double*)(ws + w.o_lslices);
    loss_slices_kernel<<<nslices, 256, 0, st>>>(lparts, (int)w.ntiles, nslices, lslices);
    EJ_LAUNCH_CHECK();
    loss_final_kernel<<<1, 256, 0, st>>>(lslices, nslices, rows, hp.vf_coef, hp.ent_coef, d_loss);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

int ej_gov_policy_forward(const ej_mlp_desc* m, int32_t K, const float* d_params, const uint16_t* d_work,
                          const float* d_gov_obs, const float* d_scale, int64_t E, uint64_t seed, uint64_t ctr,
                          const uint64_t* d_ctr_base, int32_t* d_levels, float* d_logp, float* d_val, float* d_ent,
                          uint16_t* d_obs_bf16, float* d_logits, void* stream)
{
    MlpDims d;
    int rc = gov_dims(m, K, &d);
    if (rc != EJ_OK) return rc;
    if (!d_params || !d_work || !d_gov_obs || !d_scale || !d_levels || !d_logp || !d_val || !d_ent || E < 0)
        return EJ_EINVAL;
    if (!aligned16(d_params) || !aligned16(d_work)) return EJ_EINVAL;
    if (E == 0) return EJ_OK;
    hipStream_t st = (hipStream_t)stream;
    const unsigned blocks = (unsigned)((E + 63) / 64);
#define EJ_GOV_FWD(HH)                                                                                              \
    gov_forward_kernel<HH><<<blocks, 256, gov_forward_lds_bytes<HH>(), st>>>(d, K, d_params, d_work, d_gov_obs,    \
                                                                              d_scale, E, seed, ctr, d_ctr_base,    \
                                                                              d_levels, d_logp, d_val, d_ent,       \
                                                                              d_obs_bf16, d_logits)
    switch (m->H) {
    case 64: EJ_GOV_FWD(64); break;
    case 128: EJ_GOV_FWD(128); break;
    default: EJ_GOV_FWD(256); break;
    }
#undef EJ_GOV_FWD
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

int ej_sum_steps(const float* d_x, int32_t t_begin, int32_t t_end, int64_t E, float* d_out, void* stream)
{
    if (!d_x || !d_out || t_begin < 0 || t_end < t_begin || E < 0) return EJ_EINVAL;
    if (E == 0) return EJ_OK;
    int64_t blocks = (E + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    sum_steps_kernel<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(d_x, t_begin, t_end, E, d_out);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

int ej_gov_ppo_workspace_size(const ej_mlp_desc* m, int32_t K, int64_t rows, int64_t* bytes)
{
    MlpDims d;
    int rc = gov_dims(m, K, &d);
    if (rc != EJ_OK) return rc;
    if (!bytes || rows <= 0) return EJ_EINVAL;
    PpoWorkspace w;
    ppo_workspace(d, rows, &w, false);  // the government's rows kernel writes every operand as m-blocks
    *bytes = (int64_t)w.bytes;
    return EJ_OK;
}

int ej_gov_ppo_backward(const ej_mlp_desc* m, int32_t K, const float* d_params, const uint16_t* d_work,
                        const ej_ppo_batch* b, const ej_ppo_hparams* hp, void* d_workspace, int64_t workspace_bytes,
                        float* d_grads, float* d_loss, void* stream)
{
    MlpDims d;
    int rc = gov_dims(m, K, &d);
    if (rc != EJ_OK) return rc;
    if (!d_params || !d_work || !b || !hp || !d_workspace || !d_grads || !d_loss) return EJ_EINVAL;
    if (!b->obs || !b->act || !b->logp_old || !b->val_old || !b->adv || !b->ret) return EJ_EINVAL;
    if (!aligned16(d_params) || !aligned16(d_work) || !aligned16(b->obs) || !aligned16(d_workspace) ||
        !aligned16(d_grads))
        return EJ_EINVAL;
    if (b->M_total <= 0 || b->M_total > INT32_MAX || b->rows <= 0 || b->perm_a <= 0 || b->perm_c < 0 ||
        b->row_begin < 0 || b->row_begin + b->rows > INT32_MAX || b->row_offset < 0 ||
        (b->row_stride > 0 && b->row_offset >= b->row_stride))
        return EJ_EINVAL;
    PpoWorkspace w;
    ppo_workspace(d, b->rows, &w, false);
    if (workspace_bytes < (int64_t)w.bytes) return EJ_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    unsigned char* ws = (unsigned char*)d_workspace;
    const int64_t a = b->M_total == 1 ? 1 : b->perm_a % b->M_total;
    if (a == 0) return EJ_EINVAL;
    PpoBatchDev B{b->obs, nullptr, b->act, b->logp_old, b->val_old, b->adv, b->ret, b->M_total, a,
                  b->perm_c % b->M_total, b->row_begin, b->rows, UINT64_MAX / (uint64_t)b->M_total,
                  b->row_stride > 0 ? b->row_stride : 1, b->row_offset, nullptr, 0, 0, 0};
    PpoHp h{hp->clip, hp->vclip, hp->vf_coef, hp->ent_coef};
    double* advp = (double*)(ws + w.o_adv);
    float* stats = (float*)(ws + w.o_stats);
    launch_adv_stats(B, advp, stats, st);
    EJ_LAUNCH_CHECK();
    uint16_t* T[6] = {(uint16_t*)(ws + w.o_obs), (uint16_t*)(ws + w.o_h1), (uint16_t*)(ws + w.o_h2),
                      (uint16_t*)(ws + w.o_dy), (uint16_t*)(ws + w.o_dh2), (uint16_t*)(ws + w.o_dh1)};
    float* lparts = (float*)(ws + w.o_loss);
#define EJ_GOV_ROWS(HH)                                                                                              \
    gov_rows_kernel<HH><<<(unsigned)w.ntiles, 256, gov_rows_lds_bytes<HH>(), st>>>(d, K, d_params, d_work, B, h,     \
                                                                                    stats, T[0], T[1], T[2], T[3],   \
                                                                                    T[4], T[5], lparts)
    switch (m->H) {
    case 64: EJ_GOV_ROWS(64); break;
    case 128: EJ_GOV_ROWS(128); break;
    default: EJ_GOV_ROWS(256); break;
    }
#undef EJ_GOV_ROWS
    EJ_LAUNCH_CHECK();
    return ppo_weight_grads_and_loss(d, w, ws, b->rows, *hp, d_params, d_work, d_grads, d_loss, st);
}

int ej_ppo_backward(const ej_mlp_desc* m, const float* d_params, const uint16_t* d_work, const ej_ppo_batch* b,
                    const ej_ppo_hparams* hp, void* d_workspace, int64_t workspace_bytes, float* d_grads,
                    float* d_loss, void* stream)
{
    return ppo_backward_impl(m, d_params, d_work, b, hp, d_workspace, workspace_bytes, d_grads, d_loss, stream);
}

int ej_ppo_backward_static(const ej_mlp_desc* m, const float* d_params, const uint16_t* d_work,
                           const ej_ppo_batch* b, const ej_ppo_hparams* hp, float* d_grads, float* d_loss,
                           void* stream)
{
    if (!m || !b) return EJ_EINVAL;
    int64_t need = 0;
    int rc = ej_ppo_workspace_size(m, b->rows, &need);
    if (rc != EJ_OK) return rc;
    if (need > (int64_t)EJ_PPO_STATIC_SCRATCH_BYTES) return EJ_ESCRATCH;
    void* ws = nullptr;
    if ((rc = static_scratch_address(&ws)) != EJ_OK) return rc;
    return ppo_backward_impl(m, d_params, d_work, b, hp, ws, (int64_t)EJ_PPO_STATIC_SCRATCH_BYTES, d_grads, d_loss,
                             stream);
}

int ej_adam(float* d_params, const float* d_grads, float* d_m, float* d_v, int64_t n, int32_t step, float lr,
            float beta1, float beta2, float eps, void* stream)
{
    if (!d_params || !d_grads || !d_m || !d_v || n <= 0 || step <= 0) return EJ_EINVAL;
    const float c1 = (float)(1.0 - pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - pow((double)beta2, (double)step));
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    adam_kernel<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(d_params, d_grads, d_m, d_v, n, lr, beta1, beta2,
                                                                  eps, c1, c2);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

}  // extern "C"
