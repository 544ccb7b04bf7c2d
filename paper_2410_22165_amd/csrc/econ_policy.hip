// econ_policy.hip -- the shared population policy on gfx950: one fused
// kernel runs the three bf16 MFMA layers of a row tile, then a masked
// softmax over the action logits that never leaves the chip, and samples an
// action per row.  Also the weight-layout sync kernel and the MLP part of
// the C ABI.
//
// The paper trains all population agents with one shared actor-critic
// network (Sec. 4 "Experimental details"), masks invalid actions to zero
// probability (Sec. 3 "Action masking"), and uses PPO (Table 2).
//
// Sampling rule (exact for the categorical distribution): logits are
// processed in chunks of 128 actions.  Chunk c has weight S_c (sum of
// exp(z - m) over its allowed actions) and two uniforms (u1_c, u2_c).  A
// running total W accumulates S_c; the chunk becomes the candidate when
// u1_c * W < S_c (weighted reservoir: chunk c ends chosen with probability
// S_c / sum S).  Inside a candidate chunk the action is the first allowed
// action whose cumulative weight exceeds u2_c * S_c (inverse CDF), walking
// the chunk's actions in the fixed order c 128 + 16 t + j for j = 0..15
// (outer) and t = 0..7 (inner) -- the order of the MFMA accumulator layout.
#include "econ_mlp.h"

namespace econ {

// per-row sampling uniforms of the current chunk (LDS, RS_N floats per row)
enum { RS_U1 = 0, RS_U2, RS_N };

// LDS weight staging: only the logit layer (128 columns at a time) goes
// through LDS; double-buffered for 128-row tiles
template <int H, int RPW>
constexpr int policy_wbuf() { return (MlpTile<H, RPW>::DB ? 2 : 1) * 128 * WSTRIDE; }

// 64-row tiles with H <= 256 take 47 KB of LDS: three workgroups per CU
template <int H, int RPW_>
__global__ void __launch_bounds__(256, (RPW_ == 16 && H <= 256) ? 3 : 1)
policy_forward_kernel(const MlpDims d, const float* __restrict__ params, const uint16_t* __restrict__ work,
                      const uint16_t* __restrict__ obs, const uint32_t* __restrict__ mask, int64_t M, int W,
                      uint64_t seed, uint64_t ctr_arg, const uint64_t* __restrict__ ctr_base,
                      int32_t* __restrict__ act, float* __restrict__ logp, float* __restrict__ val,
                      float* __restrict__ ent, float* __restrict__ logits)
{
    const uint64_t ctr = ctr_arg + (ctr_base ? *ctr_base : 0ull);
    using T = MlpTile<H, RPW_>;
    constexpr int RT = T::RT, RPW = T::RPW, TILE = T::TILE, HS = T::HS;
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t* hbuf = (uint16_t*)smem;
    uint16_t* wbuf = hbuf + TILE * HS;
    uint32_t* smask = (uint32_t*)(wbuf + policy_wbuf<H, RPW_>());  // [TILE][W]
    float* rstate = (float*)(smask + TILE * W);      // [TILE][RS_N] uniforms of the current chunk
    float* sbias = rstate + TILE * RS_N;              // b1 [H], b2 [H], b3 [A1p] (zero padded)
    const int wave = threadIdx.x >> 6, l = lane_id();
    const int64_t row0 = (int64_t)blockIdx.x * TILE;
    const int arow0 = wave * RPW;

    // first chunk of the logit layer's weights in flight while the tile loads
    ECON_Q8_DECL;
    chunk_gload<128>(work + d.oW3f, ECON_Q8_ARGS);
    // observation tile -> activation buffer columns [0, K1p); mask rows -> LDS
    const int ppr = d.K1p / 8;
    for (int p = threadIdx.x; p < TILE * ppr; p += 256) {
        const int r = p / ppr, cc = p - r * ppr;
        const int64_t row = row0 + r;
        uint4 v = {0u, 0u, 0u, 0u};
        if (row < M && cc * 8 < d.Ds) v = *(const uint4*)(obs + row * d.Ds + cc * 8);
        *(uint4*)(hbuf + r * HS + cc * 8) = v;
    }
    for (int p = threadIdx.x; p < TILE * W; p += 256) {
        const int64_t row = row0 + p / W;
        smask[p] = row < M ? mask[row0 * W + p] : 0u;
    }
    for (int p = threadIdx.x; p < 2 * H + d.A1p; p += 256)
        sbias[p] = p < H ? params[d.ob1 + p] : p < 2 * H ? params[d.ob2 + p - H] : (p - 2 * H < d.A1 ? params[d.ob3 + p - 2 * H] : 0.f);

    // hidden layers split by columns: wave w computes every row of the tile
    // for columns [w H / 4, (w + 1) H / 4)
    {
        constexpr int TR = TILE / 16, CTW = H / 64;
        const int col0 = wave * (H / 4);
        f32x4 acc[TR][CTW];
        __syncthreads();  // observation tile in LDS
        dense_cs<TR, CTW, 2>(acc, hbuf, HS, work + d.oW1f, (int64_t)H * 32, col0);  // K1p = 64
        __syncthreads();  // every wave is done reading the observations
        epilogue_relu_cs<TR, CTW>(acc, sbias, hbuf, HS, col0);
        __syncthreads();
        dense_cs<TR, CTW, H / 32>(acc, hbuf, HS, work + d.oW2f, (int64_t)H * 32, col0);
        __syncthreads();
        epilogue_relu_cs<TR, CTW>(acc, sbias + H, hbuf, HS, col0);
        // the logit layer's first barrier publishes these rows
    }

    // The logits are consumed in the MFMA accumulator layout: lane l owns rows
    // 4 (l / 16) + i of each 16-row tile, so the 16 lanes of a DPP row share
    // one matrix row.  Every lane of a DPP row keeps the running state of its
    // rows in registers (the row reductions leave the result in all 16
    // lanes); the row loop has no branches, so the reduction chains of the
    // wave's rows interleave.
    const float NEG = -__builtin_huge_valf();
    float sM[RT][4], sS[RT][4], sT[RT][4], sW[RT][4], sV[RT][4], sZ[RT][4];
    int sA[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            sM[rt][i] = NEG;
            sS[rt][i] = sT[rt][i] = sW[rt][i] = sV[rt][i] = sZ[rt][i] = 0.f;
            sA[rt][i] = 0;
        }
    for (int c = 0; c < d.NC; ++c) {
        f32x4 acc3[RT][8];
        const uint16_t* next = c + 1 < d.NC ? work + d.oW3f + (int64_t)(c + 1) * 128 * 32 : nullptr;
        dense_layer_pf<RT, 128, 128, T::DB>(acc3, hbuf, HS, arow0, H, work + d.oW3f + (int64_t)c * 128 * 32,
                                            (int64_t)d.A1p * 32, wbuf, true, next, ECON_Q8_ARGS);
        // uniforms of chunk c: lane j < RPW draws for the wave's row j
        if (l < RPW) {
            u64x4 w = philox(seed, PURPOSE_SAMPLE, (uint64_t)(row0 + arow0 + l), ctr, (uint64_t)(c >> 1), 0);
            rstate[(arow0 + l) * RS_N + RS_U1] = unif24(word_of(w, 2 * (c & 1)));
            rstate[(arow0 + l) * RS_N + RS_U2] = unif24(word_of(w, 2 * (c & 1) + 1));
        }
        wave_lds_fence();
        float bcol[8];
#pragma unroll
        for (int ct = 0; ct < 8; ++ct) {
            const int col = c * 128 + ct * 16 + (l & 15);
            bcol[ct] = sbias[2 * H + col];
        }
        if (logits) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t row = row0 + arow0 + rt * 16 + 4 * (l >> 4) + i;
                    if (row < M)
#pragma unroll
                        for (int ct = 0; ct < 8; ++ct) {
                            const int col = c * 128 + ct * 16 + (l & 15);
                            if (col < d.A) logits[row * d.A + col] = acc3[rt][ct][i] + bcol[ct];
                        }
                }
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int rloc = arow0 + rt * 16 + 4 * (l >> 4) + i;  // row within the tile
                const float u1 = rstate[rloc * RS_N + RS_U1], u2 = rstate[rloc * RS_N + RS_U2];
                float z[8];
                bool ok[8];
                float zval = 0.f, zmax = NEG;
#pragma unroll
                for (int ct = 0; ct < 8; ++ct) {
                    const int col = c * 128 + ct * 16 + (l & 15);
                    const int wi = c * 4 + (ct >> 1);
                    const uint32_t mw = wi < W ? smask[rloc * W + wi] : 0u;
                    z[ct] = acc3[rt][ct][i] + bcol[ct];
                    ok[ct] = col < d.A && ((mw >> (col & 31)) & 1u);
                    zval = col == d.A ? z[ct] : zval;
                    zmax = ok[ct] ? fmaxf(zmax, z[ct]) : zmax;
                }
                const float zv = row16_sum(zval);  // the value head sits right after the logits
                const float mc = row16_max(zmax);
                const bool any = mc != NEG;
                // Walk order inside the chunk: lane-major (lane j's eight actions
                // j, 16 + j, ..., 112 + j, then lane j + 1's): a lane-local prefix
                // plus one 16-lane scan of the lane totals.
                float e[8], P[8], own = 0.f, tl = 0.f;
#pragma unroll
                for (int ct = 0; ct < 8; ++ct) {
                    e[ct] = ok[ct] ? __expf(z[ct] - mc) : 0.f;
                    tl += ok[ct] ? e[ct] * (z[ct] - mc) : 0.f;
                    own += e[ct];
                    P[ct] = own;
                }
                const float incl = row16_scan(own);
                const float before = incl - own;
                const float Sc = row16_sum(own);
#pragma unroll
                for (int ct = 0; ct < 8; ++ct) P[ct] += before;
                const float Tc = row16_sum(tl);
                const float m = sM[rt][i], S0 = sS[rt][i], T0 = sT[rt][i], W0 = sW[rt][i];
                const float mn = any ? fmaxf(m, mc) : m;
                const float fo = (m == NEG) ? 0.f : __expf(m - mn), fc = any ? __expf(mc - mn) : 0.f;
                const float Tn = (m == NEG ? 0.f : fo * (T0 + (m - mn) * S0)) + (any ? fc * (Tc + (mc - mn) * Sc) : 0.f);
                const float Sn = S0 * fo + Sc * fc;
                const float Wn = W0 * fo + Sc * fc;
                const bool take = any && u1 * Wn < Sc * fc;
                // first allowed action whose cumulative weight exceeds u2 * Sc
                const float target = u2 * Sc;
                // position in the walk: (lane, ct) -> 8 lane + ct
                int key = 1 << 20, last = -1;
#pragma unroll
                for (int ct = 7; ct >= 0; --ct) {
                    key = (ok[ct] && P[ct] > target) ? 8 * (l & 15) + ct : key;
                    last = (ok[ct] && last < 0) ? 8 * (l & 15) + ct : last;
                }
                key = row16_min_i(key);
                const int top = row16_max_i(last);
                key = key == (1 << 20) ? top : key;  // rounding put the target at the top
                float zk = 0.f;
#pragma unroll
                for (int ct = 0; ct < 8; ++ct) zk = 8 * (l & 15) + ct == key ? z[ct] : zk;
                zk = row16_sum(zk);
                key = (key & 7) * 16 + (key >> 3);  // walk position -> column in the chunk
                sM[rt][i] = mn;
                sS[rt][i] = Sn;
                sT[rt][i] = Tn;
                sW[rt][i] = Wn;
                sV[rt][i] += zv;
                sA[rt][i] = take ? c * 128 + key : sA[rt][i];
                sZ[rt][i] = take ? zk : sZ[rt][i];
            }
    }
    // outputs: sampled action, its log-probability, entropy, value (lane 0 of each DPP row)
    if ((l & 15) == 0) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t row = row0 + arow0 + rt * 16 + 4 * (l >> 4) + i;
                if (row >= M) continue;
                const float S = sS[rt][i];
                int a = sA[rt][i];
                float lp = 0.f, h = 0.f;
                if (S > 0.f) {
                    const float lS = __logf(S);
                    lp = sZ[rt][i] - sM[rt][i] - lS;
                    h = lS - sT[rt][i] / S;
                } else {
                    a = 0;
                }
                act[row] = a;
                logp[row] = lp;
                ent[row] = h;
                val[row] = sV[rt][i];
            }
    }
}

// fp32 parameters -> bf16 K-chunk layouts (forward W1f, W2f, W3f; backward W3b, W2b)
__global__ void mlp_sync_kernel(const MlpDims d, const float* __restrict__ p, uint16_t* __restrict__ w)
{
    const int64_t n = d.n_work;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.f;
        int64_t j = idx;
        if (j < d.oW2f) {  // W1f [K1p/32][H][32]: (k, n) = W1[k][n]
            const int kk = (int)(j % 32), nn = (int)((j / 32) % d.H), kt = (int)(j / (32 * (int64_t)d.H));
            const int k = kt * 32 + kk;
            if (k < d.D) v = p[d.oW1 + (int64_t)k * d.H + nn];
        } else if (j < d.oW3f) {  // W2f [H/32][H][32]
            j -= d.oW2f;
            const int kk = (int)(j % 32), nn = (int)((j / 32) % d.H), kt = (int)(j / (32 * (int64_t)d.H));
            v = p[d.oW2 + (int64_t)(kt * 32 + kk) * d.H + nn];
        } else if (j < d.oW3b) {  // W3f [H/32][A1p][32]: (k, n) = W3[k][n]
            j -= d.oW3f;
            const int kk = (int)(j % 32), nn = (int)((j / 32) % d.A1p), kt = (int)(j / (32 * (int64_t)d.A1p));
            if (nn < d.A1) v = p[d.oW3 + (int64_t)(kt * 32 + kk) * d.A1 + nn];
        } else if (j < d.oW2b) {  // W3b [A1p/32][H][32]: (k = a, n = j) = W3[j][a]
            j -= d.oW3b;
            const int kk = (int)(j % 32), nn = (int)((j / 32) % d.H), kt = (int)(j / (32 * (int64_t)d.H));
            const int a = kt * 32 + kk;
            if (a < d.A1) v = p[d.oW3 + (int64_t)nn * d.A1 + a];
        } else {  // W2b [H/32][H][32]: (k, n = j) = W2[j][k]
            j -= d.oW2b;
            const int kk = (int)(j % 32), nn = (int)((j / 32) % d.H), kt = (int)(j / (32 * (int64_t)d.H));
            v = p[d.oW2 + (int64_t)nn * d.H + kt * 32 + kk];
        }
        w[idx] = f32_to_bf16(v);
    }
}

template <int H, int RPW>
size_t policy_lds_bytes(int W, int A1p)
{
    using T = MlpTile<H, RPW>;
    return (size_t)T::TILE * T::HS * 2 + (size_t)policy_wbuf<H, RPW>() * 2 + (size_t)T::TILE * W * 4 +
           (size_t)T::TILE * RS_N * 4 + (size_t)(2 * H + A1p) * 4;
}

template <int H, int RPW>
int launch_policy_forward(const MlpDims& d, const float* params, const uint16_t* work, const uint16_t* obs,
                          const uint32_t* mask, int64_t M, int W, uint64_t seed, uint64_t ctr, const uint64_t* ctr_base,
                          int32_t* act, float* logp, float* val, float* ent, float* logits, hipStream_t st)
{
    using T = MlpTile<H, RPW>;
    const int64_t blocks = (M + T::TILE - 1) / T::TILE;
    const size_t lds = policy_lds_bytes<H, RPW>(W, d.A1p);
    policy_forward_kernel<H, RPW><<<(unsigned)blocks, 256, lds, st>>>(d, params, work, obs, mask, M, W, seed, ctr, ctr_base,
                                                                  act, logp, val, ent, logits);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

}  // namespace econ

using namespace econ;

static int desc_dims(const ej_mlp_desc* m, MlpDims* d)
{
    if (!m) return EJ_EINVAL;
    if (m->tile_rows != 0 && m->tile_rows != 64 && !(m->tile_rows == 128 && m->H <= 256)) return EJ_EUNSUPPORTED;
    return mlp_dims(m->D, m->D_stride, m->H, m->A, d);
}

extern "C" {

int ej_mlp_layout(const ej_mlp_desc* m, ej_mlp_layout_t* out)
{
    MlpDims d;
    int rc = desc_dims(m, &d);
    if (rc != EJ_OK) return rc;
    if (!out) return EJ_EINVAL;
    out->n_params = d.n_params;
    out->n_work = d.n_work;
    out->W1 = d.oW1;
    out->b1 = d.ob1;
    out->W2 = d.oW2;
    out->b2 = d.ob2;
    out->W3 = d.oW3;
    out->b3 = d.ob3;
    return EJ_OK;
}

int ej_mlp_sync_weights(const ej_mlp_desc* m, const float* d_params, uint16_t* d_work, void* stream)
{
    MlpDims d;
    int rc = desc_dims(m, &d);
    if (rc != EJ_OK) return rc;
    if (!d_params || !d_work) return EJ_EINVAL;
    int64_t blocks = (d.n_work + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    mlp_sync_kernel<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(d, d_params, d_work);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

__global__ void counter_add_kernel(uint64_t* c, uint64_t inc)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *c += inc;
}

int ej_counter_add(uint64_t* d_counter, uint64_t inc, void* stream)
{
    if (!d_counter) return EJ_EINVAL;
    counter_add_kernel<<<1, 64, 0, (hipStream_t)stream>>>(d_counter, inc);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

int ej_policy_forward(const ej_mlp_desc* m, const float* d_params, const uint16_t* d_work, const uint16_t* d_obs,
                      const uint32_t* d_mask, int64_t M, uint64_t seed, uint64_t ctr, const uint64_t* d_ctr_base,
                      int32_t* d_act, float* d_logp, float* d_val, float* d_ent, float* d_logits, void* stream)
{
    MlpDims d;
    int rc = desc_dims(m, &d);
    if (rc != EJ_OK) return rc;
    if (M < 0 || !d_params || !d_work || !d_obs || !d_mask || !d_act || !d_logp || !d_val || !d_ent) return EJ_EINVAL;
    if (M == 0) return EJ_OK;
    const int W = (m->A + 31) / 32;
    hipStream_t st = (hipStream_t)stream;
    const bool small = m->tile_rows == 64 || m->H == 512;
#define EJ_POLICY(HH, RR) \
    launch_policy_forward<HH, RR>(d, d_params, d_work, d_obs, d_mask, M, W, seed, ctr, d_ctr_base, d_act, d_logp, d_val, \
                                  d_ent, d_logits, st)
    switch (m->H) {
    case 64: return small ? EJ_POLICY(64, 16) : EJ_POLICY(64, 32);
    case 128: return small ? EJ_POLICY(128, 16) : EJ_POLICY(128, 32);
    case 256: return small ? EJ_POLICY(256, 16) : EJ_POLICY(256, 32);
    default: return EJ_POLICY(512, 16);
    }
#undef EJ_POLICY
}

}  // extern "C"
