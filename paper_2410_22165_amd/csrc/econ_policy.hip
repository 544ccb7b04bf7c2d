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
// action whose cumulative weight exceeds u2_c * S_c (inverse CDF).
#include "econ_mlp.h"

namespace econ {

// per-row running state of the online softmax (LDS, one slot of 8 floats per row)
enum { RS_M = 0, RS_S, RS_T, RS_W, RS_ACT, RS_Z, RS_VAL, RS_N };

// Consume one 128-wide logit chunk of 16 rows that the wave staged in
// `scr` [16][128] (logit + bias; columns >= A1 hold junk and are ignored).
__device__ inline void softmax_chunk_rows(const MlpDims& d, const float* scr, float* rstate, int c, int64_t grow0,
                                          int64_t M, const uint32_t* __restrict__ mask, int W, float u1_lane,
                                          float u2_lane)
{
    const int l = lane_id();
    const float NEG = -__builtin_huge_valf();
    for (int r = 0; r < 16; ++r) {
        const int64_t row = grow0 + r;
        if (row >= M) break;
        const float2 z = *(const float2*)(scr + r * 128 + 2 * l);
        const int a0 = c * 128 + 2 * l, a1 = a0 + 1;
        const uint32_t mw = (a0 < d.A) ? mask[row * W + (a0 >> 5)] : 0u;
        const bool ok0 = a0 < d.A && ((mw >> (a0 & 31)) & 1u);
        const bool ok1 = a1 < d.A && ((mw >> (a1 & 31)) & 1u);
        float* st = rstate + r * RS_N;
        if (a0 == d.A) st[RS_VAL] = z.x;  // the value head sits right after the logits
        if (a1 == d.A) st[RS_VAL] = z.y;
        float mc = wave_max(fmaxf(ok0 ? z.x : NEG, ok1 ? z.y : NEG));
        if (mc == NEG) continue;  // nothing allowed in this chunk
        const float e0 = ok0 ? __expf(z.x - mc) : 0.f;
        const float e1 = ok1 ? __expf(z.y - mc) : 0.f;
        const float incl = wave_inclusive_scan(e0 + e1);
        const float Sc = __shfl(incl, 63, 64);
        const float Tc = wave_sum(e0 * (z.x - mc) + e1 * (z.y - mc));
        const float m = st[RS_M], S = st[RS_S], T = st[RS_T], Wr = st[RS_W];
        const float mn = fmaxf(m, mc);
        const float fo = (m == NEG) ? 0.f : __expf(m - mn), fc = __expf(mc - mn);
        const float Sn = S * fo + Sc * fc;
        const float Tn = (m == NEG ? 0.f : fo * (T + (m - mn) * S)) + fc * (Tc + (mc - mn) * Sc);
        const float Wn = Wr * fo + Sc * fc;
        const float u1 = __shfl(u1_lane, r, 64), u2 = __shfl(u2_lane, r, 64);
        bool take = u1 * Wn < Sc * fc;
        int pick = -1;
        float zpick = 0.f;
        if (take) {
            const float target = u2 * Sc;
            const uint64_t hit = __ballot(incl > target);
            int ln;
            if (hit) {
                ln = __builtin_ctzll(hit);
            } else {  // rounding put the target at the very top: the last allowed action
                ln = 63 - __builtin_clzll(__ballot(ok0 || ok1));
            }
            const float ex = __shfl(incl - (e0 + e1), ln, 64);
            const float f0 = __shfl(e0, ln, 64), f1 = __shfl(e1, ln, 64);
            const float z0 = __shfl(z.x, ln, 64), z1 = __shfl(z.y, ln, 64);
            const bool first = (hit && ex + f0 > target) || (!hit && f1 == 0.f);
            pick = c * 128 + 2 * ln + (first ? 0 : 1);
            zpick = first ? z0 : z1;
        }
        if (l == 0) {
            st[RS_M] = mn;
            st[RS_S] = Sn;
            st[RS_T] = Tn;
            st[RS_W] = Wn;
            if (take) {
                st[RS_ACT] = __int_as_float(pick);
                st[RS_Z] = zpick;
            }
        }
        wave_lds_fence();
    }
}

template <int H>
__global__ void __launch_bounds__(256)
policy_forward_kernel(const MlpDims d, const float* __restrict__ params, const uint16_t* __restrict__ work,
                      const uint16_t* __restrict__ obs, const uint32_t* __restrict__ mask, int64_t M, int W,
                      uint64_t seed, uint64_t ctr, int32_t* __restrict__ act, float* __restrict__ logp,
                      float* __restrict__ val, float* __restrict__ ent, float* __restrict__ logits)
{
    using T = MlpTile<H>;
    constexpr int RT = T::RT, RPW = T::RPW, TILE = T::TILE, HS = T::HS;
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t* hbuf = (uint16_t*)smem;
    uint16_t* wbuf = hbuf + TILE * HS;
    float* scratch = (float*)(wbuf + T::WREG);  // [4 waves][16][128]
    float* rstate = scratch + 4 * 16 * 128;       // [4 waves][RPW][RS_N]
    const int wave = threadIdx.x >> 6, l = lane_id();
    const int64_t row0 = (int64_t)blockIdx.x * TILE;
    const int arow0 = wave * RPW;
    float* scr = scratch + wave * 16 * 128;
    float* rs = rstate + wave * RPW * RS_N;

    // observation tile -> activation buffer columns [0, K1p)
    const int ppr = d.K1p / 8;
    for (int p = threadIdx.x; p < TILE * ppr; p += 256) {
        const int r = p / ppr, cc = p - r * ppr;
        const int64_t row = row0 + r;
        uint4 v = {0u, 0u, 0u, 0u};
        if (row < M && cc * 8 < d.Ds) v = *(const uint4*)(obs + row * d.Ds + cc * 8);
        *(uint4*)(hbuf + r * HS + cc * 8) = v;
    }
    for (int j = l; j < RPW * RS_N; j += 64) {
        const int k = j % RS_N;
        rs[j] = (k == RS_M) ? -__builtin_huge_valf() : (k == RS_ACT ? __int_as_float(0) : 0.f);
    }

    f32x4 acc[RT][H / 16];
    dense_layer<RT, H>(acc, hbuf, HS, arow0, d.K1p, work + d.oW1f, (int64_t)H * 32, wbuf);
    epilogue_relu<RT, H / 16>(acc, params + d.ob1, hbuf, HS, arow0);
    dense_layer<RT, H>(acc, hbuf, HS, arow0, H, work + d.oW2f, (int64_t)H * 32, wbuf);
    epilogue_relu<RT, H / 16>(acc, params + d.ob2, hbuf, HS, arow0);

    for (int c = 0; c < d.NC; ++c) {
        f32x4 acc3[RT][8];
        dense_layer<RT, 128>(acc3, hbuf, HS, arow0, H, work + d.oW3f + (int64_t)c * 128 * 32, (int64_t)d.A1p * 32,
                             wbuf);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int64_t grow0 = row0 + arow0 + rt * 16;
            // per-row uniforms: lane r < 16 draws for row grow0 + r
            float u1 = 0.f, u2 = 0.f;
            if (l < 16) {
                u64x4 w = philox(seed, PURPOSE_SAMPLE, (uint64_t)(grow0 + l), ctr, (uint64_t)(c >> 1), 0);
                u1 = unif24(word_of(w, 2 * (c & 1)));
                u2 = unif24(word_of(w, 2 * (c & 1) + 1));
            }
#pragma unroll
            for (int ct = 0; ct < 8; ++ct) {
                const int col = c * 128 + ct * 16 + (l & 15);
                const float b = col < d.A1 ? params[d.ob3 + col] : 0.f;
#pragma unroll
                for (int i = 0; i < 4; ++i) scr[(4 * (l >> 4) + i) * 128 + ct * 16 + (l & 15)] = acc3[rt][ct][i] + b;
            }
            wave_lds_fence();
            if (logits) {
                for (int r = 0; r < 16; ++r) {
                    const int64_t row = grow0 + r;
                    if (row >= M) break;
                    for (int j = l; j < 128; j += 64) {
                        const int a = c * 128 + j;
                        if (a < d.A) logits[row * d.A + a] = scr[r * 128 + j];
                    }
                }
            }
            softmax_chunk_rows(d, scr, rs + rt * 16 * RS_N, c, grow0, M, mask, W, u1, u2);
            wave_lds_fence();
        }
    }
    // outputs: log-probability of the sampled action, entropy, value
    for (int r = l; r < RPW; r += 64) {
        const int64_t row = row0 + arow0 + r;
        if (row >= M) continue;
        const float* st = rs + r * RS_N;
        const float S = st[RS_S];
        int a = __float_as_int(st[RS_ACT]);
        float lp = 0.f, h = 0.f;
        if (S > 0.f) {
            const float lS = __logf(S);
            lp = st[RS_Z] - st[RS_M] - lS;
            h = lS - st[RS_T] / S;
        } else {
            a = 0;
        }
        act[row] = a;
        logp[row] = lp;
        ent[row] = h;
        val[row] = st[RS_VAL];
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

template <int H>
size_t policy_lds_bytes()
{
    using T = MlpTile<H>;
    return (size_t)T::TILE * T::HS * 2 + (size_t)T::WREG * 2 + 4 * 16 * 128 * 4 + 4 * (size_t)T::RPW * RS_N * 4;
}

template <int H>
int launch_policy_forward(const MlpDims& d, const float* params, const uint16_t* work, const uint16_t* obs,
                          const uint32_t* mask, int64_t M, int W, uint64_t seed, uint64_t ctr, int32_t* act,
                          float* logp, float* val, float* ent, float* logits, hipStream_t st)
{
    using T = MlpTile<H>;
    const int64_t blocks = (M + T::TILE - 1) / T::TILE;
    const size_t lds = policy_lds_bytes<H>();
    policy_forward_kernel<H><<<(unsigned)blocks, 256, lds, st>>>(d, params, work, obs, mask, M, W, seed, ctr, act,
                                                                  logp, val, ent, logits);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

}  // namespace econ

using namespace econ;

static int desc_dims(const ej_mlp_desc* m, MlpDims* d)
{
    if (!m) return EJ_EINVAL;
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

int ej_policy_forward(const ej_mlp_desc* m, const float* d_params, const uint16_t* d_work, const uint16_t* d_obs,
                      const uint32_t* d_mask, int64_t M, uint64_t seed, uint64_t ctr, int32_t* d_act, float* d_logp,
                      float* d_val, float* d_ent, float* d_logits, void* stream)
{
    MlpDims d;
    int rc = desc_dims(m, &d);
    if (rc != EJ_OK) return rc;
    if (M < 0 || !d_params || !d_work || !d_obs || !d_mask || !d_act || !d_logp || !d_val || !d_ent) return EJ_EINVAL;
    if (M == 0) return EJ_OK;
    const int W = (m->A + 31) / 32;
    hipStream_t st = (hipStream_t)stream;
    switch (m->H) {
    case 64: return launch_policy_forward<64>(d, d_params, d_work, d_obs, d_mask, M, W, seed, ctr, d_act, d_logp, d_val, d_ent, d_logits, st);
    case 128: return launch_policy_forward<128>(d, d_params, d_work, d_obs, d_mask, M, W, seed, ctr, d_act, d_logp, d_val, d_ent, d_logits, st);
    case 256: return launch_policy_forward<256>(d, d_params, d_work, d_obs, d_mask, M, W, seed, ctr, d_act, d_logp, d_val, d_ent, d_logits, st);
    default: return launch_policy_forward<512>(d, d_params, d_work, d_obs, d_mask, M, W, seed, ctr, d_act, d_logp, d_val, d_ent, d_logits, st);
    }
}

}  // extern "C"
