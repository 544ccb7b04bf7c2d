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
// action, in action order, whose cumulative weight exceeds u2_c * S_c
// (inverse CDF).
#include "econ_mlp.h"

namespace econ {

// Weight sets and row layout of a grouped launch: group g reads parameters at
// g * pstride and bf16 work at g * wstride, and owns rows q * rstride + g
struct PolicyGroups {
    int64_t rstride, pstride, wstride;
};

// stacked weight sets start 16 bytes apart at least: n rounded up to a multiple of `m`
__host__ inline int64_t group_stride(int64_t n, int64_t m) { return (n + m - 1) / m * m; }

// LDS bytes: activations (aliased by the logit chunk when there is only one
// chunk), mask words, uniforms, biases
template <int H, int RPW>
size_t policy_lds_bytes(int W, int A1p)
{
    using T = MlpTile<H, RPW>;
    const size_t hb = (size_t)T::TILE * T::HS * 2, zb = (size_t)T::TILE * ZS * 4;
    const size_t region = A1p == 128 ? (hb > zb ? hb : zb) : hb + zb;
    return region + (size_t)T::TILE * W * 4 + (size_t)T::TILE * 4 * 4 + (size_t)A1p * 4;
}

// The workgroup's threads talk through LDS only (its barriers order LDS).
// 64-row tiles with H <= 256 take 38.5 KB of LDS and 128 VGPRs: four workgroups per CU.
// K1: first-layer input columns (64, or 128 for wide observation rows).
template <int H, int RPW_, int K1>
__global__ void __launch_bounds__(256, (RPW_ == 16 && H <= 256) ? 4 : 1)
policy_forward_kernel(const MlpDims d, const float* __restrict__ params_all, const uint16_t* __restrict__ work_all,
                      const uint16_t* __restrict__ obs, const uint32_t* __restrict__ mask, int64_t M, int64_t row_base,
                      int W, uint64_t seed, uint64_t ctr_arg, const uint64_t* __restrict__ ctr_base,
                      int32_t* __restrict__ act, float* __restrict__ logp, float* __restrict__ val,
                      float* __restrict__ ent, float* __restrict__ logits, const PolicyGroups grp)
{
    const uint64_t ctr = ctr_arg + (ctr_base ? *ctr_base : 0ull);
    // group g = blockIdx.y owns weight set g and the rows q * rstride + g of
    // its M local rows q (one group with stride 1: the shared network)
    const int64_t g = blockIdx.y;
    const float* __restrict__ params = params_all + g * grp.pstride;
    const uint16_t* __restrict__ work = work_all + g * grp.wstride;
    auto grow = [&](int64_t q) { return q * grp.rstride + g; };
    using T = MlpTile<H, RPW_>;
    constexpr int RPW = T::RPW, TILE = T::TILE, HS = T::HS, TR = TILE / 16;
    extern __shared__ __align__(16) unsigned char smem[];
    const size_t hb = (size_t)TILE * HS * 2, zb = (size_t)TILE * ZS * 4;
    const size_t region = d.A1p == 128 ? (hb > zb ? hb : zb) : hb + zb;
    uint16_t* hbuf = (uint16_t*)smem;
    float* zbuf = (float*)(smem + (d.A1p == 128 ? 0 : hb));  // logit chunk [TILE][ZS]
    uint32_t* smask = (uint32_t*)(smem + region);            // [TILE][W]
    float* urow = (float*)(smask + TILE * W);                 // [TILE][4] uniforms of the current chunk pair
    float* sb3 = urow + TILE * 4;                             // b3 [A1p] (zero padded)
    const int wave = threadIdx.x >> 6, l = lane_id();
    const int64_t row0 = (int64_t)blockIdx.x * TILE;

    // One Philox call gives the uniforms (u1, u2) of two chunks for one row.
    // A single wave draws for the whole tile (lane j takes rows j, j + 64):
    // the generator is ~450 vector instructions, whatever the number of
    // active lanes.  The drawing wave rotates with the workgroup, so every
    // SIMD gets its share.  The first pair is drawn here, under the latency
    // of the tile loads; LDS barriers separate the draws from their readers.
    const int draw_wave = (int)(blockIdx.x & 3);
    auto draw_uniforms = [&](int c) {
        if (wave == draw_wave) {
            for (int rl = l; rl < TILE; rl += 64) {
                u64x4 w = philox(seed, PURPOSE_SAMPLE, (uint64_t)(row_base + grow(row0 + rl)), ctr, (uint64_t)(c >> 1), 0);
#pragma unroll
                for (int k = 0; k < 4; ++k) urow[rl * 4 + k] = unif24(word_of(w, k));
            }
        }
    };
    draw_uniforms(0);
    // observation tile -> activation buffer columns [0, K1p), 64 columns at a
    // time (TILE x 8 pieces of 16 bytes: every load of a half is issued before
    // its first store); mask rows -> LDS
    constexpr int NPC = TILE * (K1P / 8) / 256;
    for (int h = 0; h < K1 / K1P; ++h) {
        uint4 pv[NPC];
#pragma unroll
        for (int i = 0; i < NPC; ++i) {
            const int p = threadIdx.x + 256 * i, r = p >> 3, cc = h * 8 + (p & 7);
            const int64_t row = row0 + r;
            pv[i] = (row < M && cc * 8 < d.Ds) ? *(const uint4*)(obs + grow(row) * d.Ds + cc * 8)
                                                : uint4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int i = 0; i < NPC; ++i) {
            const int p = threadIdx.x + 256 * i;
            *(uint4*)(hbuf + (p >> 3) * HS + (h * 8 + (p & 7)) * 8) = pv[i];
        }
    }
    for (int p = threadIdx.x; p < TILE * W; p += 256) {
        const int r = p / W;
        const int64_t row = row0 + r;
        smask[p] = row < M ? mask[grow(row) * W + (p - r * W)] : 0u;
    }
    for (int p = threadIdx.x; p < d.A1p; p += 256) sb3[p] = p < d.A1 ? params[d.ob3 + p] : 0.f;

    // All three layers are split by columns: wave w computes every row of the
    // tile for a quarter of the output columns, with weight fragments loaded
    // from L2 straight into registers.  The accumulators are transposed
    // (TRANS): a lane holds 4 adjacent columns of one row, stored at once,
    // and start at the bias.
    {
        constexpr int CTW = H / 64;
        const int col0 = wave * (H / 4);
        f32x4 acc[TR][CTW];
        bias_init_t<TR, CTW>(acc, params + d.ob1, col0);
        lds_barrier();  // observation tile in LDS
        dense_cs<TR, CTW, K1 / 32, false, 2, false, true>(acc, hbuf, HS, work + d.oW1f, (int64_t)H * 32, col0);
        lds_barrier();  // every wave is done reading the observations
        relu_store_t<TR, CTW>(acc, hbuf, HS, col0);
        bias_init_t<TR, CTW>(acc, params + d.ob2, col0);
        lds_barrier();
        dense_cs<TR, CTW, H / 32, false, 2, false, true>(acc, hbuf, HS, work + d.oW2f, (int64_t)H * 32, col0);
        lds_barrier();
        relu_store_t<TR, CTW>(acc, hbuf, HS, col0);
        lds_barrier();
    }

    // Logits, 128 actions (one chunk) at a time: wave w computes columns
    // [32 w, 32 w + 32) of the chunk for every row and leaves them in LDS
    // (fp32).  Then four lanes share a row (q = lane % 4 takes the chunk's
    // columns 32 q .. 32 q + 31 in order), so every row reduction is a
    // two-step quad reduction.  Each lane keeps its rows' running state.
    const float NEG = -__builtin_huge_valf();
    constexpr int SR = RPW / 16;  // softmax rows per lane
    const int q = l & 3;
    float sM[SR], sS[SR], sT[SR], sW[SR], sV[SR], sZ[SR];
    int sA[SR];
#pragma unroll
    for (int k = 0; k < SR; ++k) {
        sM[k] = NEG;
        sS[k] = sT[k] = sW[k] = sV[k] = sZ[k] = 0.f;
        sA[k] = 0;
    }
    for (int c = 0; c < d.NC; ++c) {
        {
            f32x4 acc3[TR][2];
            dense_cs<TR, 2, H / 32, true, 2, false, true>(acc3, hbuf, HS, work + d.oW3f + (int64_t)c * 128 * 32,
                                                          (int64_t)d.A1p * 32, 32 * wave);
            if (c > 0 && (c & 1) == 0) draw_uniforms(c);  // the next pair of chunks
            if (d.A1p == 128) lds_barrier();  // the logit chunk overwrites the activations
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
                const int cc = 32 * wave + ct * 16 + 4 * (l >> 4);  // 4 adjacent columns of row l % 16
                const float4 b = *(const float4*)(sb3 + c * 128 + cc);
#pragma unroll
                for (int rt = 0; rt < TR; ++rt)
                    *(float4*)(zbuf + (rt * 16 + (l & 15)) * ZS + zcol(l & 15, cc)) =
                        float4{acc3[rt][ct][0] + b.x, acc3[rt][ct][1] + b.y, acc3[rt][ct][2] + b.z,
                               acc3[rt][ct][3] + b.w};
            }
        }
        lds_barrier();  // the chunk's logits and uniforms are in LDS
        const int colq = c * 128 + 32 * q;  // first action of this lane's quarter
#pragma unroll
        for (int k = 0; k < SR; ++k) {
            const int rloc = wave * RPW + k * 16 + (l >> 2);
            const float* zrow = zbuf + rloc * ZS;
            float z[32];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float4 v = *(const float4*)(zrow + q * ZQ + 4 * (j ^ zsw(rloc)));
                z[4 * j] = v.x;
                z[4 * j + 1] = v.y;
                z[4 * j + 2] = v.z;
                z[4 * j + 3] = v.w;
            }
            if (logits && row0 + rloc < M) {
#pragma unroll
                for (int j = 0; j < 32; ++j)
                    if (colq + j < d.A) logits[grow(row0 + rloc) * d.A + colq + j] = z[j];
            }
            // allowed actions of this lane's quarter (bits past the last action cleared)
            const int wi = c * 4 + q, nact = d.A - colq;
            uint32_t mw = wi < W ? smask[rloc * W + wi] : 0u;
            mw = nact >= 32 ? mw : (nact <= 0 ? 0u : mw & ((1u << nact) - 1u));
            const float u1 = urow[rloc * 4 + 2 * (c & 1)], u2 = urow[rloc * 4 + 2 * (c & 1) + 1];
            // masked logits -> MASKED, a finite stand-in for -inf (the
            // network's logits are finite): exp(MASKED - ms) is exactly 0, and
            // so is its product with MASKED - ms, so the weight and entropy
            // sums below need no select.  Bit j of the mask word, spread to a
            // whole word, picks the logit or MASKED (extract + bit insert).
            constexpr float MASKED = -1e30f;
            float zmax = MASKED;
#pragma unroll
            for (int j = 0; j < 32; ++j) {
                const int keep = __builtin_amdgcn_sbfe((int)mw, j, 1);  // opaque to the select folding
                z[j] = __int_as_float((__float_as_int(z[j]) & keep) | (__float_as_int(MASKED) & ~keep));
                zmax = fmaxf(zmax, z[j]);
            }
            const float mc = quad_max(zmax);
            const bool any = mc > MASKED;
            const float ms = any ? mc : 0.f;
            // weights exp(z - mc), kept in z; their sum and sum of w (z - mc)
            float own = 0.f, tl = 0.f;
#pragma unroll
            for (int j = 0; j < 32; ++j) {
                const float dz = z[j] - ms;
                const float e = __expf(dz);
                tl = __builtin_fmaf(e, dz, tl);
                own += e;
                z[j] = e;
            }
            const float before = quad_scan(own, q) - own;
            const float Sc = quad_sum(own);
            const float Tc = quad_sum(tl);
            const float m = sM[k], S0 = sS[k], T0 = sT[k], W0 = sW[k];
            const float mn = any ? fmaxf(m, mc) : m;
            const float fo = (m == NEG) ? 0.f : __expf(m - mn), fc = any ? __expf(mc - mn) : 0.f;
            const float Tn = (m == NEG ? 0.f : fo * (T0 + (m - mn) * S0)) + (any ? fc * (Tc + (mc - mn) * Sc) : 0.f);
            const float Sn = S0 * fo + Sc * fc;
            const float Wn = W0 * fo + Sc * fc;
            const bool take = any && u1 * Wn < Sc * fc;
            // inverse CDF inside the chunk (action order): the first allowed
            // action whose cumulative weight exceeds u2 * Sc.  The running sum
            // never decreases, so the actions where it exceeds the target form
            // a suffix of the quarter; its first element is allowed (its weight
            // is positive) unless the suffix is the whole quarter, where the
            // first allowed action is taken.
            const float target = u2 * Sc;
            float cum = before;
            int below = 0;  // actions of the quarter where the running sum is still <= target
#pragma unroll
            for (int j = 0; j < 32; ++j) {
                cum += z[j];
                below += cum <= target ? 1 : 0;
            }
            constexpr int NONE = 1 << 20;
            int key = below == 32 ? NONE : below > 0 ? 32 * q + below : mw ? 32 * q + __builtin_ctz(mw) : NONE;
            key = quad_min_i(key);
            const int top = quad_max_i(mw ? 32 * q + 31 - __builtin_clz(mw) : -1);
            key = key == NONE ? top : key;  // rounding put the target at the top
            const float zk = zrow[zcol(rloc, key < 0 ? 0 : key)];  // the chosen action's logit
            sM[k] = mn;
            sS[k] = Sn;
            sT[k] = Tn;
            sW[k] = Wn;
            if (c == d.NC - 1) sV[k] = zrow[zcol(rloc, d.A - c * 128)];  // the value head sits right after the logits
            sA[k] = take ? c * 128 + key : sA[k];
            sZ[k] = take ? zk : sZ[k];
        }
        if (c + 1 < d.NC) lds_barrier();  // before the next chunk overwrites the logits and uniforms
    }
    // outputs: sampled action, its log-probability, entropy, value (lane 0 of each quad)
    if (q == 0) {
#pragma unroll
        for (int k = 0; k < SR; ++k) {
            const int64_t q_row = row0 + wave * RPW + k * 16 + (l >> 2);
            if (q_row >= M) continue;
            const int64_t row = grow(q_row);
            const float S = sS[k];
            int a = sA[k];
            float lp = 0.f, h = 0.f;
            if (S > 0.f) {
                const float lS = __logf(S);
                lp = sZ[k] - sM[k] - lS;
                h = lS - sT[k] / S;
            } else {
                a = 0;
            }
            act[row] = a;
            logp[row] = lp;
            ent[row] = h;
            val[row] = sV[k];
        }
    }
}

// fp32 parameters -> bf16 K-chunk layouts (forward W1f, W2f, W3f; backward W3b, W2b)
__global__ void mlp_sync_kernel(const MlpDims d, const float* __restrict__ p_all, uint16_t* __restrict__ w_all,
                                int64_t pstride, int64_t wstride)
{
    const float* __restrict__ p = p_all + (int64_t)blockIdx.y * pstride;
    uint16_t* __restrict__ w = w_all + (int64_t)blockIdx.y * wstride;
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
int launch_policy_forward(const MlpDims& d, const float* params, const uint16_t* work, const uint16_t* obs,
                          const uint32_t* mask, int64_t M, int64_t row_base, int W, uint64_t seed, uint64_t ctr,
                          const uint64_t* ctr_base, int32_t* act, float* logp, float* val, float* ent, float* logits,
                          hipStream_t st, int groups = 1, PolicyGroups grp = PolicyGroups{1, 0, 0})
{
    using T = MlpTile<H, RPW>;
    const int64_t blocks = (M + T::TILE - 1) / T::TILE;
    const size_t lds = policy_lds_bytes<H, RPW>(W, d.A1p);
    const dim3 grid((unsigned)blocks, (unsigned)groups);
    if (d.K1p == K1P) {
        policy_forward_kernel<H, RPW, K1P><<<grid, 256, lds, st>>>(d, params, work, obs, mask, M, row_base, W, seed, ctr,
                                                                 ctr_base, act, logp, val, ent, logits, grp);
    } else {
        // wide rows (mlp_dims: H >= 128; desc_dims: 64-row tiles)
        if constexpr (RPW == 16 && H >= 128)
            policy_forward_kernel<H, RPW, K1P_WIDE><<<grid, 256, lds, st>>>(d, params, work, obs, mask, M, row_base, W,
                                                                          seed, ctr, ctr_base, act, logp, val, ent,
                                                                          logits, grp);
        else
            return EJ_EUNSUPPORTED;
    }
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

}  // namespace econ

using namespace econ;

static int desc_dims(const ej_mlp_desc* m, MlpDims* d)
{
    if (!m) return EJ_EINVAL;
    if (m->tile_rows != 0 && m->tile_rows != 64 && !(m->tile_rows == 128 && m->H <= 256 && m->D_stride <= K1P))
        return EJ_EUNSUPPORTED;
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
    out->params_stride = group_stride(d.n_params, 4);
    out->work_stride = group_stride(d.n_work, 8);
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
    mlp_sync_kernel<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(d, d_params, d_work, 0, 0);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

int ej_mlp_sync_weights_grouped(const ej_mlp_desc* m, int32_t groups, const float* d_params, uint16_t* d_work,
                                void* stream)
{
    MlpDims d;
    int rc = desc_dims(m, &d);
    if (rc != EJ_OK) return rc;
    if (!d_params || !d_work || groups <= 0 || groups > 65535) return EJ_EINVAL;
    int64_t blocks = (d.n_work + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    mlp_sync_kernel<<<dim3((unsigned)blocks, (unsigned)groups), 256, 0, (hipStream_t)stream>>>(
        d, d_params, d_work, group_stride(d.n_params, 4), group_stride(d.n_work, 8));
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
                      const uint32_t* d_mask, int64_t M, int64_t row_base, uint64_t seed, uint64_t ctr,
                      const uint64_t* d_ctr_base, int32_t* d_act, float* d_logp, float* d_val, float* d_ent,
                      float* d_logits, void* stream)
{
    MlpDims d;
    int rc = desc_dims(m, &d);
    if (rc != EJ_OK) return rc;
    if (M < 0 || row_base < 0 || !d_params || !d_work || !d_obs || !d_mask || !d_act || !d_logp || !d_val || !d_ent)
        return EJ_EINVAL;
    if (!aligned16(d_params) || !aligned16(d_work) || !aligned16(d_obs)) return EJ_EINVAL;
    if (M == 0) return EJ_OK;
    const int W = (m->A + 31) / 32;
    hipStream_t st = (hipStream_t)stream;
    const bool small = m->tile_rows != 128 || m->H == 512;  // 64-row tiles unless 128 is asked for
#define EJ_POLICY(HH, RR) \
    launch_policy_forward<HH, RR>(d, d_params, d_work, d_obs, d_mask, M, row_base, W, seed, ctr, d_ctr_base, d_act, d_logp, \
                                  d_val, d_ent, d_logits, st)
    switch (m->H) {
    case 64: return small ? EJ_POLICY(64, 16) : EJ_POLICY(64, 32);
    case 128: return small ? EJ_POLICY(128, 16) : EJ_POLICY(128, 32);
    case 256: return small ? EJ_POLICY(256, 16) : EJ_POLICY(256, 32);
    default: return EJ_POLICY(512, 16);
    }
#undef EJ_POLICY
}

int ej_policy_forward_grouped(const ej_mlp_desc* m, int32_t groups, const float* d_params, const uint16_t* d_work,
                              const uint16_t* d_obs, const uint32_t* d_mask, int64_t rows_per_group,
                              int64_t row_stride, uint64_t seed, uint64_t ctr, const uint64_t* d_ctr_base,
                              int32_t* d_act, float* d_logp, float* d_val, float* d_ent, float* d_logits, void* stream)
{
    MlpDims d;
    int rc = desc_dims(m, &d);
    if (rc != EJ_OK) return rc;
    if (groups <= 0 || groups > 65535 || rows_per_group < 0 || row_stride < groups || !d_params || !d_work || !d_obs ||
        !d_mask || !d_act || !d_logp || !d_val || !d_ent)
        return EJ_EINVAL;
    if (!aligned16(d_params) || !aligned16(d_work) || !aligned16(d_obs)) return EJ_EINVAL;
    if (rows_per_group == 0) return EJ_OK;
    const int W = (m->A + 31) / 32;
    hipStream_t st = (hipStream_t)stream;
    const PolicyGroups grp{row_stride, group_stride(d.n_params, 4), group_stride(d.n_work, 8)};
#define EJ_POLICY_G(HH)                                                                                              \
    launch_policy_forward<HH, 16>(d, d_params, d_work, d_obs, d_mask, rows_per_group, 0, W, seed, ctr, d_ctr_base,   \
                                  d_act, d_logp, d_val, d_ent, d_logits, st, groups, grp)
    switch (m->H) {
    case 64: return EJ_POLICY_G(64);
    case 128: return EJ_POLICY_G(128);
    case 256: return EJ_POLICY_G(256);
    default: return EJ_POLICY_G(512);
    }
#undef EJ_POLICY_G
}

}  // extern "C"
