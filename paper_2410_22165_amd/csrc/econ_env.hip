// econ_env.hip -- gfx950 kernels of the EconoJax economy step and the
// economy half of the C ABI (ej_env_*).
//
// One workgroup owns one economy for the whole step.  Agent state is SoA in
// HBM (field-major, each economy's agents contiguous and 64-byte aligned) and
// lives in registers during the step; the order book of the economy is
// rebuilt every step in LDS as a histogram over (resource, side, price,
// age) buckets laid out in matching-priority order, so that exclusive scans
// give every live order its global priority rank without sorting.
//
// Paper passages implemented (Ponse et al., EconoJax, AAMAS 2025):
//   Sec. 3 "Population Agents": gathering, crafting, trading with escrow,
//     matching priority (price, then age, then random), optional NOOP;
//   Eq. (1)-(2): isoelastic utility minus labor, reward = utility change;
//   Sec. 3 "Government Agent", Eqs. (3)-(5): social welfare Eq * Prod;
//   Sec. 3 "Setting tax rates": marginal bracket tax on the period's
//     earnings, uniform redistribution;
//   Sec. 3 "Action masking"; Appendix A: trade price of the later order.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "econ_common.h"

namespace econ {

static thread_local int g_last_hip = 0;
void set_last_hip_error(hipError_t e) { g_last_hip = (int)e; }

// ---------------------------------------------------------------------------
// parameters and state handed to every kernel (by value)
// ---------------------------------------------------------------------------
struct EnvParams {
    int32_t N, R, P, X, max_orders, P_tax, K, T;
    int32_t R_kappa, R_d, kappa_c, start_coin;
    int32_t labor_gather, labor_craft, labor_trade, allow_noop;
    int32_t A, W, D, Ds, Dg, HB;
    double eta, omega;
    uint64_t seed;
    uint64_t gov_seed;  // government levels drawn in the step when gov_draw != 0 and no levels are passed
    uint64_t div_X, div_P;  // reciprocal multipliers 2^32 / X, 2^32 / P rounded up: j / X = (j div_X) >> 32 for j < 2^27
    int32_t gov_draw;
    int32_t apw;   // agents per wavefront in the step (64, 32 or 16; lanes beyond it idle)
    int32_t metrics;  // episode statistics accumulated by the step (ej_env_enable_metrics)
    int32_t skill_mode;  // EJ_SKILL_NORMAL / EJ_SKILL_GROWTH bits
    int64_t Ntot;  // stride between two state fields
    int32_t prices[EJ_MAX_P];
    int32_t cutoffs[EJ_MAX_K];
    ej_obs_scales sc;
};

// longest observation row (bf16 features, padded to a multiple of 8)
constexpr int EJ_MAX_DS = 8 * ((7 + 7 * EJ_MAX_R + EJ_MAX_K + 7) / 8);

struct EnvState {
    int32_t* field;          // [NF][Ntot]
    int32_t* env_t;          // [E]
    int32_t* env_ep;         // [E]
    int32_t* env_rates;      // [E][K]
    const int32_t* env_n;    // [E]
    const int32_t* env_off;  // [E]   first state slot of the economy
    const int32_t* env_row;  // [E+1] first row of the economy
    int64_t* invalid;        // [E][2] rejected population actions / government levels
    double* ug;              // [E]   social welfare of the current state (NaN: not known)
    double* u;               // [slots] utility of each agent's current state (NaN: not known)
    unsigned int* queue;     // [2]   persistent launch: next queue slot, finished workgroups
    const int32_t* order;    // [E]   persistent launch: economies by decreasing population
    int32_t E;
    int64_t* macc;           // [E][EJ_NACC] this episode's action counts, trades, price sums
    double* mlast;           // [E][EJ_NMET] record of the last completed episode
};

// episode statistics: counts per economy (action categories 3R + 3, trades R,
// price sums R) and the record layout (6 measures, then those counts)
constexpr int EJ_NACC = 5 * EJ_MAX_R + 3;
constexpr int EJ_NMET = EJ_NACC + 6;

// state field indices
__host__ __device__ inline int F_COIN_INV() { return 0; }
__host__ __device__ inline int F_COIN_ESC() { return 1; }
__host__ __device__ inline int F_LABOR() { return 2; }
__host__ __device__ inline int F_SNAP() { return 3; }
__host__ __device__ inline int F_SC() { return 4; }
__host__ __device__ inline int F_RES_INV(int R, int r) { return 5 + r + 0 * R; }
__host__ __device__ inline int F_RES_ESC(int R, int r) { return 5 + R + r; }
__host__ __device__ inline int F_SG(int R, int r) { return 5 + 2 * R + r; }
__host__ __device__ inline int F_SLOT(int R, int s) { return 5 + 3 * R + s; }
__host__ __device__ inline int n_fields(int R, int X) { return 5 + 3 * R + X; }

// packed order slot: valid | side | r (6) | p (8) | placement rank (16)
__host__ __device__ inline uint32_t slot_pack(int side, int r, int p, int rank)
{
    return 0x80000000u | ((uint32_t)side << 30) | ((uint32_t)r << 24) | ((uint32_t)p << 16) | (uint32_t)rank;
}
__host__ __device__ inline bool slot_valid(uint32_t s) { return (s >> 31) != 0; }
__host__ __device__ inline int slot_side(uint32_t s) { return (int)((s >> 30) & 1u); }
__host__ __device__ inline int slot_r(uint32_t s) { return (int)((s >> 24) & 63u); }
__host__ __device__ inline int slot_p(uint32_t s) { return (int)((s >> 16) & 255u); }
__host__ __device__ inline int slot_rank(uint32_t s) { return (int)(s & 0xffffu); }

// Pareto(4) skill in Q16.16 from one 64-bit word: x = U^(-1/4), U in (0, 1], x <= 5
__host__ __device__ inline int32_t skill_q16(uint64_t w)
{
    double u = (double)((w >> 11) + 1) * (1.0 / 9007199254740992.0);
    double x = 1.0 / sqrt(sqrt(u));
    x = x > 5.0 ? 5.0 : x;
    return (int32_t)(x * 65536.0 + 0.5);
}

// Skills of the multi-agent variant: near 1 with spread 1 as the sum of
// twelve 24-bit uniforms (both 32-bit halves of six words of two draws, top
// 24 bits each) minus six, plus one: floor(S / 2^8) - 5 * 2^16 in Q16, clipped
// to [0, 5].  Integer arithmetic only, so every device and host agrees.
__device__ inline int32_t normal_skill_q16(uint64_t seed, int e, int ep, int i, int s)
{
    const u64x4 a = philox(seed, PURPOSE_SKILL, (uint64_t)e, (uint64_t)ep, (uint64_t)i, (uint64_t)(64 + 2 * s));
    const u64x4 b = philox(seed, PURPOSE_SKILL, (uint64_t)e, (uint64_t)ep, (uint64_t)i, (uint64_t)(65 + 2 * s));
    const uint64_t w[6] = {a.x, a.y, a.z, a.w, b.x, b.y};
    int64_t S = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) S += (int64_t)(w[k] >> 40) + (int64_t)((w[k] & 0xFFFFFFFFull) >> 8);
    int64_t q = (S >> 8) - 5 * 65536;
    q = q < 0 ? 0 : (q > 5 * 65536 ? 5 * 65536 : q);
    return (int32_t)q;
}

// skill growth with use: s + floor(s (5 - s) / (200 * 5)) in Q16 (0.5 %
// shrinking to nothing at the maximum 5)
__device__ inline int32_t grown_skill_q16(int32_t s)
{
    const int64_t smax = 5 * 65536;
    const int64_t d = ((int64_t)s * (smax - (int64_t)s)) / (200 * smax);
    const int64_t v = (int64_t)s + (d > 0 ? d : 0);
    return (int32_t)(v > smax ? smax : v);
}

// ---------------------------------------------------------------------------
// per-agent registers
// ---------------------------------------------------------------------------
template <int RM, int XM>
struct Agent {
    int32_t coin_inv, coin_esc, labor, snap, sc;
    int32_t res_inv[RM], res_esc[RM], sg[RM];
    uint32_t slot[XM];
};

template <int RM>
__device__ inline int32_t rget(const int32_t (&a)[RM], int r)
{
    int32_t v = 0;
#pragma unroll
    for (int j = 0; j < RM; ++j)
        if (j == r) v = a[j];
    return v;
}
template <int RM>
__device__ inline void radd(int32_t (&a)[RM], int r, int32_t d)
{
#pragma unroll
    for (int j = 0; j < RM; ++j)
        if (j == r) a[j] += d;
}

template <int RM, int XM>
__device__ inline int n_active(const Agent<RM, XM>& ag, int X)
{
    int c = 0;
#pragma unroll
    for (int s = 0; s < XM; ++s)
        if (s < X && slot_valid(ag.slot[s])) ++c;
    return c;
}

template <int RM, int XM>
__device__ inline void load_agent(const EnvParams& P, const EnvState& S, int64_t g, Agent<RM, XM>& ag)
{
    const int32_t* f = S.field;
    const int64_t st = P.Ntot;
    ag.coin_inv = f[F_COIN_INV() * st + g];
    ag.coin_esc = f[F_COIN_ESC() * st + g];
    ag.labor = f[F_LABOR() * st + g];
    ag.snap = f[F_SNAP() * st + g];
    ag.sc = f[F_SC() * st + g];
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        if (r < P.R) {
            ag.res_inv[r] = f[F_RES_INV(P.R, r) * st + g];
            ag.res_esc[r] = f[F_RES_ESC(P.R, r) * st + g];
            ag.sg[r] = f[F_SG(P.R, r) * st + g];
        } else {
            ag.res_inv[r] = 0;
            ag.res_esc[r] = 0;
            ag.sg[r] = 0;
        }
    }
#pragma unroll
    for (int s = 0; s < XM; ++s) ag.slot[s] = s < P.X ? (uint32_t)f[F_SLOT(P.R, s) * st + g] : 0u;
}

// skills: also store the craft and gather skills (they change only when an
// episode starts)
template <int RM, int XM>
__device__ inline void store_agent(const EnvParams& P, const EnvState& S, int64_t g, const Agent<RM, XM>& ag,
                                   bool skills)
{
    int32_t* f = S.field;
    const int64_t st = P.Ntot;
    f[F_COIN_INV() * st + g] = ag.coin_inv;
    f[F_COIN_ESC() * st + g] = ag.coin_esc;
    f[F_LABOR() * st + g] = ag.labor;
    f[F_SNAP() * st + g] = ag.snap;
    if (skills) f[F_SC() * st + g] = ag.sc;
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        if (r < P.R) {
            f[F_RES_INV(P.R, r) * st + g] = ag.res_inv[r];
            f[F_RES_ESC(P.R, r) * st + g] = ag.res_esc[r];
            if (skills) f[F_SG(P.R, r) * st + g] = ag.sg[r];
        }
    }
#pragma unroll
    for (int s = 0; s < XM; ++s)
        if (s < P.X) f[F_SLOT(P.R, s) * st + g] = (int32_t)ag.slot[s];
}

// reset state of one agent at episode `ep` of economy e
template <int RM, int XM>
__device__ inline void reset_agent(const EnvParams& P, int e, int ep, int i, Agent<RM, XM>& ag)
{
    ag.coin_inv = P.start_coin;
    ag.coin_esc = 0;
    ag.labor = 0;
    ag.snap = P.start_coin;
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        ag.res_inv[r] = 0;
        ag.res_esc[r] = 0;
    }
#pragma unroll
    for (int s = 0; s < XM; ++s) ag.slot[s] = 0u;
    // skill words s = 0..R-1 gathering, s = R crafting; four words per draw
    u64x4 w = philox(P.seed, PURPOSE_SKILL, (uint64_t)e, (uint64_t)ep, (uint64_t)i, 0);
#pragma unroll
    for (int s = 0; s <= RM; ++s) {
        if (s > P.R) break;
        if (s > 0 && (s & 3) == 0) w = philox(P.seed, PURPOSE_SKILL, (uint64_t)e, (uint64_t)ep, (uint64_t)i, (uint64_t)(s >> 2));
        int32_t q = (P.skill_mode & EJ_SKILL_NORMAL) ? normal_skill_q16(P.seed, e, ep, i, s)
                                                    : skill_q16(word_of(w, s & 3));
        if (s < P.R) {
#pragma unroll
            for (int r = 0; r < RM; ++r)
                if (r == s) ag.sg[r] = q;
        } else {
            ag.sc = q;
        }
    }
}

// Eq. (1)
__device__ inline double utility(int64_t coin, int32_t labor_q, double eta)
{
    const double one_m = 1.0 - eta;
    return (pow((double)coin, one_m) - 1.0) / one_m - (double)labor_q / 20.0;
}

// marginal bracket tax in whole coin: floor(sum_b level_b overlap_b / 20)
__device__ inline int64_t bracket_tax(int64_t income, const int32_t* levels, const int32_t* cutoffs, int K)
{
    if (income <= 0 || K <= 0) return 0;
    int64_t acc = 0, lo = 0;
    for (int b = 0; b < K; ++b) {
        int64_t hi = b < K - 1 ? (int64_t)cutoffs[b] : INT64_MAX;
        int64_t top = income < hi ? income : hi;
        if (top > lo) acc += (int64_t)levels[b] * (top - lo);
        lo = hi;
        if (income <= hi) break;
    }
    return acc / 20;
}

// decoded action
struct Act {
    int type, r, p;  // type: 0 noop, 1 gather, 2 craft, 3 buy, 4 sell
};

__device__ inline Act decode_action(const EnvParams& P, int a)
{
    Act d{0, 0, 0};
    if (a <= 0) return d;
    if (a <= P.R) {
        d.type = 1;
        d.r = a - 1;
        return d;
    }
    if (a == P.R + 1) {
        d.type = 2;
        return d;
    }
    int b = a - (P.R + 2);
    const int RP = P.R * P.P;
    if (b < RP) {
        d.type = 3;
    } else {
        d.type = 4;
        b -= RP;
    }
    d.r = (int)(((uint64_t)(uint32_t)b * P.div_P) >> 32);  // b / P (b < 2 R P)
    d.p = b - d.r * P.P;
    return d;
}

template <int RM, int XM>
__device__ inline bool craft_possible(const EnvParams& P, const Agent<RM, XM>& ag)
{
    int ok = 0;
#pragma unroll
    for (int r = 0; r < RM; ++r)
        if (r < P.R && ag.res_inv[r] >= P.R_kappa) ++ok;
    return ok >= P.R_d;
}

template <int RM, int XM>
__device__ inline bool action_allowed(const EnvParams& P, const Agent<RM, XM>& ag, int nact, int a,
                                      const int32_t* s_prices)
{
    if (a < 0 || a >= P.A) return false;
    Act d = decode_action(P, a);
    switch (d.type) {
    case 0: return P.allow_noop != 0;
    case 1: return true;
    case 2: return craft_possible(P, ag);
    case 3: return nact < P.max_orders && ag.coin_inv >= s_prices[d.p];
    default: return nact < P.max_orders && rget(ag.res_inv, d.r) >= 1;
    }
}

// ---------------------------------------------------------------------------
// block primitives (blockDim.x a multiple of 64)
// ---------------------------------------------------------------------------
__device__ inline int64_t block_sum_i64(int64_t v, int64_t* red)
{
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    lds_barrier();
    if (lane_id() == 0) red[w] = v;
    lds_barrier();
    int64_t tot = 0;
    for (int j = 0; j < nw; ++j) tot += red[j];
    return tot;
}

__device__ inline double block_sum_f64(double v, int64_t* red)
{
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double* dr = (double*)red;
    v = wave_sum(v);
    lds_barrier();
    if (lane_id() == 0) dr[w] = v;
    lds_barrier();
    double tot = 0.0;
    for (int j = 0; j < nw; ++j) tot += dr[j];
    return tot;
}

// int64 key with the order of the double (finite values): the sign-magnitude
// bits of a negative double are flipped so that larger keys are larger values
__device__ inline int64_t f64_order_key(double d)
{
    const int64_t b = __double_as_longlong(d);
    return b < 0 ? (b ^ 0x7FFFFFFFFFFFFFFFll) : b;
}
__device__ inline double f64_from_order_key(int64_t k)
{
    return __longlong_as_double(k < 0 ? (k ^ 0x7FFFFFFFFFFFFFFFll) : k);
}

// three block-wide sums at the cost of one (two barriers); red holds 48 entries
__device__ inline void block_sum3_i64(int64_t& a, int64_t& b, int64_t& c, int64_t* red)
{
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    lds_barrier();
    if (lane_id() == 0) {
        red[w] = a;
        red[16 + w] = b;
        red[32 + w] = c;
    }
    lds_barrier();
    a = b = c = 0;
    for (int j = 0; j < nw; ++j) {
        a += red[j];
        b += red[16 + j];
        c += red[32 + j];
    }
}

// exclusive scans of `nseg` segments of `len` ints (src -> dst); waves take
// segments round-robin; the caller synchronises before and after.
// A wave takes U of its segments at once so that their load and scan
// chains overlap (absent segments scan zeros).
template <int U>
__device__ inline void seg_exclusive_scan(const int32_t* src, int32_t* dst, int nseg, int len)
{
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = lane_id();
    if (len <= 256) {
        // four consecutive entries per lane (one 16-byte word when len is a
        // multiple of 4): a local prefix, then one wave scan of the lane
        // totals per segment
        const bool vec = (len & 3) == 0;
        for (int s0 = w; s0 < nseg; s0 += U * nw) {
            int32_t v[U][4], tot[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int sg = s0 + u * nw;
                const bool seg = sg < nseg;
                if (vec) {
                    const int4 x = (seg && 4 * lane < len) ? *(const int4*)(src + sg * len + 4 * lane) : int4{0, 0, 0, 0};
                    v[u][0] = x.x;
                    v[u][1] = x.y;
                    v[u][2] = x.z;
                    v[u][3] = x.w;
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int j = 4 * lane + i;
                        v[u][i] = (seg && j < len) ? src[sg * len + j] : 0;
                    }
                }
                tot[u] = v[u][0] + v[u][1] + v[u][2] + v[u][3];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int sg = s0 + u * nw;
                const int32_t e0 = wave_scan_i(tot[u]) - tot[u];  // entries before this lane's four
                const int32_t e1 = e0 + v[u][0], e2 = e1 + v[u][1], e3 = e2 + v[u][2];
                if (sg >= nseg) continue;
                if (vec) {
                    if (4 * lane < len) *(int4*)(dst + sg * len + 4 * lane) = int4{e0, e1, e2, e3};
                } else {
                    const int32_t e[4] = {e0, e1, e2, e3};
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (4 * lane + i < len) dst[sg * len + 4 * lane + i] = e[i];
                }
            }
        }
        return;
    }
    for (int s0 = w; s0 < nseg; s0 += U * nw) {
        int32_t carry[U];
#pragma unroll
        for (int u = 0; u < U; ++u) carry[u] = 0;
        for (int c = 0; c < len; c += 64) {
            const int j = c + lane;
            int32_t v[U], inc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int sg = s0 + u * nw;
                v[u] = (sg < nseg && j < len) ? src[sg * len + j] : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) inc[u] = wave_scan_i(v[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int sg = s0 + u * nw;
                if (sg < nseg && j < len) dst[sg * len + j] = carry[u] + inc[u] - v[u];
                carry[u] += __builtin_amdgcn_readlane(inc[u], 63);
            }
        }
    }
}

// in-place ascending bitonic sort of `n2` (power of two) int64 keys in LDS
__device__ inline void bitonic_sort_i64(int64_t* a, int n2)
{
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n2; i += blockDim.x) {
                int l = i ^ j;
                if (l > i) {
                    int64_t x = a[i], y = a[l];
                    bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        a[i] = y;
                        a[l] = x;
                    }
                }
            }
            lds_barrier();
        }
    }
}

__host__ __device__ inline int next_pow2(int n)
{
    int p = 64;
    while (p < n) p <<= 1;
    return p;
}

// ---------------------------------------------------------------------------
// LDS carve-up shared by host (sizing) and device
// ---------------------------------------------------------------------------
struct Lds {
    int32_t *hcnt, *hmin, *hexc;     // [HB] order-book buckets
    int32_t *nbcnt, *nboff;          // [2 R P] new orders per (side, r, p)
    int32_t *ncode, *ntab;           // [NL] new-order bucket per agent; agents by bucket rank
    uint32_t* nkey;                  // [NL] new-order tie key
    int64_t* sortbuf;                // [S2]
    int32_t *prices, *cutoffs, *rates, *kr, *mstat, *misc;
    uint32_t* tmpl;                  // [EJ_MAX_DS / 2] economy-wide words of an observation row
    int64_t* red;                    // [32]
    double* dred;                    // [4]
    int32_t* met;                    // [EJ_NACC] this step's action counts, trades, price sums
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// Byte offsets of the LDS arrays; `base` null only sizes the layout.
__host__ __device__ __forceinline__ size_t lds_layout(const EnvParams& P, int NL, unsigned char* base, Lds* L)
{
    const size_t NB = 2 * (size_t)P.R * (size_t)P.P, HB = (size_t)P.HB, nl = (size_t)NL;
    const size_t S2 = (size_t)next_pow2(NL);
    const size_t o_hcnt = 0;
    const size_t o_hmin = align16(o_hcnt + 4 * HB);
    const size_t o_hexc = align16(o_hmin + 4 * HB);
    const size_t o_nbcnt = align16(o_hexc + 4 * HB);
    const size_t o_nboff = align16(o_nbcnt + 4 * NB);
    const size_t o_ncode = align16(o_nboff + 4 * NB);
    const size_t o_ntab = align16(o_ncode + 4 * nl);
    const size_t o_nkey = align16(o_ntab + 4 * nl);
    const size_t o_sort = align16(o_nkey + 4 * nl);
    const size_t o_prices = align16(o_sort + 8 * S2);
    const size_t o_cut = align16(o_prices + 4 * EJ_MAX_P);
    const size_t o_rates = align16(o_cut + 4 * EJ_MAX_K);
    const size_t o_kr = align16(o_rates + 4 * EJ_MAX_K);
    const size_t o_mstat = align16(o_kr + 4 * EJ_MAX_R);
    const size_t o_misc = align16(o_mstat + 16 * EJ_MAX_R);
    const size_t o_tmpl = align16(o_misc + 4 * 16);
    const size_t o_red = align16(o_tmpl + 2 * EJ_MAX_DS);
    const size_t o_dred = align16(o_red + 8 * 48);
    const size_t o_met = align16(o_dred + 8 * 4);
    const size_t total = align16(o_met + 4 * EJ_NACC);
    if (base) {
        L->hcnt = (int32_t*)(base + o_hcnt);
        L->hmin = (int32_t*)(base + o_hmin);
        L->hexc = (int32_t*)(base + o_hexc);
        L->nbcnt = (int32_t*)(base + o_nbcnt);
        L->nboff = (int32_t*)(base + o_nboff);
        L->ncode = (int32_t*)(base + o_ncode);
        L->ntab = (int32_t*)(base + o_ntab);
        L->nkey = (uint32_t*)(base + o_nkey);
        L->sortbuf = (int64_t*)(base + o_sort);
        L->prices = (int32_t*)(base + o_prices);
        L->cutoffs = (int32_t*)(base + o_cut);
        L->rates = (int32_t*)(base + o_rates);
        L->kr = (int32_t*)(base + o_kr);
        L->mstat = (int32_t*)(base + o_mstat);
        L->misc = (int32_t*)(base + o_misc);
        L->tmpl = (uint32_t*)(base + o_tmpl);
        L->red = (int64_t*)(base + o_red);
        L->dred = (double*)(base + o_dred);
        L->met = (int32_t*)(base + o_met);
    }
    return total;
}

// age of the order in slot s (0 <= s < X) when t mod X = tX: (tX - s) mod X,
// from tX - s + X in [1, 2X) without a division
__device__ inline int slot_age(int tX, int s, int X)
{
    const int a = tX - s + X;
    return a >= X ? a - X : a;
}

// bucket position in matching-priority order within the (r, side) segment
__device__ inline int bucket_pos(const EnvParams& P, int side, int p, int age)
{
    return side == 0 ? (P.P - 1 - p) * P.X + (P.X - 1 - age) : p * P.X + (P.X - 1 - age);
}

// Gini numerator sum_k (2k - n + 1) x_(k) and coin sum of the economy from
// the coin values in sortbuf (n live entries, padded with INT64_MAX to S2),
// then the social welfare.  Small economies take each value's rank by
// counting (ties ordered by index: any order of equal values gives the same
// sum); larger ones sort in LDS.
// sort-buffer entry of agent li holding coin C: unique keys while the
// welfare ranks by counting (n <= 256), the plain value for the sort
__device__ inline int64_t welfare_key(int64_t C, int li, int n) { return n <= 256 ? C * 256 + li : C; }

// `extra` (nullable): one more per-thread count, summed over the block in the
// same reduction
__device__ inline double social_welfare_block(const EnvParams& P, const Lds& L, int n, int S2,
                                              int64_t* extra = nullptr, int64_t* num_sum = nullptr)
{
    int64_t num = 0, sum = 0;
    if (n <= 256) {
        // The buffer holds unique keys 256 C + agent (welfare_key), so a
        // value's rank in the sorted order (ties by agent) is the number of
        // smaller keys.  Entries n.. hold INT64_MAX, so the count runs over
        // whole groups of 8 (S2 >= that).
        const int n8 = (n + 7) & ~7;
        const longlong2* sb2 = (const longlong2*)L.sortbuf;  // two keys per 16-byte read
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int64_t key = L.sortbuf[i];
            const int64_t x = key >> 8;
            int rank = 0;
#pragma unroll 4
            for (int j = 0; j < n8 / 2; j += 4) {
                longlong2 y[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) y[q] = sb2[j + q];
#pragma unroll
                for (int q = 0; q < 4; ++q) rank += (y[q].x < key) + (y[q].y < key);
            }
            num += (int64_t)(2 * rank - n + 1) * x;
            sum += x;
        }
    } else {
        bitonic_sort_i64(L.sortbuf, S2);
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            int64_t x = L.sortbuf[k];
            num += (int64_t)(2 * k - n + 1) * x;
            sum += x;
        }
    }
    int64_t x = extra ? *extra : 0;
    block_sum3_i64(num, sum, x, L.red);
    if (extra) *extra = x;
    if (num_sum) {
        num_sum[0] = num;
        num_sum[1] = sum;
    }
    double gini = 0.0;
    if (sum > 0) gini = (double)num / ((double)n * (double)sum);
    double eq = (1.0 - P.omega) + P.omega * (1.0 - gini);
    return eq * (double)sum;
}

// market statistics after the step from the bucket histogram:
// mstat[4r + 0..3] = best bid price, best ask price, #bids, #asks
// `kr` null -> no fills; `skip_age` >= 0 -> that age has expired.
__device__ inline void market_stats(const EnvParams& P, const Lds& L, const int32_t* kr, int skip_age)
{
    // a wave takes up to four (r, side) segments at once (independent chains)
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = lane_id();
    const int PX = P.P * P.X, nseg = 2 * P.R;
    for (int s0 = w; s0 < nseg; s0 += 4 * nw) {
        int best[4], count[4], k[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int sg = s0 + u * nw;
            best[u] = INT_MAX;
            count[u] = 0;
            k[u] = (sg < nseg && kr) ? kr[sg >> 1] : 0;
        }
        const uint64_t mgX = P.div_X;
        for (int c = 0; c < PX; c += 64) {
            const int pos = c + lane;
            const int age = P.X - 1 - (pos - (int)(((uint64_t)(uint32_t)pos * mgX) >> 32) * P.X);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int sg = s0 + u * nw;
                if (sg < nseg && pos < PX) {
                    const int b = sg * PX + pos;
                    const int cnt = L.hcnt[b];
                    int fill = k[u] - L.hexc[b];
                    fill = fill < 0 ? 0 : (fill > cnt ? cnt : fill);
                    const int alive = age == skip_age ? 0 : cnt - fill;
                    if (alive > 0 && pos < best[u]) best[u] = pos;
                    count[u] += alive;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            best[u] = wave_min_i(best[u]);
            count[u] = wave_sum_i(count[u]);
        }
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int sg = s0 + u * nw;
                if (sg >= nseg) continue;
                const int r = sg >> 1, side = sg & 1;
                int price = 0;
                if (best[u] != INT_MAX) {
                    const int pl = best[u] / P.X;
                    const int p = side == 0 ? P.P - 1 - pl : pl;
                    price = L.prices[p];
                }
                L.mstat[4 * r + side] = price;
                L.mstat[4 * r + 2 + side] = count[u];
            }
        }
    }
}

// packs consecutive bf16 features into 32-bit stores
struct RowWriter {
    uint32_t* base;
    uint32_t pend;
    int d;
    __device__ inline void put(float v)
    {
        uint32_t b = f32_to_bf16(v);
        if (d & 1) base[d >> 1] = pend | (b << 16);
        else pend = b;
        ++d;
    }
};

template <int RM, int XM>
__device__ inline void write_obs_row(const EnvParams& P, const Lds& L, const Agent<RM, XM>& ag, int t,
                                     uint16_t* row)
{
    const ej_obs_scales& s = P.sc;
    RowWriter w{(uint32_t*)row, 0u, 0};
    const int nact = n_active(ag, P.X);
    w.put((float)ag.coin_inv * s.coin);
    w.put((float)ag.coin_esc * s.coin);
    w.put((float)ag.labor * s.labor);
    w.put((float)nact * s.orders);
    w.put((float)(ag.coin_inv + ag.coin_esc - ag.snap) * s.coin);
#pragma unroll
    for (int r = 0; r < RM; ++r)
        if (r < P.R) w.put((float)ag.res_inv[r] * s.res);
#pragma unroll
    for (int r = 0; r < RM; ++r)
        if (r < P.R) w.put((float)ag.res_esc[r] * s.res);
#pragma unroll
    for (int r = 0; r < RM; ++r)
        if (r < P.R) w.put((float)ag.sg[r] * s.skill);
    w.put((float)ag.sc * s.skill);
    for (int b = 0; b < P.K; ++b) w.put((float)L.rates[b] * s.rate);
    w.put((float)(t % P.P_tax) * s.phase);
    for (int r = 0; r < P.R; ++r) {
        w.put((float)L.mstat[4 * r + 0] * s.price);
        w.put((float)L.mstat[4 * r + 1] * s.price);
        w.put((float)L.mstat[4 * r + 2] * s.count);
        w.put((float)L.mstat[4 * r + 3] * s.count);
    }
    while (w.d < P.Ds) w.put(0.0f);
}

// bits [lo, hi) of mask word `wd`
__device__ inline uint32_t range_bits(int wd, int lo, int hi)
{
    int a = lo - 32 * wd, b = hi - 32 * wd;
    a = a < 0 ? 0 : a;
    b = b > 32 ? 32 : b;
    if (a >= b) return 0u;
    uint32_t hi_mask = b == 32 ? 0xffffffffu : ((1u << b) - 1u);
    return hi_mask & ~((1u << a) - 1u);
}

// Features 0 .. 6 + 3R - 1 of an observation row belong to the agent; the
// rest (tax rates, phase, market statistics, zero padding) are the same for
// every agent of the economy.
__host__ __device__ inline int obs_own_features(int R) { return 6 + 3 * R; }

// bf16 bits of row feature f >= obs_own_features(R)
__device__ inline uint32_t obs_shared_bits(const EnvParams& P, const Lds& L, int f, int t)
{
    const ej_obs_scales& s = P.sc;
    const int q = f - obs_own_features(P.R);
    float v;
    if (q < P.K) {
        v = (float)L.rates[q] * s.rate;
    } else if (q == P.K) {
        v = (float)(t % P.P_tax) * s.phase;
    } else if (q < P.K + 1 + 4 * P.R) {
        const int m = q - P.K - 1;
        v = (float)L.mstat[m] * ((m & 3) < 2 ? s.price : s.count);
    } else {
        return 0u;
    }
    return f32_to_bf16(v);
}

// 32-bit word c of a row that holds no agent feature
__device__ inline uint32_t obs_shared_word(const EnvParams& P, const Lds& L, int c, int t)
{
    return obs_shared_bits(P, L, 2 * c, t) | (obs_shared_bits(P, L, 2 * c + 1, t) << 16);
}

// the words of a row that hold the agent's own features (the last one may
// also hold the first economy-wide feature)
template <int RM, int XM>
__device__ inline void write_obs_own_words(const EnvParams& P, const Lds& L, const Agent<RM, XM>& ag, int t,
                                           uint32_t* row)
{
    const ej_obs_scales& s = P.sc;
    RowWriter w{row, 0u, 0};
    w.put((float)ag.coin_inv * s.coin);
    w.put((float)ag.coin_esc * s.coin);
    w.put((float)ag.labor * s.labor);
    w.put((float)n_active(ag, P.X) * s.orders);
    w.put((float)(ag.coin_inv + ag.coin_esc - ag.snap) * s.coin);
#pragma unroll
    for (int r = 0; r < RM; ++r)
        if (r < P.R) w.put((float)ag.res_inv[r] * s.res);
#pragma unroll
    for (int r = 0; r < RM; ++r)
        if (r < P.R) w.put((float)ag.res_esc[r] * s.res);
#pragma unroll
    for (int r = 0; r < RM; ++r)
        if (r < P.R) w.put((float)ag.sg[r] * s.skill);
    w.put((float)ag.sc * s.skill);
    if (w.d & 1) row[w.d >> 1] = w.pend | (obs_shared_bits(P, L, w.d, t) << 16);
}

template <int RM, int XM>
__device__ inline void write_mask_row(const EnvParams& P, const Lds& L, const Agent<RM, XM>& ag, uint32_t* row)
{
    const int nact = n_active(ag, P.X);
    const bool can_order = nact < P.max_orders;
    // affordable price levels form a prefix: prices strictly increase
    int lo = 0, hi = P.P;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (L.prices[mid] <= ag.coin_inv) lo = mid + 1;
        else hi = mid;
    }
    const int n_afford = can_order ? lo : 0;
    const bool craft = craft_possible(P, ag);
    const int base_buy = P.R + 2, base_sell = P.R + 2 + P.R * P.P;
    for (int wd = 0; wd < P.W; ++wd) {
        const int w0 = 32 * wd, w1 = w0 + 32;
        uint32_t bits = 0;
        if (P.allow_noop) bits |= range_bits(wd, 0, 1);
        bits |= range_bits(wd, 1, P.R + 1);
        if (craft) bits |= range_bits(wd, P.R + 1, P.R + 2);
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            if (r < P.R) {
                // a resource's buy and sell ranges meet at most two words: the
                // (uniform) range tests skip the others
                const int bb = base_buy + r * P.P, sb = base_sell + r * P.P;
                if (bb < w1 && bb + P.P > w0) bits |= range_bits(wd, bb, bb + n_afford);
                if (sb < w1 && sb + P.P > w0 && can_order && ag.res_inv[r] >= 1) bits |= range_bits(wd, sb, sb + P.P);
            }
        }
        row[wd] = bits;
    }
}

// uniform government level 0..20 of bracket b at step t (economy e, episode ep)
__device__ inline int32_t gov_level_draw(uint64_t seed, int e, int ep, int t, int b)
{
    u64x4 w = philox(seed, PURPOSE_GOV, (uint64_t)e, (uint64_t)ep, (uint64_t)t, (uint64_t)(b >> 2));
    return (int32_t)(((word_of(w, b & 3) >> 32) * (uint64_t)EJ_GOV_LEVELS) >> 32);
}

// ---------------------------------------------------------------------------
// the step kernel: one workgroup per economy
// ---------------------------------------------------------------------------
template <int RM, int XM, int APT>
__device__ __forceinline__ void env_step_one(const EnvParams& P, const EnvState& S, const int e,
                                             const int32_t* __restrict__ act, const int32_t* __restrict__ gov,
                                             float* __restrict__ rew, float* __restrict__ gov_rew,
                                             uint8_t* __restrict__ done_out, uint16_t* __restrict__ obs,
                                             uint32_t* __restrict__ mask, unsigned char* smem)
{
    const int NT = blockDim.x, tid = threadIdx.x;
    // agents per wavefront: in round k, wave w takes agents k NR + w apw ..
    // + apw - 1 (lanes apw .. 63 idle); NL agent slots in all
    const int apw = P.apw;
    const int NR = (NT >> 6) * apw;
    const int NL = NR * APT;
    const int lane_slot = (tid & 63) < apw ? (tid >> 6) * apw + (tid & 63) : (1 << 30);
    Lds L;
    lds_layout(P, NL, smem, &L);
    const int n = S.env_n[e];
    const int64_t off = S.env_off[e];
    const int64_t row0 = S.env_row[e];
    const int t = S.env_t[e];
    const int ep = S.env_ep[e];
    const int R = P.R, X = P.X, K = P.K, PX = P.P * P.X;
    const int S2 = next_pow2(NL);

    // The agent's state and action loads go out first and stay in flight
    // while the LDS tables are initialised (the workgroup's threads talk
    // through LDS only, so its barriers do not wait for global memory).
    Agent<RM, XM> ag[APT];
    int a_in[APT];
    double u0[APT];  // utility of the step-start state: cached by the previous step, NaN when unknown
    const double cached_ug = S.ug[e];  // social welfare of the step-start state, NaN when unknown
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int li = lane_slot + k * NR;
        a_in[k] = 0;
        u0[k] = 0.0;
        if (li < n) {
            load_agent(P, S, off + li, ag[k]);
            a_in[k] = act[row0 + li];
            u0[k] = S.u[off + li];
        }
    }
    // this bracket's rate: the government sets the period's rates at its
    // first step (kept in a register until after the first barrier, so that
    // the barrier does not wait for the loads)
    int rate = 0;
    bool bad_level = false;  // a passed level outside 0..20 (counted, the previous rate kept)
    if (tid < K) {
        rate = S.env_rates[e * K + tid];
        if (t % P.P_tax == 0) {
            const int g = gov ? gov[e * K + tid] : gov_level_draw(P.gov_seed, e, ep, t, tid);
            if (g >= 0 && g < EJ_GOV_LEVELS) rate = g;
            else bad_level = gov != nullptr;
        }
    }
    // the economy's rejection counters, updated by thread 0 at the end
    int64_t inv_act = 0, inv_gov = 0;
    if (tid == 0) {
        inv_act = S.invalid[2 * e];
        inv_gov = S.invalid[2 * e + 1];
    }
    // price grid and bracket cutoffs: read now, stored after the barrier
    // (NT >= 64 and P <= 128: at most two prices per thread)
    const int32_t pr0 = tid < P.P ? P.prices[tid] : 0;
    const int32_t pr1 = tid + NT < P.P ? P.prices[tid + NT] : 0;
    const int32_t cut = tid < K - 1 ? P.cutoffs[tid] : 0;
    for (int j = tid; j < P.HB; j += NT) {
        L.hcnt[j] = 0;
        L.hmin[j] = INT_MAX;
    }
    for (int j = tid; j < 2 * R * P.P; j += NT) L.nbcnt[j] = 0;
    for (int j = tid; j < S2; j += NT) L.sortbuf[j] = INT64_MAX;
    if (P.metrics)
        for (int j = tid; j < 5 * R + 3; j += NT) L.met[j] = 0;
    lds_barrier();

    int eff[APT];
    int my_rank[APT];
    int invalid = 0;

    if (tid < K) L.rates[tid] = rate;
    const int bad_gov = __popcll(__ballot(bad_level));  // thread 0's wave holds every bracket (K <= 16)
    if (tid < P.P) L.prices[tid] = pr0;
    if (tid + NT < P.P) L.prices[tid + NT] = pr1;
    if (tid < K - 1) L.cutoffs[tid] = cut;
    // utilities of the step-start state
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int li = lane_slot + k * NR;
        eff[k] = 0;
        my_rank[k] = 0;
        if (li < n) {
            const int64_t C = (int64_t)ag[k].coin_inv + ag[k].coin_esc;
            if (u0[k] != u0[k]) u0[k] = utility(C, ag[k].labor, P.eta);
            L.sortbuf[li] = welfare_key(C, li, n);
        }
    }
    lds_barrier();
    const double ug0 = cached_ug == cached_ug ? cached_ug : social_welfare_block(P, L, n, S2);
    // action validation against the step-start mask
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int li = lane_slot + k * NR;
        if (li >= n) continue;
        const int a = a_in[k];
        const bool ok = action_allowed(P, ag[k], n_active(ag[k], X), a, L.prices);
        if (ok) eff[k] = a;
        else ++invalid;
        if (P.metrics) {  // category of the action taken: NOOP, gather r, craft, buy r, sell r, rejected
            const Act d = decode_action(P, eff[k]);
            const int cat = !ok ? 2 + 3 * R
                                : d.type == 0 ? 0 : d.type == 1 ? 1 + d.r : d.type == 2 ? 1 + R
                                                                          : (d.type == 3 ? 2 + R : 2 + 2 * R) + d.r;
            atomicAdd(&L.met[cat], 1);
        }
    }

    // apply every agent's action; new orders go to slot t mod X
    const int slot_new = t % X;
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int li = lane_slot + k * NR;
        if (li >= n) continue;
        L.ncode[li] = -1;
        Act d = decode_action(P, eff[k]);
        Agent<RM, XM>& a = ag[k];
        // one draw serves both the gathering luck and the order tie key (the
        // same counter), taken once before the two branches split the wave
        u64x4 w{0, 0, 0, 0};
        if (d.type == 1 || d.type >= 3)
            w = philox(P.seed, PURPOSE_ENV, (uint64_t)e, (uint64_t)ep, (uint64_t)t, (uint64_t)li);
        if (d.type == 1) {  // gather: floor(SG + rho), rho ~ U[0, 1.1)
            int64_t rho_q = (int64_t)(((w.x >> 32) * 72090ull) >> 32);
            int64_t amount = ((int64_t)rget(a.sg, d.r) + rho_q) >> 16;
            radd(a.res_inv, d.r, (int32_t)amount);
            a.labor += P.labor_gather;
            if (P.skill_mode & EJ_SKILL_GROWTH) {
#pragma unroll
                for (int r = 0; r < RM; ++r)
                    if (r == d.r) a.sg[r] = grown_skill_q16(a.sg[r]);
            }
        } else if (d.type == 2) {  // craft: R_d fullest eligible types, ties to the lower id
            uint32_t used = 0;
            for (int c = 0; c < P.R_d; ++c) {
                int best = -1, bestv = -1;
#pragma unroll
                for (int r = 0; r < RM; ++r) {
                    if (r < R && !((used >> r) & 1u) && a.res_inv[r] >= P.R_kappa && a.res_inv[r] > bestv) {
                        best = r;
                        bestv = a.res_inv[r];
                    }
                }
                used |= 1u << best;
                radd(a.res_inv, best, -P.R_kappa);
            }
            a.coin_inv += (int32_t)(((int64_t)a.sc * P.kappa_c) >> 16);
            a.labor += P.labor_craft;
            if (P.skill_mode & EJ_SKILL_GROWTH) a.sc = grown_skill_q16(a.sc);
        } else if (d.type >= 3) {  // order with escrow
            const int side = d.type == 4;
            if (side == 0) {
                a.coin_inv -= L.prices[d.p];
                a.coin_esc += L.prices[d.p];
            } else {
                radd(a.res_inv, d.r, -1);
                radd(a.res_esc, d.r, 1);
            }
            a.labor += P.labor_trade;
            const int code = (side * R + d.r) * P.P + d.p;
            L.ncode[li] = code;
            L.nkey[li] = (uint32_t)(w.y >> 32);
            my_rank[k] = atomicAdd(&L.nbcnt[code], 1);  // arrival position, ranked below
        }
    }
    lds_barrier();
    seg_exclusive_scan<1>(L.nbcnt, L.nboff, 1, 2 * R * P.P);
    lds_barrier();
    // this step's orders listed per (side, r, p) in arrival order; the
    // welfare sort buffer is free until the rewards
    int32_t* ntmp = (int32_t*)L.sortbuf;
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int li = lane_slot + k * NR;
        if (li < n && L.ncode[li] >= 0) ntmp[L.nboff[L.ncode[li]] + my_rank[k]] = li;
    }
    lds_barrier();

    // placement rank of each new order within its (side, r, p) list: by tie
    // key, then agent id; the new-order table lists the orders by rank.  Then
    // the bucket histogram of every live order.
    const int tX = t % X;
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int li = lane_slot + k * NR;
        if (li >= n) continue;
        const int code = L.ncode[li];
        if (code >= 0) {
            const uint32_t key = L.nkey[li];
            const int base = L.nboff[code], cnt = L.nbcnt[code];
            int rank = 0;
            for (int q = 0; q < cnt; ++q) {
                const int j = ntmp[base + q];
                const uint32_t kj = L.nkey[j];
                rank += (kj < key) || (kj == key && j < li);
            }
            my_rank[k] = rank;
            L.ntab[base + rank] = li;
            Act d = decode_action(P, eff[k]);
#pragma unroll
            for (int s = 0; s < XM; ++s)
                if (s == slot_new) ag[k].slot[s] = slot_pack(d.type == 4, d.r, d.p, rank);
        }
#pragma unroll
        for (int s = 0; s < XM; ++s) {
            uint32_t sl = ag[k].slot[s];
            if (s < X && slot_valid(sl)) {
                int side = slot_side(sl), r = slot_r(sl), p = slot_p(sl);
                const int age = slot_age(tX, s, X);
                int b = (r * 2 + side) * PX + bucket_pos(P, side, p, age);
                atomicAdd(&L.hcnt[b], 1);
                atomicMin(&L.hmin[b], slot_rank(sl));
            }
        }
    }
    lds_barrier();
    seg_exclusive_scan<4>(L.hcnt, L.hexc, 2 * R, PX);
    lds_barrier();

    // trades per resource: k_r = max_p min(#bids >= price p, #asks <= price p)
    {
        const int w = tid >> 6, nw = NT >> 6, lane = lane_id();
        for (int r = w; r < R; r += nw) {
            int best = 0;
            for (int c = 0; c < P.P; c += 64) {
                int p = c + lane;
                if (p < P.P) {
                    int bb = (r * 2 + 0) * PX + (P.P - p) * X - 1;  // last bid bucket with price >= p
                    int ba = (r * 2 + 1) * PX + (p + 1) * X - 1;    // last ask bucket with price <= p
                    int nbid = L.hexc[bb] + L.hcnt[bb];
                    int nask = L.hexc[ba] + L.hcnt[ba];
                    int m = nbid < nask ? nbid : nask;
                    best = m > best ? m : best;
                }
            }
            best = wave_max_i(best);
            if (lane == 0) L.kr[r] = best;
        }
    }
    lds_barrier();

    // Fill rank -> bucket tables: side s of resource r holds its k_r filled
    // ranks at tab_off[r] + s k_r, tab_off[r] = 2 (k_0 + ... + k_{r-1}).
    // 16-bit entries in the sort buffer (idle until the rewards); when they do
    // not fit, settlement falls back to a binary search over the prefix sums.
    // Every entry is found by its own thread (one binary search each, all in
    // parallel), so settlement reads one entry per filled order.
    uint16_t* ftab = (uint16_t*)L.sortbuf;
    int tab_off[RM], krr[RM];
    int ftot = 0;
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        krr[r] = r < R ? L.kr[r] : 0;
        tab_off[r] = ftot;
        ftot += 2 * krr[r];
    }
    const bool use_tab = ftot <= 4 * S2;
    if (use_tab) {
        for (int j = tid; j < ftot; j += NT) {
            int r = 0;
#pragma unroll
            for (int q = 1; q < RM; ++q) r = (q < R && tab_off[q] <= j) ? q : r;
            const int kr = rget(krr, r), rel = j - rget(tab_off, r);
            const int side = rel >= kr ? 1 : 0, g = rel - side * kr;
            const int ob = (r * 2 + side) * PX;
            int lo = 0, hi = PX - 1;
            while (lo < hi) {  // largest pos with hexc <= g
                const int mid = (lo + hi + 1) >> 1;
                if (L.hexc[ob + mid] <= g) lo = mid;
                else hi = mid - 1;
            }
            ftab[j] = (uint16_t)lo;
        }
        lds_barrier();
    }

    // settlement: every agent settles its own filled orders
    const uint64_t mgX = P.div_X;
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int li = lane_slot + k * NR;
        if (li >= n) continue;
        Agent<RM, XM>& a = ag[k];
#pragma unroll
        for (int s = 0; s < XM; ++s) {
            uint32_t sl = a.slot[s];
            if (!(s < X && slot_valid(sl))) continue;
            const int side = slot_side(sl), r = slot_r(sl), p = slot_p(sl);
            const int age = slot_age(tX, s, X);
            const int b = (r * 2 + side) * PX + bucket_pos(P, side, p, age);
            const int g = L.hexc[b] + (slot_rank(sl) - L.hmin[b]);
            if (g >= L.kr[r]) continue;
            // the counterpart holds rank g on the other side
            const int ob = (r * 2 + (1 - side)) * PX;
            int opos;
            if (use_tab) {
                opos = ftab[rget(tab_off, r) + (1 - side) * rget(krr, r) + g];
            } else {
                int lo = 0, hi = PX - 1;
                while (lo < hi) {  // largest pos with hexc <= g
                    int mid = (lo + hi + 1) >> 1;
                    if (L.hexc[ob + mid] <= g) lo = mid;
                    else hi = mid - 1;
                }
                opos = lo;
            }
            const int opl = (int)(((uint64_t)(uint32_t)opos * mgX) >> 32);  // opos / X
            const int oage = X - 1 - (opos - opl * X);
            const int op = side == 0 ? opl : P.P - 1 - opl;
            const int my_price = L.prices[p], other_price = L.prices[op];
            int q;
            if (age != oage) {
                q = age < oage ? my_price : other_price;  // the younger order was placed last
            } else {
                // Both placed this step (an uncrossed book never pairs two
                // older orders): the larger (key, agent) counts as placed later.
                const int orank = L.hmin[ob + opos] + (g - L.hexc[ob + opos]);
                const int ocode = ((1 - side) * R + r) * P.P + op;
                const int idx = L.nboff[ocode] + orank;
                q = side == 0 ? my_price : other_price;
                if (age == 0 && idx >= 0 && idx < n) {
                    const int oagent = L.ntab[idx];
                    const uint32_t mk = L.nkey[li], okey = L.nkey[oagent];
                    const bool mine_later = mk > okey || (mk == okey && li > oagent);
                    q = mine_later ? my_price : other_price;
                }
            }
            if (side == 0) {
                a.coin_esc -= my_price;
                a.coin_inv += my_price - q;
                radd(a.res_inv, r, 1);
                if (P.metrics) {  // the trade, counted on its bid, at price q
                    atomicAdd(&L.met[3 + 3 * R + r], 1);
                    atomicAdd(&L.met[3 + 4 * R + r], q);
                }
            } else {
                radd(a.res_esc, r, -1);
                a.coin_inv += q;
            }
            a.slot[s] = 0u;
        }
        // expiry: the order placed at t - X + 1 has had its X clearings
        const int se = (t + 1) % X;
#pragma unroll
        for (int s = 0; s < XM; ++s) {
            if (s != se) continue;
            uint32_t sl = a.slot[s];
            if (!slot_valid(sl)) continue;
            const int r = slot_r(sl), p = slot_p(sl);
            if (slot_side(sl) == 0) {
                a.coin_esc -= L.prices[p];
                a.coin_inv += L.prices[p];
            } else {
                radd(a.res_esc, r, -1);
                radd(a.res_inv, r, 1);
            }
            a.slot[s] = 0u;
        }
    }

    // tax collection and redistribution at the last step of a period
    if ((t + 1) % P.P_tax == 0) {
        if (K > 0) {
            int64_t mine = 0;
#pragma unroll
            for (int k = 0; k < APT; ++k) {
                const int li = lane_slot + k * NR;
                if (li >= n) continue;
                Agent<RM, XM>& a = ag[k];
                int64_t C = (int64_t)a.coin_inv + a.coin_esc;
                int64_t tax = bracket_tax(C - a.snap, L.rates, L.cutoffs, K);
                if (tax > a.coin_inv) tax = a.coin_inv;
                a.coin_inv -= (int32_t)tax;
                mine += tax;
            }
            const int64_t pool = block_sum_i64(mine, L.red);
            const int64_t period = t / P.P_tax;
            const int64_t share = pool / n, rem = pool % n;
#pragma unroll
            for (int k = 0; k < APT; ++k) {
                const int li = lane_slot + k * NR;
                if (li >= n) continue;
                int64_t rot = (((int64_t)li - period) % n + n) % n;
                ag[k].coin_inv += (int32_t)(share + (rot < rem ? 1 : 0));
            }
        }
#pragma unroll
        for (int k = 0; k < APT; ++k) ag[k].snap = ag[k].coin_inv + ag[k].coin_esc;
    }

    // rewards (Eq. (2)) and the end-of-step coin for the welfare
    lds_barrier();
    for (int j = tid; j < S2; j += NT) L.sortbuf[j] = INT64_MAX;
    lds_barrier();
    double u1v[APT];
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int li = lane_slot + k * NR;
        u1v[k] = 0.0;
        if (li >= n) continue;
        const int64_t C = (int64_t)ag[k].coin_inv + ag[k].coin_esc;
        const double u1 = utility(C, ag[k].labor, P.eta);
        u1v[k] = u1;
        rew[row0 + li] = (float)(u1 - u0[k]);
        S.u[off + li] = t + 1 >= P.T ? __builtin_nan("") : u1;  // the next step starts from this state
        L.sortbuf[li] = welfare_key(C, li, n);
    }
    lds_barrier();
    int64_t n_invalid = invalid;  // summed over the block with the welfare
    int64_t num_sum[2];
    const double ug1 = social_welfare_block(P, L, n, S2, &n_invalid, num_sum);
    if (tid == 0) {
        gov_rew[e] = (float)(ug1 - ug0);
        S.invalid[2 * e] = inv_act + n_invalid;
        S.invalid[2 * e + 1] = inv_gov + bad_gov;
    }

    // time advance; automatic reset at the episode end
    const int t1 = t + 1;
    const bool done = t1 >= P.T;
    if (P.metrics) {
        // episode statistics: this step's counts join the episode's; at its
        // end the record (productivity, 1 - gini, Eq * Prod, mean and lower
        // median return = end utility minus the reset-state utility)
        double mean_ret = 0.0, med_ret = 0.0;
        if (done) {
            const double u_start = utility(P.start_coin, 0, P.eta);
            lds_barrier();  // the welfare is done with the sort buffer
            for (int j = tid; j < S2; j += NT) L.sortbuf[j] = INT64_MAX;
            lds_barrier();
            double part = 0.0;
#pragma unroll
            for (int k = 0; k < APT; ++k) {
                const int li = lane_slot + k * NR;
                if (li >= n) continue;
                part += u1v[k] - u_start;
                L.sortbuf[li] = f64_order_key(u1v[k] - u_start);
            }
            mean_ret = block_sum_f64(part, L.red) / (double)n;
            bitonic_sort_i64(L.sortbuf, S2);
            med_ret = f64_from_order_key(L.sortbuf[(n - 1) >> 1]);
        }
        const int nm = 5 * R + 3;
        int64_t* acc = S.macc + (int64_t)e * EJ_NACC;
        double* rec = S.mlast + (int64_t)e * EJ_NMET;
        for (int j = tid; j < nm; j += NT) {
            const int64_t v = acc[j] + L.met[j];
            acc[j] = done ? 0 : v;
            if (done) rec[6 + j] = (double)v;
        }
        if (done && tid == 0) {
            const double gini = num_sum[1] > 0 ? (double)num_sum[0] / ((double)n * (double)num_sum[1]) : 0.0;
            rec[0] = (double)ep;
            rec[1] = (double)num_sum[1];
            rec[2] = 1.0 - gini;
            rec[3] = ug1;
            rec[4] = mean_ret;
            rec[5] = med_ret;
        }
    }
    const int t_next = done ? 0 : t1;
    const int ep_next = done ? ep + 1 : ep;
    if (done) {
        if (tid < K) L.rates[tid] = 0;
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            const int li = lane_slot + k * NR;
            if (li < n) reset_agent(P, e, ep_next, li, ag[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int li = lane_slot + k * NR;
        if (li >= n) continue;
        // skills change only at a reset, unless they grow with use
        store_agent(P, S, off + li, ag[k], done || (P.skill_mode & EJ_SKILL_GROWTH) != 0);
        done_out[row0 + li] = done ? 1 : 0;
    }
    if (tid == 0) {
        S.env_t[e] = t_next;
        S.env_ep[e] = ep_next;
        S.ug[e] = done ? __builtin_nan("") : ug1;  // the next step starts from this state
    }
    if (tid < K) S.env_rates[e * K + tid] = L.rates[tid];

    if (obs == nullptr && mask == nullptr) return;
    // observation of the post-step state (the book is empty after a reset)
    if (done) {
        for (int j = tid; j < 4 * R; j += NT) L.mstat[j] = 0;
    } else {
        market_stats(P, L, L.kr, X - 1);
    }
    lds_barrier();
    // Rows go through LDS (the bucket arrays are free now) so that the whole
    // economy's rows leave in coalesced stores; direct stores when they do
    // not fit.  Staged, an agent writes only the 32-bit words that hold its
    // own features (odd LDS stride: no bank conflicts); the words made of
    // economy-wide features (tax rates, phase, market statistics) are the
    // same in every row and are built once.
    const int dw = P.Ds >> 1;                     // row length in 32-bit words
    const int c_own = (obs_own_features(R) + 1) >> 1;
    const int os = c_own | 1, ms = P.W | 1;
    const size_t obs_lds = obs ? (size_t)n * os * 4 : 0, mask_lds = mask ? (size_t)n * ms * 4 : 0;
    const bool staged = obs_lds + mask_lds <= (size_t)3 * P.HB * 4;
    uint32_t* so = (uint32_t*)L.hcnt;
    uint32_t* smk = so + (obs ? (size_t)n * os : 0);
    if (staged && obs)
        for (int c = c_own + tid; c < dw; c += NT) L.tmpl[c] = obs_shared_word(P, L, c, t_next);
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int li = lane_slot + k * NR;
        if (li >= n) continue;
        if (staged) {  // separate calls keep the LDS and global address spaces apart
            if (obs) write_obs_own_words(P, L, ag[k], t_next, so + li * os);
            if (mask) write_mask_row(P, L, ag[k], smk + li * ms);
        } else {
            if (obs) write_obs_row(P, L, ag[k], t_next, obs + (row0 + li) * (int64_t)P.Ds);
            if (mask) write_mask_row(P, L, ag[k], mask + (row0 + li) * (int64_t)P.W);
        }
    }
    if (!staged) return;
    lds_barrier();
    if (obs) {
        // A row is dw = Ds / 2 words, a multiple of 4 (Ds is a multiple of 8),
        // and the economy's rows are contiguous: its block leaves in 16-byte
        // pieces, none of which straddles two rows.
        uint4* dst = (uint4*)(obs + row0 * (int64_t)P.Ds);
        const int q4 = dw >> 2;                                 // pieces per row
        const uint64_t mg = 0xFFFFFFFFull / (uint64_t)q4 + 1ull;  // j / q4 = (j mg) >> 32 for j < 2^27
        for (int j = tid; j < n * q4; j += NT) {
            const int row = (int)(((uint64_t)(uint32_t)j * mg) >> 32), c0 = 4 * (j - row * q4);
            uint32_t v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = c0 + i < c_own ? so[row * os + c0 + i] : L.tmpl[c0 + i];
            dst[j] = uint4{v[0], v[1], v[2], v[3]};
        }
    }
    if (mask) {
        uint32_t* dst = mask + row0 * (int64_t)P.W;
        const uint32_t mg = 0xFFFFFFFFu / (uint32_t)P.W + 1u;
        for (int j = tid; j < n * P.W; j += NT) {
            const int row = (int)__umulhi((uint32_t)j, mg);
            dst[j] = smk[row * ms + (j - row * P.W)];
        }
    }
}

// plain launch: one workgroup per economy.  MAXT bounds the workgroup size:
// 256 leaves the compiler 256 VGPRs per lane (no spills), 1024 allows
// populations of up to 1024 agents with 128.
template <int RM, int XM, int APT, int MAXT>
__global__ void __launch_bounds__(MAXT)
env_step_kernel(const EnvParams P, const EnvState S, const int32_t* __restrict__ act,
                const int32_t* __restrict__ gov, float* __restrict__ rew, float* __restrict__ gov_rew,
                uint8_t* __restrict__ done_out, uint16_t* __restrict__ obs, uint32_t* __restrict__ mask, int e_begin)
{
    extern __shared__ __align__(16) unsigned char smem[];
    env_step_one<RM, XM, APT>(P, S, e_begin + (int)blockIdx.x, act, gov, rew, gov_rew, done_out, obs, mask, smem);
}

// Persistent launch: a fixed set of workgroups takes economies from a work
// queue (largest populations first).  The last workgroup to run dry resets
// the queue, so consecutive launches (and replays of a captured graph) need
// no host-side reset.
template <int RM, int XM, int APT, int MAXT>
__global__ void __launch_bounds__(MAXT)
env_step_persistent_kernel(const EnvParams P, const EnvState S, const int32_t* __restrict__ act,
                           const int32_t* __restrict__ gov, float* __restrict__ rew, float* __restrict__ gov_rew,
                           uint8_t* __restrict__ done_out, uint16_t* __restrict__ obs,
                           uint32_t* __restrict__ mask, int)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_slot;
    for (;;) {
        lds_barrier();  // everyone has read the previous slot
        if (threadIdx.x == 0) s_slot = (int)atomicAdd(&S.queue[0], 1u);
        lds_barrier();
        const int k = s_slot;
        if (k >= S.E) break;
        env_step_one<RM, XM, APT>(P, S, S.order[k], act, gov, rew, gov_rew, done_out, obs, mask, smem);
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned int finished = atomicAdd(&S.queue[1], 1u);
        if (finished + 1 == gridDim.x) {  // every workgroup has drained the queue
            atomicExch(&S.queue[0], 0u);
            atomicExch(&S.queue[1], 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// observation of the current state (population rows, masks, government)
// ---------------------------------------------------------------------------
template <int RM, int XM, int APT>
__global__ void __launch_bounds__(1024 / APT)
env_observe_kernel(const EnvParams P, const EnvState S, uint16_t* __restrict__ obs, uint32_t* __restrict__ mask,
                   float* __restrict__ gov_obs)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int e = blockIdx.x;
    const int NT = blockDim.x, tid = threadIdx.x;
    const int NL = NT * APT;
    Lds L;
    lds_layout(P, NL, smem, &L);
    const int n = S.env_n[e];
    const int64_t off = S.env_off[e];
    const int64_t row0 = S.env_row[e];
    const int t = S.env_t[e];
    const int R = P.R, X = P.X, K = P.K, PX = P.P * P.X;
    const int S2 = next_pow2(NL);
    for (int j = tid; j < P.P; j += NT) L.prices[j] = P.prices[j];
    if (tid < K) L.rates[tid] = S.env_rates[e * K + tid];
    for (int j = tid; j < P.HB; j += NT) {
        L.hcnt[j] = 0;
        L.hexc[j] = 0;
    }
    lds_barrier();
    Agent<RM, XM> ag[APT];
    const int tX = t % X;
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int li = tid + k * NT;
        if (li >= n) continue;
        load_agent(P, S, off + li, ag[k]);
#pragma unroll
        for (int s = 0; s < XM; ++s) {
            uint32_t sl = ag[k].slot[s];
            if (s < X && slot_valid(sl)) {
                int side = slot_side(sl), r = slot_r(sl), p = slot_p(sl);
                const int age = slot_age(tX, s, X);
                atomicAdd(&L.hcnt[(r * 2 + side) * PX + bucket_pos(P, side, p, age)], 1);
            }
        }
    }
    lds_barrier();
    market_stats(P, L, nullptr, -1);
    lds_barrier();
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int li = tid + k * NT;
        if (li >= n) continue;
        write_obs_row(P, L, ag[k], t, obs + (row0 + li) * (int64_t)P.Ds);
        write_mask_row(P, L, ag[k], mask + (row0 + li) * (int64_t)P.W);
    }
    if (gov_obs == nullptr) return;
    float* g = gov_obs + (int64_t)e * P.Dg;
    for (int feat = 0; feat < 3 + R; ++feat) {
        lds_barrier();
        for (int j = tid; j < S2; j += NT) L.sortbuf[j] = INT64_MAX;
        lds_barrier();
        int64_t s1 = 0, s2 = 0;
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            const int li = tid + k * NT;
            if (li >= n) continue;
            const Agent<RM, XM>& a = ag[k];
            int64_t C = (int64_t)a.coin_inv + a.coin_esc;
            int64_t v = feat == 0 ? C : feat == 1 ? C - a.snap : feat == 2 ? (int64_t)a.labor
                                                                              : (int64_t)rget(a.res_inv, feat - 3);
            L.sortbuf[li] = v;
            s1 += v;
            s2 += v * v;
        }
        s1 = block_sum_i64(s1, L.red);
        s2 = block_sum_i64(s2, L.red + 16);
        bitonic_sort_i64(L.sortbuf, S2);
        if (tid == 0) {
            double mean = (double)s1 / (double)n;
            double var = (double)s2 / (double)n - mean * mean;
            if (var < 0.0) var = 0.0;
            g[3 * feat + 0] = (float)mean;
            g[3 * feat + 1] = (float)sqrt(var);
            g[3 * feat + 2] = (float)L.sortbuf[(n - 1) / 2];
        }
    }
    if (tid == 0) {
        int d = 3 * (3 + R);
        for (int b = 0; b < K; ++b) g[d++] = (float)L.rates[b] * P.sc.rate;
        g[d++] = (float)(t % P.P_tax) * P.sc.phase;
        for (int r = 0; r < R; ++r)
            for (int j = 0; j < 4; ++j) g[d++] = (float)L.mstat[4 * r + j];
    }
}

template <int RM, int XM, int APT>
__global__ void __launch_bounds__(1024 / APT) env_reset_kernel(const EnvParams P, const EnvState S, int ep)
{
    const int e = blockIdx.x;
    const int n = S.env_n[e];
    const int64_t off = S.env_off[e];
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int li = threadIdx.x + k * blockDim.x;
        if (li >= n) continue;
        Agent<RM, XM> ag;
        reset_agent(P, e, ep, li, ag);
        store_agent(P, S, off + li, ag, true);
        S.u[off + li] = __builtin_nan("");
    }
    if (threadIdx.x == 0) {
        S.env_t[e] = 0;
        S.env_ep[e] = ep;
        S.ug[e] = __builtin_nan("");
    }
    if ((int)threadIdx.x < P.K) S.env_rates[e * P.K + threadIdx.x] = 0;
    if (S.macc && (int)threadIdx.x < EJ_NACC) S.macc[(int64_t)e * EJ_NACC + threadIdx.x] = 0;  // a new episode
}

// record of the last completed episode of every economy, packed to 5 R + 9 doubles
__global__ void env_metrics_copy_kernel(const double* __restrict__ mlast, int E, int len, double* __restrict__ out)
{
    const int64_t n = (int64_t)E * len;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = i / len, j = i - e * len;
        out[i] = mlast[e * EJ_NMET + j];
    }
}

__global__ void env_random_actions_kernel(const EnvParams P, const EnvState S, uint64_t act_seed,
                                          int32_t* __restrict__ act, int32_t* __restrict__ gov)
{
    const int e = blockIdx.x;
    const int n = S.env_n[e];
    const int64_t row0 = S.env_row[e];
    const int t = S.env_t[e], ep = S.env_ep[e];
    if (act) {
        for (int li = threadIdx.x; li < n; li += blockDim.x) {
            u64x4 w = philox(act_seed, PURPOSE_ACT, (uint64_t)e, (uint64_t)ep, (uint64_t)t, (uint64_t)li);
            act[row0 + li] = (int32_t)(((w.x >> 32) * (uint64_t)P.A) >> 32);
        }
    }
    if ((int)threadIdx.x < P.K) {
        gov[e * P.K + threadIdx.x] = gov_level_draw(act_seed, e, ep, t, threadIdx.x);
    }
}

// government levels only: one thread per (economy, bracket)
__global__ void env_random_gov_kernel(const EnvParams P, const EnvState S, uint64_t act_seed, int32_t* __restrict__ gov)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S.E * P.K) return;
    const int e = j / P.K, b = j - e * P.K;
    gov[j] = gov_level_draw(act_seed, e, S.env_ep[e], S.env_t[e], b);
}

}  // namespace econ

// ===========================================================================
// host side: the handle and the C ABI
// ===========================================================================
using namespace econ;

struct ej_env {
    EnvParams P;
    int E = 0, NT = 64, APT = 1, variant = 0;  // variant 0: R<=4, X<=16; 1: R<=8, X<=32; 2: R<=16, X<=32
    int64_t M = 0;
    std::vector<int32_t> n, off, row;
    int32_t* d_field = nullptr;
    int32_t* d_t = nullptr;
    int32_t* d_ep = nullptr;
    int32_t* d_rates = nullptr;
    int32_t* d_n = nullptr;
    int32_t* d_off = nullptr;
    int32_t* d_row = nullptr;
    int64_t* d_invalid = nullptr;
    double* d_ug = nullptr;
    double* d_u = nullptr;
    unsigned int* d_queue = nullptr;
    int32_t* d_order = nullptr;
    int64_t* d_macc = nullptr;  // episode statistics (allocated by ej_env_enable_metrics)
    double* d_mlast = nullptr;
    int mode = 0, persistent_wg = 0;  // mode 0: one workgroup per economy; 1: persistent work queue
    size_t lds = 0;
    int step_NT = 64;      // workgroup size of the step: ceil(N / apw) waves
    size_t step_lds = 0;
    EnvState state() const
    {
        return EnvState{d_field, d_t, d_ep, d_rates, d_n,   d_off,   d_row, d_invalid,
                        d_ug,    d_u, d_queue, d_order, E, d_macc, d_mlast};
    }
};

static int choose_launch(ej_env* h, int apt)
{
    const int N = h->P.N;
    int nt = (N + apt - 1) / apt;
    nt = (nt + 63) / 64 * 64;
    if (nt > 1024 / apt) return EJ_EUNSUPPORTED;
    h->APT = apt;
    h->NT = nt;
    h->lds = lds_layout(h->P, nt * apt, nullptr, nullptr);
    h->P.apw = 64;
    h->step_NT = h->NT;
    h->step_lds = h->lds;
    return EJ_OK;
}

// step workgroup for `apw` agents per wavefront: ceil(N / apw) waves
static int choose_step_shape(ej_env* h, int apw)
{
    if (apw != 64 && apw != 32 && apw != 16) return EJ_EINVAL;
    const int waves = (h->P.N + apw - 1) / apw;
    if (waves * 64 > (h->variant == 2 ? 256 : 1024)) return EJ_EUNSUPPORTED;
    h->P.apw = apw;
    h->step_NT = waves * 64;
    h->step_lds = lds_layout(h->P, waves * apw * h->APT, nullptr, nullptr);
    return EJ_OK;
}

// Kernels are instantiated for one agent per thread (APT = 1): with several
// agents per thread the register arrays of the agent state spill.
#define EJ_DISPATCH(h, KERNEL, ...)                                                                        \
    do {                                                                                                    \
        if ((h)->variant == 0) KERNEL<4, 16, 1><<<(h)->E, (h)->NT, (h)->lds, st>>>(__VA_ARGS__);           \
        else if ((h)->variant == 1) KERNEL<8, 32, 1><<<(h)->E, (h)->NT, (h)->lds, st>>>(__VA_ARGS__);      \
        else KERNEL<16, 32, 1><<<(h)->E, (h)->NT, (h)->lds, st>>>(__VA_ARGS__);                            \
    } while (0)

extern "C" {

const char* ej_strerror(int code)
{
    switch (code) {
    case EJ_OK: return "ok";
    case EJ_EINVAL: return "invalid argument or configuration";
    case EJ_ENOMEM: return "out of memory";
    case EJ_EHIP: return "HIP runtime error";
    case EJ_EUNSUPPORTED: return "configuration outside the supported limits";
    case EJ_ESCRATCH: return "request larger than the static scratch of the allocation-free entry point";
    default: return "unknown error";
    }
}

int ej_last_hip_error(void) { return g_last_hip; }

static int validate(const ej_env_config* c)
{
    if (!c) return EJ_EINVAL;
    if (c->E <= 0 || c->N <= 0 || c->R <= 0 || c->P <= 0 || c->X <= 0 || c->P_tax <= 0 || c->T <= 0 || c->K < 0)
        return EJ_EINVAL;
    if (c->N > EJ_MAX_N || c->R > EJ_MAX_R || c->P > EJ_MAX_P || c->K > EJ_MAX_K || c->X > EJ_MAX_X)
        return EJ_EUNSUPPORTED;
    if ((int64_t)c->R * 2 * c->P * c->X > 8192) return EJ_EUNSUPPORTED;
    if (c->R_d < 0 || c->R_d > c->R || c->R_kappa < 1 || c->max_orders < 0 || c->start_coin < 0) return EJ_EINVAL;
    if (c->labor_gather < 0 || c->labor_craft < 0 || c->labor_trade < 0) return EJ_EINVAL;
    if (c->skill_mode & ~(EJ_SKILL_NORMAL | EJ_SKILL_GROWTH)) return EJ_EINVAL;
    if (!(c->eta >= 0.0) || c->eta == 1.0 || !(c->omega >= 0.0 && c->omega <= 1.0)) return EJ_EINVAL;
    for (int p = 0; p < c->P; ++p) {
        if (c->prices[p] <= 0) return EJ_EINVAL;
        if (p > 0 && c->prices[p] <= c->prices[p - 1]) return EJ_EINVAL;
    }
    for (int b = 0; b + 1 < c->K; ++b) {
        if (c->cutoffs[b] <= 0) return EJ_EINVAL;
        if (b > 0 && c->cutoffs[b] <= c->cutoffs[b - 1]) return EJ_EINVAL;
    }
    return EJ_OK;
}

int ej_env_create(const ej_env_config* cfg, const int32_t* h_n_per_env, ej_env** out)
{
    if (!out) return EJ_EINVAL;
    *out = nullptr;
    int rc = validate(cfg);
    if (rc != EJ_OK) return rc;
    ej_env* h = new (std::nothrow) ej_env();
    if (!h) return EJ_ENOMEM;
    EnvParams& P = h->P;
    std::memset(&P, 0, sizeof(P));
    P.N = cfg->N; P.R = cfg->R; P.P = cfg->P; P.X = cfg->X; P.max_orders = cfg->max_orders;
    // exact for every numerator below 2^27 (the error of the rounded-up multiplier stays below 1 / divisor)
    P.div_X = cfg->X > 0 ? 0xFFFFFFFFull / (uint64_t)cfg->X + 1ull : 0;
    P.div_P = cfg->P > 0 ? 0xFFFFFFFFull / (uint64_t)cfg->P + 1ull : 0;
    P.P_tax = cfg->P_tax; P.K = cfg->K; P.T = cfg->T; P.R_kappa = cfg->R_kappa; P.R_d = cfg->R_d;
    P.kappa_c = cfg->kappa_c; P.start_coin = cfg->start_coin; P.labor_gather = cfg->labor_gather;
    P.labor_craft = cfg->labor_craft; P.labor_trade = cfg->labor_trade; P.allow_noop = cfg->allow_noop;
    P.skill_mode = cfg->skill_mode;
    P.A = 2 + P.R + 2 * P.R * P.P;
    P.W = (P.A + 31) / 32;
    P.D = 7 + 7 * P.R + P.K;
    P.Ds = (P.D + 7) / 8 * 8;
    P.Dg = 3 * (3 + P.R) + P.K + 1 + 4 * P.R;
    P.HB = P.R * 2 * P.P * P.X;
    P.eta = cfg->eta; P.omega = cfg->omega; P.seed = cfg->seed;
    std::memcpy(P.prices, cfg->prices, sizeof(P.prices));
    std::memcpy(P.cutoffs, cfg->cutoffs, sizeof(P.cutoffs));
    P.sc = cfg->scales;
    h->E = cfg->E;
    h->variant = (P.R <= 4 && P.X <= 16) ? 0 : P.R <= 8 ? 1 : 2;
    h->n.resize(h->E);
    h->off.resize(h->E);
    h->row.resize(h->E + 1);
    int64_t slots = 0, rows = 0;
    for (int e = 0; e < h->E; ++e) {
        int ne = h_n_per_env ? h_n_per_env[e] : P.N;
        if (ne <= 0 || ne > P.N) {
            delete h;
            return EJ_EINVAL;
        }
        h->n[e] = ne;
        h->off[e] = (int32_t)slots;
        h->row[e] = (int32_t)rows;
        slots += (ne + 15) / 16 * 16;  // 64-byte aligned economies
        rows += ne;
    }
    h->row[h->E] = (int32_t)rows;
    if (slots > INT32_MAX || rows > INT32_MAX) {
        delete h;
        return EJ_EUNSUPPORTED;
    }
    h->M = rows;
    P.Ntot = slots;
    rc = choose_launch(h, 1);
    if (rc == EJ_OK && h->variant == 2 && h->NT > 256) rc = EJ_EUNSUPPORTED;  // R > 8: populations of <= 256
    if (rc != EJ_OK) {
        delete h;
        return rc;
    }
    const size_t nf = (size_t)n_fields(P.R, P.X);
    bool ok = hipMalloc(&h->d_field, nf * (size_t)slots * 4) == hipSuccess &&
              hipMalloc(&h->d_t, 4 * (size_t)h->E) == hipSuccess && hipMalloc(&h->d_ep, 4 * (size_t)h->E) == hipSuccess &&
              hipMalloc(&h->d_rates, 4 * (size_t)h->E * (size_t)(P.K > 0 ? P.K : 1)) == hipSuccess &&
              hipMalloc(&h->d_n, 4 * (size_t)h->E) == hipSuccess && hipMalloc(&h->d_off, 4 * (size_t)h->E) == hipSuccess &&
              hipMalloc(&h->d_row, 4 * (size_t)(h->E + 1)) == hipSuccess &&
              hipMalloc(&h->d_invalid, 16 * (size_t)h->E) == hipSuccess &&
              hipMalloc(&h->d_ug, 8 * (size_t)h->E) == hipSuccess && hipMalloc(&h->d_u, 8 * (size_t)slots) == hipSuccess &&
              hipMalloc(&h->d_queue, 8) == hipSuccess && hipMalloc(&h->d_order, 4 * (size_t)h->E) == hipSuccess;
    if (!ok) {
        ej_env_destroy(h);
        return EJ_ENOMEM;
    }
    if (hipMemcpy(h->d_n, h->n.data(), 4 * (size_t)h->E, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_off, h->off.data(), 4 * (size_t)h->E, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_row, h->row.data(), 4 * (size_t)(h->E + 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(h->d_invalid, 0, 16 * (size_t)h->E) != hipSuccess || hipMemset(h->d_queue, 0, 8) != hipSuccess ||
        hipMemset(h->d_u, 0xFF, 8 * (size_t)slots) != hipSuccess ||  // all-ones: NaN, utility not known
        hipMemset(h->d_field, 0, nf * (size_t)slots * 4) != hipSuccess) {
        set_last_hip_error(hipGetLastError());
        ej_env_destroy(h);
        return EJ_EHIP;
    }
    {
        // persistent-launch order: largest populations first (stable by index)
        std::vector<int32_t> order(h->E);
        for (int e = 0; e < h->E; ++e) order[e] = e;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return h->n[a] > h->n[b]; });
        if (hipMemcpy(h->d_order, order.data(), 4 * (size_t)h->E, hipMemcpyHostToDevice) != hipSuccess) {
            set_last_hip_error(hipGetLastError());
            ej_env_destroy(h);
            return EJ_EHIP;
        }
    }
    rc = ej_env_reset(h, 0, nullptr);
    if (rc == EJ_OK && hipDeviceSynchronize() != hipSuccess) rc = EJ_EHIP;
    if (rc != EJ_OK) {
        ej_env_destroy(h);
        return rc;
    }
    *out = h;
    return EJ_OK;
}

int ej_env_destroy(ej_env* h)
{
    if (!h) return EJ_EINVAL;
    (void)hipFree(h->d_field);
    (void)hipFree(h->d_t);
    (void)hipFree(h->d_ep);
    (void)hipFree(h->d_rates);
    (void)hipFree(h->d_n);
    (void)hipFree(h->d_off);
    (void)hipFree(h->d_row);
    (void)hipFree(h->d_invalid);
    (void)hipFree(h->d_ug);
    (void)hipFree(h->d_u);
    (void)hipFree(h->d_queue);
    (void)hipFree(h->d_order);
    (void)hipFree(h->d_macc);
    (void)hipFree(h->d_mlast);
    delete h;
    return EJ_OK;
}

int ej_env_dims(const ej_env* h, ej_env_dims_t* out)
{
    if (!h || !out) return EJ_EINVAL;
    out->M = h->M;
    out->A = h->P.A;
    out->mask_words = h->P.W;
    out->D = h->P.D;
    out->D_stride = h->P.Ds;
    out->D_gov = h->P.Dg;
    out->K = h->P.K;
    out->E = h->E;
    out->D_metrics = 5 * h->P.R + 9;
    return EJ_OK;
}

const int32_t* ej_env_row_offsets(const ej_env* h) { return h ? h->row.data() : nullptr; }

int ej_env_reset(ej_env* h, int32_t episode, void* stream)
{
    if (!h || episode < 0) return EJ_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    EnvState S = h->state();
    EJ_DISPATCH(h, env_reset_kernel, h->P, S, (int)episode);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

int ej_env_step(ej_env* h, const int32_t* d_act, const int32_t* d_gov, float* d_rew, float* d_gov_rew,
                uint8_t* d_done, uint16_t* d_obs, uint32_t* d_mask, void* stream)
{
    if (!h) return EJ_EINVAL;
    return ej_env_step_range(h, 0, h->E, d_act, d_gov, d_rew, d_gov_rew, d_done, d_obs, d_mask, stream);
}

int ej_env_step_range(ej_env* h, int32_t e_begin, int32_t e_end, const int32_t* d_act, const int32_t* d_gov,
                      float* d_rew, float* d_gov_rew, uint8_t* d_done, uint16_t* d_obs, uint32_t* d_mask,
                      void* stream)
{
    if (!h || !d_act || !d_rew || !d_gov_rew || !d_done) return EJ_EINVAL;
    if (e_begin < 0 || e_end > h->E || e_begin > e_end) return EJ_EINVAL;
    if (d_obs && !aligned16(d_obs)) return EJ_EINVAL;  // observation blocks leave in 16-byte stores
    if (e_begin == e_end) return EJ_OK;
    const bool whole = e_begin == 0 && e_end == h->E;
    if (h->P.K > 0 && !d_gov && !h->P.gov_draw) return EJ_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    EnvState S = h->state();
#define EJ_STEP_LAUNCH(KERNEL, G)                                                                            \
    do {                                                                                                     \
        const int nt = h->step_NT;                                                                           \
        const size_t lds = h->step_lds;                                                                      \
        const bool small = nt <= 256;                                                                        \
        if (h->variant == 0 && small)                                                                        \
            KERNEL<4, 16, 1, 256><<<G, nt, lds, st>>>(h->P, S, d_act, d_gov, d_rew, d_gov_rew, d_done, d_obs,  \
                                                      d_mask, e_begin);                                      \
        else if (h->variant == 0)                                                                            \
            KERNEL<4, 16, 1, 1024><<<G, nt, lds, st>>>(h->P, S, d_act, d_gov, d_rew, d_gov_rew, d_done, d_obs, \
                                                       d_mask, e_begin);                                     \
        else if (h->variant == 1 && small)                                                                   \
            KERNEL<8, 32, 1, 256><<<G, nt, lds, st>>>(h->P, S, d_act, d_gov, d_rew, d_gov_rew, d_done, d_obs,  \
                                                      d_mask, e_begin);                                      \
        else if (h->variant == 1)                                                                            \
            KERNEL<8, 32, 1, 1024><<<G, nt, lds, st>>>(h->P, S, d_act, d_gov, d_rew, d_gov_rew, d_done, d_obs, \
                                                       d_mask, e_begin);                                     \
        else /* variant 2: at most 256 threads (creation and choose_step_shape) */                           \
            KERNEL<16, 32, 1, 256><<<G, nt, lds, st>>>(h->P, S, d_act, d_gov, d_rew, d_gov_rew, d_done, d_obs, \
                                                       d_mask, e_begin);                                     \
    } while (0)
    if (h->mode == 1 && whole) {
        const unsigned G = (unsigned)h->persistent_wg;
        EJ_STEP_LAUNCH(env_step_persistent_kernel, G);
    } else {
        EJ_STEP_LAUNCH(env_step_kernel, (unsigned)(e_end - e_begin));
    }
#undef EJ_STEP_LAUNCH
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

int ej_env_set_gov_draw(ej_env* h, int32_t enabled, uint64_t seed)
{
    if (!h) return EJ_EINVAL;
    h->P.gov_draw = enabled != 0;
    h->P.gov_seed = seed;
    return EJ_OK;
}

int ej_env_set_launch(ej_env* h, int32_t mode, int32_t workgroups)
{
    if (!h || mode < 0 || mode > 1 || workgroups < 0) return EJ_EINVAL;
    if (mode == 1) {
        int dev = 0, cus = 0;
        EJ_HIP(hipGetDevice(&dev));
        EJ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        int g = workgroups > 0 ? workgroups : 2 * cus;
        if (g > h->E) g = h->E;
        h->persistent_wg = g;
    }
    h->mode = mode;
    return EJ_OK;
}

int ej_env_enable_metrics(ej_env* h, int32_t enabled)
{
    if (!h) return EJ_EINVAL;
    if (enabled && !h->d_macc) {
        const size_t E = (size_t)h->E;
        if (hipMalloc(&h->d_macc, 8 * E * EJ_NACC) != hipSuccess) return EJ_ENOMEM;
        if (hipMalloc(&h->d_mlast, 8 * E * EJ_NMET) != hipSuccess) {
            (void)hipFree(h->d_macc);
            h->d_macc = nullptr;
            return EJ_ENOMEM;
        }
        std::vector<double> rec(E * EJ_NMET, 0.0);
        for (size_t e = 0; e < E; ++e) rec[e * EJ_NMET] = -1.0;  // no episode completed yet
        EJ_HIP(hipMemset(h->d_macc, 0, 8 * E * EJ_NACC));
        EJ_HIP(hipMemcpy(h->d_mlast, rec.data(), 8 * E * EJ_NMET, hipMemcpyHostToDevice));
    }
    h->P.metrics = enabled ? 1 : 0;
    return EJ_OK;
}

int ej_env_episode_metrics(ej_env* h, double* d_out, void* stream)
{
    if (!h || !d_out || !h->d_mlast) return EJ_EINVAL;
    const int len = 5 * h->P.R + 9;
    const int64_t n = (int64_t)h->E * len;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    env_metrics_copy_kernel<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(h->d_mlast, h->E, len, d_out);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

int ej_env_set_agents_per_wave(ej_env* h, int32_t agents_per_wave)
{
    if (!h) return EJ_EINVAL;
    return choose_step_shape(h, agents_per_wave);
}

int ej_env_observe(ej_env* h, uint16_t* d_obs, uint32_t* d_mask, float* d_gov_obs, void* stream)
{
    if (!h || !d_obs || !d_mask) return EJ_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    EnvState S = h->state();
    EJ_DISPATCH(h, env_observe_kernel, h->P, S, d_obs, d_mask, d_gov_obs);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

int ej_env_random_actions(ej_env* h, uint64_t act_seed, int32_t* d_act, int32_t* d_gov, void* stream)
{
    if (!h || (h->P.K > 0 && !d_gov)) return EJ_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (d_act) {
        env_random_actions_kernel<<<h->E, 256, 0, st>>>(h->P, h->state(), act_seed, d_act, d_gov);
    } else {
        if (h->P.K == 0) return EJ_OK;
        const int64_t n = (int64_t)h->E * h->P.K;
        env_random_gov_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(h->P, h->state(), act_seed, d_gov);
    }
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

int ej_env_get_state(ej_env* h, const ej_state_view* v, void* stream)
{
    if (!h || !v) return EJ_EINVAL;
    const EnvParams& P = h->P;
    const int E = h->E, K = P.K, R = P.R, X = P.X;
    const size_t nf = (size_t)n_fields(R, X);
    std::vector<int32_t> f(nf * (size_t)P.Ntot), t(E), ep(E), rates((size_t)E * (K > 0 ? K : 1));
    EJ_HIP(hipStreamSynchronize((hipStream_t)stream));
    EJ_HIP(hipMemcpy(f.data(), h->d_field, f.size() * 4, hipMemcpyDeviceToHost));
    EJ_HIP(hipMemcpy(t.data(), h->d_t, 4 * (size_t)E, hipMemcpyDeviceToHost));
    EJ_HIP(hipMemcpy(ep.data(), h->d_ep, 4 * (size_t)E, hipMemcpyDeviceToHost));
    EJ_HIP(hipMemcpy(rates.data(), h->d_rates, rates.size() * 4, hipMemcpyDeviceToHost));
    const int64_t M = h->M, st = P.Ntot;
    for (int e = 0; e < E; ++e) {
        if (v->t) v->t[e] = t[e];
        if (v->ep) v->ep[e] = ep[e];
        if (v->rates)
            for (int b = 0; b < K; ++b) v->rates[(size_t)e * K + b] = rates[(size_t)e * K + b];
        for (int i = 0; i < h->n[e]; ++i) {
            const int64_t g = h->off[e] + i, rw = h->row[e] + i;
            if (v->coin_inv) v->coin_inv[rw] = f[F_COIN_INV() * st + g];
            if (v->coin_esc) v->coin_esc[rw] = f[F_COIN_ESC() * st + g];
            if (v->labor) v->labor[rw] = f[F_LABOR() * st + g];
            if (v->snap) v->snap[rw] = f[F_SNAP() * st + g];
            if (v->sc) v->sc[rw] = f[F_SC() * st + g];
            for (int r = 0; r < R; ++r) {
                if (v->res_inv) v->res_inv[r * M + rw] = f[F_RES_INV(R, r) * st + g];
                if (v->res_esc) v->res_esc[r * M + rw] = f[F_RES_ESC(R, r) * st + g];
                if (v->sg) v->sg[r * M + rw] = f[F_SG(R, r) * st + g];
            }
            for (int s = 0; s < X; ++s) {
                uint32_t sl = (uint32_t)f[F_SLOT(R, s) * st + g];
                if (v->orders)
                    v->orders[s * M + rw] = slot_valid(sl) ? slot_side(sl) + 2 * (slot_r(sl) + R * slot_p(sl)) : -1;
            }
        }
    }
    return EJ_OK;
}

int ej_env_set_state(ej_env* h, const ej_state_view* v, void* stream)
{
    if (!h || !v || !v->t || !v->ep || !v->coin_inv || !v->coin_esc || !v->labor || !v->snap || !v->sc ||
        !v->res_inv || !v->res_esc || !v->sg || !v->orders || (h->P.K > 0 && !v->rates))
        return EJ_EINVAL;
    const EnvParams& P = h->P;
    const int E = h->E, K = P.K, R = P.R, X = P.X;
    const size_t nf = (size_t)n_fields(R, X);
    const int64_t M = h->M, st = P.Ntot;
    std::vector<int32_t> f(nf * (size_t)P.Ntot, 0);
    for (int e = 0; e < E; ++e) {
        const int te = v->t[e];
        if (te < 0 || te >= P.T || v->ep[e] < 0) return EJ_EINVAL;
        const int n = h->n[e];
        // placement ranks of live orders: rank by (tie key, agent) within (t0, side, r, p)
        struct O {
            int i, s, code, t0;
            uint32_t key;
        };
        std::vector<O> orders;
        for (int i = 0; i < n; ++i) {
            const int64_t g = h->off[e] + i, rw = h->row[e] + i;
            f[F_COIN_INV() * st + g] = v->coin_inv[rw];
            f[F_COIN_ESC() * st + g] = v->coin_esc[rw];
            f[F_LABOR() * st + g] = v->labor[rw];
            f[F_SNAP() * st + g] = v->snap[rw];
            f[F_SC() * st + g] = v->sc[rw];
            for (int r = 0; r < R; ++r) {
                f[F_RES_INV(R, r) * st + g] = v->res_inv[r * M + rw];
                f[F_RES_ESC(R, r) * st + g] = v->res_esc[r * M + rw];
                f[F_SG(R, r) * st + g] = v->sg[r * M + rw];
            }
            for (int s = 0; s < X; ++s) {
                const int code = v->orders[s * M + rw];
                if (code < 0) continue;
                if ((code >> 1) >= R * P.P) return EJ_EINVAL;
                const int t0 = te - 1 - ((((te - 1 - s) % X) + X) % X);
                if (t0 < 0 || s == te % X) return EJ_EINVAL;
                u64x4 w = philox(P.seed, PURPOSE_ENV, (uint64_t)e, (uint64_t)v->ep[e], (uint64_t)t0, (uint64_t)i);
                orders.push_back(O{i, s, code, t0, (uint32_t)(w.y >> 32)});
            }
        }
        for (size_t a = 0; a < orders.size(); ++a) {
            int rank = 0;
            for (size_t b = 0; b < orders.size(); ++b) {
                if (orders[b].code != orders[a].code || orders[b].t0 != orders[a].t0) continue;
                rank += orders[b].key < orders[a].key || (orders[b].key == orders[a].key && orders[b].i < orders[a].i);
            }
            const O& o = orders[a];
            const int side = o.code & 1, r = (o.code >> 1) % R, p = (o.code >> 1) / R;
            f[F_SLOT(R, o.s) * st + h->off[e] + o.i] = (int32_t)slot_pack(side, r, p, rank);
        }
    }
    std::vector<int32_t> rates((size_t)E * (K > 0 ? K : 1), 0);
    for (size_t j = 0; j < (size_t)E * K; ++j) rates[j] = v->rates[j];
    EJ_HIP(hipStreamSynchronize((hipStream_t)stream));
    EJ_HIP(hipMemcpy(h->d_field, f.data(), f.size() * 4, hipMemcpyHostToDevice));
    EJ_HIP(hipMemcpy(h->d_t, v->t, 4 * (size_t)E, hipMemcpyHostToDevice));
    EJ_HIP(hipMemcpy(h->d_ep, v->ep, 4 * (size_t)E, hipMemcpyHostToDevice));
    EJ_HIP(hipMemcpy(h->d_rates, rates.data(), rates.size() * 4, hipMemcpyHostToDevice));
    std::vector<double> unknown((size_t)E, __builtin_nan(""));
    EJ_HIP(hipMemcpy(h->d_ug, unknown.data(), 8 * (size_t)E, hipMemcpyHostToDevice));
    EJ_HIP(hipMemset(h->d_u, 0xFF, 8 * (size_t)h->P.Ntot));  // all-ones: NaN, utility not known
    if (h->d_macc) EJ_HIP(hipMemset(h->d_macc, 0, 8 * (size_t)E * EJ_NACC));  // episode-to-date counts unknown
    return EJ_OK;
}

int ej_env_status(ej_env* h, int64_t* h_invalid_actions, int64_t* h_invalid_gov, void* stream)
{
    if (!h) return EJ_EINVAL;
    std::vector<int64_t> c(2 * (size_t)h->E);
    EJ_HIP(hipStreamSynchronize((hipStream_t)stream));
    EJ_HIP(hipMemcpy(c.data(), h->d_invalid, c.size() * 8, hipMemcpyDeviceToHost));
    int64_t a = 0, g = 0;
    for (int e = 0; e < h->E; ++e) {
        a += c[2 * e];
        g += c[2 * e + 1];
    }
    if (h_invalid_actions) *h_invalid_actions = a;
    if (h_invalid_gov) *h_invalid_gov = g;
    return EJ_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// autotuner: launch shapes of the rollout kernels, timed with HIP events
// ---------------------------------------------------------------------------
namespace {

// device copies of everything a trial step changes: the handle's state and
// the caller's per-step buffers; restored afterwards so tuning changes no result
struct Snapshot {
    struct Piece {
        void* dst;
        void* save;
        size_t bytes;
    };
    std::vector<Piece> pieces;
    hipStream_t st = nullptr;

    int add(void* p, size_t bytes)
    {
        if (!p || bytes == 0) return EJ_OK;
        void* save = nullptr;
        if (hipMalloc(&save, bytes) != hipSuccess) return EJ_ENOMEM;
        pieces.push_back({p, save, bytes});
        EJ_HIP(hipMemcpyAsync(save, p, bytes, hipMemcpyDeviceToDevice, st));
        return EJ_OK;
    }
    int restore()
    {
        for (auto& q : pieces) EJ_HIP(hipMemcpyAsync(q.dst, q.save, q.bytes, hipMemcpyDeviceToDevice, st));
        return EJ_OK;
    }
    ~Snapshot()
    {
        (void)hipStreamSynchronize(st);
        for (auto& q : pieces) (void)hipFree(q.save);
    }
};

template <typename F>
static int time_launches(F&& launch, int reps, hipStream_t st, float* ms)
{
    hipEvent_t a = nullptr, b = nullptr;
    EJ_HIP(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return EJ_EHIP;
    }
    int rc = launch();  // warm-up (first use of a shape)
    if (rc == EJ_OK && hipEventRecord(a, st) != hipSuccess) rc = EJ_EHIP;
    for (int i = 0; i < reps && rc == EJ_OK; ++i) rc = launch();
    if (rc == EJ_OK && hipEventRecord(b, st) != hipSuccess) rc = EJ_EHIP;
    if (rc == EJ_OK && hipEventSynchronize(b) != hipSuccess) rc = EJ_EHIP;
    float t = 0.f;
    if (rc == EJ_OK && hipEventElapsedTime(&t, a, b) != hipSuccess) rc = EJ_EHIP;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = t / (float)reps;
    return rc;
}

}  // namespace

extern "C" int ej_autotune(ej_env* h, ej_mlp_desc* m, const float* d_params, const uint16_t* d_work,
                           uint16_t* d_obs, uint32_t* d_mask, int32_t* d_act, const int32_t* d_gov, float* d_logp,
                           float* d_val, float* d_ent, float* d_rew, float* d_gov_rew, uint8_t* d_done, int32_t reps,
                           ej_autotune_result* out, void* stream)
{
    if (!out || !h || reps <= 0) return EJ_EINVAL;
    if (!d_obs || !d_mask || !d_act || !d_rew || !d_gov_rew || !d_done) return EJ_EINVAL;
    if (m && (!d_params || !d_work || !d_logp || !d_val || !d_ent)) return EJ_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    std::memset(out, 0, sizeof(*out));
    const EnvParams& P = h->P;
    const size_t slots = (size_t)P.Ntot, E = (size_t)h->E, M = (size_t)h->M;
    const size_t kk = (size_t)(P.K > 0 ? P.K : 1);
    int rc = EJ_OK;
    {
        Snapshot snap;  // everything a trial launch changes; restored below
        snap.st = st;
        if ((rc = snap.add(h->d_field, (size_t)n_fields(P.R, P.X) * slots * 4)) != EJ_OK ||
            (rc = snap.add(h->d_t, 4 * E)) != EJ_OK || (rc = snap.add(h->d_ep, 4 * E)) != EJ_OK ||
            (rc = snap.add(h->d_rates, 4 * E * kk)) != EJ_OK || (rc = snap.add(h->d_invalid, 16 * E)) != EJ_OK ||
            (rc = snap.add(h->d_ug, 8 * E)) != EJ_OK || (rc = snap.add(h->d_u, 8 * slots)) != EJ_OK ||
            (rc = snap.add(d_obs, 2 * M * (size_t)P.Ds)) != EJ_OK ||
            (rc = snap.add(d_mask, 4 * M * (size_t)P.W)) != EJ_OK || (rc = snap.add(d_act, 4 * M)) != EJ_OK ||
            (rc = snap.add(d_rew, 4 * M)) != EJ_OK || (rc = snap.add(d_gov_rew, 4 * E)) != EJ_OK ||
            (rc = snap.add(d_done, M)) != EJ_OK)
            return rc;
        if (m && ((rc = snap.add(d_logp, 4 * M)) != EJ_OK || (rc = snap.add(d_val, 4 * M)) != EJ_OK ||
                  (rc = snap.add(d_ent, 4 * M)) != EJ_OK))
            return rc;
        int dev = 0, cus = 0;
        EJ_HIP(hipGetDevice(&dev));
        EJ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const int old_mode = h->mode, old_wg = h->persistent_wg, old_apw = h->P.apw;
        float best = 3.4e38f;
        int bmode = old_mode, bwg = old_wg, bapw = old_apw;
        const int apws[3] = {64, 32, 16};
        const int wgs[4] = {0, cus, 2 * cus, 4 * cus};
        for (int ai = 0; ai < 3 && rc == EJ_OK; ++ai) {
            if (choose_step_shape(h, apws[ai]) != EJ_OK) continue;  // more than 16 waves per economy
            for (int wi = 0; wi < 4 && rc == EJ_OK; ++wi) {
                const int mode = wi == 0 ? 0 : 1;
                if ((rc = ej_env_set_launch(h, mode, wgs[wi])) != EJ_OK) break;
                float ms = 0.f;
                rc = time_launches([&] { return ej_env_step(h, d_act, d_gov, d_rew, d_gov_rew, d_done, d_obs,
                                                            d_mask, stream); },
                                   reps, st, &ms);
                if (rc != EJ_OK) break;
                ++out->candidates;
                if (ms < best) {
                    best = ms;
                    bmode = mode;
                    bwg = h->persistent_wg;
                    bapw = apws[ai];
                }
            }
        }
        if (rc != EJ_OK) {
            bmode = old_mode;
            bwg = old_wg;
            bapw = old_apw;
        }
        choose_step_shape(h, bapw);
        h->mode = bmode;
        h->persistent_wg = bwg;
        out->env_mode = bmode;
        out->env_workgroups = bmode == 1 ? bwg : 0;
        out->agents_per_wave = bapw;
        out->env_ms = best;
        if (m && rc == EJ_OK) {
            const int old_rows = m->tile_rows;
            float pbest = 3.4e38f;
            int brows = old_rows;
            const int cand[2] = {64, 128};
            for (int ci = 0; ci < 2 && rc == EJ_OK; ++ci) {
                if (cand[ci] == 128 && m->H > 256) continue;
                m->tile_rows = cand[ci];
                float ms = 0.f;
                rc = time_launches([&] { return ej_policy_forward(m, d_params, d_work, d_obs, d_mask, (int64_t)M, 0, 0,
                                                                  0, nullptr, d_act, d_logp, d_val, d_ent, nullptr,
                                                                  stream); },
                                   reps, st, &ms);
                if (rc != EJ_OK) break;
                ++out->candidates;
                if (ms < pbest) {
                    pbest = ms;
                    brows = cand[ci];
                }
            }
            m->tile_rows = rc == EJ_OK ? brows : old_rows;
            out->policy_tile_rows = m->tile_rows;
            out->policy_ms = pbest;
        }
        const int rc2 = snap.restore();
        if (rc == EJ_OK) rc = rc2;
    }  // the snapshot waits for the restore before it frees its copies
    return rc;
}
