/*
 * econ_oracle.c -- plain, slow, single-threaded CPU reference of the EconoJax
 * economy (Ponse, Plaat, van Stein, Moerland, "EconoJax: A Fast & Scalable
 * Economic Simulation in JAX", AAMAS 2025, arXiv 2410.22165).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  It shares no code, header, table or constant generator
 * with the HIP path, and nothing in the product may link or load it: only the
 * tests, the smoke check and the benchmark's CPU-baseline leg do.
 *
 * Every rule is written the straightforward way: the order book is a flat list
 * of order records, each market is cleared by sorting (qsort) and pairing, the
 * Gini numerator comes from a sorted copy.  Paper passages followed:
 *   Sec. 3 "Population Agents": one action per step; gathering floor(SG+rho),
 *     rho ~ U[0, 1.1); crafting R_kappa units of R_d types, fullest types
 *     first, coin = SC x constant; trading with escrow, best prices first,
 *     then older, then random; NOOP optional.
 *   Eq. (1), Eq. (2): isoelastic utility minus labor; reward = utility change.
 *   Sec. 3 "Government Agent": Eq. (3)-(5) social welfare = Eq * Prod.
 *   Sec. 3 "Setting tax rates": marginal brackets, 21 levels of 5 %, tax on
 *     the previous period's earnings, uniform redistribution; worked example
 *     (brackets [0,50),[50,100),[100,inf), rates 10/30/50 %, income 130 -> 35).
 *   Sec. 3 "Action masking"; Table 2 (defaults); Appendix A (a trade executes
 *     at the price of the order placed last).
 * Readings of passages the paper leaves open are the ones listed in the
 * design notes (Eq. (4) read as (1-w) + w(1-gini); integer coin; labor in
 * units of 1/20; Q16.16 skills; counter-based Philox4x64-10 randomness).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OC_MAXR 16
#define OC_MAXP 128
#define OC_MAXK 16

#define OC_PURPOSE_SKILL 1u
#define OC_PURPOSE_ENV 2u
#define OC_PURPOSE_ACT 3u
#define OC_PURPOSE_GOV 4u

typedef struct {
    int32_t N, R, P, X, max_orders, P_tax, K, T;
    int32_t R_kappa, R_d, kappa_c, start_coin;
    int32_t labor_gather, labor_craft, labor_trade; /* units of 1/20 labor */
    int32_t allow_noop;
    int32_t skill_mode; /* bit 0: skills ~ N(1, 1) clipped to [0, 5]; bit 1: skills grow with use */
    double eta, omega;
    int32_t prices[OC_MAXP];
    int32_t cutoffs[OC_MAXK];
} oc_config;

typedef struct {
    int32_t agent, side, r, p, t0; /* side 0 = buy (bid), 1 = sell (ask) */
    uint32_t key;
} oc_order;

typedef struct {
    oc_config c;
    uint64_t seed;
    int32_t e;
    int32_t t, ep;
    int32_t rates[OC_MAXK];
    int32_t *coin_inv, *coin_esc, *labor, *snap, *n_active, *sc; /* [N] */
    int32_t *res_inv, *res_esc, *sg;                             /* [R][N] */
    oc_order* book;
    int32_t n_book, cap_book;
    int64_t invalid_actions, invalid_gov;
    /* episode statistics: counts of this episode so far and the record of
     * the last completed one (layout at oc_env_episode_metrics) */
    int64_t macc[5 * OC_MAXR + 3];
    double mlast[5 * OC_MAXR + 9];
} oc_env;

/* ---------------------------------------------------------------------------
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplies with a
 * Weyl-sequence key schedule.
 * ------------------------------------------------------------------------- */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void oc_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(0xD2E7470EE14C6C93ull, c0, &hi0, &lo0);
        mulhilo64(0xCA5A826395121157ull, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint32_t purpose, uint64_t a, uint64_t b, uint64_t c, uint64_t d,
                 uint64_t out[4])
{
    uint64_t ctr[4] = {a, b, c, d};
    uint64_t key[2] = {seed, (uint64_t)purpose};
    oc_philox4x64(ctr, key, out);
}

/* ---------------------------------------------------------------------------
 * Small definitions, exported so the tests can pin them one by one.
 * ------------------------------------------------------------------------- */

/* Eq. (1): u = (C^(1-eta) - 1)/(1-eta) - L, with L = labor_q / 20. */
double oc_utility(int64_t coin, int64_t labor_q, double eta)
{
    double one_m = 1.0 - eta;
    return (pow((double)coin, one_m) - 1.0) / one_m - (double)labor_q / 20.0;
}

/* Gini index numerator over a sorted copy: sum_k (2k - N + 1) x_(k), 0-based
 * ascending ranks.  gini = numerator / (N * sum x); equal to the mean
 * absolute difference sum_i sum_j |x_i - x_j| / (2 N sum x). */
static int cmp_i64(const void* a, const void* b)
{
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

int64_t oc_gini_numerator(const int64_t* x, int32_t n)
{
    int64_t* s = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    memcpy(s, x, sizeof(int64_t) * (size_t)n);
    qsort(s, (size_t)n, sizeof(int64_t), cmp_i64);
    int64_t num = 0;
    for (int32_t k = 0; k < n; ++k) num += (int64_t)(2 * k - n + 1) * s[k];
    free(s);
    return num;
}

/* Eqs. (3)-(5): u_g = Eq * Prod, Prod = sum C, Eq = (1 - w) + w (1 - gini). */
double oc_social_welfare(const int64_t* coin, int32_t n, double omega)
{
    int64_t sum = 0;
    for (int32_t i = 0; i < n; ++i) sum += coin[i];
    double gini = 0.0;
    if (sum > 0) gini = (double)oc_gini_numerator(coin, n) / ((double)n * (double)sum);
    double eq = (1.0 - omega) + omega * (1.0 - gini);
    return eq * (double)sum;
}

/* Marginal bracket tax: rates in 5 % levels (0..20), cutoffs ascending; the
 * last bracket is open.  tax = floor(sum_b level_b * overlap_b / 20). */
int64_t oc_bracket_tax(int64_t income, const int32_t* levels, const int32_t* cutoffs, int32_t K)
{
    if (income <= 0 || K <= 0) return 0;
    int64_t acc = 0, lo = 0;
    for (int32_t b = 0; b < K; ++b) {
        int64_t hi = (b < K - 1) ? (int64_t)cutoffs[b] : INT64_MAX;
        int64_t top = income < hi ? income : hi;
        if (top > lo) acc += (int64_t)levels[b] * (top - lo);
        lo = hi;
        if (income <= hi) break;
    }
    return acc / 20;
}

int32_t oc_num_actions(int32_t R, int32_t P) { return 2 + R + 2 * R * P; }

/* ---------------------------------------------------------------------------
 * Environment life cycle.
 * ------------------------------------------------------------------------- */
#define AG(arr, j, i) ((arr)[(size_t)(j) * (size_t)env->c.N + (size_t)(i)])

static int32_t skill_q16_from_word(uint64_t w)
{
    /* Pareto(alpha = 4, x_m = 1) by inversion: x = U^(-1/4), U in (0, 1];
     * clipped to the skill maximum 5; stored in Q16.16 (round half up). */
    double u = (double)((w >> 11) + 1) * (1.0 / 9007199254740992.0);
    double x = 1.0 / sqrt(sqrt(u));
    if (x > 5.0) x = 5.0;
    return (int32_t)(x * 65536.0 + 0.5);
}

/* The multi-agent variant (Sec. 5): skills start near 1 with spread 1 and
 * grow by 0.5 % with every gather (that resource's skill) or craft (the
 * crafting skill), the bonus shrinking to zero at the maximum 5.
 *
 * Normal skills: the sum of twelve uniforms minus six, whose mean is 0 and
 * variance 1 (the classical uniform-sum approximation of the standard
 * normal, Irwin-Hall with n = 12), taken in exact integer arithmetic: twelve
 * 24-bit uniforms (the top 24 bits of both 32-bit halves of six words from
 * two draws) sum to S, and x = 1 + S / 2^24 - 6, i.e. x in Q16 =
 * floor(S / 2^8) - 5 * 2^16, clipped to [0, 5]. */
static int32_t normal_skill_q16(uint64_t seed, int32_t e, int32_t ep, int32_t i, int32_t s)
{
    uint64_t w0[4], w1[4];
    draw(seed, OC_PURPOSE_SKILL, (uint64_t)e, (uint64_t)ep, (uint64_t)i, (uint64_t)(64 + 2 * s), w0);
    draw(seed, OC_PURPOSE_SKILL, (uint64_t)e, (uint64_t)ep, (uint64_t)i, (uint64_t)(65 + 2 * s), w1);
    uint64_t words[6] = {w0[0], w0[1], w0[2], w0[3], w1[0], w1[1]};
    int64_t S = 0;
    for (int k = 0; k < 6; ++k) {
        S += (int64_t)(words[k] >> 40);                  /* top 24 bits of the high half */
        S += (int64_t)((words[k] & 0xFFFFFFFFull) >> 8); /* top 24 bits of the low half */
    }
    int64_t q = (S >> 8) - 5 * 65536;
    if (q < 0) q = 0;
    if (q > 5 * 65536) q = 5 * 65536;
    return (int32_t)q;
}

/* s <- s + 0.005 s (1 - s / 5), rounded down in Q16: the 0.5 % bonus times
 * the remaining fraction of the range up to 5 (never above 5). */
static int32_t grown_skill_q16(int32_t s)
{
    const int64_t smax = 5 * 65536;
    int64_t d = ((int64_t)s * (smax - (int64_t)s)) / (200 * smax);
    int64_t v = (int64_t)s + (d > 0 ? d : 0);
    return (int32_t)(v > smax ? smax : v);
}

static void reset_episode_state(oc_env* env)
{
    const oc_config* c = &env->c;
    env->t = 0;
    for (int b = 0; b < OC_MAXK; ++b) env->rates[b] = 0;
    for (int32_t i = 0; i < c->N; ++i) {
        env->coin_inv[i] = c->start_coin;
        env->coin_esc[i] = 0;
        env->labor[i] = 0;
        env->snap[i] = c->start_coin;
        env->n_active[i] = 0;
        for (int32_t r = 0; r < c->R; ++r) {
            AG(env->res_inv, r, i) = 0;
            AG(env->res_esc, r, i) = 0;
        }
        /* skill word s: s < R -> gathering skill of resource s; s == R -> crafting */
        for (int32_t s = 0; s <= c->R; ++s) {
            uint64_t out[4];
            draw(env->seed, OC_PURPOSE_SKILL, (uint64_t)env->e, (uint64_t)env->ep, (uint64_t)i,
                 (uint64_t)(s / 4), out);
            int32_t q = (c->skill_mode & 1) ? normal_skill_q16(env->seed, env->e, env->ep, i, s)
                                            : skill_q16_from_word(out[s % 4]);
            if (s < c->R) AG(env->sg, s, i) = q;
            else env->sc[i] = q;
        }
    }
    env->n_book = 0;
    for (int j = 0; j < 5 * OC_MAXR + 3; ++j) env->macc[j] = 0;
}

oc_env* oc_env_create(const oc_config* cfg, uint64_t seed, int32_t e)
{
    oc_env* env = (oc_env*)calloc(1, sizeof(oc_env));
    env->c = *cfg;
    env->seed = seed;
    env->e = e;
    size_t n = (size_t)cfg->N, nr = (size_t)cfg->N * (size_t)cfg->R;
    env->coin_inv = (int32_t*)calloc(n, 4);
    env->coin_esc = (int32_t*)calloc(n, 4);
    env->labor = (int32_t*)calloc(n, 4);
    env->snap = (int32_t*)calloc(n, 4);
    env->n_active = (int32_t*)calloc(n, 4);
    env->sc = (int32_t*)calloc(n, 4);
    env->res_inv = (int32_t*)calloc(nr, 4);
    env->res_esc = (int32_t*)calloc(nr, 4);
    env->sg = (int32_t*)calloc(nr, 4);
    env->cap_book = cfg->N * (cfg->X + 1) + 16;
    env->book = (oc_order*)calloc((size_t)env->cap_book, sizeof(oc_order));
    env->ep = 0;
    reset_episode_state(env);
    for (int j = 0; j < 5 * OC_MAXR + 9; ++j) env->mlast[j] = 0.0;
    env->mlast[0] = -1.0;
    return env;
}

void oc_env_destroy(oc_env* env)
{
    if (!env) return;
    free(env->coin_inv); free(env->coin_esc); free(env->labor); free(env->snap);
    free(env->n_active); free(env->sc); free(env->res_inv); free(env->res_esc);
    free(env->sg); free(env->book); free(env);
}

/* Restart at episode `ep` (fresh skills from the counter-based generator). */
void oc_env_reset(oc_env* env, int32_t ep)
{
    env->ep = ep;
    reset_episode_state(env);
}

/* ---------------------------------------------------------------------------
 * Action decoding.  0 = NOOP, 1..R = gather r, R+1 = craft,
 * R+2 + r P + p = buy (r, p), R+2 + R P + r P + p = sell (r, p).
 * ------------------------------------------------------------------------- */
enum { A_NOOP = 0, A_GATHER = 1, A_CRAFT = 2, A_BUY = 3, A_SELL = 4 };

static void decode(const oc_config* c, int32_t a, int32_t* type, int32_t* r, int32_t* p)
{
    *r = 0; *p = 0;
    if (a == 0) { *type = A_NOOP; return; }
    if (a >= 1 && a <= c->R) { *type = A_GATHER; *r = a - 1; return; }
    if (a == c->R + 1) { *type = A_CRAFT; return; }
    int32_t b = a - (c->R + 2);
    if (b < c->R * c->P) { *type = A_BUY; *r = b / c->P; *p = b % c->P; return; }
    b -= c->R * c->P;
    *type = A_SELL; *r = b / c->P; *p = b % c->P;
}

static int craft_possible(const oc_env* env, int32_t i)
{
    int32_t n_ok = 0;
    for (int32_t r = 0; r < env->c.R; ++r)
        if (AG(env->res_inv, r, i) >= env->c.R_kappa) ++n_ok;
    return n_ok >= env->c.R_d;
}

/* Action mask of agent i on the current state (Sec. 3 "Action masking"). */
static int action_valid(const oc_env* env, int32_t i, int32_t a)
{
    const oc_config* c = &env->c;
    if (a < 0 || a >= oc_num_actions(c->R, c->P)) return 0;
    int32_t type, r, p;
    decode(c, a, &type, &r, &p);
    switch (type) {
    case A_NOOP: return c->allow_noop != 0;
    case A_GATHER: return 1;
    case A_CRAFT: return craft_possible(env, i);
    case A_BUY: return env->n_active[i] < c->max_orders && env->coin_inv[i] >= c->prices[p];
    default: return env->n_active[i] < c->max_orders && AG(env->res_inv, r, i) >= 1;
    }
}

/* ---------------------------------------------------------------------------
 * Market clearing (Sec. 3 "Trading", Appendix A).
 * ------------------------------------------------------------------------- */
static const oc_order* g_sort_book;

static int cmp_bid(const void* a, const void* b)
{
    const oc_order* x = &g_sort_book[*(const int32_t*)a];
    const oc_order* y = &g_sort_book[*(const int32_t*)b];
    if (x->p != y->p) return x->p > y->p ? -1 : 1; /* higher bid first */
    if (x->t0 != y->t0) return x->t0 < y->t0 ? -1 : 1; /* older first */
    if (x->key != y->key) return x->key < y->key ? -1 : 1; /* then at random */
    return x->agent < y->agent ? -1 : (x->agent > y->agent);
}

static int cmp_ask(const void* a, const void* b)
{
    const oc_order* x = &g_sort_book[*(const int32_t*)a];
    const oc_order* y = &g_sort_book[*(const int32_t*)b];
    if (x->p != y->p) return x->p < y->p ? -1 : 1; /* lower ask first */
    if (x->t0 != y->t0) return x->t0 < y->t0 ? -1 : 1;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->agent < y->agent ? -1 : (x->agent > y->agent);
}

/* Placement order: (t0, key, agent) ascending; the larger one was placed last. */
static int placed_later(const oc_order* x, const oc_order* y)
{
    if (x->t0 != y->t0) return x->t0 > y->t0;
    if (x->key != y->key) return x->key > y->key;
    return x->agent > y->agent;
}

/* Clears one resource of a flat list of orders.  `filled[j]` is set for
 * orders that trade; `price_paid[j]` receives the trade price (the price of
 * the later-placed order of the pair); `partner[j]` the index of the other
 * order.  Returns the number of trades.  Exported for the matching tests. */
int32_t oc_clear_orders(const oc_order* book, int32_t n, int32_t r, const int32_t* prices,
                        int32_t* filled, int32_t* price_paid, int32_t* partner)
{
    int32_t* bids = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t* asks = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t nb = 0, na = 0;
    for (int32_t j = 0; j < n; ++j) {
        filled[j] = 0; price_paid[j] = 0; partner[j] = -1;
        if (book[j].r != r) continue;
        if (book[j].side == 0) bids[nb++] = j;
        else asks[na++] = j;
    }
    g_sort_book = book;
    qsort(bids, (size_t)nb, sizeof(int32_t), cmp_bid);
    qsort(asks, (size_t)na, sizeof(int32_t), cmp_ask);
    int32_t k = 0;
    while (k < nb && k < na && prices[book[bids[k]].p] >= prices[book[asks[k]].p]) {
        const oc_order* b = &book[bids[k]];
        const oc_order* s = &book[asks[k]];
        int32_t q = placed_later(b, s) ? prices[b->p] : prices[s->p];
        filled[bids[k]] = 1; filled[asks[k]] = 1;
        price_paid[bids[k]] = q; price_paid[asks[k]] = q;
        partner[bids[k]] = asks[k]; partner[asks[k]] = bids[k];
        ++k;
    }
    free(bids); free(asks);
    return k;
}

static void remove_order(oc_env* env, int32_t j)
{
    env->book[j] = env->book[env->n_book - 1];
    env->n_book -= 1;
}

/* ---------------------------------------------------------------------------
 * One environment step.  Order of sub-steps:
 *   utilities of the step-start state; action validation against the
 *   step-start mask (invalid -> NOOP, no labor); government rates at the
 *   first step of a period; every agent's action; clearing of every market;
 *   expiry of orders that have lived X clearings; tax collection and
 *   redistribution at the last step of a period; rewards; time advance with
 *   automatic reset at the episode end.
 * ------------------------------------------------------------------------- */
/* ---------------------------------------------------------------------------
 * Episode statistics, the measures the paper reports at the end of an
 * episode (Sec. 4 results): productivity (Eq. (5)), equality 1 - gini, the
 * government utility Eq * Prod (Eq. (3)), the mean and median episode
 * return of the population, the distribution of actions taken and the
 * trades and their prices per resource.  The return of an agent over an
 * episode is the sum of its rewards, i.e. (Eq. (2) telescopes) its utility
 * at the end minus its utility at the reset state.
 * Record (doubles): [0] index of the episode, [1] Prod, [2] 1 - gini,
 * [3] Eq * Prod, [4] mean return, [5] lower median return, [6 + j] actions of
 * category j (j = 0 NOOP, 1 + r gather r, 1 + R craft, 2 + R + r buy r,
 * 2 + 2R + r sell r, 2 + 3R rejected), [9 + 3R + r] trades of resource r,
 * [9 + 4R + r] the sum of their prices.
 * ------------------------------------------------------------------------- */
static int cmp_f64(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

static void episode_record(oc_env* env, const int64_t* coins, double ug)
{
    const oc_config* c = &env->c;
    const int32_t N = c->N, R = c->R;
    int64_t prod = 0;
    for (int32_t i = 0; i < N; ++i) prod += coins[i];
    double gini = prod > 0 ? (double)oc_gini_numerator(coins, N) / ((double)N * (double)prod) : 0.0;
    double u_start = oc_utility(c->start_coin, 0, c->eta);
    double* ret = (double*)malloc(sizeof(double) * (size_t)N);
    double sum = 0.0;
    for (int32_t i = 0; i < N; ++i) {
        ret[i] = oc_utility(coins[i], env->labor[i], c->eta) - u_start;
        sum += ret[i];
    }
    qsort(ret, (size_t)N, sizeof(double), cmp_f64);
    double* m = env->mlast;
    m[0] = (double)env->ep;
    m[1] = (double)prod;
    m[2] = 1.0 - gini;
    m[3] = ug;
    m[4] = sum / (double)N;
    m[5] = ret[(N - 1) / 2];
    for (int32_t j = 0; j < 5 * R + 3; ++j) m[6 + j] = (double)env->macc[j];
    free(ret);
}

int32_t oc_metrics_len(int32_t R) { return 5 * R + 9; }

void oc_env_episode_metrics(const oc_env* env, double* out)
{
    memcpy(out, env->mlast, sizeof(double) * (size_t)oc_metrics_len(env->c.R));
}

int32_t oc_env_step(oc_env* env, const int32_t* act, const int32_t* gov, float* rew, float* gov_rew,
                    int32_t* done)
{
    const oc_config* c = &env->c;
    const int32_t N = c->N, R = c->R, t = env->t;
    double* u0 = (double*)malloc(sizeof(double) * (size_t)N);
    int64_t* coins = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    int32_t* eff = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);

    /* utilities at the start of the step (Eq. (1), Eqs. (3)-(5)) */
    for (int32_t i = 0; i < N; ++i) {
        coins[i] = (int64_t)env->coin_inv[i] + env->coin_esc[i];
        u0[i] = oc_utility(coins[i], env->labor[i], c->eta);
    }
    double ug0 = oc_social_welfare(coins, N, c->omega);

    /* validation against the step-start state; every agent's action is
     * counted in its category for the episode statistics */
    for (int32_t i = 0; i < N; ++i) {
        if (action_valid(env, i, act[i])) {
            int32_t type, r, p;
            eff[i] = act[i];
            decode(c, eff[i], &type, &r, &p);
            int32_t cat = type == A_NOOP ? 0 : type == A_GATHER ? 1 + r : type == A_CRAFT ? 1 + R
                          : type == A_BUY ? 2 + R + r : 2 + 2 * R + r;
            env->macc[cat] += 1;
        } else {
            eff[i] = 0;
            env->invalid_actions += 1;
            env->macc[2 + 3 * R] += 1;
        }
    }

    /* government: new rates at the first step of each period */
    if (c->K > 0 && t % c->P_tax == 0) {
        for (int32_t b = 0; b < c->K; ++b) {
            if (gov[b] >= 0 && gov[b] <= 20) env->rates[b] = gov[b];
            else env->invalid_gov += 1;
        }
    }

    /* population actions */
    for (int32_t i = 0; i < N; ++i) {
        int32_t type, r, p;
        decode(c, eff[i], &type, &r, &p);
        if (type == A_NOOP) continue;
        if (type == A_GATHER) {
            uint64_t w[4];
            draw(env->seed, OC_PURPOSE_ENV, (uint64_t)env->e, (uint64_t)env->ep, (uint64_t)t,
                 (uint64_t)i, w);
            /* rho uniform in [0, 1.1) in Q16: 1.1 * 65536 = 72090 (rounded) */
            int64_t rho_q = (int64_t)(((w[0] >> 32) * 72090ull) >> 32);
            int64_t amount = ((int64_t)AG(env->sg, r, i) + rho_q) >> 16; /* floor(SG + rho) */
            AG(env->res_inv, r, i) += (int32_t)amount;
            env->labor[i] += c->labor_gather;
            if (c->skill_mode & 2) AG(env->sg, r, i) = grown_skill_q16(AG(env->sg, r, i));
        } else if (type == A_CRAFT) {
            /* pick R_d types with at least R_kappa units, fullest first, ties to the lower id */
            int32_t used[OC_MAXR] = {0};
            for (int32_t k = 0; k < c->R_d; ++k) {
                int32_t best = -1;
                for (int32_t q = 0; q < R; ++q) {
                    if (used[q] || AG(env->res_inv, q, i) < c->R_kappa) continue;
                    if (best < 0 || AG(env->res_inv, q, i) > AG(env->res_inv, best, i)) best = q;
                }
                used[best] = 1;
                AG(env->res_inv, best, i) -= c->R_kappa;
            }
            env->coin_inv[i] += (int32_t)(((int64_t)env->sc[i] * c->kappa_c) >> 16);
            env->labor[i] += c->labor_craft;
            if (c->skill_mode & 2) env->sc[i] = grown_skill_q16(env->sc[i]);
        } else {
            uint64_t w[4];
            draw(env->seed, OC_PURPOSE_ENV, (uint64_t)env->e, (uint64_t)env->ep, (uint64_t)t,
                 (uint64_t)i, w);
            oc_order o;
            o.agent = i; o.side = (type == A_SELL); o.r = r; o.p = p; o.t0 = t;
            o.key = (uint32_t)(w[1] >> 32);
            if (type == A_BUY) {
                env->coin_inv[i] -= c->prices[p];
                env->coin_esc[i] += c->prices[p];
            } else {
                AG(env->res_inv, r, i) -= 1;
                AG(env->res_esc, r, i) += 1;
            }
            env->book[env->n_book++] = o;
            env->n_active[i] += 1;
            env->labor[i] += c->labor_trade;
        }
    }

    /* clear every market */
    if (env->n_book > 0) {
        int32_t* filled = (int32_t*)malloc(sizeof(int32_t) * (size_t)env->n_book);
        int32_t* paid = (int32_t*)malloc(sizeof(int32_t) * (size_t)env->n_book);
        int32_t* partner = (int32_t*)malloc(sizeof(int32_t) * (size_t)env->n_book);
        for (int32_t r = 0; r < R; ++r) {
            oc_clear_orders(env->book, env->n_book, r, c->prices, filled, paid, partner);
            for (int32_t j = 0; j < env->n_book; ++j) {
                if (!filled[j]) continue;
                const oc_order* o = &env->book[j];
                int32_t i = o->agent;
                if (o->side == 0) { /* buyer: escrowed bid price leaves, change returned */
                    env->coin_esc[i] -= c->prices[o->p];
                    env->coin_inv[i] += c->prices[o->p] - paid[j];
                    AG(env->res_inv, o->r, i) += 1;
                    env->macc[3 + 3 * R + o->r] += 1;        /* one trade, counted on its bid */
                    env->macc[3 + 4 * R + o->r] += paid[j];  /* at its price */
                } else { /* seller: escrowed unit leaves, trade price received */
                    AG(env->res_esc, o->r, i) -= 1;
                    env->coin_inv[i] += paid[j];
                }
                env->n_active[i] -= 1;
            }
            for (int32_t j = env->n_book - 1; j >= 0; --j) /* descending keeps indices valid */
                if (filled[j]) remove_order(env, j);
            /* removal reorders the list, so refresh the flags for the next resource */
            for (int32_t j = 0; j < env->n_book; ++j) filled[j] = 0;
        }
        free(filled); free(paid); free(partner);
    }

    /* expiry: an order placed at t0 takes part in clearings t0 .. t0 + X - 1 */
    for (int32_t j = env->n_book - 1; j >= 0; --j) {
        const oc_order* o = &env->book[j];
        if (o->t0 != t - c->X + 1) continue;
        int32_t i = o->agent;
        if (o->side == 0) {
            env->coin_esc[i] -= c->prices[o->p];
            env->coin_inv[i] += c->prices[o->p];
        } else {
            AG(env->res_esc, o->r, i) -= 1;
            AG(env->res_inv, o->r, i) += 1;
        }
        env->n_active[i] -= 1;
        remove_order(env, j);
    }

    /* tax collection and redistribution at the last step of a period */
    if ((t + 1) % c->P_tax == 0) {
        if (c->K > 0) {
            int64_t pool = 0;
            for (int32_t i = 0; i < N; ++i) {
                int64_t C = (int64_t)env->coin_inv[i] + env->coin_esc[i];
                int64_t income = C - env->snap[i];
                int64_t tax = oc_bracket_tax(income, env->rates, c->cutoffs, c->K);
                if (tax > env->coin_inv[i]) tax = env->coin_inv[i]; /* escrow is not taxed */
                env->coin_inv[i] -= (int32_t)tax;
                pool += tax;
            }
            int64_t period = t / c->P_tax;
            int64_t share = pool / N, rem = pool % N;
            for (int32_t i = 0; i < N; ++i) {
                int64_t rot = (((int64_t)i - period) % N + N) % N;
                env->coin_inv[i] += (int32_t)(share + (rot < rem ? 1 : 0));
            }
        }
        for (int32_t i = 0; i < N; ++i) env->snap[i] = env->coin_inv[i] + env->coin_esc[i];
    }

    /* rewards: change of utility (Eq. (2)), fp64 difference rounded to fp32 */
    for (int32_t i = 0; i < N; ++i) {
        coins[i] = (int64_t)env->coin_inv[i] + env->coin_esc[i];
        double u1 = oc_utility(coins[i], env->labor[i], c->eta);
        rew[i] = (float)(u1 - u0[i]);
    }
    double ug1 = oc_social_welfare(coins, N, c->omega);
    *gov_rew = (float)(ug1 - ug0);

    /* time advance, automatic reset at the episode end */
    env->t = t + 1;
    *done = 0;
    if (env->t >= c->T) {
        episode_record(env, coins, ug1);
        *done = 1;
        env->ep += 1;
        reset_episode_state(env);
    }
    free(u0); free(coins); free(eff);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Observations (the layout is this project's proposal: the paper's figure
 * that lists the observation space is not available; Sec. 3, Appendix A say
 * the market part holds highest / lowest prices and numbers of orders, and
 * the government sees population mean / std / median).
 * ------------------------------------------------------------------------- */
static uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7fffu + lsb) >> 16);
}

int32_t oc_obs_dim(int32_t R, int32_t K) { return 7 + 7 * R + K; }
int32_t oc_gov_obs_dim(int32_t R, int32_t K) { return 3 * (3 + R) + K + 1 + 4 * R; }

/* market statistics of resource r: best bid, best ask (0 if none), counts */
static void market_stats(const oc_env* env, int32_t r, int32_t* best_bid, int32_t* best_ask,
                         int32_t* n_bid, int32_t* n_ask)
{
    *best_bid = 0; *best_ask = 0; *n_bid = 0; *n_ask = 0;
    for (int32_t j = 0; j < env->n_book; ++j) {
        const oc_order* o = &env->book[j];
        if (o->r != r) continue;
        int32_t pr = env->c.prices[o->p];
        if (o->side == 0) {
            if (*n_bid == 0 || pr > *best_bid) *best_bid = pr;
            *n_bid += 1;
        } else {
            if (*n_ask == 0 || pr < *best_ask) *best_ask = pr;
            *n_ask += 1;
        }
    }
}

/* Population observation rows (bf16 bits, row stride `stride` >= D, zero
 * padded) and action-mask bits (W = ceil(A/32) words per row).  Feature
 * scales: the caller passes the float scale of every feature group. */
typedef struct {
    float coin, labor, orders, res, skill, rate, phase, price, count;
} oc_obs_scales;

void oc_env_observe(const oc_env* env, const oc_obs_scales* s, int32_t stride, uint16_t* obs,
                    uint32_t* mask, float* gov_obs)
{
    const oc_config* c = &env->c;
    const int32_t N = c->N, R = c->R, K = c->K, A = oc_num_actions(R, c->P);
    const int32_t W = (A + 31) / 32;
    int32_t bb[OC_MAXR], ba[OC_MAXR], nb[OC_MAXR], na[OC_MAXR];
    for (int32_t r = 0; r < R; ++r) market_stats(env, r, &bb[r], &ba[r], &nb[r], &na[r]);
    float* f = (float*)malloc(sizeof(float) * (size_t)(oc_obs_dim(R, K) + 1));
    for (int32_t i = 0; i < N; ++i) {
        int32_t d = 0;
        int32_t C = env->coin_inv[i] + env->coin_esc[i];
        f[d++] = (float)env->coin_inv[i] * s->coin;
        f[d++] = (float)env->coin_esc[i] * s->coin;
        f[d++] = (float)env->labor[i] * s->labor;
        f[d++] = (float)env->n_active[i] * s->orders;
        f[d++] = (float)(C - env->snap[i]) * s->coin;
        for (int32_t r = 0; r < R; ++r) f[d++] = (float)AG(env->res_inv, r, i) * s->res;
        for (int32_t r = 0; r < R; ++r) f[d++] = (float)AG(env->res_esc, r, i) * s->res;
        for (int32_t r = 0; r < R; ++r) f[d++] = (float)AG(env->sg, r, i) * s->skill;
        f[d++] = (float)env->sc[i] * s->skill;
        for (int32_t b = 0; b < K; ++b) f[d++] = (float)env->rates[b] * s->rate;
        f[d++] = (float)(env->t % c->P_tax) * s->phase;
        for (int32_t r = 0; r < R; ++r) {
            f[d++] = (float)bb[r] * s->price;
            f[d++] = (float)ba[r] * s->price;
            f[d++] = (float)nb[r] * s->count;
            f[d++] = (float)na[r] * s->count;
        }
        for (int32_t k = 0; k < stride; ++k)
            obs[(size_t)i * (size_t)stride + (size_t)k] = k < d ? f32_to_bf16_rne(f[k]) : 0;
        for (int32_t w = 0; w < W; ++w) mask[(size_t)i * (size_t)W + (size_t)w] = 0;
        for (int32_t a = 0; a < A; ++a)
            if (action_valid(env, i, a)) mask[(size_t)i * (size_t)W + (size_t)(a / 32)] |= 1u << (a % 32);
    }
    free(f);
    if (!gov_obs) return;
    /* government: mean, std (population), lower median of coin, period income,
     * labor (in units of 1/20) and every resource inventory */
    int64_t* x = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    int32_t d = 0;
    for (int32_t feat = 0; feat < 3 + R; ++feat) {
        int64_t s1 = 0, s2 = 0;
        for (int32_t i = 0; i < N; ++i) {
            int64_t C = (int64_t)env->coin_inv[i] + env->coin_esc[i];
            int64_t v;
            if (feat == 0) v = C;
            else if (feat == 1) v = C - env->snap[i];
            else if (feat == 2) v = env->labor[i];
            else v = AG(env->res_inv, feat - 3, i);
            x[i] = v; s1 += v; s2 += v * v;
        }
        qsort(x, (size_t)N, sizeof(int64_t), cmp_i64);
        double mean = (double)s1 / (double)N;
        double var = (double)s2 / (double)N - mean * mean;
        if (var < 0.0) var = 0.0;
        gov_obs[d++] = (float)mean;
        gov_obs[d++] = (float)sqrt(var);
        gov_obs[d++] = (float)x[(N - 1) / 2];
    }
    for (int32_t b = 0; b < K; ++b) gov_obs[d++] = (float)env->rates[b] * s->rate;
    gov_obs[d++] = (float)(env->t % c->P_tax) * s->phase;
    for (int32_t r = 0; r < R; ++r) {
        gov_obs[d++] = (float)bb[r];
        gov_obs[d++] = (float)ba[r];
        gov_obs[d++] = (float)nb[r];
        gov_obs[d++] = (float)na[r];
    }
    free(x);
}

/* ---------------------------------------------------------------------------
 * State export in a representation-neutral form: every int32 field, and per
 * (slot s = t0 mod X, agent) the live order as side + 2 (r + R p), or -1.
 * ------------------------------------------------------------------------- */
void oc_env_get_state(const oc_env* env, int32_t* scalars /* t, ep, rates[K] */, int32_t* coin_inv,
                      int32_t* coin_esc, int32_t* labor, int32_t* snap, int32_t* n_active,
                      int32_t* res_inv, int32_t* res_esc, int32_t* sg, int32_t* sc, int32_t* orders)
{
    const oc_config* c = &env->c;
    const int32_t N = c->N, R = c->R;
    scalars[0] = env->t;
    scalars[1] = env->ep;
    for (int32_t b = 0; b < c->K; ++b) scalars[2 + b] = env->rates[b];
    memcpy(coin_inv, env->coin_inv, 4 * (size_t)N);
    memcpy(coin_esc, env->coin_esc, 4 * (size_t)N);
    memcpy(labor, env->labor, 4 * (size_t)N);
    memcpy(snap, env->snap, 4 * (size_t)N);
    memcpy(n_active, env->n_active, 4 * (size_t)N);
    memcpy(sc, env->sc, 4 * (size_t)N);
    memcpy(res_inv, env->res_inv, 4 * (size_t)N * (size_t)R);
    memcpy(res_esc, env->res_esc, 4 * (size_t)N * (size_t)R);
    memcpy(sg, env->sg, 4 * (size_t)N * (size_t)R);
    for (size_t j = 0; j < (size_t)N * (size_t)c->X; ++j) orders[j] = -1;
    for (int32_t j = 0; j < env->n_book; ++j) {
        const oc_order* o = &env->book[j];
        orders[(size_t)(o->t0 % c->X) * (size_t)N + (size_t)o->agent] = o->side + 2 * (o->r + R * o->p);
    }
}

/* Inverse of oc_env_get_state: installs a state between two steps.  Live
 * orders must satisfy t - X < t0 < t; slot s holds the order with
 * t0 = t - 1 - ((t - 1 - s) mod X).  Order tie keys are re-derived from the
 * counter-based generator (they are a function of (env, episode, t0, agent)).
 * n_active is recounted from the orders. */
void oc_env_set_state(oc_env* env, const int32_t* scalars, const int32_t* coin_inv,
                      const int32_t* coin_esc, const int32_t* labor, const int32_t* snap,
                      const int32_t* res_inv, const int32_t* res_esc, const int32_t* sg,
                      const int32_t* sc, const int32_t* orders)
{
    const oc_config* c = &env->c;
    const int32_t N = c->N, R = c->R, X = c->X;
    env->t = scalars[0];
    env->ep = scalars[1];
    for (int32_t b = 0; b < c->K; ++b) env->rates[b] = scalars[2 + b];
    memcpy(env->coin_inv, coin_inv, 4 * (size_t)N);
    memcpy(env->coin_esc, coin_esc, 4 * (size_t)N);
    memcpy(env->labor, labor, 4 * (size_t)N);
    memcpy(env->snap, snap, 4 * (size_t)N);
    memcpy(env->sc, sc, 4 * (size_t)N);
    memcpy(env->res_inv, res_inv, 4 * (size_t)N * (size_t)R);
    memcpy(env->res_esc, res_esc, 4 * (size_t)N * (size_t)R);
    memcpy(env->sg, sg, 4 * (size_t)N * (size_t)R);
    env->n_book = 0;
    for (int q = 0; q < 5 * OC_MAXR + 3; ++q) env->macc[q] = 0; /* episode-to-date counts unknown */
    for (int32_t i = 0; i < N; ++i) env->n_active[i] = 0;
    for (int32_t s = 0; s < X; ++s) {
        for (int32_t i = 0; i < N; ++i) {
            int32_t code = orders[(size_t)s * (size_t)N + (size_t)i];
            if (code < 0) continue;
            int32_t t0 = env->t - 1 - ((((env->t - 1 - s) % X) + X) % X);
            uint64_t w[4];
            draw(env->seed, OC_PURPOSE_ENV, (uint64_t)env->e, (uint64_t)env->ep, (uint64_t)t0,
                 (uint64_t)i, w);
            oc_order o;
            o.agent = i; o.side = code & 1; o.r = (code >> 1) % R; o.p = (code >> 1) / R;
            o.t0 = t0; o.key = (uint32_t)(w[1] >> 32);
            env->book[env->n_book++] = o;
            env->n_active[i] += 1;
        }
    }
}

int64_t oc_env_invalid_actions(const oc_env* env) { return env->invalid_actions; }
int64_t oc_env_invalid_gov(const oc_env* env) { return env->invalid_gov; }

/* ---------------------------------------------------------------------------
 * Synthetic workload actions: uniform over the action space from the
 * counter-based generator, keyed (seed, env, episode, step, agent); the
 * government draws uniform levels 0..20 per bracket.
 * ------------------------------------------------------------------------- */
void oc_random_actions(const oc_config* c, uint64_t seed, int32_t e, int32_t ep, int32_t t,
                       int32_t* act, int32_t* gov)
{
    const uint64_t A = (uint64_t)oc_num_actions(c->R, c->P);
    for (int32_t i = 0; i < c->N; ++i) {
        uint64_t w[4];
        draw(seed, OC_PURPOSE_ACT, (uint64_t)e, (uint64_t)ep, (uint64_t)t, (uint64_t)i, w);
        act[i] = (int32_t)(((w[0] >> 32) * A) >> 32);
    }
    for (int32_t b = 0; b < c->K; ++b) {
        uint64_t w[4];
        draw(seed, OC_PURPOSE_GOV, (uint64_t)e, (uint64_t)ep, (uint64_t)t, (uint64_t)(b / 4), w);
        gov[b] = (int32_t)(((w[b % 4] >> 32) * 21ull) >> 32);
    }
}

/* Runs `steps` steps of one environment on its own synthetic action stream
 * (the action seed is separate from the environment seed).  Used for the
 * CPU baseline timing; rewards are summed into *rew_sum. */
int32_t oc_env_run_random(oc_env* env, uint64_t act_seed, int32_t steps, double* rew_sum)
{
    const oc_config* c = &env->c;
    int32_t* act = (int32_t*)malloc(sizeof(int32_t) * (size_t)c->N);
    int32_t gov[OC_MAXK];
    float* rew = (float*)malloc(sizeof(float) * (size_t)c->N);
    double acc = 0.0;
    for (int32_t s = 0; s < steps; ++s) {
        float gr;
        int32_t done;
        oc_random_actions(c, act_seed, env->e, env->ep, env->t, act, gov);
        oc_env_step(env, act, gov, rew, &gr, &done);
        for (int32_t i = 0; i < c->N; ++i) acc += rew[i];
    }
    *rew_sum = acc;
    free(act); free(rew);
    return 0;
}
