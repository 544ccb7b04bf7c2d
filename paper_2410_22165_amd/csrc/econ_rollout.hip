// econ_rollout.hip -- the T-step rollout captured as one HIP graph.
//
// A rollout step is the shared policy forward over every agent's current
// observation followed by the economy step (Sec. 3: every population agent
// acts each step; Table 2: rollout length before each PPO update).  The
// economies never interact, so they are cut into G contiguous groups, each
// with its own stream: group g's chain policy(t) -> step(t) -> policy(t+1)
// ... only waits for itself, and one group's policy forward overlaps another
// group's economy step.  The whole rollout -- T x (policy, step) per group,
// the last-value forward, GAE and the sampling-counter advance -- is
// recorded once by stream capture and replayed with one hipGraphLaunch.
//
// Host code only: every node is a launch of the library's own entry points.
#include <new>
#include <vector>

#include "econ_common.h"

struct ej_rollout {
    ej_env* env = nullptr;
    ej_mlp_desc m{};
    const float* params = nullptr;
    const uint16_t* work = nullptr;
    ej_rollout_config cfg{};
    ej_rollout_buffers b{};
    ej_env_dims_t dims{};
    int32_t E = 0;
    std::vector<int32_t> e0, e1;  // economy range of every group
    std::vector<int64_t> r0, r1;  // row range of every group
    hipStream_t cap = nullptr;    // capture stream (origin of the graph)
    std::vector<hipStream_t> gs;  // group streams (G > 1)
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// dst[i] = src[i], n words (the carried observation and mask slot)
__global__ void copy_words_kernel(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

int copy_words(const void* src, void* dst, int64_t n, hipStream_t st)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) return EJ_OK;
    copy_words_kernel<<<(unsigned)blocks, 256, 0, st>>>((const uint32_t*)src, (uint32_t*)dst, n);
    EJ_LAUNCH_CHECK();
    return EJ_OK;
}

// every launch of one rollout, on `origin` (G > 1: forked onto the group
// streams and joined back); under stream capture this records the graph
int issue_rollout(ej_rollout* r, hipStream_t origin)
{
    const ej_rollout_buffers& b = r->b;
    const int64_t M = r->dims.M;
    const int64_t Ds = r->dims.D_stride, W = r->dims.mask_words;
    const int G = (int)r->e0.size();
    const int T = r->cfg.T;
    int rc = EJ_OK;
    if (G > 1) {
        EJ_HIP(hipEventRecord(r->fork, origin));
        for (int g = 0; g < G; ++g) EJ_HIP(hipStreamWaitEvent(r->gs[g], r->fork, 0));
    }
    for (int t = 0; t < T; ++t) {
        for (int g = 0; g < G; ++g) {
            hipStream_t st = G > 1 ? r->gs[g] : origin;
            const int64_t lo = r->r0[g], n = r->r1[g] - r->r0[g];
            const int64_t o = (int64_t)t * M + lo;
            if (n > 0 &&
                (rc = ej_policy_forward(&r->m, r->params, r->work, b.d_obs + ((int64_t)t * M + lo) * Ds,
                                        b.d_mask + ((int64_t)t * M + lo) * W, n, lo, r->cfg.seed, (uint64_t)t,
                                        b.d_ctr, b.d_act + o, b.d_logp + o, b.d_val + o, b.d_ent + o, nullptr, st)) !=
                    EJ_OK)
                return rc;
            if ((rc = ej_env_step_range(r->env, r->e0[g], r->e1[g], b.d_act + (int64_t)t * M, nullptr,
                                        b.d_rew + (int64_t)t * M, b.d_gov_rew + (int64_t)t * r->E,
                                        b.d_done + (int64_t)t * M, b.d_obs + (int64_t)(t + 1) * M * Ds,
                                        b.d_mask + (int64_t)(t + 1) * M * W, st)) != EJ_OK)
                return rc;
        }
    }
    if (G > 1) {
        for (int g = 0; g < G; ++g) {
            EJ_HIP(hipEventRecord(r->join[g], r->gs[g]));
            EJ_HIP(hipStreamWaitEvent(origin, r->join[g], 0));
        }
    }
    if (r->cfg.last_value) {
        float* tmp = b.d_tmp;
        if ((rc = ej_policy_forward(&r->m, r->params, r->work, b.d_obs + (int64_t)T * M * Ds,
                                    b.d_mask + (int64_t)T * M * W, M, 0, r->cfg.seed, (uint64_t)T, b.d_ctr,
                                    (int32_t*)tmp, tmp + M, b.d_last_val, tmp + 2 * M, nullptr, origin)) != EJ_OK)
            return rc;
        if (b.d_adv &&
            (rc = ej_gae(b.d_rew, b.d_val, b.d_done, b.d_last_val, T, M, r->cfg.gamma, r->cfg.lam, b.d_adv, b.d_ret,
                         origin)) != EJ_OK)
            return rc;
    }
    if (r->cfg.carry) {  // the next launch starts from the state after this one
        if ((rc = copy_words(b.d_obs + (int64_t)T * M * Ds, b.d_obs, M * Ds / 2, origin)) != EJ_OK ||
            (rc = copy_words(b.d_mask + (int64_t)T * M * W, b.d_mask, M * W, origin)) != EJ_OK)
            return rc;
    }
    return ej_counter_add(b.d_ctr, (uint64_t)T + 1, origin);
}

void release(ej_rollout* r)
{
    if (r->exec) (void)hipGraphExecDestroy(r->exec);
    if (r->graph) (void)hipGraphDestroy(r->graph);
    if (r->fork) (void)hipEventDestroy(r->fork);
    for (hipEvent_t e : r->join) (void)hipEventDestroy(e);
    for (hipStream_t s : r->gs) (void)hipStreamDestroy(s);
    if (r->cap) (void)hipStreamDestroy(r->cap);
    delete r;
}

}  // namespace

extern "C" {

int ej_rollout_capture(ej_env* env, const ej_mlp_desc* m, const float* d_params, const uint16_t* d_work,
                       const ej_rollout_config* cfg, const ej_rollout_buffers* b, ej_rollout** out)
{
    if (!out) return EJ_EINVAL;
    *out = nullptr;
    if (!env || !m || !d_params || !d_work || !cfg || !b) return EJ_EINVAL;
    if (cfg->T <= 0 || cfg->groups <= 0) return EJ_EINVAL;
    if (!b->d_obs || !b->d_mask || !b->d_act || !b->d_logp || !b->d_val || !b->d_ent || !b->d_rew || !b->d_done ||
        !b->d_gov_rew || !b->d_ctr)
        return EJ_EINVAL;
    if (cfg->last_value && (!b->d_last_val || !b->d_tmp)) return EJ_EINVAL;
    if ((b->d_adv == nullptr) != (b->d_ret == nullptr)) return EJ_EINVAL;
    ej_rollout* r = new (std::nothrow) ej_rollout();
    if (!r) return EJ_ENOMEM;
    r->env = env;
    r->m = *m;
    r->params = d_params;
    r->work = d_work;
    r->cfg = *cfg;
    r->b = *b;
    int rc = ej_env_dims(env, &r->dims);
    if (rc != EJ_OK) {
        release(r);
        return rc;
    }
    if (r->dims.D != m->D || r->dims.D_stride != m->D_stride || r->dims.A != m->A) {
        release(r);
        return EJ_EINVAL;
    }
    const int32_t* rows = ej_env_row_offsets(env);
    const int E = r->dims.E;
    r->E = E;
    const int G = cfg->groups < E ? cfg->groups : E;
    for (int g = 0; g < G; ++g) {
        const int a = (int)((int64_t)E * g / G), z = (int)((int64_t)E * (g + 1) / G);
        r->e0.push_back(a);
        r->e1.push_back(z);
        r->r0.push_back(rows[a]);
        r->r1.push_back(rows[z]);
    }
    bool ok = hipStreamCreateWithFlags(&r->cap, hipStreamNonBlocking) == hipSuccess;
    if (ok && G > 1) {
        ok = hipEventCreateWithFlags(&r->fork, hipEventDisableTiming) == hipSuccess;
        for (int g = 0; g < G && ok; ++g) {
            hipStream_t s = nullptr;
            hipEvent_t e = nullptr;
            ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
            if (ok) r->gs.push_back(s);
            ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
            if (ok) r->join.push_back(e);
        }
    }
    if (!ok) {
        econ::set_last_hip_error(hipGetLastError());
        release(r);
        return EJ_EHIP;
    }
    hipError_t e = hipStreamBeginCapture(r->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        econ::set_last_hip_error(e);
        release(r);
        return EJ_EHIP;
    }
    rc = issue_rollout(r, r->cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(r->cap, &graph);
    r->graph = graph;
    if (rc == EJ_OK && e != hipSuccess) {
        econ::set_last_hip_error(e);
        rc = EJ_EHIP;
    }
    if (rc == EJ_OK) {
        e = hipGraphInstantiate(&r->exec, r->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            econ::set_last_hip_error(e);
            rc = EJ_EHIP;
        }
    }
    if (rc != EJ_OK) {
        release(r);
        return rc;
    }
    *out = r;
    return EJ_OK;
}

int ej_rollout_launch(ej_rollout* r, void* stream)
{
    if (!r || !r->exec) return EJ_EINVAL;
    hipError_t e = hipGraphLaunch(r->exec, (hipStream_t)stream);
    if (e != hipSuccess) {
        econ::set_last_hip_error(e);
        return EJ_EHIP;
    }
    return EJ_OK;
}

int ej_rollout_launch_plain(ej_rollout* r, void* stream)
{
    if (!r) return EJ_EINVAL;
    hipStream_t origin = (hipStream_t)stream;
    return issue_rollout(r, origin);
}

int ej_rollout_destroy(ej_rollout* r)
{
    if (!r) return EJ_EINVAL;
    release(r);
    return EJ_OK;
}

}  // extern "C"
