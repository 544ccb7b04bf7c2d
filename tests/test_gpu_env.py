"""GPU parity of the economy step (C ABI) against the CPU oracle.

Integer state (inventories, escrow, labor, skills, the order book, time,
episode, tax levels) must match bit for bit; rewards within 1e-5 relative;
observations (bf16 bits) and action masks exactly.  Actions are identical
on both sides: host arrays uploaded to the GPU, or the counter-based
synthetic stream that each side derives on its own."""
import numpy as np
import pytest

import workloads as W
from oracle import env as oe

pytestmark = pytest.mark.gpu

INT_FIELDS = ("coin_inv", "coin_esc", "labor", "snap", "sc", "res_inv", "res_esc", "sg", "orders", "n_active")


def _torch():
    import torch
    return torch


def make_env(cfg, n_per_env=None):
    from paper_2410_22165_amd import binding
    print(f"[gpu] env E={cfg['E']} N={cfg['N']} R={cfg['R']} P={cfg['P']} X={cfg['X']} K={cfg['K']}", flush=True)
    return binding.Env(cfg, W.obs_scales(cfg), n_per_env)


def compare_state(g, o, where=""):
    assert g["t"] == o["t"] and g["ep"] == o["ep"], f"{where}: t/ep {g['t']},{g['ep']} vs {o['t']},{o['ep']}"
    assert np.array_equal(g["rates"], o["rates"]), f"{where}: rates"
    for k in INT_FIELDS:
        if not np.array_equal(np.asarray(g[k]), np.asarray(o[k])):
            bad = np.argwhere(np.asarray(g[k]) != np.asarray(o[k]))[:5]
            raise AssertionError(f"{where}: field {k} differs at {bad.tolist()}: "
                                 f"gpu {np.asarray(g[k])[tuple(bad.T)]} oracle {np.asarray(o[k])[tuple(bad.T)]}")


def assert_rew_close(g, o, where=""):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    ok = np.abs(g - o) <= 1e-5 * np.abs(o)
    assert ok.all(), f"{where}: rewards {g[~ok][:5]} vs {o[~ok][:5]}"


def run_lockstep(cfg, steps, actions="masked", seed=0, check_obs=True, n_per_env=None):
    """Steps the GPU batch and one oracle economy per GPU economy in lockstep,
    comparing everything after every step."""
    torch = _torch()
    env = make_env(cfg, n_per_env)
    E = cfg["E"]
    ns = [cfg["N"]] * E if n_per_env is None else list(n_per_env)
    orc = [oe.OracleEnv(cfg, e=e, seed=cfg["seed"], n_agents=ns[e]) for e in range(E)]
    b = env.buffers()
    sc, Ds = W.obs_scales(cfg), env.Ds
    rng = np.random.default_rng(seed)
    A = env.A
    for step in range(steps):
        acts, govs = [], []
        for e in range(E):
            if actions == "masked":
                _, m, _ = orc[e].observe(sc, Ds, with_gov=False)
                bits = ((m[:, np.arange(A) // 32] >> (np.arange(A) % 32).astype(np.uint32)) & 1).astype(bool)
                a = np.array([rng.choice(np.flatnonzero(bits[i])) if bits[i].any() else 0 for i in range(ns[e])])
                if rng.random() < 0.1:  # a few invalid and out-of-range actions
                    a[rng.integers(ns[e])] = rng.integers(-3, A + 3)
            else:
                a = rng.integers(0, A, size=ns[e])
            acts.append(a.astype(np.int32))
            govs.append(rng.integers(-1, 22, size=max(cfg["K"], 1)).astype(np.int32))
        b["act"].copy_(torch.from_numpy(np.concatenate(acts)))
        if cfg["K"] > 0:
            b["gov"].copy_(torch.from_numpy(np.concatenate([g[:cfg["K"]] for g in govs])))
        env.step(b["act"], b["gov"], b["rew"], b["gov_rew"], b["done"], b["obs"], b["mask"])
        torch.cuda.synchronize()
        gst = env.get_state()
        rew = b["rew"].cpu().numpy()
        grew = b["gov_rew"].cpu().numpy()
        done = b["done"].cpu().numpy()
        obs = b["obs"].cpu().numpy().view(np.uint16)
        mask = b["mask"].cpu().numpy().view(np.uint32)
        for e in range(E):
            r_o, g_o, d_o = orc[e].step(acts[e], govs[e][:cfg["K"]])
            lo, hi = int(env.row_offsets[e]), int(env.row_offsets[e + 1])
            where = f"step {step} env {e}"
            compare_state(env.env_state(gst, e), orc[e].state(), where)
            assert_rew_close(rew[lo:hi], r_o, where)
            assert_rew_close([grew[e]], [g_o], where + " gov")
            assert (done[lo:hi] == d_o).all(), where
            if check_obs:
                o_obs, o_mask, _ = orc[e].observe(sc, Ds, with_gov=False)
                assert np.array_equal(obs[lo:hi], o_obs), where + " obs"
                assert np.array_equal(mask[lo:hi], o_mask), where + " mask"
    ia, ig = env.status()
    oa = sum(o.invalid_counts()[0] for o in orc)
    og = sum(o.invalid_counts()[1] for o in orc)
    assert (ia, ig) == (oa, og)
    env.close()


def test_parity_econ_e1_n4_full_episode_and_reset():
    """The parity workload (one economy of 4 agents, 2 resources, 10 prices,
    7 brackets, tax period 10) over 1.5 episodes, uniform actions."""
    cfg = W.workload("econ_e1_n4")["env"]
    run_lockstep(cfg, 150, actions="uniform", seed=1)


@pytest.mark.parametrize("variant", range(5))
def test_parity_small_configs_masked_actions(variant):
    cfgs = [
        W.env_config(E=3, N=4, R=2, P=10, X=10, P_tax=10, K=7, T=100),
        W.env_config(E=2, N=7, R=3, P=4, X=3, max_orders=2, P_tax=5, K=3, T=37, R_d=2),
        W.env_config(E=2, N=5, R=1, P=3, X=1, P_tax=4, K=1, T=20, R_d=1, R_kappa=1),
        W.env_config(E=2, N=6, R=5, P=3, X=30, max_orders=15, P_tax=7, K=0, T=50, R_d=3, allow_noop=0),
        W.env_config(E=2, N=70, R=8, P=6, X=20, max_orders=9, P_tax=9, K=16, T=60, R_d=3, seed=5),
    ]
    run_lockstep(cfgs[variant], 80, actions="masked", seed=variant)


def test_parity_uneven_populations_small():
    cfg = W.env_config(E=5, N=130, R=3, P=5, X=4, P_tax=6, K=3, T=40)
    run_lockstep(cfg, 45, actions="masked", seed=9, n_per_env=[1, 64, 65, 130, 17])


def test_parity_max_population():
    cfg = W.env_config(E=1, N=1024, R=2, P=8, X=6, P_tax=10, K=4, T=30)
    run_lockstep(cfg, 12, actions="masked", seed=3, check_obs=True)


def _sampled_parity(cfg, steps, sample, n_per_env=None, act_seed=77, check_every=100):
    """Full-size batch driven by the synthetic action stream; the oracle
    replays only the sampled economies (each side derives the actions).
    Every step also writes the next observations and masks (the launch
    configuration of the throughput run); at every state check they are
    compared with the oracle's, bf16 bits and mask words exactly."""
    torch = _torch()
    env = make_env(cfg, n_per_env)
    b = env.buffers()
    ns = [cfg["N"]] * cfg["E"] if n_per_env is None else list(n_per_env)
    orc = {e: oe.OracleEnv(cfg, e=e, seed=cfg["seed"], n_agents=ns[e]) for e in sample}
    sc, Ds = W.obs_scales(cfg), env.Ds
    for step in range(steps):
        env.random_actions(act_seed, b["act"], b["gov"])
        env.step(b["act"], b["gov"], b["rew"], b["gov_rew"], b["done"], b["obs"], b["mask"])
        rew = b["rew"].cpu().numpy()
        act = b["act"].cpu().numpy()
        grew = b["gov_rew"].cpu().numpy()
        for e, o in orc.items():
            a_o, g_o = o.random_actions(act_seed)
            lo, hi = int(env.row_offsets[e]), int(env.row_offsets[e + 1])
            assert np.array_equal(act[lo:hi], a_o), f"step {step} env {e}: action stream"
            r_o, gr_o, _ = o.step(a_o, g_o)
            assert_rew_close(rew[lo:hi], r_o, f"step {step} env {e}")
            assert_rew_close([grew[e]], [gr_o], f"step {step} env {e} gov")
        if (step + 1) % check_every == 0 or step == steps - 1 or step < 3:
            gst = env.get_state()
            obs = b["obs"].cpu().numpy().view(np.uint16)
            mask = b["mask"].cpu().numpy().view(np.uint32)
            for e, o in orc.items():
                where = f"step {step} env {e}"
                compare_state(env.env_state(gst, e), o.state(), where)
                lo, hi = int(env.row_offsets[e]), int(env.row_offsets[e + 1])
                o_obs, o_mask, _ = o.observe(sc, Ds, with_gov=False)
                assert np.array_equal(obs[lo:hi], o_obs), where + " obs"
                assert np.array_equal(mask[lo:hi], o_mask), where + " mask"
    env.close()


@pytest.mark.slow
def test_parity_econ_e1024_n100_sampled():
    """Full-size plain-env workload (1024 x 100, 3 resources, 20 prices),
    1100 steps (covers tax periods and the auto-reset), 3 sampled economies."""
    cfg = W.workload("econ_e1024_n100")["env"]
    _sampled_parity(cfg, 1100, sample=[0, 517, 1023])


@pytest.mark.slow
def test_parity_uneven_512_sampled():
    wl = W.workload("econ_e512_uneven")
    cfg = wl["env"]
    ns = W.uneven_populations(cfg["E"], wl["n_min"], wl["n_max"])
    sample = [int(np.argmin(ns)), int(np.argmax(ns)), 255]
    _sampled_parity(cfg, 250, sample=sample, n_per_env=ns)


@pytest.mark.slow
def test_parity_econ_e256_n1000_sampled():
    cfg = W.workload("econ_e256_n1000_ppo")["env"]
    _sampled_parity(cfg, 220, sample=[3, 200])


def test_observe_matches_oracle_including_government():
    torch = _torch()
    cfg = W.env_config(E=3, N=37, R=3, P=5, X=4, P_tax=6, K=3, T=40)
    env = make_env(cfg)
    b = env.buffers()
    orc = [oe.OracleEnv(cfg, e=e, seed=cfg["seed"]) for e in range(3)]
    rng = np.random.default_rng(0)
    for step in range(25):
        acts = [rng.integers(0, env.A, size=37).astype(np.int32) for _ in range(3)]
        govs = [rng.integers(0, 21, size=3).astype(np.int32) for _ in range(3)]
        b["act"].copy_(torch.from_numpy(np.concatenate(acts)))
        b["gov"].copy_(torch.from_numpy(np.concatenate(govs)))
        env.step(b["act"], b["gov"], b["rew"], b["gov_rew"], b["done"])
        for e in range(3):
            orc[e].step(acts[e], govs[e])
    env.observe(b["obs"], b["mask"], b["gov_obs"])
    obs = b["obs"].cpu().numpy().view(np.uint16)
    mask = b["mask"].cpu().numpy().view(np.uint32)
    gobs = b["gov_obs"].cpu().numpy()
    for e in range(3):
        o_obs, o_mask, o_gov = orc[e].observe(W.obs_scales(cfg), env.Ds, with_gov=True)
        assert np.array_equal(obs[37 * e:37 * (e + 1)], o_obs)
        assert np.array_equal(mask[37 * e:37 * (e + 1)], o_mask)
        assert np.allclose(gobs[e], o_gov, rtol=1e-6, atol=0), (gobs[e], o_gov)
    env.close()


def test_determinism_and_checkpoint_resume():
    torch = _torch()
    cfg = W.env_config(E=64, N=100, R=3, P=20, X=10, P_tax=100, K=7, T=1000)

    def run(env, b, steps):
        out = []
        for _ in range(steps):
            env.random_actions(5, b["act"], b["gov"])
            env.step(b["act"], b["gov"], b["rew"], b["gov_rew"], b["done"], b["obs"], b["mask"])
            out.append(b["rew"].clone())
        return torch.stack(out).cpu().numpy()

    e1 = make_env(cfg)
    b1 = e1.buffers()
    r_first = run(e1, b1, 120)
    mid = e1.get_state()
    r_second = run(e1, b1, 130)
    end1 = e1.get_state()
    e2 = make_env(cfg)
    b2 = e2.buffers()
    r_again = run(e2, b2, 250)
    end2 = e2.get_state()
    assert np.array_equal(np.concatenate([r_first, r_second]), r_again)
    for k in end1:
        assert np.array_equal(end1[k], end2[k])
    e3 = make_env(cfg)
    b3 = e3.buffers()
    e3.set_state(mid)
    r_resumed = run(e3, b3, 130)
    assert np.array_equal(r_resumed, r_second)
    end3 = e3.get_state()
    for k in end1:
        assert np.array_equal(end1[k], end3[k]), k
    # the same handle rewound: values the step caches from the state it last
    # wrote (welfare, utilities) must not survive set_state
    e1.set_state(mid)
    r_rewound = run(e1, b1, 130)
    assert np.array_equal(r_rewound, r_second)
    for e in (e1, e2, e3):
        e.close()


def test_create_rejects_bad_configs():
    from paper_2410_22165_amd import binding
    base = W.env_config(E=2, N=4)
    bad = [dict(N=2000), dict(R=17), dict(X=33), dict(K=17), dict(prices=[4, 2] + [6] * 8), dict(E=0),
           dict(P=128, X=32, R=8), dict(R=12, N=300)]  # (more than 8 resources: populations of <= 256)
    for kv in bad:
        cfg = dict(base)
        cfg.update(kv)
        if "P" in kv and "prices" not in kv:
            cfg["prices"] = W.default_prices(cfg["P"])
        with pytest.raises(binding.EconError):
            binding.Env(cfg, W.obs_scales(cfg))


def test_reset_after_steps_equals_fresh_handle():
    """ej_env_reset on a handle that has stepped: the following steps equal
    those of a fresh handle bit for bit (no cached welfare or utility of the
    old state survives the reset)."""
    torch = _torch()
    cfg = W.env_config(E=16, N=100, R=3, P=20, X=10, P_tax=100, K=7, T=1000)

    def run(env, b, steps):
        out = []
        for _ in range(steps):
            env.random_actions(9, b["act"], b["gov"])
            env.step(b["act"], b["gov"], b["rew"], b["gov_rew"], b["done"], b["obs"], b["mask"])
            out.append(torch.cat([b["rew"], b["gov_rew"]]).clone())
        return torch.stack(out).cpu().numpy()

    e1 = make_env(cfg)
    b1 = e1.buffers()
    run(e1, b1, 60)
    e1.reset(0)
    r1 = run(e1, b1, 40)
    e2 = make_env(cfg)
    b2 = e2.buffers()
    r2 = run(e2, b2, 40)
    assert np.array_equal(r1, r2)
    s1, s2 = e1.get_state(), e2.get_state()
    for k in s1:
        assert np.array_equal(s1[k], s2[k]), k
    for e in (e1, e2):
        e.close()


@pytest.mark.parametrize("variant", range(3))
def test_episode_metrics_match_oracle(variant):
    """Episode statistics (ej_env_enable_metrics / ej_env_episode_metrics)
    against the oracle's record at every episode end over 2.5 episodes:
    episode index, productivity, action counts, trades and price sums
    exactly; equality and Eq * Prod exactly (the same integer Gini sums);
    mean return within 1e-12 relative (summation order) and the median
    within 1e-9 (utilities by each side's pow).  Uneven populations, invalid
    actions, one economy above 256 agents (the sorted-welfare path)."""
    torch = _torch()
    cases = [
        (W.env_config(E=3, N=37, R=3, P=6, X=4, P_tax=5, K=3, T=23, seed=1), [37, 5, 20]),
        (W.env_config(E=2, N=300, R=2, P=5, X=3, P_tax=4, K=2, T=14, seed=2), [300, 257]),
        (W.env_config(E=2, N=9, R=5, P=3, X=6, P_tax=7, K=0, T=11, seed=3), None),
    ]
    cfg, ns = cases[variant]
    env = make_env(cfg, ns)
    env.enable_metrics()
    E = cfg["E"]
    ns = [cfg["N"]] * E if ns is None else ns
    orc = [oe.OracleEnv(cfg, e=e, seed=cfg["seed"], n_agents=ns[e]) for e in range(E)]
    b = env.buffers()
    rng = np.random.default_rng(variant)
    A = env.A
    assert (env.episode_metrics().cpu().numpy()[:, 0] == -1).all()
    ends = 0
    for step in range(int(2.5 * cfg["T"])):
        acts = [rng.integers(-1, A + 1, size=ns[e]).astype(np.int32) for e in range(E)]
        govs = [rng.integers(0, 21, size=max(cfg["K"], 1)).astype(np.int32) for e in range(E)]
        b["act"].copy_(torch.from_numpy(np.concatenate(acts)))
        if cfg["K"] > 0:
            b["gov"].copy_(torch.from_numpy(np.concatenate([g[:cfg["K"]] for g in govs])))
        env.step(b["act"], b["gov"], b["rew"], b["gov_rew"], b["done"], b["obs"], b["mask"])
        done = False
        for e in range(E):
            _, _, d = orc[e].step(acts[e], govs[e][:cfg["K"]])
            done = done or bool(d)
        if not done:
            continue
        ends += 1
        g = env.episode_metrics().cpu().numpy()
        R = cfg["R"]
        for e in range(E):
            o = orc[e].episode_metrics()
            where = f"step {step} economy {e}"
            exact = np.r_[0, 1, 2, 3, np.arange(6, 9 + 5 * R)]
            assert np.array_equal(g[e][exact], o[exact]), (where, g[e][exact], o[exact])
            assert abs(g[e][4] - o[4]) <= 1e-12 * max(1.0, abs(o[4])), (where, g[e][4], o[4])
            assert abs(g[e][5] - o[5]) <= 1e-9 * max(1.0, abs(o[5])), (where, g[e][5], o[5])
    assert ends == 2
    env.close()


@pytest.mark.parametrize("R", [4, 8, 12, 16])
def test_parity_multi_agent_variant_lockstep(R):
    """The multi-agent variant (Sec. 5): skills near 1 with spread 1 that
    grow with every gather and craft, taxes off, prices 3, 6, 9, R_d from R;
    state (skills included), rewards, observations and masks against the
    oracle after every step, over an episode end (new skills drawn).  R = 16
    is the largest resource count (114 actions, 122-feature observations)."""
    cfg = W.variant_config(R=R, N=23, E=3, X=7, T=35, seed=4)
    run_lockstep(cfg, 50, actions="masked", seed=R, n_per_env=[23, 9, 16])


@pytest.mark.slow
@pytest.mark.parametrize("R", [4, 12])
def test_parity_multi_agent_variant_sampled(R):
    """64 economies of 100 agents with 4 or 12 resources (30 or 86 actions),
    order lifetime 30, 1100 steps (an episode end at 1000), 2 sampled
    economies."""
    cfg = W.variant_config(R=R, N=100, E=64, seed=2)
    _sampled_parity(cfg, 1100, sample=[0, 41])
