"""Throughput of the batched economy rollout step on one MI355X.

A step is one pass of the hot path over the 1024-economy x 100-agent
synthetic workload (3 resources, 20 price levels, order lifetime 10, tax
period 100, 1000-step episodes): the shared policy network samples every
agent's action from the current observation (35 -> 256 -> 256 -> 125 + 1,
bf16 MFMA), and the economy step draws the government's tax levels, applies
the actions, clears the markets, taxes and redistributes, computes
the rewards and writes the next observation and action mask.  Inputs are
resident in HBM before the timed region starts.

Prints one JSON line (metric, value, ms_per_step, roofline of the dominant
kernel measured with HIP events, CPU-oracle baseline on a bounded sample).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
WORKLOAD = "econ_e1024_n100"
POLICY_WORKLOAD = "econ_e4096_n100_ppo"  # the policy network shape (hidden 256)


def env_bytes_per_agent_step(cfg, D, A) -> int:
    """Algorithmic HBM bytes one agent-step of the economy must move:
    mutable state read and written (coin in inventory and escrow, labor,
    period snapshot, R inventories, R escrows, X order slots: int32), the
    skills read (R + 1 int32), the action read, the reward and done flag
    written, the bf16 observation (D features) and the mask bits written."""
    R, X = cfg["R"], cfg["X"]
    mutable = 4 * (4 + 2 * R + X)
    return 2 * mutable + 4 * (R + 1) + 4 + 4 + 1 + 2 * D + 4 * ((A + 31) // 32)


def policy_flops_per_row(D, H, A) -> int:
    return 2 * (D * H + H * H + H * (A + 1))


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    counter passes (scaled by a 256 MiB copy), or None when the kernel's
    sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{WORKLOAD}.json")
    try:
        with open(path) as f:
            rec = json.load(f)["kernels"][kernel]
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
    except (OSError, KeyError, ValueError):
        return None
    return rec["bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def _oracle_worker(args):
    """One host core's share of the CPU baseline: economies e0.. of the
    workload stepped with the oracle policy until the budget is spent."""
    cfg, weights, economies, budget_s = args
    from threadpoolctl import threadpool_limits

    from oracle import env as oe
    from oracle import policy as op

    sc = W.obs_scales(cfg)
    Ds = W.obs_stride(cfg)
    A = W.num_actions(cfg)
    D = W.obs_dim(cfg)
    envs = [(e, oe.OracleEnv(cfg, e=e, seed=cfg["seed"])) for e in economies]
    wb = op.bf16_weights(weights)
    agent_steps = 0
    steps = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            for e, env in envs:
                obs, mask, _ = env.observe(sc, Ds, with_gov=False)
                x = oe.bf16_bits_to_f32(obs[:, :D]).astype(np.float64)
                logits, _ = op.mlp(x, wb)
                lp = op.masked_log_softmax(logits, op.unpack_mask(mask, A))
                u1, u2 = oe.sample_uniforms(1, np.arange(cfg["N"]) + e * cfg["N"], steps, 1)
                act, _ = op.sample_chunked(np.concatenate([lp, np.full((cfg["N"], 128 - A), -np.inf)], 1), u1, u2)
                _, gov = env.random_actions(2)
                env.step(act.astype(np.int32), gov)
                agent_steps += cfg["N"]
            steps += 1
        dt = time.perf_counter() - t0
    return agent_steps, dt, steps


def cpu_baseline(cfg, weights, budget_s: float = 12.0):
    """The oracle as it stands (C economy, float64 numpy policy with its own
    sampler) on a bounded sample of the same workload: first one thread on 4
    economies, then one process per host core (the cores this process may
    run on), 4 economies each, for the same time budget."""
    import multiprocessing as mp

    n1, dt1, steps1 = _oracle_worker((cfg, weights, range(4), budget_s / 2))
    # the host cores this process may run on (its affinity mask), at most 16
    cores = min(len(os.sched_getaffinity(0)), 16)
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(cfg, weights, range(4 * c, 4 * c + 4), budget_s / 2) for c in range(cores)])
    total = sum(r[0] for r in res)
    wall = max(r[1] for r in res)
    return dict(value=total / wall, unit="agent-steps/s", cores=cores, kind="oracle",
                one_thread=round(n1 / dt1, 1),
                sample=f"{cores} processes x 4 economies x {cfg['N']} agents of the same workload for "
                       f"{budget_s / 2:.0f} s each (C economy step + float64 numpy policy and sampler; "
                       f"{min(r[2] for r in res)}+ steps per economy); one thread alone: 4 economies x "
                       f"{steps1} steps")


def ppo_benchmark(updates: int = 1, groups: int = 4, name: str = POLICY_WORKLOAD):
    """PPO samples/s on a learning workload (default: 4096 economies x 100
    agents, rollout of 128 steps as one captured graph + 4 epochs x 8
    minibatches of the hand-written backward with activation recompute, and
    Adam): one warm-up update, then `updates` timed ones."""
    import torch

    from paper_2410_22165_amd.ppo import PPOTrainer

    wl = W.workload(name)
    cfg = wl["env"]
    tr = PPOTrainer(cfg, W.obs_scales(cfg), hidden=wl["hidden"], rollout=wl["rollout"], epochs=wl["epochs"],
                    minibatches=wl["minibatches"], gamma=wl["gamma"], lam=wl["lam"], clip=wl["clip"],
                    vf_coef=wl["vf_coef"], vclip=wl["vclip"], ent_coef=wl["ent_coef"], lr=wl["lr"], seed=0,
                    total_updates=updates + 1, groups=groups)
    tr.collect(graph=True)
    tr.update()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    # the same rollout from per-step host launches, for the graph's speed-up
    ev[0].record(s)
    tr.collect(graph=False)
    ev[1].record(s)
    torch.cuda.synchronize()
    t_plain = ev[0].elapsed_time(ev[1])
    tr.next_rollout()
    t_roll = t_upd = 0.0
    for _ in range(updates):
        ev[0].record(s)
        tr.collect(graph=True)
        ev[1].record(s)
        tr.update()
        ev[2].record(s)
        torch.cuda.synchronize()
        t_roll += ev[0].elapsed_time(ev[1])
        t_upd += ev[1].elapsed_time(ev[2])
    samples = tr.M_total * updates
    terms = tr.loss_terms.cpu().numpy().tolist()
    tr.close()
    return {"value": round(samples / ((t_roll + t_upd) / 1e3), 1), "unit": "samples/s",
            "update_only": round(samples / (t_upd / 1e3), 1), "rollout_ms": round(t_roll / updates, 3),
            "update_ms": round(t_upd / updates, 3), "samples_per_update": tr.M_total,
            "rollout_plain_ms": round(t_plain, 3), "rollout_x_vs_plain": round(t_plain / (t_roll / updates), 4),
            "workload": f"{name}: E={cfg['E']} N={cfg['N']} T={wl['rollout']} "
                        f"{wl['epochs']}x{wl['minibatches']} minibatches, hidden {wl['hidden']}",
            "rollout_groups": groups,
            "last_loss_terms": [round(x, 5) for x in terms]}


def timed_launches(fn, reps: int) -> float:
    """Milliseconds per call of fn, from HIP events on the current stream."""
    import torch
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(s)
    for _ in range(reps):
        fn()
    b.record(s)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def graph_rollouts(env, mlp, T: int, reps: int, group_counts, seed: int = 1):
    """The rollout of T steps as the library captures it (ej_rollout_capture,
    carry on: each replay continues from the last), against the same
    launches issued one by one with one group (plain per-step launches).
    Returns (plain ms/step, {groups: graph ms/step})."""
    from paper_2410_22165_amd import binding

    bufs = binding.rollout_storage(env, T)
    plain = binding.Rollout(env, mlp, bufs, T, seed, groups=1, last_value=False, carry=True)
    plain.launch_plain()
    ms_plain = timed_launches(plain.launch_plain, reps) / T
    plain.close()
    graph_ms = {}
    for ng in group_counts:
        r = binding.Rollout(env, mlp, bufs, T, seed, groups=ng, last_value=False, carry=True)
        r.launch()
        graph_ms[ng] = timed_launches(r.launch, reps) / T
        r.close()
    del bufs
    return ms_plain, graph_ms


def rollout_benchmark(name: str, H: int, graph_steps: int = 20, reps: int = 2, n_per_env=None,
                      group_counts=(1, 2, 4)):
    """Rollout steps (policy forward + economy step with its government draw)
    on one workload: plain per-step launches with one workgroup per economy
    against the autotuned launch shapes replayed from the library's captured
    graph of `graph_steps` steps, with the economies in 1, 2 or 4 groups on
    their own streams (fastest kept)."""
    import torch

    from paper_2410_22165_amd import binding

    wl = W.workload(name)
    cfg = wl["env"]
    env = binding.Env(cfg, W.obs_scales(cfg), n_per_env)
    b = env.buffers()
    M, A, D, Ds = env.M, env.A, env.D, env.Ds
    mlp = binding.Mlp(D, Ds, H, A, W.policy_weights(D, H, A, seed=0))
    dev = torch.device("cuda")
    act = torch.zeros(M, dtype=torch.int32, device=dev)
    logp, val, ent = (torch.zeros(M, device=dev) for _ in range(3))
    env.observe(b["obs"], b["mask"])
    env.set_gov_draw(True, 2)
    env.set_launch(0, 0)
    ms_plain, _ = graph_rollouts(env, mlp, graph_steps, reps, ())
    tuned = binding.autotune(env, mlp, dict(obs=b["obs"], mask=b["mask"], act=act, logp=logp, val=val, ent=ent,
                                            rew=b["rew"], gov_rew=b["gov_rew"], done=b["done"]))
    _, graph_ms = graph_rollouts(env, mlp, graph_steps, reps, group_counts)
    best = min(graph_ms, key=graph_ms.get)
    ms_graph = graph_ms[best]
    env.close()
    return {"workload": name, "economies": cfg["E"], "agents": int(M), "hidden": H,
            "value": round(M / (ms_graph / 1e3), 1), "unit": "agent-steps/s",
            "plain_ms_per_step": round(ms_plain, 5), "graph_ms_per_step": round(ms_graph, 5),
            "graph_steps": graph_steps, "x_vs_plain": round(ms_plain / ms_graph, 4), "groups": best,
            "graph_ms_per_step_by_groups": {str(k): round(v, 5) for k, v in graph_ms.items()},
            "autotune": tuned}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ppo", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the uneven-population and 1000-agent rollouts")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--graph-steps", type=int, default=50)
    ap.add_argument("--groups", type=int, nargs="+", default=[1, 2, 3, 4],
                    help="economy-group counts tried for the graph-replayed step")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (one process, one MI355X)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2410_22165_amd import binding

    torch.cuda.set_device(0)
    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = W.workload(WORKLOAD)
    cfg = wl["env"]
    H = W.workload(POLICY_WORKLOAD)["hidden"]
    env = binding.Env(cfg, W.obs_scales(cfg))
    b = env.buffers()
    M, A, D, Ds = env.M, env.A, env.D, env.Ds
    weights = W.policy_weights(D, H, A, seed=0)
    mlp = binding.Mlp(D, Ds, H, A, weights)
    dev = torch.device("cuda")
    act = torch.zeros(M, dtype=torch.int32, device=dev)
    logp, val, ent = (torch.zeros(M, device=dev) for _ in range(3))
    ctr_base = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    env.observe(b["obs"], b["mask"])

    def policy(i):
        mlp.forward(b["obs"], b["mask"], M, 1, i, act, logp, val, ent, ctr_base=ctr_base)

    env.set_gov_draw(True, 2)  # uniform government levels drawn inside the step

    def economy():
        env.step(act, None, b["rew"], b["gov_rew"], b["done"], b["obs"], b["mask"])

    # launch shapes chosen by the autotuner (everything a trial changes is restored)
    tuned = binding.autotune(env, mlp, dict(obs=b["obs"], mask=b["mask"], act=act, logp=logp, val=val, ent=ent,
                                            rew=b["rew"], gov_rew=b["gov_rew"], done=b["done"]))

    for i in range(args.warmup):
        policy(i)
        economy()
    torch.cuda.synchronize()

    # plain: one launch per kernel per step; graph: the rollout of G steps as
    # the library captures it, the economies split into groups whose policy ->
    # step chains run on their own streams (one group's policy overlaps
    # another's step); the group count giving the fastest replay is kept
    G = max(1, min(args.graph_steps, args.steps))
    reps = max(1, args.steps // G)
    ms_plain, graph_ms = graph_rollouts(env, mlp, G, reps, args.groups)
    best_groups = min(graph_ms, key=graph_ms.get)
    ms_graph = graph_ms[best_groups]
    timed_steps = reps * G

    ms_step = min(ms_plain, ms_graph)
    value = M / (ms_step / 1e3)

    # per-kernel durations with HIP events on the launch stream
    n_k = min(args.steps, 100)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(n_k)]
    for i in range(n_k):
        ev[i][0].record(stream)
        policy(10 ** 6 + i)
        ev[i][1].record(stream)
        ev[i][2].record(stream)
        env.step(act, None, b["rew"], b["gov_rew"], b["done"], b["obs"], b["mask"])
        ev[i][3].record(stream)
    torch.cuda.synchronize()
    ms_pol = float(np.mean([ev[i][0].elapsed_time(ev[i][1]) for i in range(n_k)]))
    ms_env = float(np.mean([ev[i][2].elapsed_time(ev[i][3]) for i in range(n_k)]))

    env_bytes = env_bytes_per_agent_step(cfg, D, A) * M
    pol_flops = policy_flops_per_row(D, H, A) * M
    env_gbs = env_bytes / (ms_env / 1e3) / 1e9
    pol_tflops = pol_flops / (ms_pol / 1e3) / 1e12
    env_kernel = "env_step_persistent_kernel" if tuned["env_mode"] == 1 else "env_step_kernel"
    kernels = {
        env_kernel: {"bound": "hbm", "achieved": env_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": env_gbs / HBM_PEAK_GBS, "ms": ms_env,
                            "algorithmic_bytes_per_launch": env_bytes},
        "policy_forward_kernel": {"bound": "mfma", "achieved": pol_tflops, "peak": BF16_PEAK_TFLOPS,
                                  "unit": "TFLOP/s", "frac": pol_tflops / BF16_PEAK_TFLOPS, "ms": ms_pol,
                                  "algorithmic_flops_per_launch": pol_flops},
    }
    dom = env_kernel if ms_env >= ms_pol else "policy_forward_kernel"
    k = kernels[dom]
    for name, kk in kernels.items():
        kk["hbm_bytes_per_launch"] = measured_traffic(name)
    roofline = {"kernel": dom, "bound": k["bound"], "achieved": round(k["achieved"], 3), "peak": k["peak"],
                "unit": k["unit"], "frac": round(k["frac"], 5), "traffic": k["hbm_bytes_per_launch"]}

    out = {
        "metric": "agent-steps/sec (env+policy) at E×N=1024×100",
        "value": round(value, 1),
        "unit": "agent-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+bf16",
        "data": "synthetic (seed-generated economies; random-init policy weights)",
        "config": {"workload": WORKLOAD, "E": cfg["E"], "N": cfg["N"], "R": cfg["R"], "P": cfg["P"],
                   "X": cfg["X"], "P_tax": cfg["P_tax"], "K": cfg["K"], "T": cfg["T"],
                   "policy": f"{D}->{H}->{H}->{A}+1", "parallelism": "one workgroup per economy",
                   "launch": (f"hipGraph of {G} steps, {best_groups} economy group(s) on their own streams"
                              if ms_graph <= ms_plain else "per-step launches"),
                   "autotune": tuned},
        "x_vs_plain": round(ms_plain / ms_graph, 4),
        "plain_ms_per_step": round(ms_plain, 5),
        "graph_ms_per_step": round(ms_graph, 5),
        "graph_timed_steps": timed_steps,
        "graph_ms_per_step_by_groups": {str(k): round(v, 5) for k, v in graph_ms.items()},
        "roofline": roofline,
        "kernels": {n: {kk: (round(v, 5) if isinstance(v, float) else v) for kk, v in d.items()}
                    for n, d in kernels.items()},
    }
    env.close()
    if not args.no_ppo:
        out["ppo"] = ppo_benchmark()
        if not args.no_extra:  # 256 economies x 1000 agents, 5 resources, 50 prices, hidden 512, T = 256
            out["ppo_large"] = ppo_benchmark(name="econ_e256_n1000_ppo")
    if not args.no_extra:
        wl4 = W.workload("econ_e512_uneven")
        ns = W.uneven_populations(wl4["env"]["E"], wl4["n_min"], wl4["n_max"], seed=0)
        out["uneven"] = rollout_benchmark("econ_e512_uneven", 256, graph_steps=1000, reps=1, n_per_env=ns)
        out["large"] = rollout_benchmark("econ_e256_n1000_ppo", W.workload("econ_e256_n1000_ppo")["hidden"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, weights, args.cpu_budget)
        out["cpu_baseline"]["value"] = round(out["cpu_baseline"]["value"], 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
