"""Autotuner for the launch shapes of the rollout kernels.

Two knobs, both measured with HIP events on the stream the kernels run on:
  * the economy step: one workgroup per economy, or a persistent set of
    workgroups (1, 2 or 4 per compute unit) pulling economies from a work
    queue, largest populations first;
  * the policy forward: 128-row tiles (one workgroup per CU, weight
    fragments reused across two MFMA row tiles) or 64-row tiles (half the
    LDS, two workgroups per CU).
The economy state is restored after tuning, so tuning changes no result.
Choices are cached per (shape, device architecture) in memory and in
$XDG_CACHE_HOME/econ_mi355x/autotune.json.
"""
from __future__ import annotations

import json
import os

_CACHE: dict = {}


def _cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "econ_mi355x", "autotune.json")


def _load():
    if _CACHE:
        return
    try:
        with open(_cache_path()) as f:
            _CACHE.update(json.load(f))
    except (OSError, ValueError):
        pass


def _store():
    try:
        os.makedirs(os.path.dirname(_cache_path()), exist_ok=True)
        with open(_cache_path(), "w") as f:
            json.dump(_CACHE, f, indent=1, sort_keys=True)
    except OSError:
        pass


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name)


def _time(fn, reps: int) -> float:
    import torch
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    a.record(s)
    for _ in range(reps):
        fn()
    b.record(s)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_env(env, buf: dict, reps: int = 10, use_cache: bool = True) -> dict:
    """Picks the economy-step launch shape; returns {"mode", "workgroups", "ms"}."""
    import torch
    _load()
    cfg = env.cfg
    key = f"env|{_arch()}|E{cfg['E']}|N{cfg['N']}|R{cfg['R']}|P{cfg['P']}|X{cfg['X']}|n{int(env.M)}"
    if use_cache and key in _CACHE:
        best = _CACHE[key]
        env.set_launch(best["mode"], best["workgroups"])
        return best
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    saved = env.get_state()
    results = []
    for mode, wg in [(0, 0), (1, cus), (1, 2 * cus), (1, 4 * cus)]:
        env.set_launch(mode, wg)

        def step():
            env.step(buf["act"], buf["gov"], buf["rew"], buf["gov_rew"], buf["done"], buf["obs"], buf["mask"])

        results.append(dict(mode=mode, workgroups=wg, ms=_time(step, reps)))
    env.set_state(saved)
    best = min(results, key=lambda r: r["ms"])
    env.set_launch(best["mode"], best["workgroups"])
    best = dict(best, candidates=results)
    _CACHE[key] = best
    _store()
    return best


def tune_policy(mlp, obs, mask, M: int, outs: tuple, reps: int = 10, use_cache: bool = True) -> dict:
    """Picks the policy-forward row tile; returns {"tile_rows", "ms"}."""
    _load()
    key = f"policy|{_arch()}|D{mlp.D}|H{mlp.H}|A{mlp.A}|M{M}"
    if use_cache and key in _CACHE:
        best = _CACHE[key]
        mlp.set_tile_rows(best["tile_rows"])
        return best
    cands = [128, 64] if mlp.H <= 256 else [64]
    results = []
    for rows in cands:
        mlp.set_tile_rows(rows)
        results.append(dict(tile_rows=rows, ms=_time(lambda: mlp.forward(obs, mask, M, 0, 0, *outs), reps)))
    best = min(results, key=lambda r: r["ms"])
    mlp.set_tile_rows(best["tile_rows"])
    best = dict(best, candidates=results)
    _CACHE[key] = best
    _store()
    return best
