"""ctypes binding of libecon_mi355x.so (argument marshalling only).

Every step of the path runs in the library's HIP kernels; this module turns
torch tensors into device pointers and HIP streams, and raises on any error
code.  It loads the in-tree build and fails loudly when it is missing: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libecon_mi355x.so")

EJ_MAX_P, EJ_MAX_K = 128, 16
PPO_LOSS_TERMS = 5  # surrogate, value, entropy, clipped fraction, loss


class EjObsScales(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("coin", "labor", "orders", "res", "skill", "rate", "phase", "price",
                                          "count")]


class EjEnvConfig(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("E", "N", "R", "P", "X", "max_orders", "P_tax", "K", "T", "R_kappa",
                                          "R_d", "kappa_c", "start_coin", "labor_gather", "labor_craft",
                                          "labor_trade", "allow_noop", "skill_mode")] + [
        ("eta", C.c_double), ("omega", C.c_double), ("seed", C.c_uint64),
        ("prices", C.c_int32 * EJ_MAX_P), ("cutoffs", C.c_int32 * EJ_MAX_K), ("scales", EjObsScales)]


class EjEnvDims(C.Structure):
    _fields_ = [("M", C.c_int64), ("A", C.c_int32), ("mask_words", C.c_int32), ("D", C.c_int32),
                ("D_stride", C.c_int32), ("D_gov", C.c_int32), ("K", C.c_int32), ("E", C.c_int32),
                ("D_metrics", C.c_int32)]


_STATE_FIELDS = ("t", "ep", "rates", "coin_inv", "coin_esc", "labor", "snap", "sc", "res_inv", "res_esc", "sg",
                 "orders")


class EjStateView(C.Structure):
    _fields_ = [(n, C.POINTER(C.c_int32)) for n in _STATE_FIELDS]


class EjMlpDesc(C.Structure):
    _fields_ = [("D", C.c_int32), ("D_stride", C.c_int32), ("H", C.c_int32), ("A", C.c_int32),
                ("tile_rows", C.c_int32)]


class EjMlpLayout(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_params", "n_work", "W1", "b1", "W2", "b2", "W3", "b3", "params_stride",
                                          "work_stride")]


class EjPpoBatch(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("obs", "mask", "act", "logp_old", "val_old", "adv", "ret")] + [
        (n, C.c_int64) for n in ("M_total", "perm_a", "perm_c", "row_begin", "rows", "row_stride", "row_offset")] + [
        ("records", C.c_void_p)]


class EjPpoHparams(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("clip", "vclip", "vf_coef", "ent_coef")]


class EjRolloutBuffers(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("obs", "mask", "act", "logp", "val", "ent", "rew", "done", "gov_rew",
                                           "last_val", "adv", "ret", "tmp", "ctr")]


class EjRolloutConfig(C.Structure):
    _fields_ = [("T", C.c_int32), ("groups", C.c_int32), ("last_value", C.c_int32), ("carry", C.c_int32),
                ("seed", C.c_uint64), ("gamma", C.c_float), ("lam", C.c_float)]


class EjAutotuneResult(C.Structure):
    _fields_ = [("env_mode", C.c_int32), ("env_workgroups", C.c_int32), ("agents_per_wave", C.c_int32),
                ("policy_tile_rows", C.c_int32), ("env_ms", C.c_float), ("policy_ms", C.c_float),
                ("candidates", C.c_int32)]


class EconError(RuntimeError):
    pass


_lib = None


def lib():
    """The loaded library (in-tree build).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise EconError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    L.ej_strerror.argtypes = [C.c_int]
    L.ej_strerror.restype = C.c_char_p
    L.ej_last_hip_error.restype = C.c_int
    L.ej_env_create.argtypes = [C.POINTER(EjEnvConfig), C.POINTER(i32), C.POINTER(vp)]
    L.ej_env_destroy.argtypes = [vp]
    L.ej_env_dims.argtypes = [vp, C.POINTER(EjEnvDims)]
    L.ej_env_row_offsets.argtypes = [vp]
    L.ej_env_row_offsets.restype = C.POINTER(i32)
    L.ej_env_reset.argtypes = [vp, i32, vp]
    L.ej_env_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.ej_env_step_range.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.ej_env_observe.argtypes = [vp, vp, vp, vp, vp]
    L.ej_env_random_actions.argtypes = [vp, u64, vp, vp, vp]
    L.ej_env_get_state.argtypes = [vp, C.POINTER(EjStateView), vp]
    L.ej_env_set_state.argtypes = [vp, C.POINTER(EjStateView), vp]
    L.ej_env_status.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), vp]
    L.ej_env_set_launch.argtypes = [vp, i32, i32]
    L.ej_env_set_gov_draw.argtypes = [vp, i32, C.c_uint64]
    L.ej_env_set_agents_per_wave.argtypes = [vp, i32]
    L.ej_env_enable_metrics.argtypes = [vp, i32]
    L.ej_env_episode_metrics.argtypes = [vp, vp, vp]
    _declare_learner(L)
    _lib = L
    return L


def _declare_learner(L):
    """Signatures of the policy / learner entry points (present once built)."""
    vp, i32, i64, u64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_float
    table = {
        "ej_mlp_layout": [C.POINTER(EjMlpDesc), C.POINTER(EjMlpLayout)],
        "ej_mlp_sync_weights": [C.POINTER(EjMlpDesc), vp, vp, vp],
        "ej_policy_forward": [C.POINTER(EjMlpDesc), vp, vp, vp, vp, i64, i64, u64, u64, vp, vp, vp, vp, vp, vp, vp],
        "ej_counter_add": [vp, u64, vp],
        "ej_policy_forward_grouped": [C.POINTER(EjMlpDesc), i32, vp, vp, vp, vp, i64, i64, u64, u64, vp, vp, vp, vp,
                                      vp, vp, vp],
        "ej_mlp_sync_weights_grouped": [C.POINTER(EjMlpDesc), i32, vp, vp, vp],
        "ej_gae": [vp, vp, vp, vp, i32, i64, f32, f32, vp, vp, vp],
        "ej_ppo_workspace_size": [C.POINTER(EjMlpDesc), i64, C.POINTER(i64)],
        "ej_ppo_record_bytes": [C.POINTER(EjMlpDesc), C.POINTER(i64)],
        "ej_ppo_pack": [C.POINTER(EjMlpDesc), C.POINTER(EjPpoBatch), vp, vp],
        "ej_ppo_backward": [C.POINTER(EjMlpDesc), vp, vp, C.POINTER(EjPpoBatch), C.POINTER(EjPpoHparams), vp, i64,
                            vp, vp, vp],
        "ej_ppo_backward_static": [C.POINTER(EjMlpDesc), vp, vp, C.POINTER(EjPpoBatch), C.POINTER(EjPpoHparams),
                                   vp, vp, vp],
        "ej_adam": [vp, vp, vp, vp, i64, i32, f32, f32, f32, f32, vp],
        "ej_gov_policy_forward": [C.POINTER(EjMlpDesc), i32, vp, vp, vp, vp, i64, u64, u64, vp, vp, vp, vp, vp, vp,
                                  vp, vp],
        "ej_gov_ppo_workspace_size": [C.POINTER(EjMlpDesc), i32, i64, C.POINTER(i64)],
        "ej_gov_ppo_backward": [C.POINTER(EjMlpDesc), i32, vp, vp, C.POINTER(EjPpoBatch), C.POINTER(EjPpoHparams),
                                vp, i64, vp, vp, vp],
        "ej_sum_steps": [vp, i32, i32, i64, vp, vp],
        "ej_rollout_capture": [vp, C.POINTER(EjMlpDesc), vp, vp, C.POINTER(EjRolloutConfig),
                               C.POINTER(EjRolloutBuffers), C.POINTER(vp)],
        "ej_rollout_launch": [vp, vp],
        "ej_rollout_launch_plain": [vp, vp],
        "ej_rollout_destroy": [vp],
        "ej_autotune": [vp, C.POINTER(EjMlpDesc), vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32,
                        C.POINTER(EjAutotuneResult), vp],
    }
    for name, args in table.items():
        fn = getattr(L, name, None)
        if fn is not None:
            fn.argtypes = args


def check(rc: int, what: str = ""):
    if rc != 0:
        msg = lib().ej_strerror(rc).decode()
        hip = lib().ej_last_hip_error()
        raise EconError(f"{what}: {msg} (code {rc}, hip error {hip})")


def ptr(t) -> int | None:
    """Device pointer of a torch tensor (None passes NULL)."""
    if t is None:
        return None
    return t.data_ptr()


def stream_ptr(stream=None) -> int | None:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def make_env_config(cfg: dict, scales: dict) -> EjEnvConfig:
    c = EjEnvConfig()
    for n in ("E", "N", "R", "P", "X", "max_orders", "P_tax", "K", "T", "R_kappa", "R_d", "kappa_c",
              "start_coin", "labor_gather", "labor_craft", "labor_trade", "allow_noop"):
        setattr(c, n, int(cfg[n]))
    c.skill_mode = int(cfg.get("skill_mode", 0))
    c.eta, c.omega, c.seed = float(cfg["eta"]), float(cfg["omega"]), int(cfg.get("seed", 0))
    for i, v in enumerate(cfg["prices"]):
        c.prices[i] = int(v)
    for i, v in enumerate(cfg["cutoffs"]):
        c.cutoffs[i] = int(v)
    c.scales = EjObsScales(**{k: float(v) for k, v in scales.items()})
    return c


class Env:
    """A batch of E economies on the GPU (thin owner of an ej_env handle)."""

    def __init__(self, cfg: dict, scales: dict, n_per_env=None):
        import torch
        self.cfg = dict(cfg)
        self._c = make_env_config(cfg, scales)
        h = C.c_void_p()
        arr = None
        if n_per_env is not None:
            arr = np.ascontiguousarray(n_per_env, dtype=np.int32)
            check(lib().ej_env_create(C.byref(self._c), arr.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(h)),
                  "ej_env_create")
        else:
            check(lib().ej_env_create(C.byref(self._c), None, C.byref(h)), "ej_env_create")
        self._h = h
        d = EjEnvDims()
        check(lib().ej_env_dims(h, C.byref(d)), "ej_env_dims")
        self.M, self.A, self.W, self.D, self.Ds, self.Dg, self.K = (int(d.M), d.A, d.mask_words, d.D, d.D_stride,
                                                                      d.D_gov, d.K)
        self.E = int(cfg["E"])
        ro = lib().ej_env_row_offsets(h)
        self.row_offsets = np.array([ro[i] for i in range(self.E + 1)], np.int64)
        self.device = torch.device("cuda")

    def close(self):
        if getattr(self, "_h", None):
            lib().ej_env_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- buffers ----
    def buffers(self):
        import torch
        dev = self.device
        return dict(
            act=torch.zeros(self.M, dtype=torch.int32, device=dev),
            gov=torch.zeros(max(self.E * self.K, 1), dtype=torch.int32, device=dev),
            rew=torch.zeros(self.M, dtype=torch.float32, device=dev),
            gov_rew=torch.zeros(self.E, dtype=torch.float32, device=dev),
            done=torch.zeros(self.M, dtype=torch.uint8, device=dev),
            obs=torch.zeros((self.M, self.Ds), dtype=torch.int16, device=dev),
            mask=torch.zeros((self.M, self.W), dtype=torch.int32, device=dev),
            gov_obs=torch.zeros((self.E, self.Dg), dtype=torch.float32, device=dev),
        )

    # ---- entry points ----
    def reset(self, episode: int = 0, stream=None):
        check(lib().ej_env_reset(self._h, episode, stream_ptr(stream)), "ej_env_reset")

    def step(self, act, gov, rew, gov_rew, done, obs=None, mask=None, stream=None, economies=None):
        """One step of every economy, or of economies [begin, end) when
        `economies` is given (arrays keep the whole batch's layout)."""
        if economies is None:
            check(lib().ej_env_step(self._h, ptr(act), ptr(gov), ptr(rew), ptr(gov_rew), ptr(done), ptr(obs),
                                    ptr(mask), stream_ptr(stream)), "ej_env_step")
        else:
            check(lib().ej_env_step_range(self._h, economies[0], economies[1], ptr(act), ptr(gov), ptr(rew),
                                          ptr(gov_rew), ptr(done), ptr(obs), ptr(mask), stream_ptr(stream)),
                  "ej_env_step_range")

    def observe(self, obs, mask, gov_obs=None, stream=None):
        check(lib().ej_env_observe(self._h, ptr(obs), ptr(mask), ptr(gov_obs), stream_ptr(stream)), "ej_env_observe")

    def random_actions(self, act_seed: int, act, gov, stream=None):
        check(lib().ej_env_random_actions(self._h, act_seed, ptr(act), ptr(gov), stream_ptr(stream)),
              "ej_env_random_actions")

    def enable_metrics(self, enabled: bool = True):
        check(lib().ej_env_enable_metrics(self._h, 1 if enabled else 0), "ej_env_enable_metrics")

    def episode_metrics(self, out=None, stream=None):
        """[E, 5 R + 9] float64 device tensor: every economy's record of its
        last completed episode (layout in the header)."""
        import torch
        if out is None:
            out = torch.zeros((self.E, 5 * self.cfg["R"] + 9), dtype=torch.float64, device="cuda")
        check(lib().ej_env_episode_metrics(self._h, ptr(out), stream_ptr(stream)), "ej_env_episode_metrics")
        return out

    def set_agents_per_wave(self, apw: int):
        """Agents per wavefront of the step (64, 32 or 16; same results)."""
        check(lib().ej_env_set_agents_per_wave(self._h, apw), "ej_env_set_agents_per_wave")

    def set_launch(self, mode: int, workgroups: int = 0):
        """mode 0: one workgroup per economy; 1: persistent work queue."""
        check(lib().ej_env_set_launch(self._h, mode, workgroups), "ej_env_set_launch")

    def set_gov_draw(self, enabled: bool, seed: int = 0):
        """Let step() draw uniform government levels itself (gov=None)."""
        check(lib().ej_env_set_gov_draw(self._h, int(enabled), seed), "ej_env_set_gov_draw")

    def status(self, stream=None):
        a, g = C.c_int64(), C.c_int64()
        check(lib().ej_env_status(self._h, C.byref(a), C.byref(g), stream_ptr(stream)), "ej_env_status")
        return a.value, g.value

    def _view(self, arrays):
        v = EjStateView()
        for n in _STATE_FIELDS:
            setattr(v, n, arrays[n].ctypes.data_as(C.POINTER(C.c_int32)))
        return v

    def get_state(self, stream=None) -> dict:
        E, M, R, X, K = self.E, self.M, self.cfg["R"], self.cfg["X"], self.K
        a = dict(t=np.zeros(E, np.int32), ep=np.zeros(E, np.int32), rates=np.zeros((E, max(K, 1)), np.int32))
        for n in ("coin_inv", "coin_esc", "labor", "snap", "sc"):
            a[n] = np.zeros(M, np.int32)
        for n in ("res_inv", "res_esc", "sg"):
            a[n] = np.zeros((R, M), np.int32)
        a["orders"] = np.zeros((X, M), np.int32)
        v = self._view(a)
        check(lib().ej_env_get_state(self._h, C.byref(v), stream_ptr(stream)), "ej_env_get_state")
        a["rates"] = a["rates"][:, :K]
        return a

    def set_state(self, st: dict, stream=None):
        E, K = self.E, self.K
        a = {n: np.ascontiguousarray(st[n], dtype=np.int32) for n in _STATE_FIELDS}
        if K == 0:
            a["rates"] = np.zeros((E, 1), np.int32)
        v = self._view(a)
        check(lib().ej_env_set_state(self._h, C.byref(v), stream_ptr(stream)), "ej_env_set_state")

    def env_state(self, st: dict, e: int) -> dict:
        """The state of economy e in the oracle's per-economy layout."""
        lo, hi = int(self.row_offsets[e]), int(self.row_offsets[e + 1])
        out = dict(t=int(st["t"][e]), ep=int(st["ep"][e]), rates=st["rates"][e].copy())
        for n in ("coin_inv", "coin_esc", "labor", "snap", "sc"):
            out[n] = st[n][lo:hi].copy()
        for n in ("res_inv", "res_esc", "sg", "orders"):
            out[n] = st[n][:, lo:hi].copy()
        out["n_active"] = (out["orders"] >= 0).sum(axis=0).astype(np.int32)
        return out


class Mlp:
    """Shared policy network parameters on the GPU: the flat fp32 vector and
    its bf16 work copy (both torch tensors; the kernels own the layouts)."""

    def __init__(self, D: int, D_stride: int, H: int, A: int, weights: dict | None = None, tile_rows: int = 0):
        import torch
        self.desc = EjMlpDesc(D, D_stride, H, A, tile_rows)
        lay = EjMlpLayout()
        check(lib().ej_mlp_layout(C.byref(self.desc), C.byref(lay)), "ej_mlp_layout")
        self.layout = {n: int(getattr(lay, n)) for n, _ in EjMlpLayout._fields_}
        self.D, self.Ds, self.H, self.A = D, D_stride, H, A
        self.params = torch.zeros(self.layout["n_params"], dtype=torch.float32, device="cuda")
        self.work = torch.zeros(self.layout["n_work"], dtype=torch.int16, device="cuda")
        if weights is not None:
            self.load(weights)

    def flat(self, weights: dict) -> np.ndarray:
        v = np.zeros(self.layout["n_params"], np.float32)
        for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
            a = np.asarray(weights[k], np.float32).ravel()
            v[self.layout[k]:self.layout[k] + a.size] = a
        return v

    def unflat(self, v) -> dict:
        v = np.asarray(v, np.float32)
        D, H, A1 = self.D, self.H, self.A + 1
        shapes = dict(W1=(D, H), b1=(H,), W2=(H, H), b2=(H,), W3=(H, A1), b3=(A1,))
        return {k: v[self.layout[k]:self.layout[k] + int(np.prod(s))].reshape(s) for k, s in shapes.items()}

    def load(self, weights: dict, stream=None):
        import torch
        self.params.copy_(torch.from_numpy(self.flat(weights)))
        self.sync(stream)

    def set_tile_rows(self, rows: int):
        """Row tile of the policy forward (0: default, 64 or 128)."""
        self.desc.tile_rows = rows

    def sync(self, stream=None):
        check(lib().ej_mlp_sync_weights(C.byref(self.desc), ptr(self.params), ptr(self.work), stream_ptr(stream)),
              "ej_mlp_sync_weights")

    def forward(self, obs, mask, M: int, seed: int, ctr: int, act, logp, val, ent, logits=None, stream=None,
                ctr_base=None, row_base: int = 0):
        check(lib().ej_policy_forward(C.byref(self.desc), ptr(self.params), ptr(self.work), ptr(obs), ptr(mask), M,
                                      row_base, seed, ctr, ptr(ctr_base), ptr(act), ptr(logp), ptr(val), ptr(ent),
                                      ptr(logits), stream_ptr(stream)), "ej_policy_forward")


def gae(rew, val, done, last_val, T: int, M: int, gamma: float, lam: float, adv, ret, stream=None):
    check(lib().ej_gae(ptr(rew), ptr(val), ptr(done), ptr(last_val), T, M, gamma, lam, ptr(adv), ptr(ret),
                       stream_ptr(stream)), "ej_gae")


def adam(params, grads, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(lib().ej_adam(ptr(params), ptr(grads), ptr(m), ptr(v), params.numel(), step, lr, beta1, beta2, eps,
                        stream_ptr(stream)), "ej_adam")


def ppo_workspace_bytes(mlp: "Mlp", rows: int) -> int:
    out = C.c_int64()
    check(lib().ej_ppo_workspace_size(C.byref(mlp.desc), rows, C.byref(out)), "ej_ppo_workspace_size")
    return int(out.value)


def ppo_record_bytes(mlp: "Mlp") -> int:
    out = C.c_int64()
    check(lib().ej_ppo_record_bytes(C.byref(mlp.desc), C.byref(out)), "ej_ppo_record_bytes")
    return int(out.value)


def ppo_pack(mlp: "Mlp", storage: dict, M_total: int, records, stream=None, row_stride: int = 1,
             row_offset: int = 0):
    """ej_ppo_pack: record s of `records` (uint8, M_total * ppo_record_bytes)
    <- sample s of the storage arrays."""
    if records.numel() < M_total * ppo_record_bytes(mlp):
        raise EconError("records buffer too small")
    b = EjPpoBatch(*(ptr(storage[k]) for k in ("obs", "mask", "act", "logp_old", "val_old", "adv", "ret")),
                   M_total, 1, 0, 0, 0, row_stride, row_offset, None)
    check(lib().ej_ppo_pack(C.byref(mlp.desc), C.byref(b), ptr(records), stream_ptr(stream)), "ej_ppo_pack")


def ppo_backward(mlp: "Mlp", storage: dict, M_total: int, perm_a: int, perm_c: int, row_begin: int, rows: int,
                 hp: dict, workspace, grads, loss, stream=None, row_stride: int = 1, row_offset: int = 0,
                 params=None, work=None, records=None):
    """storage: torch tensors obs, mask, act, logp_old, val_old, adv, ret indexed by sample;
    loss: at least PPO_LOSS_TERMS floats; records: optional ppo_pack output of the same storage."""
    if loss.numel() < PPO_LOSS_TERMS:
        raise EconError(f"ej_ppo_backward writes {PPO_LOSS_TERMS} loss terms; got {loss.numel()}")
    b = EjPpoBatch(*(ptr(storage[k]) for k in ("obs", "mask", "act", "logp_old", "val_old", "adv", "ret")),
                   M_total, perm_a, perm_c, row_begin, rows, row_stride, row_offset, ptr(records))
    h = EjPpoHparams(hp["clip"], hp["vclip"], hp["vf_coef"], hp["ent_coef"])
    p_ptr = ptr(mlp.params) if params is None else params
    w_ptr = ptr(mlp.work) if work is None else work
    check(lib().ej_ppo_backward(C.byref(mlp.desc), p_ptr, w_ptr, C.byref(b), C.byref(h),
                                ptr(workspace), workspace.numel(), ptr(grads), ptr(loss), stream_ptr(stream)),
          "ej_ppo_backward")


EJ_ESCRATCH = -5
PPO_STATIC_SCRATCH_BYTES = 64 << 20


def ppo_backward_static(mlp: "Mlp", storage: dict, M_total: int, perm_a: int, perm_c: int, row_begin: int,
                        rows: int, hp: dict, grads, loss, stream=None):
    """ej_ppo_backward without a caller workspace (the library's static
    device scratch); raises when the minibatch needs more than it holds."""
    if loss.numel() < PPO_LOSS_TERMS:
        raise EconError(f"ej_ppo_backward_static writes {PPO_LOSS_TERMS} loss terms; got {loss.numel()}")
    b = EjPpoBatch(*(ptr(storage[k]) for k in ("obs", "mask", "act", "logp_old", "val_old", "adv", "ret")),
                   M_total, perm_a, perm_c, row_begin, rows)
    h = EjPpoHparams(hp["clip"], hp["vclip"], hp["vf_coef"], hp["ent_coef"])
    check(lib().ej_ppo_backward_static(C.byref(mlp.desc), ptr(mlp.params), ptr(mlp.work), C.byref(b), C.byref(h),
                                       ptr(grads), ptr(loss), stream_ptr(stream)), "ej_ppo_backward_static")


def counter_add(counter, inc: int, stream=None):
    check(lib().ej_counter_add(ptr(counter), inc, stream_ptr(stream)), "ej_counter_add")


class Rollout:
    """A T-step rollout captured by the library as one HIP graph
    (ej_rollout_capture): policy forward + economy step per step, economy
    groups on their own streams, then the last-value forward, GAE and the
    sampling-counter advance.  `bufs` holds the torch storage it writes
    (kept alive here, since the graph keeps the pointers)."""

    def __init__(self, env: "Env", mlp: "Mlp", bufs: dict, T: int, seed: int, groups: int = 1,
                 last_value: bool = True, gamma: float = 0.99, lam: float = 0.95, carry: bool = False):
        self.env, self.mlp, self.bufs = env, mlp, bufs
        b = EjRolloutBuffers(*(ptr(bufs.get(k)) for k in ("obs", "mask", "act", "logp", "val", "ent", "rew", "done",
                                                           "gov_rew", "last_val", "adv", "ret", "tmp", "ctr")))
        cfg = EjRolloutConfig(T, groups, 1 if last_value else 0, 1 if carry else 0, seed, gamma, lam)
        h = C.c_void_p()
        check(lib().ej_rollout_capture(env._h, C.byref(mlp.desc), ptr(mlp.params), ptr(mlp.work), C.byref(cfg),
                                       C.byref(b), C.byref(h)), "ej_rollout_capture")
        self._h = h

    def launch(self, stream=None):
        check(lib().ej_rollout_launch(self._h, stream_ptr(stream)), "ej_rollout_launch")

    def launch_plain(self, stream=None):
        check(lib().ej_rollout_launch_plain(self._h, stream_ptr(stream)), "ej_rollout_launch_plain")

    def close(self):
        if getattr(self, "_h", None):
            lib().ej_rollout_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(env: "Env", mlp: "Mlp | None", buf: dict, reps: int = 10, stream=None) -> dict:
    """ej_autotune: times the economy-step launch shapes (and the policy row
    tile when mlp is given) and applies the fastest; everything a trial step
    changes is restored."""
    r = EjAutotuneResult()
    check(lib().ej_autotune(env._h, C.byref(mlp.desc) if mlp is not None else None,
                            ptr(mlp.params) if mlp is not None else None, ptr(mlp.work) if mlp is not None else None,
                            ptr(buf["obs"]), ptr(buf["mask"]), ptr(buf["act"]), ptr(buf.get("gov")),
                            ptr(buf.get("logp")), ptr(buf.get("val")), ptr(buf.get("ent")), ptr(buf["rew"]),
                            ptr(buf["gov_rew"]), ptr(buf["done"]), reps, C.byref(r), stream_ptr(stream)),
          "ej_autotune")
    return {n: (float(getattr(r, n)) if n.endswith("_ms") else int(getattr(r, n))) for n, _ in r._fields_}


def rollout_storage(env: "Env", T: int, last_value: bool = False) -> dict:
    """Device arrays of a T-step rollout in the layout ej_rollout_capture
    writes; obs[0] / mask[0] hold the observation of the current state."""
    import torch
    z = dict(device="cuda")
    M, E = env.M, env.E
    b = dict(obs=torch.zeros((T + 1, M, env.Ds), dtype=torch.int16, **z),
             mask=torch.zeros((T + 1, M, env.W), dtype=torch.int32, **z),
             act=torch.zeros((T, M), dtype=torch.int32, **z), logp=torch.zeros((T, M), **z),
             val=torch.zeros((T, M), **z), ent=torch.zeros((T, M), **z), rew=torch.zeros((T, M), **z),
             done=torch.zeros((T, M), dtype=torch.uint8, **z), gov_rew=torch.zeros((T, E), **z),
             ctr=torch.zeros(1, dtype=torch.int64, **z))
    if last_value:
        b.update(last_val=torch.zeros(M, **z), adv=torch.zeros((T, M), **z), ret=torch.zeros((T, M), **z),
                 tmp=torch.zeros(3 * M, **z))
    env.observe(b["obs"][0], b["mask"][0])
    return b


def gov_policy_forward(mlp: "Mlp", K: int, gov_obs, scale, E: int, seed: int, ctr: int, levels, logp, val, ent,
                       obs_bf16=None, logits=None, ctr_base=None, stream=None):
    """ej_gov_policy_forward: the government's K tax levels per economy."""
    check(lib().ej_gov_policy_forward(C.byref(mlp.desc), K, ptr(mlp.params), ptr(mlp.work), ptr(gov_obs), ptr(scale),
                                      E, seed, ctr, ptr(ctr_base), ptr(levels), ptr(logp), ptr(val), ptr(ent),
                                      ptr(obs_bf16), ptr(logits), stream_ptr(stream)), "ej_gov_policy_forward")


def gov_ppo_workspace_bytes(mlp: "Mlp", K: int, rows: int) -> int:
    out = C.c_int64()
    check(lib().ej_gov_ppo_workspace_size(C.byref(mlp.desc), K, rows, C.byref(out)), "ej_gov_ppo_workspace_size")
    return int(out.value)


def gov_ppo_backward(mlp: "Mlp", K: int, storage: dict, M_total: int, perm_a: int, perm_c: int, row_begin: int,
                     rows: int, hp: dict, workspace, grads, loss, stream=None):
    """storage: torch tensors obs (bf16 rows), act (levels [M_total, K]), logp_old, val_old, adv, ret."""
    if loss.numel() < PPO_LOSS_TERMS:
        raise EconError(f"ej_gov_ppo_backward writes {PPO_LOSS_TERMS} loss terms; got {loss.numel()}")
    b = EjPpoBatch(ptr(storage["obs"]), None, *(ptr(storage[k]) for k in ("act", "logp_old", "val_old", "adv", "ret")),
                   M_total, perm_a, perm_c, row_begin, rows)
    h = EjPpoHparams(hp["clip"], hp["vclip"], hp["vf_coef"], hp["ent_coef"])
    check(lib().ej_gov_ppo_backward(C.byref(mlp.desc), K, ptr(mlp.params), ptr(mlp.work), C.byref(b), C.byref(h),
                                    ptr(workspace), workspace.numel(), ptr(grads), ptr(loss), stream_ptr(stream)),
          "ej_gov_ppo_backward")


def sum_steps(x, t_begin: int, t_end: int, E: int, out, stream=None):
    """out[e] = sum over t in [t_begin, t_end) of x[t, e] (ej_sum_steps)."""
    check(lib().ej_sum_steps(ptr(x), t_begin, t_end, E, ptr(out), stream_ptr(stream)), "ej_sum_steps")


class GroupedMlp:
    """G weight sets of one network stacked in one tensor (per-agent
    policies): set g's fp32 parameters at g * params_stride, its bf16 work
    copy at g * work_stride."""

    def __init__(self, D: int, D_stride: int, H: int, A: int, groups: int, weights: list | None = None):
        import torch
        self.desc = EjMlpDesc(D, D_stride, H, A, 0)
        lay = EjMlpLayout()
        check(lib().ej_mlp_layout(C.byref(self.desc), C.byref(lay)), "ej_mlp_layout")
        self.layout = {n: int(getattr(lay, n)) for n, _ in EjMlpLayout._fields_}
        self.D, self.Ds, self.H, self.A, self.G = D, D_stride, H, A, groups
        self.ps, self.wst = self.layout["params_stride"], self.layout["work_stride"]
        self.params = torch.zeros(groups * self.ps, dtype=torch.float32, device="cuda")
        self.work = torch.zeros(groups * self.wst, dtype=torch.int16, device="cuda")
        self._one = Mlp(D, D_stride, H, A)
        if weights is not None:
            for g, w in enumerate(weights):
                self.params[g * self.ps:g * self.ps + self.layout["n_params"]].copy_(
                    torch.from_numpy(self._one.flat(w)))
            self.sync()

    def set_params(self, g: int):
        """Parameter view of set g."""
        return self.params[g * self.ps:g * self.ps + self.layout["n_params"]]

    def params_ptr(self, g: int) -> int:
        return self.params.data_ptr() + 4 * g * self.ps

    def work_ptr(self, g: int) -> int:
        return self.work.data_ptr() + 2 * g * self.wst

    def unflat(self, g: int, v=None) -> dict:
        return self._one.unflat(self.set_params(g).cpu().numpy() if v is None else v)

    def sync(self, stream=None):
        check(lib().ej_mlp_sync_weights_grouped(C.byref(self.desc), self.G, ptr(self.params), ptr(self.work),
                                                stream_ptr(stream)), "ej_mlp_sync_weights_grouped")

    def forward(self, obs, mask, rows_per_group: int, row_stride: int, seed: int, ctr: int, act, logp, val, ent,
                logits=None, ctr_base=None, stream=None):
        check(lib().ej_policy_forward_grouped(C.byref(self.desc), self.G, ptr(self.params), ptr(self.work), ptr(obs),
                                              ptr(mask), rows_per_group, row_stride, seed, ctr, ptr(ctr_base),
                                              ptr(act), ptr(logp), ptr(val), ptr(ent), ptr(logits),
                                              stream_ptr(stream)), "ej_policy_forward_grouped")
