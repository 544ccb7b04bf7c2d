"""The C-ABI library loads on the CPU and exports every function the public
header declares (no compute calls: this host has no GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(ej_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ej_env_create", "ej_env_reset", "ej_env_step", "ej_env_observe", "ej_policy_forward",
                     "ej_ppo_backward", "ej_gae", "ej_adam"):
        assert required in names, required


def test_library_exports_every_declared_symbol():
    from paper_2410_22165_amd import binding
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_without_gpu():
    from paper_2410_22165_amd import binding
    lib = binding.lib()
    assert lib.ej_strerror(0) == b"ok"
    assert lib.ej_strerror(-4).startswith(b"configuration")


def test_static_scratch_backward_rejects_oversize_on_the_host():
    """ej_ppo_backward_static sizes the minibatch's workspace before any HIP
    call: one that does not fit the static scratch returns EJ_ESCRATCH (no
    device needed), and a NULL descriptor returns EJ_EINVAL."""
    import ctypes as C
    from paper_2410_22165_amd import binding
    L = binding.lib()
    desc = binding.EjMlpDesc(35, 40, 256, 125, 64)
    need = C.c_int64(0)
    assert L.ej_ppo_workspace_size(C.byref(desc), 100000, C.byref(need)) == 0
    assert need.value > binding.PPO_STATIC_SCRATCH_BYTES
    b = binding.EjPpoBatch(*([None] * 7), 100000, 1, 0, 0, 100000)
    h = binding.EjPpoHparams(0.2, 10.0, 0.25, 0.01)
    rc = L.ej_ppo_backward_static(C.byref(desc), None, None, C.byref(b), C.byref(h), None, None, None)
    assert rc == binding.EJ_ESCRATCH
    assert L.ej_ppo_backward_static(None, None, None, C.byref(b), C.byref(h), None, None, None) == -1


def test_mlp_layout_limits_on_the_host():
    """ej_mlp_layout (host only): rows of up to 64 features take a 64-column
    first layer, wider rows (up to 128, H >= 128) a 128-column one; the
    12-resource multi-agent economy gives 7 + 7 * 12 = 91 features."""
    import ctypes as C
    from paper_2410_22165_amd import binding
    L = binding.lib()
    out = binding.EjMlpLayout()
    for D, Ds, H, ok in ((35, 40, 256, True), (64, 64, 64, True), (91, 96, 256, True), (128, 128, 512, True),
                         (91, 96, 64, False), (129, 136, 256, False), (40, 36, 256, False)):
        rc = L.ej_mlp_layout(C.byref(binding.EjMlpDesc(D, Ds, H, 86, 0)), C.byref(out))
        assert (rc == 0) == ok, (D, Ds, H, rc)
        if ok:
            k1 = 64 if Ds <= 64 else 128
            assert out.W1 == 0 and out.b1 == D * H and out.n_work == k1 * H + H * H + H * 128 + 128 * H + H * H
    # 128-row tiles take rows of at most 64 features
    assert L.ej_mlp_layout(C.byref(binding.EjMlpDesc(91, 96, 256, 86, 128)), C.byref(out)) != 0


def test_ppo_record_bytes_on_the_host():
    """Record size of ej_ppo_pack (host only): observation row padded to 16
    bytes, mask words, five 4-byte scalars, rounded up to 128 bytes."""
    import ctypes as C
    from paper_2410_22165_amd import binding
    L = binding.lib()
    out = C.c_int64()
    for (D, Ds, H, A), want in (((35, 40, 256, 125), 128), ((49, 56, 512, 507), 256), ((91, 96, 256, 86), 256),
                                ((64, 64, 128, 1000), 384), ((11, 16, 64, 9), 128)):
        assert L.ej_ppo_record_bytes(C.byref(binding.EjMlpDesc(D, Ds, H, A, 0)), C.byref(out)) == 0
        assert out.value == want, (D, Ds, A, out.value)
