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
