"""The C ABI without a GPU: the built library loads and exports every
function include/pamc.h declares, the Python binding covers them, and the
binding refuses to run without the library (no fallback path exists)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pamc.h")
LIB = os.path.join(ROOT, "paper_2606_25203_amd", "libpamc.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pamc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for must in ("pamc_create_instance_csr", "pamc_create_instance_dense_i8", "pamc_create_instance_dense_random",
                 "pamc_anneal", "pamc_sweep", "pamc_resample", "pamc_cluster_move", "pamc_best",
                 "pamc_get_state", "pamc_anneal_batch", "pamc_server_create", "pamc_server_submit",
                 "pamc_server_poll", "pamc_server_destroy", "pamc_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_exports_are_c_symbols():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for n in declared():
        assert n in syms, f"{n} is not an unmangled exported function"


def test_binding_covers_the_header(lib):
    sys.path.insert(0, ROOT)
    from paper_2606_25203_amd import pamc
    assert sorted(pamc.EXPORTED) == declared()


def test_last_error_without_gpu(lib):
    lib.pamc_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.pamc_last_error(), bytes)


def test_binding_fails_loudly_without_library(tmp_path):
    """Load the binding's module text against a path with no library: it
    must raise, not fall back to anything else."""
    src = open(os.path.join(ROOT, "paper_2606_25203_amd", "pamc.py")).read()
    mod = tmp_path / "pamc_copy.py"
    mod.write_text(src)
    code = f"import sys; sys.path.insert(0, {str(tmp_path)!r}); import pamc_copy"
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert r.returncode != 0 and "missing" in r.stderr


def test_invalid_arguments_rejected_on_host(lib):
    """Argument checks that run before any device call."""
    sys.path.insert(0, ROOT)
    from paper_2606_25203_amd import pamc
    out = ctypes.c_void_p()
    cfg = pamc.pamc_config(0, 100, 0, 0, None, 0)      # replicas not a multiple of 64
    st = lib.pamc_create_instance_csr(4, None, None, None, 0, 0, ctypes.byref(cfg), ctypes.byref(out))
    assert st == pamc.PAMC_ERR_INVALID_ARG
    cfg = pamc.pamc_config(0, 64, 7, 0, None, 0)       # unknown rule
    st = lib.pamc_create_instance_csr(4, None, None, None, 0, 0, ctypes.byref(cfg), ctypes.byref(out))
    assert st == pamc.PAMC_ERR_INVALID_ARG
    assert lib.pamc_anneal(None, None, None) == pamc.PAMC_ERR_INVALID_ARG
    assert lib.pamc_server_tick(None, 0, None, None) == pamc.PAMC_ERR_INVALID_ARG
    assert lib.pamc_anneal_batch(None, None, 0, None) == pamc.PAMC_OK
