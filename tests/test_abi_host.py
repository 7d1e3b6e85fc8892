"""Host-side checks of the C ABI (no GPU): the library loads, exports every entry point that
include/ace.h declares, and rejects bad arguments before touching the device."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ace.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+([a-z_]+)\s*\(", text, flags=re.M)))


def test_header_and_binding_agree():
    from paper_2405_01522_amd import _lib
    decl = _declared()
    assert "ace_build" in decl and "tda_coupling" in decl and "pair_poisson_batched" in decl
    assert set(decl) == set(_lib.SIGNATURES)


def test_library_exports_every_symbol():
    from paper_2405_01522_amd import _lib
    lib = _lib.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True).stdout
    for name in _declared():
        assert re.search(r"\bT %s\b" % name, out), name


def test_size_table_and_messages():
    from paper_2405_01522_amd import _lib
    lib = _lib.lib()
    for n in (8, 9, 10, 12, 16, 20, 24, 32, 40, 48, 56, 64):
        assert lib.ace_size_supported(n, 1) == 1          # FP32 complex
    for n in (8, 9, 10, 12, 16, 20, 24, 32, 40, 48, 56, 64):
        assert lib.ace_size_supported(n, 0) == 1          # FP64 complex (56, 64: column strips)
    assert lib.ace_size_supported(11, 1) == 0             # radix 11 not compiled
    assert lib.ace_size_supported(16, 7) == 0             # bad dtype
    assert lib.ace_strerror(-5).decode() == "-M is not positive definite"


def test_invalid_arguments_rejected_on_host():
    from paper_2405_01522_amd import _lib
    lib = _lib.lib()
    h = ctypes.c_void_p()
    assert lib.ace_ctx_create(16, 0.0, 0, None, ctypes.byref(h)) == -1
    assert lib.ace_ctx_create(16, 0.3, 9, None, ctypes.byref(h)) == -1
    assert lib.ace_ctx_create(11, 0.3, 0, None, ctypes.byref(h)) == -2
    assert lib.ace_ctx_create(16, 0.3, 0, None, None) == -1
    assert lib.ace_build(None, None, 1, None, None, None) == -1
    assert lib.ace_apply(None, None, 1, None, 1, None) == -1
    assert lib.pair_poisson_batched(None, None, 1, None, 1, None, 1, None) == -1
    assert lib.pair_poisson_batched_dev(None, None, 1, None, 1, None, 1, None) == -1
    assert lib.tda_coupling(None, None, 1, None, 1, 2, None) == -1
    assert lib.ace_ctx_destroy(None) == 0


@pytest.mark.slow
def test_register_dft_and_two_step_transform_on_host(tmp_path):
    """The register DFTs and the P = P1*P2 two-step transform of the Poisson passes, run on the
    CPU against a naive long-double DFT (the routines are __host__ __device__)."""
    exe = tmp_path / "dft_check"
    src = os.path.join(ROOT, "tests", "native", "dft_host_check.hip")
    res = subprocess.run(["hipcc", "-O1", "-std=c++17", "-o", str(exe), src],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True)
    assert run.returncode == 0 and "OK" in run.stdout, run.stdout


@pytest.mark.slow
def test_abi_layer_under_address_and_ub_sanitizers(tmp_path):
    """The host side of the C ABI (abi.cpp, batch.cpp, scf_driver.cpp) rebuilt with ASan and
    UBSan, linked with the kernels' objects, and driven through every entry point's argument
    checks and, on a machine without a GPU, the failure paths of context / batch / network
    creation (partial set-up released).  Any sanitizer report fails the run."""
    from paper_2405_01522_amd import build
    exe = build.build_sanitized_driver(os.path.join(ROOT, "tests", "native", "abi_sanitize.cpp"),
                                       str(tmp_path), jobs=8)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0 and "OK" in run.stdout, (run.stdout + run.stderr)[-4000:]


def test_binding_rejects_wrong_result_tensors():
    """Caller-supplied result tensors are checked before their pointers reach the library:
    a wrong dtype for M or a result block of the wrong shape is a ValueError, not a write past
    the end of an allocation."""
    import torch
    from paper_2405_01522_amd import api
    dev = torch.device("cpu")
    ok = torch.zeros((8, 8), dtype=torch.complex128)
    assert api.check_out(ok, "m_out", (8, 8), torch.complex128, dev) is not None
    with pytest.raises(ValueError, match="dtype"):
        api.check_out(torch.zeros((8, 8), dtype=torch.float32), "m_out", (8, 8),
                      torch.complex128, dev)
    with pytest.raises(ValueError, match="shape"):
        api.check_out(torch.zeros((16, 16), dtype=torch.float64), "out", (512, 512),
                      torch.float64, dev)
    with pytest.raises(ValueError, match="contiguous"):
        api.check_out(torch.zeros((8, 16), dtype=torch.float64)[:, ::2], "out", (8, 8),
                      torch.float64, dev)
    with pytest.raises(ValueError, match="expected cuda"):
        api.check_out(ok, "m_out", (8, 8), torch.complex128, torch.device("cuda", 0))
