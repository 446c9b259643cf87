"""Host-side checks of the C ABI library (no GPU needed): it loads, and it exports every
function the public header declares; the binding refuses to run without it."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sw2d.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sw2d_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1711_04471_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return ctypes.CDLL(_lib.LIB_PATH)


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("sw2d_create", "sw2d_step", "sw2d_reduce", "sw2d_destroy", "sw2d_workspace_bytes"):
        assert core in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_1711_04471_amd import _lib
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


def test_host_only_calls(lib):
    from paper_1711_04471_amd import _lib
    L = _lib.load()
    p = _lib.sw2d_params(66, 66, 100.0, 100.0, 9.81, 5.0, 0.05, 0)
    assert L.sw2d_workspace_bytes(ctypes.byref(p)) > 66 * 66 * 4
    bad = _lib.sw2d_params(66, 66, 100.0, 100.0, 9.81, 5.0, 1.5, 0)
    assert L.sw2d_workspace_bytes(ctypes.byref(bad)) == 0
    # rows wider than 2^28 cells are refused (32-bit row byte offsets), 2^28 itself is not
    wide = _lib.sw2d_params((1 << 28) + 2, 3, 100.0, 100.0, 9.81, 5.0, 0.05, 0)
    assert L.sw2d_workspace_bytes(ctypes.byref(wide)) == 0
    edge = _lib.sw2d_params(1 << 28, 3, 100.0, 100.0, 9.81, 5.0, 0.05, 0)
    assert L.sw2d_workspace_bytes(ctypes.byref(edge)) > 0
    assert L.sw2d_ring_capacity() >= 1000
    assert L.sw2d_strerror(-5).decode().startswith("workspace")
    assert L.sw2d_destroy(None) == 0
    assert L.sw2d_step(None, 1) == _lib.SW2D_ESTATE


def test_variant_flags_are_checked_on_the_host(lib):
    """Wetting and drying is taken alone with a finite hmin >= 0; unknown flags are refused."""
    from paper_1711_04471_amd import _lib
    from paper_1711_04471_amd.sw2d import ADVECTION, FILTER_UV, FRICTION, WETDRY, params
    L = _lib.load()

    def ws(**kw):
        return L.sw2d_workspace_bytes(ctypes.byref(params(66, 66, 100.0, 100.0, 9.81, 5.0, 0.05, **kw)))

    assert ws(flags=WETDRY, hmin=0.05) > 0 and ws(flags=WETDRY, hmin=0.0) > 0
    assert ws(flags=FRICTION | FILTER_UV | ADVECTION, cd=0.002) > 0
    for flags in (WETDRY | FRICTION, WETDRY | FILTER_UV, WETDRY | ADVECTION, 16):
        assert ws(flags=flags) == 0, flags
    for hmin in (-0.01, float("nan"), float("inf")):
        assert ws(flags=WETDRY, hmin=hmin) == 0
    assert ws(flags=FRICTION, cd=-1.0) == 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1711_04471_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(OSError, match="no CPU fallback"):
        _lib.load()


def test_sor_argument_checks_need_no_gpu():
    """Invalid SOR parameters are refused on the host before any device call."""
    import ctypes

    from paper_1711_04471_amd import _lib
    lib = _lib.load()
    bad = [(2, 5, 5, 1.0, 1.0, 1.0, 1.5), (5, 5, 5, 0.0, 1.0, 1.0, 1.5), (5, 5, 5, 1.0, 1.0, 1.0, 2.0),
           (5, 5, 5, 1.0, 1.0, 1.0, 0.0), (5, 5, 5, 1.0, float("nan"), 1.0, 1.0)]
    for args in bad:
        p = _lib.sw2d_sor_params(*args)
        assert lib.sw2d_sor_workspace_bytes(ctypes.byref(p), 10) == 0
        assert lib.sw2d_sor_run(ctypes.byref(p), None, None, 10, None, None, 0, None) == -1
    assert lib.sw2d_sor_workspace_bytes(ctypes.byref(_lib.sw2d_sor_params(5, 5, 5, 1.0, 1.0, 1.0, 1.5, 2)), 10) == 0
    fused = _lib.sw2d_sor_params(300, 300, 90, 4.0, 4.0, 2.0, 1.7, 1)
    assert lib.sw2d_sor_workspace_bytes(ctypes.byref(fused), 50) > 0
    good = _lib.sw2d_sor_params(300, 300, 90, 4.0, 4.0, 2.0, 1.7)
    nb = lib.sw2d_sor_workspace_bytes(ctypes.byref(good), 50)
    assert nb > 0
    assert lib.sw2d_sor_workspace_bytes(ctypes.byref(good), -1) == 0
    # a short workspace is refused before any launch
    assert lib.sw2d_sor_run(ctypes.byref(good), ctypes.c_void_p(16), ctypes.c_void_p(16), 50, None,
                            ctypes.c_void_p(16), nb - 1, None) == -5


def test_surrogate_entry_points_check_arguments_on_the_host(lib):
    """The one-kernel network and the corrected-step loop refuse missing pointers, bad
    normalisation and a missing handle before any device call."""
    import ctypes

    from paper_1711_04471_amd import _lib
    L = _lib.load()
    fp = ctypes.POINTER(ctypes.c_float)
    mean = (ctypes.c_float * 5)(0, 0, 0, 0, 0)
    std = (ctypes.c_float * 5)(1, 1, 1, 1, 1)
    bad_std = (ctypes.c_float * 5)(1, 1, 0, 1, 1)
    dummy = ctypes.c_void_p(256)
    wk = (ctypes.c_void_p * 4)(256, 256, 256, 256)
    bias = (ctypes.c_void_p * 4)(256, 256, 256, 256)
    no_w = (ctypes.c_void_p * 4)(256, None, 256, 256)
    args = [dummy] * 5
    assert L.sw2d_cnn_forward(*args, 8, 8, mean, std, wk, bias, None, None) == _lib.SW2D_EINVAL
    assert L.sw2d_cnn_forward(*args, 8, 8, mean, bad_std, wk, bias, dummy, None) == _lib.SW2D_EINVAL
    assert L.sw2d_cnn_forward(*args, 8, 8, mean, std, no_w, bias, dummy, None) == _lib.SW2D_EINVAL
    assert L.sw2d_cnn_forward(*args, 0, 8, mean, std, wk, bias, dummy, None) == _lib.SW2D_EINVAL
    t_std = (ctypes.c_float * 3)(1, 1, 1)
    assert L.sw2d_surrogate_advance(None, 1, dummy, dummy, mean, std, wk, bias, t_std, dummy) == _lib.SW2D_ESTATE
    assert L.sw2d_surrogate_advance_noalloc(None, 1, dummy, dummy, mean, std, wk, bias, t_std) == _lib.SW2D_ESTATE


def test_plain_c_client_builds_and_links(lib, tmp_path):
    """The header compiles as C99 with warnings as errors, and a C program linked against the
    library and the HIP runtime alone starts (its usage path makes no HIP call)."""
    import subprocess

    from tests.c_client import build as c_client
    exe = c_client.build()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage:" in r.stderr
    r = subprocess.run([exe, str(tmp_path), "8", "8", "1", "1", "9.81", "0.1", "0.05", "1", "1", "0"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2  # no input files: refused before any device call
