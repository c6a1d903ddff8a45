"""Host-side checks of the C-ABI library: it loads, exports every symbol the
header declares, sizes workspaces, and rejects bad arguments before touching
the GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("lbm_create", "lbm_set_metric", "lbm_step", "lbm_moments", "lbm_wall_force", "lbm_backward"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_1803_07822_amd import lbm

    lib = ctypes.CDLL(lbm.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(declared_symbols()) == set(lbm.SYMBOLS)


def test_workspace_bytes():
    from paper_1803_07822_amd import lbm

    b64 = lbm.lbm_workspace_bytes(256, 128, 128, lbm.LBM_FP64)
    b32 = lbm.lbm_workspace_bytes(256, 128, 128, lbm.LBM_FP32_DEV)
    N = 256 * 126 * 128
    assert b32 < b64
    # at least populations A/B, history, geometry, moments in the storage type
    assert b64 > 8 * N * (2 * 19 + 10 + 28 + 4)
    assert b32 > 4 * N * (2 * 19 + 10 + 28 + 4)
    assert lbm.lbm_workspace_bytes(8, 3, 8) == 0  # too few layers
    assert lbm.lbm_workspace_bytes(0, 8, 8) == 0
    # 32-bit offsets over a pair of FP64 planes: 2^28 fluid nodes and above are refused
    assert lbm.lbm_workspace_bytes(1024, 2 + 256, 1024) == 0
    assert lbm.lbm_workspace_bytes(1024, 2 + 255, 1024) > 0
    assert lbm.lbm_workspace_bytes(8, 8, 8, lbm.LBM_FP64, 10, 11) == 0  # ckpt_every > K
    adj = lbm.lbm_workspace_bytes(16, 10, 8, lbm.LBM_FP64, 20, 5)
    assert adj > lbm.lbm_workspace_bytes(16, 10, 8, lbm.LBM_FP64)


def test_create_rejects_bad_arguments_without_gpu():
    from paper_1803_07822_amd import lbm

    lib = lbm._lib
    h = ctypes.c_void_p()
    g = lbm.lbm_grid(8, 8, 8)
    fake = ctypes.c_void_p(4096)  # never dereferenced: argument checks fail first
    assert lib.lbm_create(ctypes.byref(h), ctypes.byref(g), 19, 0.5, 0, fake, 1 << 40, None) == -1  # tau
    assert lib.lbm_create(ctypes.byref(h), ctypes.byref(g), 27, 0.8, 0, fake, 1 << 40, None) == -1  # lattice
    assert lib.lbm_create(ctypes.byref(h), ctypes.byref(g), 19, 0.8, 7, fake, 1 << 40, None) == -1  # precision
    assert lib.lbm_create(ctypes.byref(h), ctypes.byref(g), 19, 0.8, 0, None, 1 << 40, None) == -1  # workspace
    assert lib.lbm_create(ctypes.byref(h), ctypes.byref(g), 19, 0.8, 0, fake, 16, None) == -2  # too small
    bad = lbm.lbm_grid(8, 3, 8)
    assert lib.lbm_create(ctypes.byref(h), ctypes.byref(bad), 19, 0.8, 0, fake, 1 << 40, None) == -1
    assert lib.lbm_step(None, 1) == -1
    assert lib.lbm_destroy(None) == -1
    assert lbm.lbm_last_error(None) == "null context"


def test_oracle_library_is_separate():
    """The oracle and the HIP library share no object code."""
    import oracle

    from paper_1803_07822_amd import lbm

    assert os.path.dirname(oracle.lib_path()) != os.path.dirname(lbm.LIB_PATH)
    lib = ctypes.CDLL(oracle.lib_path())
    assert not hasattr(lib, "lbm_step")


def test_stream_probe_argument_errors():
    """The calibration entry point rejects bad arguments before any device call."""
    from paper_1803_07822_amd import lbm

    for args in ((lbm.LBM_FP32_DEV, 0), (lbm.LBM_FP32_DEV, -5), (7, 100), (lbm.LBM_FP64, 1 << 28)):
        assert lbm._lib.lbm_stream_probe(args[0], args[1], None, None, None) == -1



def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more it exits with status 2 and
    says so, before touching any device."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_paper_values_fixture_is_cited():
    """Every number in tests/golden/paper_values.json carries the passage it
    comes from."""
    import json

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.json")
    with open(path) as fh:
        data = json.load(fh)
    entries = {k: v for k, v in data.items() if isinstance(v, dict)}
    assert entries
    for k, v in entries.items():
        assert isinstance(v["value"], (int, float)), k
        assert re.search(r"(Sec\.|App\.|Fig\.)", v["cite"]), k
