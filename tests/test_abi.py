"""The C ABI library loads and exports every symbol that include/swmi.h
declares; host-only entry points behave as documented (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2302_14720_amd as sw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "swmi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sw_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sw.LIB_PATH):
        from paper_2302_14720_amd import build
        build.build()
    return sw.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "sw_create" in names and "sw_sweep" in names and "sw_observables" in names
    for name in names:
        assert hasattr(lib, name), name
        assert name in sw._SIGNATURES, f"binding lacks {name}"


def test_binding_covers_only_declared_symbols():
    assert sorted(sw._SIGNATURES) == _declared()


def test_workspace_sizes_and_validation(lib):
    n64 = sw.sw_workspace_bytes(64)
    n1024 = sw.sw_workspace_bytes(1024)
    assert n64 > 2 * 64 * 64 and n1024 > 2 * 1024 * 1024
    assert n1024 > n64
    for bad in (0, 16, 33, 100, 65536):
        assert sw.sw_workspace_bytes(bad) == 0
    cfg = sw.sw_config_init(96, 0.44, 1.0, 1)
    assert sw.sw_workspace_bytes_ex(cfg) > 0
    cfg.tile = 64  # 96 is not a multiple of 64
    assert sw.sw_workspace_bytes_ex(cfg) == 0
    assert "tile 64" in sw.sw_last_error()
    cfg = sw.sw_config_init(64, -1.0, 1.0, 1)
    assert sw.sw_workspace_bytes_ex(cfg) == 0
    cfg = sw.sw_config_init(64, 0.4, 0.0, 1)
    assert sw.sw_workspace_bytes_ex(cfg) == 0
    cfg = sw.sw_config_init(64, float("nan"), 1.0, 1)
    assert sw.sw_workspace_bytes_ex(cfg) == 0
    cfg = sw.sw_config_init(64, 0.4, 1.0, 1, flags=sw.SW_FLAG_LABELS | sw.SW_FLAG_DENSE_HIST)
    plain = sw.sw_config_init(64, 0.4, 1.0, 1)
    assert sw.sw_workspace_bytes_ex(cfg) >= sw.sw_workspace_bytes_ex(plain) + 64 * 64 * 4 + (64 * 64 + 1) * 8
    cfg = sw.sw_config_init(64, 0.4, 1.0, 1, flags=8)
    assert sw.sw_workspace_bytes_ex(cfg) == 0


def test_create_rejects_bad_arguments_before_touching_the_gpu(lib):
    h = ctypes.c_void_p()
    assert lib.sw_create(48, 0.4, 1.0, 1, ctypes.byref(h)) == sw.SW_EINVAL
    assert h.value is None
    assert lib.sw_create(64, 0.4, -1.0, 1, ctypes.byref(h)) == sw.SW_EINVAL
    assert lib.sw_create_in(64, 0.4, 1.0, 1, None, 0, None, ctypes.byref(h)) == sw.SW_EINVAL
    assert lib.sw_sweep(None, 1) == sw.SW_EINVAL
    assert lib.sw_observables(None, None) == sw.SW_EINVAL
    lib.sw_destroy(None)  # no-op


def test_batch_workspace_sizes_and_validation():
    lib = sw.lib()
    L = np.array([64, 128, 256], dtype=np.int32)
    n1 = sw.sw_batch_workspace_bytes(L)
    assert n1 > sum(sw.sw_workspace_bytes(int(x)) // 4 for x in L)
    assert sw.sw_batch_workspace_bytes(L, ring=4096) > n1
    assert sw.sw_batch_workspace_bytes(L, tile=32) > n1  # more, smaller tiles
    assert sw.sw_batch_workspace_bytes(np.array([64, 96], dtype=np.int32), tile=64) == 0
    assert sw.sw_batch_workspace_bytes(L, tile=48) == 0
    assert sw.sw_batch_workspace_bytes(np.array([64, 100], dtype=np.int32)) == 0
    assert sw.sw_batch_workspace_bytes(np.zeros(0, dtype=np.int32)) == 0
    assert sw.sw_batch_workspace_bytes(np.full(4097, 64, dtype=np.int32)) == 0
    # per-replica tile widths and merges
    mixed = np.array([64, 96, 512], dtype=np.int32)
    assert sw.sw_batch_workspace_bytes(mixed, tiles=[64, 32, 64], merge=[1, 1, 2]) > 0
    assert sw.sw_batch_workspace_bytes(mixed, tiles=[64, 64, 64]) == 0  # 96 needs 32-wide tiles
    assert "replica 1" in sw.sw_last_error()
    assert sw.sw_batch_workspace_bytes(mixed, merge=[0, 0, sw.SW_MERGE_LDS]) == 0  # 64 tiles: too many for LDS
    assert "LDS merge" in sw.sw_last_error()
    assert sw.sw_batch_workspace_bytes(mixed, merge=[0, 3, 0]) == 0
    assert sw.sw_batch_workspace_bytes(mixed, q=[0, 3, 9], tiles=0) == 0
    # creation is refused before any device call for invalid replicas
    h = ctypes.c_void_p()
    b = np.array([0.4, 0.4]), np.array([1.0, 1.0])
    s = np.array([1, 2], dtype=np.uint64)
    bad_L = np.array([64, 33], dtype=np.int32)
    rc = lib.sw_batch_create(2, bad_L.ctypes.data_as(ctypes.c_void_p), b[0].ctypes.data_as(ctypes.c_void_p),
                             b[1].ctypes.data_as(ctypes.c_void_p), s.ctypes.data_as(ctypes.c_void_p), 0, 0, 0,
                             None, 0, None, ctypes.byref(h))
    assert rc == sw.SW_EINVAL and b"replica 1" in lib.sw_last_error()
    rc = lib.sw_batch_create(0, None, None, None, None, 0, 0, 0, None, 0, None, ctypes.byref(h))
    assert rc == sw.SW_EINVAL
    assert lib.sw_batch_size(None) == 0 and lib.sw_batch_next_sweep(None) == -1


def test_server_job_bytes():
    assert sw.Server.job_bytes(128, 100) > 2 * 128 * 128
    assert sw.Server.job_bytes(128, 10000) > sw.Server.job_bytes(128, 100)
    assert sw.Server.job_bytes(100, 100) == 0
    assert sw.Server.job_bytes(128, 0) == 0
    assert sw.sw_last_error is not None


def test_server_potts_job_bytes():
    assert sw.Server.job_bytes(128, 100, q=3) == sw.Server.job_bytes(128, 100) > 0  # same 64-wide tile layout
    assert sw.Server.job_bytes(96, 100, q=5) > 0  # 32-wide tiles above q = 4
    assert sw.Server.job_bytes(128, 100, q=1) == 0 and sw.Server.job_bytes(128, 100, q=9) == 0


_RUNTIMES = r"""
import sys
sys.path.insert(0, sys.argv[1])
import paper_2302_14720_amd as sw
sw.lib()
import torch
maps = {line.split()[-1] for line in open("/proc/self/maps") if "/" in line}
for tag in ("libamdhip64", "libhsa-runtime64"):
    print(tag, len([m for m in maps if tag in m.rsplit("/", 1)[-1]]))
"""


def test_library_shares_torch_hip_runtime(lib):
    """Loading the library before anything else imports torch must still
    leave one HIP and one HSA runtime in the process (torch's): a second
    copy would not see the device torch holds, nor torch's streams."""
    import subprocess
    import sys

    out = subprocess.run([sys.executable, "-c", _RUNTIMES, ROOT], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    counts = dict(line.split() for line in out.stdout.splitlines())
    assert counts == {"libamdhip64": "1", "libhsa-runtime64": "1"}, out.stdout


def test_model_and_lattice_validation(lib):
    """Potts and cubic configurations are checked on the host: tile widths,
    lattice sides, q and dims ranges; workspaces grow with the sites."""
    ok = lambda **kw: sw.sw_workspace_bytes_ex(sw.sw_config_init(kw.pop("L", 64), 0.5, 1.0, 1, **kw))
    assert ok(q=3) > 0 and ok(q=3, tile=64) > 0 and ok(q=8, tile=32) > 0
    assert ok(q=5, tile=64) == 0 and "32-wide" in sw.sw_last_error()
    assert ok(q=1) == 0 and ok(q=9) == 0
    assert ok(q=5, tile=64, flags=sw.SW_FLAG_LABEL_EQUIV) > 0  # tile unused there
    # cubic: L a multiple of 16 in [16, 1616]; labels kept for every site
    n16, n32 = ok(L=16, dims=3), ok(L=32, dims=3)
    assert n16 > 16 ** 3 * 9 and n32 > 32 ** 3 * 9 and n32 > n16
    assert ok(L=32, dims=3, flags=sw.SW_FLAG_LABEL_EQUIV) > 0
    assert ok(L=1616, dims=3) > 1616 ** 3 * 9
    for bad in (8, 24, 1632):
        assert ok(L=bad, dims=3) == 0
    assert ok(L=48, dims=2) == 0  # the square lattice needs multiples of 32
    assert ok(L=64, dims=2) == ok(L=64, dims=0) > 0
    assert ok(dims=1) == 0 and ok(dims=4) == 0


def test_potts_batch_workspace_validation(lib):
    L = np.array([64, 128, 96], dtype=np.int32)
    assert sw.sw_batch_workspace_bytes(L, q=[2, 3, 8]) > 0
    assert sw.sw_batch_workspace_bytes(L, q=[2, 3, 9]) == 0
    assert sw.sw_batch_workspace_bytes(L, q=[2, 1, 3]) == 0
    assert sw.sw_batch_workspace_bytes(np.array([64, 128], dtype=np.int32), q=[3, 4], tile=64) > 0
    assert sw.sw_batch_workspace_bytes(np.array([64, 128], dtype=np.int32), q=[3, 5], tile=64) == 0
    assert lib.sw_batch_workspace_bytes_potts(2, L.ctypes.data_as(ctypes.c_void_p), None, 0, 0) == 0
