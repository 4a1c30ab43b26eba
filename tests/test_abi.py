"""The C-ABI library loads, exports every declared entry point, and validates
arguments on the host (no device call is made by these checks)."""
import ctypes as C
import subprocess

import pytest

from paper_2604_19501_amd import _lib as L
from paper_2604_19501_amd.solver import make_grid, make_mg


def test_exports_every_declared_symbol():
    names = L.declared_symbols()
    assert len(names) >= 17
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIBPATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(L.lib, n)


def test_status_strings():
    for code in (0, -1, -2, -3, -4, -5, 1, 2):
        assert L.lib.helm_status_str(code)
    assert L.lib.helm_status_str(123) == b"unknown status"


def _bytes(n, layer=None, **mg):
    layer = layer or tuple((2, 2) for _ in n)
    g = make_grid(n, 1.0 / n[0], layer, 2.0)
    m = make_mg(**mg)
    b = C.c_size_t()
    return L.lib.helm_workspace_bytes(C.byref(g), C.byref(m), C.byref(b)), b.value


def test_workspace_query_and_validation():
    st, b = _bytes((32, 32))
    assert st == 0 and b > 0
    st3, b3 = _bytes((16, 16, 16))
    assert st3 == 0 and b3 > 0
    assert _bytes((30, 32))[0] == L.HELM_EINVAL            # not a multiple of 4
    assert b"multiple of 4" in L.lib.helm_last_error()
    assert _bytes((32, 32), layer=((20, 20), (2, 2)))[0] == L.HELM_EINVAL   # layers overlap
    assert _bytes((32, 32), restart=0)[0] == L.HELM_EINVAL
    assert _bytes((32, 32), restart=65)[0] == L.HELM_EINVAL
    assert _bytes((32, 32), nu=(5, 1))[0] == L.HELM_EINVAL
    assert _bytes((32, 32), cycle=3)[0] == L.HELM_EINVAL
    assert b"cycle must be" in L.lib.helm_last_error()
    # larger grids and more Krylov vectors need more workspace
    assert _bytes((64, 64))[1] > b
    assert _bytes((32, 32), restart=40)[1] > b


def test_lockstep_capacity_workspace():
    """a single-instance context with lock-step capacity r needs more workspace than r = 1;
    the capacity is capped at 16, and r < 1 is rejected before any device work"""
    g = make_grid((32, 32), 1 / 32, ((2, 2), (2, 2)), 2.0)
    m = make_mg()
    sizes = {}
    for r in (1, 4, 16, 64):
        b = C.c_size_t()
        assert L.lib.helm_workspace_bytes_multi(C.byref(g), C.byref(m), r, C.byref(b)) == 0
        sizes[r] = b.value
    single = C.c_size_t()
    assert L.lib.helm_workspace_bytes(C.byref(g), C.byref(m), C.byref(single)) == 0
    assert sizes[1] == single.value
    assert sizes[1] < sizes[4] < sizes[16] == sizes[64]
    b = C.c_size_t()
    assert L.lib.helm_workspace_bytes_multi(C.byref(g), C.byref(m), 0, C.byref(b)) == L.HELM_EINVAL
    ctx = C.c_void_p()
    s = L.Shift(1.0, 1.0, 0.0)
    assert L.lib.helm_setup_multi(C.byref(g), None, 10.0, C.byref(s), C.byref(m), 0, None, 0, None,
                                  C.byref(ctx)) == L.HELM_EINVAL


def test_setup_rejects_bad_arguments_before_device_work():
    g = make_grid((32, 32), 1 / 32, ((2, 2), (2, 2)), 2.0)
    m = make_mg()
    s = L.Shift(1.1, 1.0, 0.0)
    ctx = C.c_void_p()
    # NULL slowness / workspace are refused on the host
    assert L.lib.helm_setup(C.byref(g), None, 10.0, C.byref(s), C.byref(m), None, 0, None, C.byref(ctx)) == L.HELM_EINVAL
    assert L.lib.helm_setup(C.byref(g), C.c_void_p(256), 10.0, C.byref(s), C.byref(m), None, 0, None,
                            C.byref(ctx)) == L.HELM_EWORKSPACE
    assert L.lib.helm_setup(C.byref(g), C.c_void_p(256), -1.0, C.byref(s), C.byref(m), C.c_void_p(256), 1 << 30, None,
                            C.byref(ctx)) == L.HELM_EINVAL
    assert L.lib.helm_setup(C.byref(g), C.c_void_p(256), 10.0, C.byref(s), C.byref(m), C.c_void_p(257), 1 << 30, None,
                            C.byref(ctx)) == L.HELM_EWORKSPACE
    assert L.lib.helm_destroy(None) == 0
    assert L.lib.helm_apply(None, 0, 0, None, None, None) == L.HELM_EINVAL
    assert L.lib.helm_solve(None, 0, None, None, 1e-6, 10, None, None) == L.HELM_EINVAL
    v = (C.c_longlong * 21)()
    assert L.lib.helm_get_instance_info(None, 0, v, 21) == L.HELM_EINVAL
    assert L.lib.helm_level_size(None, 0, 1) == -1


def test_tuning_cache_changes_the_plan(tmp_path, monkeypatch):
    """the coarsest-solve schedule is read from the autotuner's cache when the context is
    planned (visible on the CPU through the workspace size, which depends on the leaf size)."""
    import json
    def ws():
        st, b = _bytes((256, 256), cycle_prec="f32")
        assert st == 0
        return b
    monkeypatch.delenv("HELM_TUNE_CACHE", raising=False)
    base = ws()
    path = tmp_path / "cache.json"
    key = "nd:2:256x256x0:f32"
    sizes = {}
    for leaf in (16, 64):
        path.write_text(json.dumps({key: {"leaf": leaf, "root": 1100, "cuts": "1"}}))
        monkeypatch.setenv("HELM_TUNE_CACHE", str(path))
        sizes[leaf] = ws()
    assert sizes[16] != sizes[64]
    monkeypatch.setenv("HELM_TUNE_CACHE", str(tmp_path / "missing.json"))
    assert ws() == base
    path.write_text("{ not json")
    monkeypatch.setenv("HELM_TUNE_CACHE", str(path))
    assert ws() == base


def test_tune_cache_members_are_read_at_the_top_level(monkeypatch, tmp_path):
    """the planner reads the cached schedule's own members: nested objects and arrays
    (per-class timings, runners-up) before and after them, holding members of the same
    names, are skipped.  Checked through helm_workspace_bytes, which plans on the host."""
    import json
    n = (256, 256)
    key = "nd:2:256x256x0:f32"
    monkeypatch.setenv("HELM_TUNE_CACHE", str(tmp_path / "none.json"))
    monkeypatch.setenv("HELM_ND_ROOT", "100")
    monkeypatch.setenv("HELM_ND_LEAF", "8")
    st8, b8 = _bytes(n)
    monkeypatch.setenv("HELM_ND_LEAF", "64")
    st64, b64 = _bytes(n)
    monkeypatch.delenv("HELM_ND_LEAF")
    monkeypatch.delenv("HELM_ND_ROOT")
    assert st8 == st64 == 0 and b8 != b64
    entry = {"a_nested": {"leaf": 8, "root": 1}, "leaf": 64, "merge": "none", "root": 100,
             "runners_up": [{"leaf": 8, "splitk_kb": 1}], "splitk_kb": 4096, "cuts": ""}
    path = tmp_path / "cache.json"
    path.write_text(json.dumps({key: entry}, indent=1, sort_keys=True))
    monkeypatch.setenv("HELM_TUNE_CACHE", str(path))
    st, b = _bytes(n)
    assert st == 0 and b == b64
    entry["leaf"] = 8
    path.write_text(json.dumps({key: entry}, indent=1, sort_keys=True))
    st, b = _bytes(n)
    assert st == 0 and b == b8
