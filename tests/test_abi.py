"""The C-ABI library loads and exports every symbol its header declares; host-side
argument validation returns the documented status codes without touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1601_06274_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            txt = open(os.path.join(inc, fn)).read()
            names |= set(re.findall(r"^\s*(?:int|size_t|void|const char\*)\s+(dm_\w+)\s*\(", txt, re.M))
    return names


def test_library_exports_declared_symbols():
    lib = L.lib()
    declared = _declared()
    assert declared, "no declarations found"
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    # and the binding knows every declared symbol
    assert declared <= set(L.exported_names())


def test_status_strings():
    lib = L.lib()
    for code in range(-7, 1):
        assert lib.dm_status_string(code)
    assert b"gfx950" in lib.dm_version()


def _params(**kw):
    from paper_1601_06274_amd.ops import discrete_params
    return discrete_params(**kw)


def test_workspace_query_and_validation():
    lib = L.lib()
    p = _params(T=3, n_iters=2)
    sz = lib.dm_solve_discrete_workspace(L.DmShape(128, 96, 32), L.DM_F32, ctypes.byref(p))
    assert sz >= 128 * 96 * 32 * 4
    assert lib.dm_solve_discrete_workspace(L.DmShape(0, 96, 32), L.DM_F32, ctypes.byref(p)) == 0
    assert lib.dm_solve_discrete_workspace(L.DmShape(8, 8, 257), L.DM_F32, ctypes.byref(p)) == 0


def _solve(shape, p, cost=1, dual=1, ws=None, ws_bytes=0, dtype=L.DM_F32):
    lib = L.lib()
    fake = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    return lib.dm_solve_discrete(fake if cost else None, dtype, fake, fake, shape, ctypes.byref(p), None, None,
                                 fake if dual else None, None, None, ws, ctypes.c_size_t(ws_bytes), None)


@pytest.mark.parametrize("kw,code", [
    (dict(T=0), -3),
    (dict(gammas=(0.25, 0.5)), -3),          # last gamma must be 1
    (dict(gammas=(0.0, 1.0)), -3),
    (dict(gammas=(0.1,) * 8 + (1.0,)), -3),  # too many passes (max_pass 9 -> clipped list)
    (dict(n_iters=-1), -3),
    (dict(tile=(64, 2)), -6),                # tile not compiled in
    (dict(tile=(4, 1)), -3),                 # tile too small for K
])
def test_param_validation(kw, code):
    p = _params(**kw)
    if "gammas" in kw and len(kw["gammas"]) > 8:
        p.max_pass = 9
    assert _solve(L.DmShape(16, 8, 8), p) == code
    assert L.lib().dm_last_error_message()


def test_null_and_shape_and_workspace_errors():
    p = _params()
    assert _solve(L.DmShape(16, 8, 8), p, cost=0) == -1
    assert _solve(L.DmShape(16, 8, 8), p, dual=0) == -1
    assert _solve(L.DmShape(16, 0, 8), p) == -2
    assert _solve(L.DmShape(16, 8, 300), p) == -2
    assert _solve(L.DmShape(16384, 16384, 4), p) == -2  # FP32 volume beyond 32-bit offsets
    assert _solve(L.DmShape(16384, 16300, 4), p) == -2  # 4272947200 bytes > 0xFE000000
    assert "offset range" in L.lib().dm_last_error_message().decode()
    assert _solve(L.DmShape(16, 8, 8), p, dtype=7) == -4
    assert _solve(L.DmShape(16, 8, 8), p, ws=ctypes.c_void_p(4096), ws_bytes=16) == -5


def test_cost_volume_validation():
    lib = L.lib()
    cp = L.DmCostParams(4, 0.3, 0.1, 0.1)  # even window
    fake = ctypes.c_void_p(4096)
    assert lib.dm_build_cost_volume(fake, fake, L.DmShape(8, 8, 4), ctypes.byref(cp), 0, fake, None, None, None) == -3
    cp = L.DmCostParams(3, 0.3, 0.1, 0.1)
    assert lib.dm_build_cost_volume(None, fake, L.DmShape(8, 8, 4), ctypes.byref(cp), 0, fake, None, None, None) == -1
    assert lib.dm_build_cost_volume(fake, fake, L.DmShape(8, 8, 4), ctypes.byref(cp), 5, fake, None, None, None) == -4


def test_default_tile_host_query():
    lib = L.lib()
    g, l = ctypes.c_int(0), ctypes.c_int(0)
    for K, want in [(192, (64, 3)), (128, (32, 4)), (5, (4, 2)), (1, (4, 1)), (256, (64, 4)), (96, (32, 3))]:
        assert lib.dm_default_tile(K, ctypes.byref(g), ctypes.byref(l)) == 0
        assert (g.value, l.value) == want, K
        assert g.value * l.value >= K
    assert lib.dm_default_tile(300, ctypes.byref(g), ctypes.byref(l)) == -2
    assert lib.dm_default_tile(8, None, ctypes.byref(l)) == -1
