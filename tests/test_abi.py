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


def _al(x, a=256):
    return (x + a - 1) // a * a


def _tape_bytes(W, H, K, T, tile, recompute):
    """One selection tape: G lanes x ceil(LPL/4) dwords per pixel, when the window reaches at
    most one lane across (and the caller did not ask for recomputation)."""
    G, lpl = tile
    need = (T - 1 + lpl - 1) // lpl
    if recompute or min(need, G - 1) > 1:
        return 0
    b = _al(W * H * G * ((lpl + 3) // 4) * 4)
    return b if b <= 0xFE000000 else 0


@pytest.mark.parametrize("keep", [0, 1, 2])
@pytest.mark.parametrize("T,tile,recompute", [(3, (64, 3), False), (3, (64, 3), True), (5, (4, 1), False),
                                              (5, (8, 4), False), (1, (4, 2), False)])
def test_checkpoint_and_tape_workspace_sizes(keep, T, tile, recompute):
    """Forward and backward workspace sizes for every checkpoint mode, with and without
    selection tapes (the layouts the solver and its adjoint index into)."""
    lib = L.lib()
    W, H, K, it = 40, 24, tile[0] * tile[1] - 1, 3
    P = 3  # update passes of the iterative minorant (1/4, 1/4, 1)
    p = _params(T=T, n_iters=it, tile=tile, keep_checkpoints=keep, recompute_selections=recompute)
    S = 2 * it
    vol = _al(W * H * K * 4)
    tb = _tape_bytes(W, H, K, T, tile, recompute)
    head = _al(_al(_al(vol + (S + 2) * max(W, H) * 8) + 1024 * 8) + W * H * 4)
    if keep == 0:
        slab = 0
    elif keep == 1:
        slab = vol
    else:
        slab = vol + (P + 1) * tb if tb else (1 + (P + 1) + (P - 1)) * vol
    assert lib.dm_solve_discrete_workspace(L.DmShape(W, H, K), L.DM_F16, ctypes.byref(p)) == head + S * slab
    if keep == 0:
        return
    Pb = 1 if keep == 2 else P
    body = ((1 if tb else Pb + 1) + (((1 if tb else Pb - 1)) if Pb > 1 else 0)) * vol + ((Pb + 1) * tb if tb else 0)
    body += 3 * vol + _al(H * (W - 1) * 8) + _al((H - 1) * W * 8) + _al(W * H * 4)
    assert lib.dm_solve_discrete_backward_workspace(L.DmShape(W, H, K), ctypes.byref(p)) == body


def test_census_and_lr_check_validation():
    lib = L.lib()
    fake = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    s = L.DmShape(8, 8, 4)
    for window, trunc, view, dtype, code in [(9, 1.0, 0, 0, -3), (4, 1.0, 0, 0, -3), (5, 0.0, 0, 0, -3),
                                             (5, 1.5, 0, 0, -3), (5, 1.0, 2, 0, -3), (5, 1.0, 0, 3, -4)]:
        cp = L.DmCostParams(window, trunc, 0.1, 0.1)
        assert lib.dm_build_cost_volume_census(fake, fake, s, ctypes.byref(cp), view, dtype, fake, None, None,
                                               None) == code
    cp = L.DmCostParams(5, 1.0, 0.1, 0.1)
    assert lib.dm_build_cost_volume_census(fake, None, s, ctypes.byref(cp), 0, 0, fake, None, None, None) == -1
    assert lib.dm_build_cost_volume_census(fake, fake, L.DmShape(8, 8, 0), ctypes.byref(cp), 0, 0, fake, None, None,
                                           None) == -2
    assert lib.dm_lr_check(fake, None, 8, 8, 1.0, -1.0, fake, None) == -1
    assert lib.dm_lr_check(fake, fake, 0, 8, 1.0, -1.0, fake, None) == -2
    assert lib.dm_lr_check(fake, fake, 8, 8, -1.0, -1.0, fake, None) == -3


def test_hierarchical_minorant_is_forward_only():
    lib = L.lib()
    from paper_1601_06274_amd import ops
    s = L.DmShape(16, 8, 8)
    p = ops.discrete_params(minorant="hierarchical")
    assert lib.dm_solve_discrete_workspace(s, 0, ctypes.byref(p)) > 0
    plain = ops.discrete_params(minorant="iterative")
    # a second message volume
    assert lib.dm_solve_discrete_workspace(s, 0, ctypes.byref(p)) >= \
        lib.dm_solve_discrete_workspace(s, 0, ctypes.byref(plain)) + 16 * 8 * 8 * 4
    pk = ops.discrete_params(minorant="hierarchical", keep_checkpoints=True)
    assert lib.dm_solve_discrete_workspace(s, 0, ctypes.byref(pk)) == 0
    fake = ctypes.c_void_p(4096)
    assert lib.dm_solve_discrete(fake, 0, fake, fake, s, ctypes.byref(pk), None, None, fake, None, None, fake,
                                 ctypes.c_size_t(1 << 30), None) == -6
