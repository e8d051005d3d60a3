"""dm_solve_discrete_noalloc (the entry point for callers that cannot allocate) against
dm_solve_discrete with a caller workspace: both run the same kernels, so every output is
equal bit for bit.  Two calls in a row on the library's scratch array, the second on a
smaller problem (the array keeps the first call's contents), then the first again."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")


def _lib():
    from paper_1601_06274_amd import _lib as L
    return L, L.lib()


def test_noalloc_limit_and_rejection():
    """Host-side checks (no launch): the stated limit, and a problem whose workspace
    exceeds it fails with DM_ERR_WORKSPACE before anything is enqueued."""
    L, lib = _lib()
    from paper_1601_06274_amd import ops
    limit = int(lib.dm_solve_discrete_noalloc_limit())
    assert limit == 256 << 20
    p = ops.discrete_params(T=3, n_iters=2)
    big = L.DmShape(2048, 1024, 64)   # 512 MiB of messages
    assert lib.dm_solve_discrete_workspace(big, L.DM_F32, ctypes.byref(p)) > limit
    fake = ctypes.c_void_p(4096)
    st = lib.dm_solve_discrete_noalloc(fake, L.DM_F32, fake, fake, big, ctypes.byref(p), None, None, fake, None, None,
                                       None)
    assert st == -5
    assert b"no-allocation" in lib.dm_last_error_message()
    bad = L.DmShape(8, 8, 0)
    assert lib.dm_solve_discrete_noalloc(fake, L.DM_F32, fake, fake, bad, ctypes.byref(p), None, None, fake, None,
                                         None, None) == -2


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _noalloc(cost, w_h, w_v, p):
    L, lib = _lib()
    H, W, K = cost.shape
    dev = cost.device
    out = dict(labels=torch.full((H, W), -1, dtype=torch.int32, device=dev),
               minmarg=torch.full((H, W, K), float("nan"), dtype=torch.float32, device=dev),
               dual=torch.full((H, W, K), float("nan"), dtype=torch.float32, device=dev),
               bounds=torch.full((2,), float("nan"), dtype=torch.float64, device=dev),
               trace=torch.full((2 * p.n_iters,), float("nan"), dtype=torch.float64, device=dev))
    dt = L.DM_F16 if cost.dtype == torch.float16 else L.DM_F32
    st = lib.dm_solve_discrete_noalloc(_ptr(cost), dt, _ptr(w_h), _ptr(w_v), L.DmShape(W, H, K), ctypes.byref(p),
                                       _ptr(out["labels"]), _ptr(out["minmarg"]), _ptr(out["dual"]),
                                       _ptr(out["bounds"]), _ptr(out["trace"]),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    L.check("dm_solve_discrete_noalloc", st)
    return out


CASES = [  # (H, W, K, cost dtype, minorant): a larger problem, then a smaller one
    (96, 128, 32, torch.float32, "iterative"),
    (37, 53, 19, torch.float16, "iterative"),
    (20, 24, 48, torch.float32, "hierarchical"),
]


@pytest.mark.gpu
def test_noalloc_equals_workspace_call():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1601_06274_amd import ops
    for (H, W, K, dtype, minorant) in CASES + CASES[:1]:
        print(f"[case] noalloc {H}x{W}x{K} {dtype} {minorant}", flush=True)
        theta, w_h, w_v = synth.tiny_instance(H, W, K, seed=H + W + K, w_max=0.4)
        cost = torch.from_numpy(theta).to("cuda", dtype)
        wh, wv = torch.from_numpy(w_h).cuda(), torch.from_numpy(w_v).cuda()
        kw = dict(T=3, n_iters=4, minorant=minorant)
        ref = ops.solve_discrete(cost, wh, wv, want_trace=True, **kw)
        got = _noalloc(cost, wh, wv, ops.discrete_params(**kw))
        torch.cuda.synchronize()
        assert torch.equal(got["labels"], ref.labels)
        assert torch.equal(got["minmarg"], ref.minmarg)
        assert torch.equal(got["dual"], ref.dual)
        assert torch.equal(got["bounds"], ref.bounds)
        assert torch.equal(got["trace"], ref.lb_trace)
