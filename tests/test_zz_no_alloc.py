"""so2dr_run_noalloc (the static-workspace variant of so2dr_run, for callers
that cannot allocate device memory) against so2dr_run on the caller's arena:
bit-identical results on two calls in a row, the second with a smaller grid,
and E_BUDGET for a plan larger than the static workspace."""
import ctypes

import numpy as np
import pytest

from conftest import gpu_available
from helpers import pinned_copy, to_storage

pytestmark = pytest.mark.gpu


def _case(nx, ny, nz, T, storage, seed, shape="star", radius=1, chunks=4, tb=4, k_on=0):
    import workloads
    from paper_2309_08864_amd import stencil_offsets
    offs = stencil_offsets(3, shape, radius)
    w = workloads.fp32_rounded(workloads.centre_arm_weights(offs, 0.4, [0.1] * radius)
                               if shape == "star" else workloads.random_box_weights(offs, seed))
    kw = dict(ndim=3, nx=nx, ny=ny, nz=nz, shape=shape, radius=radius, weights=list(w), T=T,
              tb_depth=tb, n_chunks=chunks, k_on=k_on, budget=64 << 20, storage=storage)
    u0 = workloads.uniform((nz, ny, nx), seed=seed)
    return kw, to_storage(u0, storage)


def _noalloc(plan, host):
    """so2dr_run_noalloc through the C ABI on the library's per-process streams."""
    from paper_2309_08864_amd import _lib
    from paper_2309_08864_amd.plan import _plan_streams
    streams = _plan_streams("cuda", 3)
    arr = (ctypes.c_void_p * 3)(*[s.cuda_stream for s in streams])
    st = _lib.Stats()
    rc = _lib.lib().so2dr_run_noalloc(plan._h, ctypes.c_void_p(host.data_ptr()), arr, 3,
                                      ctypes.byref(st))
    return rc, st


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_noalloc_matches_run_two_calls():
    import torch
    from paper_2309_08864_amd import Plan
    from paper_2309_08864_amd._lib import NOALLOC_MAX_BYTES
    cases = [
        # a larger grid first, then a smaller one: the second call's
        # workspace holds the first call's leftovers
        _case(200, 72, 60, T=9, storage="f32", seed=11, chunks=5, tb=4),
        _case(96, 40, 24, T=6, storage="bf16", seed=12, shape="star", radius=2, chunks=2, tb=3),
    ]
    for i, (kw, u) in enumerate(cases):
        print(f"no-alloc case {i}: {kw['nx']}x{kw['ny']}x{kw['nz']} {kw['storage']}", flush=True)
        ref_plan = Plan(**kw).bind()
        h_ref = pinned_copy(u)
        ref_plan.run(h_ref)
        ref_plan.close()
        plan = Plan(**kw)
        assert plan.info()["workspace_bytes"] <= NOALLOC_MAX_BYTES
        h = pinned_copy(u)
        rc, st = _noalloc(plan, h)
        assert rc == 0, plan_error()
        assert st.rounds_done == plan.info()["n_rounds"]
        assert torch.equal(h, h_ref), f"case {i}: so2dr_run_noalloc differs from so2dr_run"
        assert not torch.equal(h, u)
        plan.close()


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_noalloc_bound_plan_and_budget_error():
    import torch
    from paper_2309_08864_amd import Plan, _lib
    kw, u = _case(128, 48, 32, T=8, storage="f32", seed=13, chunks=4, tb=4)
    plan = Plan(**kw).bind()
    h1 = pinned_copy(u)
    plan.run(h1)
    h2 = pinned_copy(u)
    rc, _ = _noalloc(plan, h2)
    assert rc == 0, plan_error()
    h3 = pinned_copy(u)
    plan.run(h3)        # the caller's binding is intact after the static-workspace call
    assert torch.equal(h1, h2) and torch.equal(h1, h3)
    plan.close()
    # a plan whose workspace exceeds the static array is refused before any work
    big = dict(kw, nx=2048, ny=1024, nz=64, budget=1 << 30, n_chunks=2)
    p = Plan(**big)
    assert p.info()["workspace_bytes"] > _lib.NOALLOC_MAX_BYTES
    hb = torch.zeros((64, 1024, 2048), dtype=torch.float32, pin_memory=True)
    rc, _ = _noalloc(p, hb)
    assert rc == _lib.E_BUDGET
    assert "static workspace" in _lib.lib().so2dr_last_error().decode()
    assert float(hb.abs().sum()) == 0.0
    p.close()


def plan_error():
    from paper_2309_08864_amd import _lib
    return _lib.lib().so2dr_last_error().decode()
