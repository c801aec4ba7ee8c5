"""GPU adjoint: loss, dL/du0 and dL/dw from the out-of-core reverse sweep
against the FP64 oracle adjoint (itself pinned by finite differences and
torch autograd in test_oracle_pins.py), plus finite differences taken with
the GPU forward sweep itself in FP64 storage."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from helpers import fp32_weights, pinned_copy, rel_l2, to_storage
from paper_2309_08864_amd import Plan, adjoint_buffers_needed

pytestmark = pytest.mark.gpu


def _gw_err(g, ref):
    """per component |g - ref| / max(|ref|, 1e-3 ||ref||_inf)"""
    ref = np.asarray(ref)
    den = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return float(np.max(np.abs(np.asarray(g) - ref) / den))


def _run_adjoint(kw, u0, y, ckpt_every):
    p = Plan(adjoint=True, **kw).bind()
    loss, gu, gw, st = p.adjoint(pinned_copy(u0), pinned_copy(y), ckpt_every)
    p.close()
    return loss, gu.clone(), gw, st


@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("ndim,shape,r,per,T,K,d,ckpt", [
    (3, "star", 1, (0, 0, 0), 12, 4, 3, 8),
    (3, "star", 1, (0, 0, 0), 11, 3, 4, 5),
    (3, "box", 1, (1, 1, 0), 9, 4, 2, 9),
    (3, "star", 2, (0, 0, 0), 8, 2, 3, 4),
    (2, "star", 1, (0, 0, 0), 10, 4, 3, 6),
    (2, "box", 2, (1, 0, 0), 7, 3, 2, 7),
])
def test_adjoint_vs_oracle(storage, ndim, shape, r, per, T, K, d, ckpt):
    rng = np.random.default_rng(T * 13 + K)
    offs = oracle.stencil_offsets(ndim, shape, r)
    w = rng.uniform(0.2, 1, len(offs))
    w = w / w.sum()
    if storage == "f32":
        w = fp32_weights(w)
    nx, ny, nz = (70, 37, 31) if ndim == 3 else (300, 45, 1)
    shp = (nz, ny, nx) if ndim == 3 else (ny, nx)
    u0 = to_storage(rng.random(shp), storage)
    y = to_storage(rng.random(shp), storage)
    kw = dict(ndim=ndim, nx=nx, ny=ny, nz=nz, shape=shape, radius=r, weights=list(w), T=T,
              tb_depth=K, n_chunks=d, k_on=2 if r == 1 else 1, budget=1 << 30, storage=storage,
              bc=per)
    loss, gu, gw, st = _run_adjoint(kw, u0, y, ckpt)
    rl, rgu, rgw, _ = oracle.adjoint(u0.double().numpy(), y.double().numpy(), offs, w, T, per)
    tol = 1e-4 if storage == "f32" else 1e-10
    e_loss = abs(loss - rl) / abs(rl)
    e_gu = rel_l2(gu.double().numpy(), rgu)
    e_gw = _gw_err(gw, rgw)
    print(f"[{storage} {ndim}D {shape} r={r}] loss {e_loss:.2e} grad_u0 {e_gu:.2e} grad_w {e_gw:.2e}",
          flush=True)
    assert e_loss <= tol and e_gu <= tol and e_gw <= tol


def test_adjoint_checkpoint_interval_invariance():
    """Different checkpoint intervals, chunk counts and depths agree (F64)."""
    rng = np.random.default_rng(3)
    offs = oracle.stencil_offsets(3, "star", 1)
    w = list(workloads.centre_arm_weights(offs, 0.4, [0.1]))
    nx, ny, nz, T = 33, 29, 40, 14
    u0 = to_storage(rng.random((nz, ny, nx)), "f64")
    y = to_storage(rng.random((nz, ny, nx)), "f64")
    res = []
    for K, d, ckpt in [(14, 1, 14), (4, 3, 8), (3, 5, 3), (5, 2, 7), (2, 6, 1)]:
        kw = dict(ndim=3, nx=nx, ny=ny, nz=nz, shape="star", radius=1, weights=w, T=T, tb_depth=K,
                  n_chunks=d, budget=1 << 30, storage="f64")
        res.append(_run_adjoint(kw, u0, y, ckpt))
    for other in res[1:]:
        assert abs(other[0] - res[0][0]) <= 1e-12 * abs(res[0][0])
        assert rel_l2(other[1].numpy(), res[0][1].numpy()) <= 1e-12
        assert _gw_err(other[2], res[0][2]) <= 1e-10


def test_adjoint_copy_engines_bitwise():
    """The gradient with host copies by copy kernels equals the one with DMA
    copies bit for bit (loss, dL/du0, dL/dw)."""
    rng = np.random.default_rng(73)
    offs = oracle.stencil_offsets(3, "star", 1)
    w = rng.uniform(0.05, 0.2, len(offs))
    nx, ny, nz = 40, 24, 30
    kw = dict(ndim=3, nx=nx, ny=ny, nz=nz, shape="star", radius=1, weights=list(w), T=10,
              tb_depth=4, n_chunks=3, budget=1 << 30)
    u0 = to_storage(rng.random((nz, ny, nx)), "f32")
    y = to_storage(rng.random((nz, ny, nx)), "f32")
    res = []
    for engine in ("dma", "kernel", "kernel_out"):
        p = Plan(adjoint=True, copy_engine=engine, **kw).bind()
        assert p.info()["copy_engine"] == {"dma": 1, "kernel": 2, "kernel_out": 3}[engine]
        loss, gu, gw, _ = p.adjoint(pinned_copy(u0), pinned_copy(y), 4)
        res.append((loss, gu.clone(), gw))
        p.close()
    for r in res[1:]:
        assert res[0][0] == r[0]
        assert torch.equal(res[0][1], r[1])
        assert np.array_equal(res[0][2], r[2])


def _gpu_loss(kw, u0, y):
    p = Plan(**kw).bind()
    h = pinned_copy(u0)
    p.run(h)
    p.close()
    d = h.double().numpy() - y.double().numpy()
    return 0.5 * float(np.sum(d * d))


def test_adjoint_finite_differences_32cube():
    """The adjoint workload's FD instance: 32^3, T = 128, checkpoints every
    16 steps, 7-point weights; GPU F64 storage.  Directional difference in
    u0 (exact: L is quadratic in u0) and central differences in every weight,
    all evaluated with the GPU forward sweep."""
    offs = oracle.stencil_offsets(3, "star", 1)
    w = workloads.centre_arm_weights(offs, 0.4, [0.1])
    n, T = 32, 128
    u0n = workloads.uniform((n, n, n), seed=5)
    yn = oracle.sweep(u0n, offs, workloads.perturbed(w, 50), T)
    u0, y = to_storage(u0n, "f64"), to_storage(yn, "f64")
    kw = dict(ndim=3, nx=n, ny=n, nz=n, shape="star", radius=1, T=T, tb_depth=8, n_chunks=2,
              budget=1 << 30, storage="f64")
    loss, gu, gw, _ = _run_adjoint(dict(kw, weights=list(w)), u0, y, 16)
    v = np.random.default_rng(9).standard_normal((n, n, n))
    lp = _gpu_loss(dict(kw, weights=list(w)), to_storage(u0n + v, "f64"), y)
    lm = _gpu_loss(dict(kw, weights=list(w)), to_storage(u0n - v, "f64"), y)
    fd = (lp - lm) / 2.0
    assert abs(fd - float(np.sum(gu.numpy() * v))) <= 1e-9 * abs(fd)
    for k in range(len(w)):
        h = 1e-6 * abs(w[k])
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fdk = (_gpu_loss(dict(kw, weights=list(wp)), u0, y) - _gpu_loss(dict(kw, weights=list(wm)), u0, y)) / (2 * h)
        assert abs(fdk - gw[k]) <= 1e-5 * np.abs(gw).max(), (k, fdk, gw[k])
    # and the F32 adjoint on the same instance is within 1e-4 of the FP64 reference
    w32 = fp32_weights(w)
    rl, rgu, rgw, _ = oracle.adjoint(to_storage(u0n, "f32").double().numpy(),
                                     to_storage(yn, "f32").double().numpy(), offs, w32, T, ckpt=16)
    l32, gu32, gw32, _ = _run_adjoint(dict(kw, weights=list(w32), storage="f32"),
                                      to_storage(u0n, "f32"), to_storage(yn, "f32"), 16)
    assert abs(l32 - rl) / rl <= 1e-4
    assert rel_l2(gu32.double().numpy(), rgu) <= 1e-4
    assert _gw_err(gw32, rgw) <= 1e-4


def test_stencil_loss_autograd():
    from paper_2309_08864_amd import StencilLoss
    rng = np.random.default_rng(4)
    offs = oracle.stencil_offsets(3, "star", 1)
    w0 = fp32_weights(workloads.centre_arm_weights(offs, 0.4, [0.1]))
    nx, ny, nz, T = 24, 20, 30, 6
    u0 = pinned_copy(to_storage(rng.random((nz, ny, nx)), "f32"))
    y = pinned_copy(to_storage(rng.random((nz, ny, nx)), "f32"))
    u0.requires_grad_(True)
    w = torch.tensor(w0, dtype=torch.float64, requires_grad=True)
    spec = dict(ndim=3, nx=nx, ny=ny, nz=nz, shape="star", radius=1, T=T, tb_depth=3, n_chunks=3,
                budget=1 << 30, storage="f32", ckpt_every=3)
    L = StencilLoss.apply(u0, w, y, spec)
    (2.0 * L).backward()
    rl, rgu, rgw, _ = oracle.adjoint(u0.detach().double().numpy(), y.double().numpy(), offs, w0, T)
    assert abs(L.item() - rl) <= 1e-5 * rl
    assert rel_l2(u0.grad.double().numpy(), 2 * rgu) <= 1e-4
    assert _gw_err(w.grad.numpy(), 2 * rgw) <= 1e-4


def test_adjoint_256cube_per_component_vs_fp64_reference():
    """The gradient workload's form at 256^3: 7-point weights 0.4 / 0.1,
    T = 128, host checkpoints every 16 steps, K = 8, 4 or more chunks, FP32
    storage; target from the same sweep with perturbed weights.  The loss,
    every dL/dw_k (per component, |g - g_ref| / max(|g_ref|, 1e-3
    ||g_ref||_inf)) and dL/du0 (relative L2) against the FP64 oracle's full
    reverse sweep, each within 1e-4."""
    offs = oracle.stencil_offsets(3, "star", 1)
    w = fp32_weights(workloads.centre_arm_weights(offs, 0.4, [0.1]))
    wt = fp32_weights(workloads.perturbed(w, 50))
    n, T = 256, 128
    u0n = workloads.uniform((n, n, n), seed=5).astype(np.float32).astype(np.float64)
    u0 = to_storage(u0n, "f32")
    yh = pinned_copy(u0)
    pt = Plan(ndim=3, nx=n, ny=n, nz=n, shape="star", radius=1, weights=list(wt), T=T, tb_depth=8,
              n_chunks=4, budget=1 << 30).bind()
    pt.run(yh)
    pt.close()
    kw = dict(ndim=3, nx=n, ny=n, nz=n, shape="star", radius=1, weights=list(w), T=T, tb_depth=8,
              n_chunks=0, budget=160 << 20)
    p = Plan(adjoint=True, **kw)
    info = p.info()
    p.close()
    assert info["n_chunks"] >= 4 and info["tb_depth"] == 8, info
    loss, gu, gw, st = _run_adjoint(kw, u0, yh, 16)
    rl, rgu, rgw, _ = oracle.adjoint(u0n, yh.double().numpy(), offs, w, T, ckpt=16)
    e_loss = abs(loss - rl) / abs(rl)
    e_gu = rel_l2(gu.double().numpy(), rgu)
    den = np.maximum(np.abs(rgw), 1e-3 * np.abs(rgw).max())
    e_comp = np.abs(np.asarray(gw) - rgw) / den
    print(f"[256^3 T=128, {info['n_chunks']} chunks, {info['n_slots']} slots] loss {e_loss:.2e}, "
          f"grad_u0 rel L2 {e_gu:.2e}, grad_w per component " +
          " ".join(f"{e:.1e}" for e in e_comp), flush=True)
    assert e_loss <= 1e-4 and e_gu <= 1e-4
    assert np.all(e_comp <= 1e-4), e_comp
