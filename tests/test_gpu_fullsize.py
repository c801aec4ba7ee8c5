"""Parity at the workloads' full sizes, in the launch configurations the
benchmark uses and in the plans the cost model picks: sampled output boxes
against the FP64 oracle's light-cone sub-box sweep (it reads only each box's
dependency cone of u0) and bit for bit against the C model of the documented
arithmetic, bit-for-bit in-core vs out-of-core for every plan and storage
type, and for the adjoint, identities that hold at any size.

Large pinned host fields: 2D 5-point 1024^2; 3D 7-point and 27-point
2048x1024x1024 (8 GiB per FP32 field); 13-point 2048^3 (32 GiB FP32);
adjoint 1024^3 (4 GiB per field, 8 checkpoints)."""
import time

import numpy as np
import pytest
import torch

import oracle
import workloads
from helpers import pinned_copy, rel_l2
from paper_2309_08864_amd import Plan, So2drError, stencil_offsets

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

WL = workloads.CONFIGS


@pytest.fixture(autouse=True)
def _release_pinned():
    """Each test pins tens of GiB of host memory; hand it back afterwards
    instead of leaving it in torch's pinned-block cache."""
    yield
    import gc
    gc.collect()
    if hasattr(torch._C, "_host_emptyCache"):
        torch._C._host_emptyCache()


def _log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def _weights(wl, offs):
    tag = wl.weights.split(":")
    if tag[0] == "const":
        w = workloads.const_weights(offs, float(tag[1]))
    elif tag[0] == "centre_arm":
        w = workloads.centre_arm_weights(offs, float(tag[1]), [float(x) for x in tag[2:]])
    else:
        w = workloads.random_box_weights(offs, wl.seed)
    return w


def _pinned(shape, dtype):
    return torch.empty(shape, dtype=dtype, pin_memory=True)


def _sample_boxes(nx, ny, nz, n_chunks, rng, size=3, extra=4):
    """Boxes at the corners, across chunk boundaries and at random places."""
    boxes = []
    corners = [(0, 0, 0), (nx - size, ny - size, nz - size), (0, ny - size, nz // 2),
               (nx - size, 0, 0)]
    for c in corners:
        boxes.append(c)
    for i in range(1, min(n_chunks, 3)):
        z = nz * i // n_chunks - size // 2
        boxes.append((int(rng.integers(0, nx - size)), int(rng.integers(0, ny - size)), z))
    for _ in range(extra):
        boxes.append(tuple(int(rng.integers(0, n - size + 1)) for n in (nx, ny, nz)))
    return [(b, tuple(v + size for v in b)) for b in boxes]


def _check_boxes(u0_np, got_np, offs, w, T, per, boxes, tol, tag):
    worst = 0.0
    for lo, hi in boxes:
        ref = oracle.sweep_box_from_field(u0_np, offs, w, T, lo, hi, per)
        g = got_np[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].astype(np.float64)
        e = rel_l2(g, ref)
        worst = max(worst, e)
        assert e <= tol, f"{tag}: box {lo}-{hi} rel L2 {e:.3e}"
    _log(f"{tag}: {len(boxes)} boxes, worst rel L2 vs FP64 oracle {worst:.3e}")
    return worst


def test_c1_2d5pt_full():
    """2D 5-point, 1024^2, 4 row chunks, TB depth 4, 4 MiB budget, FP32; FP64
    with the same chunks needs 4.19 MiB with two ping-pong buffers, so the
    planner refuses it under 4 MiB and it runs with 8 chunks instead."""
    wl = WL["c1_2d5pt"]
    offs = stencil_offsets(2, "star", 1)
    w = _weights(wl, offs)
    u64 = workloads.uniform((wl.ny, wl.nx), seed=wl.seed)
    base = dict(ndim=2, nx=wl.nx, ny=wl.ny, nz=1, shape="star", radius=1, T=wl.T,
                tb_depth=wl.tb_depth, budget=wl.budget)
    # FP32, 4 chunks, 4 MiB
    w32 = workloads.fp32_rounded(w)
    u32 = torch.from_numpy(u64.astype(np.float32))
    p = Plan(weights=list(w32), n_chunks=4, **base).bind()
    assert p.info()["workspace_bytes"] <= 4 << 20 and p.info()["n_chunks"] == 4
    h = pinned_copy(u32)
    p.run(h)
    p.close()
    ref = oracle.sweep(u32.double().numpy(), offs, w32, wl.T)
    e32 = rel_l2(h.double().numpy(), ref)
    _log(f"c1 FP32 rel L2 {e32:.3e}")
    assert e32 <= 1e-5
    # in-core bitwise
    pin = Plan(weights=list(w32), n_chunks=1, **dict(base, tb_depth=wl.T, budget=64 << 20)).bind()
    hi = pinned_copy(u32)
    pin.run(hi)
    pin.close()
    assert torch.equal(hi, h)
    # FP64: two buffers per slot would need 4.19 MiB, so the planner takes the
    # one-buffer layout (sub-block launches writing below what they read)
    p = Plan(weights=list(w), n_chunks=4, storage="f64", **base).bind()
    info = p.info()
    assert info["workspace_bytes"] <= 4 << 20 and info["n_chunks"] == 4 and info["lean"] == 1
    h = pinned_copy(torch.from_numpy(u64))
    p.run(h)
    p.close()
    e64 = rel_l2(h.numpy(), oracle.sweep(u64, offs, w, wl.T))
    _log(f"c1 FP64 (4 chunks, one buffer per slot) rel L2 {e64:.3e}")
    assert e64 <= 1e-12
    pin = Plan(weights=list(w), n_chunks=1, storage="f64", **dict(base, tb_depth=wl.T, budget=64 << 20)).bind()
    hi = pinned_copy(torch.from_numpy(u64))
    pin.run(hi)
    pin.close()
    assert torch.equal(hi, h)


def _check_bits(u0_np, got_np, offs, w, T, per, boxes, storage, tag, round_after=None):
    """Sampled boxes bit for bit against the C model of the documented
    arithmetic (light-cone windows; the grid's interior boxes come from the
    kernels' interior path)."""
    from oracle import emulator
    for lo, hi in boxes:
        ref = emulator.sweep_bits_box_from_field(u0_np, offs, w, T, lo, hi, storage, per,
                                                 round_after=round_after)
        g = got_np[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        g = np.ascontiguousarray(g.float().numpy() if isinstance(g, torch.Tensor) else g,
                                 dtype=np.float32)
        diff = int(np.sum(g.view(np.uint32) != ref.view(np.uint32)))
        assert diff == 0, f"{tag}: box {lo}-{hi}: {diff} cells differ from the arithmetic model"
    _log(f"{tag}: {len(boxes)} boxes bit-identical to the arithmetic model")


def _full_3d(name, plans):
    """The workload's field, run out of core under each plan of `plans`
    (keyword overrides of the workload's tb_depth / n_chunks / k_on /
    n_slots), checked on sampled boxes against the FP64 oracle and bit for
    bit against the arithmetic model, and each bit for bit against the
    in-core run."""
    wl = WL[name]
    offs = stencil_offsets(3, wl.shape, wl.radius)
    w = workloads.fp32_rounded(_weights(wl, offs))
    shp = (wl.nz, wl.ny, wl.nx)
    h_in = _pinned(shp, torch.float32)
    t0 = time.time()
    if wl.init == "uniform":
        workloads.uniform_into(h_in.numpy(), wl.seed)
    elif wl.init == "fourier":
        workloads.fourier_modes_into(h_in.numpy(), wl.seed)
    _log(f"{name}: input ready in {time.time() - t0:.1f} s")
    kw = dict(ndim=3, nx=wl.nx, ny=wl.ny, nz=wl.nz, shape=wl.shape, radius=wl.radius,
              weights=list(w), T=wl.T, bc=wl.periodic)
    pin = Plan(tb_depth=wl.T, n_chunks=1, budget=24 << 30, **kw).bind()
    h_ic = _pinned(shp, torch.float32)
    pin.run_steps(h_in, h_ic, wl.T)
    pin.close()
    h_out = _pinned(shp, torch.float32)
    rng = np.random.default_rng(7)
    uniq = []
    for over in plans:   # suggest() may pick a plan already listed
        if over not in uniq:
            uniq.append(over)
    for i, over in enumerate(uniq):
        plan_kw = dict(dict(tb_depth=wl.tb_depth, n_chunks=wl.n_chunks, k_on=0, n_slots=0,
                            budget=wl.budget), **over)
        p = Plan(**plan_kw, **kw).bind()
        info = p.info()
        assert info["workspace_bytes"] <= wl.budget
        for k in ("tb_depth", "n_chunks", "k_on", "n_slots"):
            if over.get(k):
                assert info[k] == over[k], (k, info[k], over[k])
        st = p.run_steps(h_in, h_out, wl.T)
        p.close()
        tag = (f"{name} K={info['tb_depth']} d={info['n_chunks']} k_on={info['k_on']} "
               f"slots={info['n_slots']}")
        _log(f"{tag}: out-of-core {st['wall_ms']:.0f} ms")
        assert torch.equal(h_ic, h_out), f"{tag}: out-of-core differs from in-core"
        _log(f"{tag}: out-of-core == in-core bit for bit")
        if i == 0:
            boxes = _sample_boxes(wl.nx, wl.ny, wl.nz, info["n_chunks"], rng)
            _check_boxes(h_in.numpy(), h_out.numpy(), offs, w, wl.T, wl.periodic, boxes, 1e-5, name)
            _check_bits(h_in.numpy(), h_out.numpy(), offs, w, wl.T, wl.periodic, boxes, "f32", name)


def _suggested(name):
    """The plan so2dr_plan_suggest picks for the workload with the round
    depth, chunk count, fused depth and slot count all free."""
    from paper_2309_08864_amd import suggest
    wl = WL[name]
    offs = stencil_offsets(3, wl.shape, wl.radius)
    w = workloads.fp32_rounded(_weights(wl, offs))
    kw, pred = suggest(ndim=3, nx=wl.nx, ny=wl.ny, nz=wl.nz, shape=wl.shape, radius=wl.radius,
                       weights=list(w), T=wl.T, budget=wl.budget, bc=wl.periodic)
    auto = {k: kw[k] for k in ("tb_depth", "n_chunks", "k_on", "n_slots")}
    _log(f"{name}: suggest() -> {auto}, predicted {pred:.0f} ms")
    return auto


def test_c2_3d7pt_full():
    """The benchmark's plan (K = 8, 16 chunks, k_on = 3, 3 slots); the cost
    model's plan with the round depth free as measured (K = 24, 16 chunks,
    k_on = 3, 2 slots: 64-plane chunks carrying a 48-plane halo); and
    whatever so2dr_plan_suggest picks now."""
    _full_3d("c2_3d7pt", [{}, dict(tb_depth=24, n_chunks=16, k_on=3, n_slots=2),
                          _suggested("c2_3d7pt")])


def test_c3_3d27pt_full():
    """The workload's plan (K = 4, 16 chunks); the cost model's measured plan
    (K = 16, 29 ragged chunks, k_on = 2, 3 slots); and what so2dr_plan_suggest
    picks now."""
    _full_3d("c3_3d27pt", [{}, dict(tb_depth=16, n_chunks=29, k_on=2, n_slots=3),
                           _suggested("c3_3d27pt")])


def test_c4_3d13pt_full_precision():
    """2048^3 13-point star in BF16 (rounded every step and at store), FP16
    and FP32 storage (the FP32 field, from the FP64 recipe rounded once, is
    the input; BF16 / FP16 inputs are its roundings).  Per storage type and
    rounding: the workload's plan (K = 8, 32 chunks)
    and, for FP32 and BF16, also the cost model's plan (FP32: K = 24, 19
    chunks, 1 slot; BF16: K = 16, 22 chunks, k_on = 1) are bit-identical to
    the in-core run of that type; sampled boxes are
    bit-identical to the arithmetic model and, against the FP64 oracle run
    from the same input, within the rigorous per-step rounding bound; the
    error against the oracle run from the FP32 input is reported.  At most
    one field (32 GiB) is pinned at a time; the input and the out-of-core
    result are kept in pageable memory."""
    import gc
    wl = WL["c4_3d13pt"]
    offs = stencil_offsets(3, "star", 2)
    w = workloads.fp32_rounded(_weights(wl, offs))
    shp = (wl.nz, wl.ny, wl.nx)
    master = np.empty(shp, np.float32)
    t0 = time.time()
    workloads.gaussian_bump_into(master, wl.seed)
    tm = torch.from_numpy(master)
    _log(f"c4: input ready in {time.time() - t0:.1f} s")
    max_u0 = max(float(master.max()), -float(master.min()))
    rng = np.random.default_rng(11)
    boxes = _sample_boxes(wl.nx, wl.ny, wl.nz, 32, rng, size=2, extra=3)
    refs32 = [oracle.sweep_box_from_field(master, offs, w, wl.T, lo, hi) for lo, hi in boxes]
    base = dict(ndim=3, nx=wl.nx, ny=wl.ny, nz=wl.nz, shape="star", radius=2, weights=list(w),
                T=wl.T)
    dts = {"bf16": torch.bfloat16, "f16": torch.float16, "f32": torch.float32}
    own_refs = {}
    for name, rounding in (("bf16", "every_step"), ("bf16", "at_store"), ("f16", "every_step"),
                           ("f32", "every_step")):
        tag = f"c4 {name}" + (" at store" if rounding == "at_store" else "")
        h = _pinned(shp, dts[name])

        def load():
            for z0 in range(0, wl.nz, 64):
                h[z0:z0 + 64].copy_(tm[z0:z0 + 64])

        load()
        if name not in own_refs:
            own_refs[name] = refs32 if name == "f32" else \
                [oracle.sweep_box_from_field(h, offs, w, wl.T, lo, hi) for lo, hi in boxes]
        refs_own = own_refs[name]
        p = Plan(storage=name, tb_depth=wl.tb_depth, n_chunks=wl.n_chunks, budget=wl.budget,
                 rounding=rounding, **base).bind()
        info = p.info()
        st = p.run(h)
        p.close()
        _log(f"{tag} K=8 d=32: {st['wall_ms']:.0f} ms")
        unit = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}[name]
        worst_arith, worst_total = 0.0, 0.0
        for k, ((lo, hi), r32, ref_own) in enumerate(zip(boxes, refs32, refs_own)):
            g = h[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].double().numpy()
            worst_total = max(worst_total, rel_l2(g, r32))
            err = np.abs(g - ref_own).max()
            # weights >= 0 summing to 1: ||A||_inf <= 1, so the error is at most
            # the per-step roundings summed: T (u_storage + P 2^-24) max|u0|
            bound = wl.T * (unit + 13 * 2.0 ** -24) * max_u0
            worst_arith = max(worst_arith, err)
            assert err <= bound, f"{tag}: box {lo} max err {err:.3e} > bound {bound:.3e}"
        _log(f"{tag}: worst total rel L2 vs FP64 oracle (FP32 input) {worst_total:.3e}; "
             f"worst arithmetic max err {worst_arith:.3e}")
        if name == "f32":
            assert worst_total <= 1e-5
        ooc = h.clone()                  # pageable copy of the out-of-core result
        load()
        from helpers import store_steps
        ra = store_steps(wl.T, wl.tb_depth, info["k_on"]) if rounding == "at_store" else None
        _check_bits(h, ooc, offs, w, wl.T, (0, 0, 0), boxes, name, tag, round_after=ra)
        if name == "f32":
            p = Plan(storage=name, tb_depth=24, n_chunks=19, k_on=2, n_slots=1, budget=wl.budget,
                     **base).bind()
            info = p.info()
            assert (info["tb_depth"], info["n_chunks"], info["n_slots"]) == (24, 19, 1)
            st = p.run(h)
            p.close()
            _log(f"c4 f32 K=24 d=19 1 slot: {st['wall_ms']:.0f} ms")
            assert torch.equal(h, ooc), "c4 f32: the cost model's plan differs from K=8 d=32"
            load()
        if name == "bf16" and rounding == "every_step":
            # the cost model's BF16 plan (round depth 16, 22 ragged chunks,
            # single-step launches): every-step rounding makes the result
            # independent of K, k_on and the chunking
            p = Plan(storage=name, tb_depth=16, n_chunks=22, k_on=1, budget=wl.budget, **base).bind()
            info2 = p.info()
            assert (info2["tb_depth"], info2["n_chunks"], info2["k_on"]) == (16, 22, 1)
            st = p.run(h)
            p.close()
            _log(f"c4 bf16 K=16 d=22 k_on=1 {info2['n_slots']} slots: {st['wall_ms']:.0f} ms")
            assert torch.equal(h, ooc), "c4 bf16: the cost model's plan differs from K=8 d=32"
            load()
        esz = h.element_size()
        # (at store: the same k_on, and K = 8 a multiple of it, give the same
        # store schedule in and out of core)
        pin = Plan(storage=name, tb_depth=wl.T, n_chunks=1, k_on=info["k_on"], rounding=rounding,
                   budget=2 * wl.nx * wl.ny * wl.nz * esz + (2 << 30), **base).bind()
        st = pin.run(h)
        pin.close()
        _log(f"{tag} in-core: {st['wall_ms']:.0f} ms")
        assert torch.equal(h, ooc), f"{tag}: out-of-core differs from in-core"
        _log(f"{tag}: out-of-core == in-core bit for bit")
        del h, ooc
        gc.collect()
        if hasattr(torch._C, "_host_emptyCache"):
            torch._C._host_emptyCache()


def test_c5_adjoint_full():
    """Adjoint of the 7-point sweep at 1024^3, T = 128, checkpoints every 16
    steps, 2 GiB budget.  Checks: the loss against 1/2 ||u_T - y||^2 from a
    forward run; the exact identities <grad_u0, u0> = <u_T - y, u_T> (u_T is
    linear in u0) and sum_k w_k dL/dw_k = T <u_T - y, u_T> (u_T is
    homogeneous of degree T in w); and dL/du0 on a sampled box against the
    FP64 oracle's light-cone reverse sweep."""
    wl = WL["c5_adjoint"]
    offs = stencil_offsets(3, "star", 1)
    w = workloads.fp32_rounded(_weights(wl, offs))
    wt = workloads.fp32_rounded(workloads.perturbed(w, wl.extra["target_seed"]))
    n, T = wl.nx, wl.T
    shp = (n, n, n)
    u0 = _pinned(shp, torch.float32)
    workloads.uniform_into(u0.numpy(), wl.seed)
    base = dict(ndim=3, nx=n, ny=n, nz=n, shape="star", radius=1, T=T, tb_depth=wl.tb_depth,
                budget=wl.budget)
    y = _pinned(shp, torch.float32)
    pt = Plan(weights=list(wt), **base).bind()
    pt.run_steps(u0, y, T)
    pt.close()
    uT = _pinned(shp, torch.float32)
    pf = Plan(weights=list(w), **base).bind()
    pf.run_steps(u0, uT, T)
    pf.close()
    pa = Plan(weights=list(w), adjoint=True, **base).bind()
    _log(f"c5 plan {pa.info()}")
    t0 = time.time()
    loss, gu, gw, st = pa.adjoint(u0, y, wl.extra["ckpt_every"])
    pa.close()
    _log(f"c5 adjoint {time.time() - t0:.1f} s")
    d = uT.numpy().astype(np.float64) - y.numpy()
    ref_loss = 0.5 * float(np.sum(d * d))
    inner = float(np.sum(d * uT.numpy()))
    e_loss = abs(loss - ref_loss) / ref_loss
    e_u0 = abs(float(np.sum(gu.numpy().astype(np.float64) * u0.numpy())) - inner) / abs(inner)
    e_w = abs(float(np.dot(w, gw)) - T * inner) / abs(T * inner)
    _log(f"c5 loss {e_loss:.2e}; <grad_u0,u0> identity {e_u0:.2e}; sum w dL/dw identity {e_w:.2e}")
    assert e_loss <= 1e-10 and e_u0 <= 1e-4 and e_w <= 1e-4
    # sampled box: lambda_0 = (A^T)^T (u_T - y) on B needs u_T - y on B + T r,
    # i.e. u_T from u0 on B + 2 T r; y is the shared input array
    lo, hi = np.array([500, 11, 700]), np.array([502, 13, 702])
    R = T
    lo1, hi1 = lo - R, hi + R
    uTb = oracle.sweep_box_from_field(u0.numpy(), offs, w, T, lo1, hi1)
    yb = oracle.extract_window(y.numpy(), lo1, hi1, (0, 0, 0))
    lamT = uTb - yb
    neg = [(-a, -b, -c) for a, b, c in offs]
    lam0 = oracle.sweep_box_window(lamT, (n, n, n), neg, w, T, lo, hi)
    g = gu.numpy()[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].astype(np.float64)
    e_box = rel_l2(g, lam0)
    _log(f"c5 grad_u0 sampled box rel L2 vs FP64 oracle {e_box:.2e}")
    assert e_box <= 1e-4


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_paper_box2d_full(r):
    """The paper's out-of-core workloads at full size (box2d{r}r, 38400^2
    FP32, 640 steps, 4 chunks, S_TB 160/160/80/40, 10 GB budget): the SO2DR
    plan and the ResReu comparison plan are bit-identical to the in-core
    run; for radius 1 and 2 also sampled boxes against the FP64 oracle (the
    light cone of 640 steps: windows of 1281^2 and 2561^2 cells)."""
    wl = WL[f"paper_box2d{r}r"]
    offs = stencil_offsets(2, "box", r)
    w = workloads.fp32_rounded(_weights(wl, offs))
    shp = (wl.ny, wl.nx)
    h_in = _pinned(shp, torch.float32)
    workloads.uniform_into(h_in.numpy(), wl.seed)
    kw = dict(ndim=2, nx=wl.nx, ny=wl.ny, nz=1, shape="box", radius=r, weights=list(w), T=wl.T)
    outs = {}
    for name, over in (("in-core", dict(tb_depth=wl.T, n_chunks=1, budget=24 << 30)),
                       ("so2dr", dict(tb_depth=wl.tb_depth, n_chunks=wl.n_chunks, budget=wl.budget)),
                       ("resreu", dict(tb_depth=wl.tb_depth, n_chunks=wl.n_chunks, budget=wl.budget,
                                       method="resreu"))):
        p = Plan(**kw, **over).bind()
        info = p.info()
        h = _pinned(shp, torch.float32) if name != "resreu" else outs.pop("so2dr_buf")
        st = p.run_steps(h_in, h, wl.T)
        p.close()
        _log(f"box2d{r}r {name}: {st['wall_ms']:.0f} ms, k_on {info['k_on']}, {info['n_chunks']} chunks")
        if name == "in-core":
            outs["ref"] = h
        else:
            assert torch.equal(h, outs["ref"]), f"box2d{r}r: {name} differs from in-core"
            _log(f"box2d{r}r {name} == in-core bit for bit")
            if name == "so2dr":
                if r <= 2:
                    rng = np.random.default_rng(5 + r)
                    # a corner each way and a box across the middle chunk boundary
                    x0 = int(rng.integers(0, wl.nx - 2))
                    corners = [(0, 0), (wl.nx - 2, wl.ny - 2), (x0, wl.ny // 2 - 1)]
                    boxes = [((x, y, 0), (x + 2, y + 2, 1)) for x, y in corners]
                    worst = 0.0
                    for lo, hi in boxes:
                        ref = oracle.sweep_box_from_field(h_in.numpy(), offs, w, wl.T, lo, hi)
                        g = h.numpy()[lo[1]:hi[1], lo[0]:hi[0]].astype(np.float64)
                        worst = max(worst, rel_l2(g, ref[0] if ref.ndim == 3 else ref))
                    _log(f"box2d{r}r: {len(boxes)} boxes, worst rel L2 vs FP64 oracle {worst:.3e}")
                    assert worst <= 1e-5
                outs["so2dr_buf"] = h
