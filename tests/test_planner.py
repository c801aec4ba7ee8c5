"""Host-side tests of the planner (no GPU): geometry, Algorithm 1 counts,
budget accounting, error paths, and a schedule simulator that replays the
planner's exact operation list on host arrays with a NumPy stepper.

The simulator tracks, for every plane of every slot buffer, which time level
it holds (or that it holds nothing valid), and fails on any read of a plane
that is not valid at the level the operation needs: that is the halo
sufficiency check of the parallelogram geometry (paper Sec. IV-B).  Its
stepper is whole-array shifting in NumPy, not the oracle's code; the end
result is compared with the oracle."""
import math
import re
import os

import numpy as np
import pytest

import oracle
from paper_2309_08864_amd import Plan, So2drError
from paper_2309_08864_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _w(ndim, shape, r):
    offs = oracle.stencil_offsets(ndim, shape, r)
    rng = np.random.default_rng(len(offs))
    w = rng.uniform(0.1, 1, len(offs))
    return offs, list(w / w.sum())


def _plan(ndim=3, nx=8, ny=6, nz=40, shape="star", r=1, T=10, K=3, d=4, k_on=2, slots=0,
          budget=1 << 30, **kw):
    offs, w = _w(ndim, shape, r)
    if ndim == 2:
        ny, nz = nz, 1
    return Plan(ndim=ndim, nx=nx, ny=ny, nz=nz, shape=shape, radius=r, weights=w, T=T,
                tb_depth=K, n_chunks=d, k_on=k_on, n_slots=slots, budget=budget, **kw), offs, w


# ------------------------------------------------------------------ symbols
def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "so2dr.h")).read()
    declared = set(re.findall(r"\b(so2dr_[a-z_]+)\s*\(", hdr))
    assert declared == set(_lib.EXPORTS)
    L = _lib.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert L.so2dr_version().decode().startswith("so2dr")


# ------------------------------------------------------------------ geometry
@pytest.mark.parametrize("T,K,d,k_on,r", [(10, 3, 4, 2, 1), (16, 4, 4, 4, 1), (7, 7, 1, 3, 1),
                                          (9, 4, 3, 3, 2), (5, 8, 2, 2, 1), (1, 1, 5, 1, 1),
                                          (13, 5, 2, 4, 1)])
def test_algorithm1_counts_and_partition(T, K, d, k_on, r):
    p, _, _ = _plan(T=T, K=K, d=d, k_on=min(k_on, 2 if r == 2 else 4), r=r, nz=60)
    info = p.info()
    Kp = min(K, T)
    k_on = info["k_on"]
    n_rounds = math.ceil(T / Kp)   # Algorithm 1: N_t = ceil(n / k_off)
    assert info["n_rounds"] == n_rounds
    ops = p.ops()
    N = info["n_axis"]
    for t in range(n_rounds):
        kp = T - (n_rounds - 1) * Kp if (t == n_rounds - 1 and T % Kp) else Kp
        outs = []
        for i in range(d):
            mine = [o for o in ops if o["round"] == t and o["chunk"] == i]
            kinds = [o["kind"] for o in mine]
            assert kinds.count("H2D") == 1 and kinds.count("D2H") == 1
            # read, then write, the region-sharing buffer (Algorithm 1)
            assert kinds.count("RS_READ") == (1 if i > 0 else 0)
            assert kinds.count("RS_WRITE") == (1 if i < d - 1 else 0)
            if i > 0 and i < d - 1:
                assert kinds.index("RS_READ") < kinds.index("RS_WRITE")
            ks = [o for o in mine if o["kind"] == "KERNEL"]
            assert len(ks) == kp // k_on + (1 if kp % k_on else 0)
            assert [o["levels"] for o in ks] == [k_on] * (kp // k_on) + ([kp % k_on] if kp % k_on else [])
            assert sum(o["levels"] for o in ks) == kp
            # consecutive launches chain their areas and shrink by r per level
            for a, b in zip(ks, ks[1:]):
                assert (b["in_z0"], b["in_z1"]) == (a["z0"], a["z1"])
            for o in ks:
                lo_shrink = 0 if i == 0 else o["levels"] * r
                hi_shrink = 0 if i == d - 1 else o["levels"] * r
                assert o["z0"] - o["in_z0"] == lo_shrink and o["in_z1"] - o["z1"] == hi_shrink
            h2d = mine[kinds.index("H2D")]
            d2h = mine[kinds.index("D2H")]
            assert d2h["z0"] == ks[-1]["z0"] and d2h["z1"] == ks[-1]["z1"]
            outs.append((d2h["z0"], d2h["z1"]))
            # the shared region lies inside the previous chunk's own planes
            if i > 0:
                rs = mine[kinds.index("RS_READ")]
                assert rs["z1"] == h2d["z0"] and rs["z1"] - rs["z0"] == 2 * r * kp
        # outputs partition [0, N)
        assert outs[0][0] == 0 and outs[-1][1] == N
        for a, b in zip(outs, outs[1:]):
            assert a[1] == b[0]
    # every plane crosses the link once per round in each direction
    assert sum(o["z1"] - o["z0"] for o in ops if o["kind"] == "H2D") == N * n_rounds
    assert sum(o["z1"] - o["z0"] for o in ops if o["kind"] == "D2H") == N * n_rounds


def test_paper_configuration_fits_and_counts():
    """The paper's out-of-core setting: 38400^2 FP32, 640 steps, d = 4,
    S_TB = 160, box2d1r, 10 GB device memory, 3 streams (Sec. V-A, V-B)."""
    offs = oracle.stencil_offsets(2, "box", 1)
    p = Plan(ndim=2, nx=38400, ny=38400, nz=1, shape="box", radius=1, weights=[1 / 9] * 9, T=640,
             tb_depth=160, n_chunks=4, k_on=4, n_slots=3, budget=10 * 10 ** 9)
    info = p.info()
    assert info["n_rounds"] == 4 and info["n_chunks"] == 4 and info["n_slots"] == 3
    assert info["workspace_bytes"] <= 10 * 10 ** 9
    # halo (2 r S_TB rows) is 3.3% of a 9600-row chunk: under the paper's 20% rule
    assert 2 * 160 / 9600 < 0.2
    ops = p.ops()
    assert sum(1 for o in ops if o["kind"] == "KERNEL") == 4 * 4 * 40


@pytest.mark.parametrize("ndim,shape,r,T,K,d", [(3, "star", 1, 10, 3, 4), (3, "box", 1, 7, 4, 3),
                                                 (3, "star", 2, 6, 3, 2), (2, "box", 3, 5, 2, 3)])
def test_resreu_schedule_matches_oracle(ndim, shape, r, T, K, d):
    """The comparison method: per-step sharing through one buffer slot per
    level, single-step kernels, no recomputation."""
    nx, ny, N = 7, 5, 60
    p, offs, w = _plan(ndim=ndim, nx=nx, ny=ny, nz=N, shape=shape, r=r, T=T, K=K, d=d, k_on=0,
                       method="resreu")
    info = p.info()
    assert info["method"] == 1 and info["k_on"] == 1 and info["redundant_fraction"] == 0.0
    ops = p.ops()
    kp_first = min(K, T)
    for i in range(1, d - 1):   # every step of an inner chunk reads then writes the buffer
        kinds = [o["kind"] for o in ops if o["round"] == 0 and o["chunk"] == i]
        assert kinds.count("RS_READ") == kp_first and kinds.count("RS_WRITE") == kp_first
        assert kinds.count("KERNEL") == kp_first
    rng = np.random.default_rng(T + K)
    if ndim == 3:
        u0 = rng.random((N, ny, nx))
        ref = oracle.sweep(u0, offs, w, T)
        host, lv = simulate(p, offs, w, u0, 0, 0, 3)
    else:
        u0 = rng.random((N, 1, nx))
        ref = oracle.sweep(u0[:, 0, :], offs, w, T)[:, None, :]
        host, lv = simulate(p, offs, w, u0, 0, 0, 2)
    assert np.all(lv == T) and np.allclose(host, ref, rtol=1e-12, atol=1e-12)


def test_lean_layout_for_the_2d_fp64_workload():
    """Four 256-row FP64 chunks need 4.19 MiB with two buffers per slot; the
    one-buffer layout fits the 4 MiB budget, and its schedule replays on the
    CPU against the oracle."""
    offs, w = _w(2, "star", 1)
    w = [0.2] * 5
    p = Plan(ndim=2, nx=1024, ny=1024, nz=1, shape="star", radius=1, weights=w, T=16, tb_depth=4,
             n_chunks=4, budget=4 << 20, storage="f64")
    info = p.info()
    assert info["lean"] == 1 and info["workspace_bytes"] <= 4 << 20
    ps = Plan(ndim=2, nx=16, ny=1024, nz=1, shape="star", radius=1, weights=w, T=16, tb_depth=4,
              n_chunks=4, budget=info["workspace_bytes"] // 64, storage="f64")
    assert ps.info()["lean"] == 1
    rng = np.random.default_rng(1)
    u0 = rng.random((1024, 1, 16))
    host, lv = simulate(ps, offs, w, u0, 0, 0, 2)
    ref = oracle.sweep(u0[:, 0, :], offs, w, 16)[:, None, :]
    assert np.all(lv == 16) and np.allclose(host, ref, rtol=1e-12, atol=1e-12)


def test_budget_accounting_and_auto_plan():
    offs, w = _w(3, "star", 1)
    kw = dict(ndim=3, nx=2048, ny=1024, nz=1024, shape="star", radius=1, weights=w, T=64, tb_depth=8)
    p = Plan(budget=4 << 30, **kw)
    info = p.info()
    assert info["workspace_bytes"] <= 4 << 30
    assert info["n_chunks"] == 16 and info["n_slots"] == 3     # fewest chunks with 3 slots
    plane = 2048 * 1024 * 4
    assert info["slot_bytes"] == 2 * (64 + 16) * plane
    assert info["rs_bytes"] == 16 * plane
    assert info["workspace_bytes"] == 3 * info["slot_bytes"] + info["rs_bytes"]
    assert abs(info["redundant_fraction"] - 0.1025390625) < 1e-12
    # 8 chunks only fit one slot under 4 GiB
    p8 = Plan(budget=4 << 30, n_chunks=8, **kw)
    assert p8.info()["n_slots"] == 1
    # a whole-grid (in-core) plan when the budget allows it
    pin = Plan(budget=64 << 30, **kw)
    assert pin.info()["n_chunks"] == 1
    # the 2D 5-point FP32 workload: 4 row chunks under 4 MiB
    o2, w2 = _w(2, "star", 1)
    p2 = Plan(ndim=2, nx=1024, ny=1024, nz=1, shape="star", radius=1, weights=w2, T=16, tb_depth=4,
              n_chunks=4, budget=4 << 20)
    assert p2.info()["workspace_bytes"] <= 4 << 20


def test_error_paths():
    offs, w = _w(3, "star", 1)
    base = dict(ndim=3, nx=16, ny=16, nz=64, shape="star", radius=1, weights=w, T=8, tb_depth=4)
    with pytest.raises(So2drError, match="E_BUDGET"):
        Plan(budget=1000, **base)
    with pytest.raises(So2drError, match="E_BUDGET"):
        Plan(budget=40 * 1024, n_chunks=2, n_slots=3, **base)
    with pytest.raises(So2drError, match="E_INVALID"):
        Plan(budget=1 << 30, n_chunks=9, **base)      # chunk shorter than 2 r K
    with pytest.raises(So2drError, match="E_UNSUPPORTED"):
        Plan(budget=1 << 30, bc=(0, 0, 1), **base)    # periodic cut axis
    with pytest.raises(So2drError, match="E_INVALID"):
        Plan(budget=1 << 30, **dict(base, weights=w[:-1]))
    with pytest.raises(So2drError, match="E_UNSUPPORTED"):
        Plan(budget=1 << 30, **dict(base, shape="star", radius=3, weights=[0.1] * 19))
    with pytest.raises(So2drError, match="E_UNSUPPORTED"):
        Plan(budget=1 << 30, k_on=16, **base)
    with pytest.raises(So2drError, match="E_INVALID"):
        Plan(budget=1 << 30, **dict(base, nz=0))
    with pytest.raises(So2drError, match="E_INVALID"):
        Plan(budget=1 << 30, **dict(base, ndim=2))    # 2D grids have nz == 1
    p = Plan(budget=1 << 30, **base)
    with pytest.raises(So2drError, match="E_UNBOUND"):
        import torch
        p.run(torch.zeros(64 * 16 * 16))


def test_copy_engine_choice():
    """Automatic copy engine: copy kernels for the copy-out below 512 MiB per
    chunk copy when a run queues more than 256 copies, DMA otherwise and for
    adjoint plans; an explicit choice is kept; unknown values are refused."""
    import ctypes
    from paper_2309_08864_amd import _lib
    from paper_2309_08864_amd.plan import _make_desc
    offs, w = _w(3, "star", 1)
    base = dict(ndim=3, nx=2048, ny=1024, nz=1024, shape="star", radius=1, weights=w, T=64,
                tb_depth=8, budget=4 << 30)
    assert Plan(n_chunks=16, **base).info()["copy_engine"] == 1      # 512 MiB copies: DMA
    assert Plan(n_chunks=32, **base).info()["copy_engine"] == 3      # 256 MiB: kernels out
    assert Plan(n_chunks=32, copy_engine="dma", **base).info()["copy_engine"] == 1
    assert Plan(n_chunks=16, copy_engine="kernel", **base).info()["copy_engine"] == 2
    assert Plan(n_chunks=32, adjoint=True, **dict(base, budget=8 << 30)).info()["copy_engine"] == 1
    assert Plan(n_chunks=32, **dict(base, T=32, tb_depth=16)).info()["copy_engine"] == 1  # 128 copies
    kw = dict(base, nz=1024, tb_depth=8, n_chunks=16, k_on=0, n_slots=0, storage="f32",
              bc=(0, 0, 0), adjoint=False, method="so2dr", rounding="every_step")
    d, keep = _make_desc(**kw)
    d.copy_engine = 7
    h = ctypes.c_void_p()
    assert _lib.lib().so2dr_plan_create(ctypes.byref(d), ctypes.byref(h)) == -1
    # the cost model prices copy kernels at their own both-directions rate
    pk = Plan(n_chunks=16, copy_engine="kernel", **base)
    pd = Plan(n_chunks=16, copy_engine="dma", **base)
    m = pd.machine()
    assert m["kcopy_gbps"] < m["duplex_gbps"]
    assert pk.predict() > pd.predict() * 1.05
    po = Plan(n_chunks=16, copy_engine="kernel_out", **base)
    assert m["kcopy_gbps"] < m["kcopy_out_gbps"] < m["duplex_gbps"]
    assert pk.predict() > po.predict() > pd.predict()


def test_host_alloc_argument_paths():
    """so2dr_host_alloc / so2dr_host_free paths that make no HIP call."""
    import ctypes
    from paper_2309_08864_amd._lib import lib
    L = lib()
    assert L.so2dr_host_alloc(16, None) == -1                   # null output: E_INVALID
    p = ctypes.c_void_p(1234)
    assert L.so2dr_host_alloc(0, ctypes.byref(p)) == 0 and p.value is None
    assert L.so2dr_host_free(None) == 0


# ------------------------------------------------------------------ simulator
def _np_step(win, offs, w, per_x, per_y):
    """One step on a window of planes: win is (planes, ny, nx) FP64 of level
    s covering planes [q0 - r, q1 + r); returns planes [q0, q1) of level s+1.
    In-plane boundary by padding, cut axis by the window itself."""
    r = max(max(abs(o[0]), abs(o[1]), abs(o[2])) for o in offs)
    nzw = win.shape[0] - 2 * r
    pad = np.pad(win, ((0, 0), (r, r), (0, 0)), mode="wrap" if per_y else "constant")
    pad = np.pad(pad, ((0, 0), (0, 0), (r, r)), mode="wrap" if per_x else "constant")
    ny, nx = win.shape[1], win.shape[2]
    out = np.zeros((nzw, ny, nx))
    for o, wk in zip(offs, w):
        dz, dy, dx = o
        out += wk * pad[r + dz:r + dz + nzw, r + dy:r + dy + ny, r + dx:r + dx + nx]
    return out


def simulate(p, offs, w, u0, per_x=0, per_y=0, ndim=3):
    """Replay p.ops() on host arrays.  u0: (N, ny, nx).  Every buffer index an
    operation touches is checked against the slot size, and every plane a
    kernel needs must hold the level it expects."""
    info = p.info()
    N = info["n_axis"]
    r = max(max(abs(c) for c in o) for o in offs)
    if ndim == 2:   # 2D: rows are planes, offsets (dy, dx) act as (dz, 0, dx)
        offs = [(o[1], 0, o[2]) for o in offs]
    host = u0.copy()
    host_lvl = np.zeros(N, dtype=np.int64)          # global time level of each host plane
    S = info["slot_planes"]
    shp = u0.shape[1:]
    bufs = {}
    lvl = {}
    pool = np.zeros((2 * r * info["tb_depth"],) + shp)
    pool_lvl = np.full(pool.shape[0], -1)
    round_start = 0

    def idx(z0, z1, base):
        i0, i1 = z0 - base, z1 - base
        assert 0 <= i0 <= i1 <= S, f"buffer index [{i0}, {i1}) outside [0, {S})"
        return slice(i0, i1)

    for op in p.ops():
        sl = op["slot"]
        if sl not in bufs:
            bufs[sl] = [np.full((S,) + shp, np.nan), np.full((S,) + shp, np.nan)]
            lvl[sl] = [np.full(S, -1), np.full(S, -1)]
        z0, z1, b0 = op["z0"], op["z1"], op["buf_z0"]
        kind = op["kind"]
        if kind == "H2D":
            round_start = int(host_lvl[z0])
            assert np.all(host_lvl[z0:z1] == round_start), "host planes not at round-start level"
            bufs[sl][op["buf_out"]][idx(z0, z1, b0)] = host[z0:z1]
            lvl[sl][op["buf_out"]][idx(z0, z1, b0)] = round_start
        elif kind == "RS_READ":
            n, po = z1 - z0, op["pool_off"]
            assert 0 <= po and po + n <= pool.shape[0]
            assert np.all(pool_lvl[po:po + n] >= round_start), "stale region-sharing data"
            bufs[sl][op["buf_out"]][idx(z0, z1, b0)] = pool[po:po + n]
            lvl[sl][op["buf_out"]][idx(z0, z1, b0)] = pool_lvl[po:po + n]
        elif kind == "RS_WRITE":
            n, po = z1 - z0, op["pool_off"]
            assert 0 <= po and po + n <= pool.shape[0]
            src = bufs[sl][op["buf_in"]]
            assert np.all(lvl[sl][op["buf_in"]][idx(z0, z1, b0)] >= round_start)
            pool[po:po + n] = src[idx(z0, z1, b0)]
            pool_lvl[po:po + n] = lvl[sl][op["buf_in"]][idx(z0, z1, b0)]
        elif kind == "KERNEL":
            L = op["levels"]
            s0 = round_start + op["level_in"]
            src, slv = bufs[sl][op["buf_in"]], lvl[sl][op["buf_in"]]
            # planes this launch needs, inside the input's valid area
            cur_lo, cur_hi = max(0, z0 - L * r), min(N, z1 + L * r)
            assert op["in_z0"] <= cur_lo and cur_hi <= op["in_z1"]
            assert np.all(slv[idx(cur_lo, cur_hi, b0)] == s0), "kernel input not valid (halo too thin or overwritten)"
            cur = src[idx(cur_lo, cur_hi, b0)].copy()
            for j in range(1, L + 1):
                new_lo = max(z0 - (L - j) * r, 0)
                new_hi = min(z1 + (L - j) * r, N)
                win = np.zeros((new_hi - new_lo + 2 * r,) + shp)
                for q in range(new_lo - r, new_hi + r):
                    if 0 <= q < N:
                        assert cur_lo <= q < cur_hi, f"plane {q} needed but not loaded"
                        win[q - (new_lo - r)] = cur[q - cur_lo]
                cur = _np_step(win, offs, w, per_x, per_y)
                cur_lo, cur_hi = new_lo, new_hi
            assert (cur_lo, cur_hi) == (z0, z1)
            dst, dlv = bufs[sl][op["buf_out"]], lvl[sl][op["buf_out"]]
            if op["buf_out"] == op["buf_in"]:
                # one launch reads and writes the same buffer concurrently: the
                # index ranges must not meet
                rd = idx(max(0, z0 - L * r), min(N, z1 + L * r), b0)
                wr = idx(z0, z1, op["out_z0"])
                assert wr.stop <= rd.start or rd.stop <= wr.start, "launch overwrites its own input"
            dst[idx(z0, z1, op["out_z0"])] = cur
            dlv[idx(z0, z1, op["out_z0"])] = s0 + L
        elif kind == "D2H":
            src, slv = bufs[sl][op["buf_in"]], lvl[sl][op["buf_in"]]
            lv = slv[idx(z0, z1, b0)]
            assert np.all(lv == lv[0]) and lv[0] > round_start
            host[z0:z1] = src[idx(z0, z1, b0)]
            host_lvl[z0:z1] = lv[0]
    assert np.all(host_lvl == host_lvl[0])
    return host, host_lvl


@pytest.mark.parametrize("ndim,shape,r,T,K,d,k_on,per", [
    (3, "star", 1, 10, 3, 4, 2, (0, 0)), (3, "star", 2, 9, 4, 3, 2, (0, 0)),
    (3, "box", 1, 8, 4, 5, 3, (1, 1)), (2, "box", 2, 7, 3, 3, 2, (1, 0)),
    (2, "star", 1, 16, 4, 4, 4, (0, 0)), (3, "star", 1, 5, 5, 1, 2, (0, 0)),
    (3, "box", 1, 11, 3, 6, 3, (1, 0)), (2, "box", 4, 6, 2, 3, 1, (0, 0))])
@pytest.mark.parametrize("lean", [False, True])
def test_schedule_simulator_matches_oracle(ndim, shape, r, T, K, d, k_on, per, lean):
    nx, ny, N = 7, 5, 48
    budget = 1 << 30
    if lean:   # just under what two buffers per slot need with one slot
        p0, _, _ = _plan(ndim=ndim, nx=nx, ny=ny, nz=N, shape=shape, r=r, T=T, K=K, d=d, k_on=k_on,
                         slots=1, bc=(per[0], per[1] if ndim == 3 else 0, 0))
        budget = p0.info()["workspace_bytes"] - 1
    p, offs, w = _plan(ndim=ndim, nx=nx, ny=ny, nz=N, shape=shape, r=r, T=T, K=K, d=d, k_on=k_on,
                       slots=1 if lean else 0, budget=budget,
                       bc=(per[0], per[1] if ndim == 3 else 0, 0))
    assert p.info()["lean"] == (1 if lean else 0)
    rng = np.random.default_rng(T * 7 + K)
    if ndim == 3:
        u0 = rng.random((N, ny, nx))
        ref = oracle.sweep(u0, offs, w, T, (per[0], per[1], 0))
        host, lv = simulate(p, offs, w, u0, per[0], per[1], 3)
    else:
        u0 = rng.random((N, 1, nx))
        ref = oracle.sweep(u0[:, 0, :], offs, w, T, (per[0], 0, 0))[:, None, :]
        host, lv = simulate(p, offs, w, u0, per[0], 0, 2)
    assert np.all(lv == T)
    assert np.allclose(host, ref, rtol=1e-12, atol=1e-12)
