"""Benchmark: out-of-core 3D 7-point Jacobi sweep on one MI355X.

Workload (default): 2048 x 1024 x 1024 FP32 grid (8 GiB per field) in pinned
host memory, zero Dirichlet boundary, weights 0.4 centre / 0.1 neighbours,
U[0,1) input from seed 2, T = 64 steps, 8 steps per HBM residency, 16 chunks
along z, device budget capped at 4 GiB.  One "step" of this benchmark is one
whole out-of-core run of T time steps over the grid (host -> HBM -> host).

Prints one JSON line with
  * the whole-job GCell-updates/s of the timed runs;
  * `roofline`: the dominant kernel (the fused depth with the most kernel
    time) -- algorithmic bytes per launch over its mean HIP-event launch
    time on the kernel's own stream, against 8 TB/s; beside it, when a
    committed rocprofv3 summary covers this configuration and kernel
    sources, its traced mean duration and counter-measured HBM traffic;
  * `link`: host-link bytes over wall time, against the vendor PCIe 5.0
    figure and against the pinned-copy rates measured in this run;
  * `precision` (default workload only): the 13-point 2048^3 workload in
    FP32, BF16, FP16 and BF16 rounded at store: GCell-updates/s, speedup over
    FP32 and the error against the FP64 oracle on sampled boxes;
  * `cpu_baseline`: the FP64 CPU oracle on a bounded slab of the same sweep
    (median of three runs on all host threads, plus one single-thread run).
"""
import argparse
import glob
import hashlib
import json
import os
import statistics
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, vendor figure
LINK_PEAK_GBPS = 2 * 63.0       # PCIe 5.0 x16, both directions, vendor figure
TORCH_DT = {"f32": "float32", "f64": "float64", "bf16": "bfloat16", "f16": "float16"}


def committed_profile(config_key):
    """Figures for this configuration from the committed rocprofv3 summaries
    under profiles/ (machine-readable `key=value` lines), provided the kernel
    sources still hash to the value recorded there: the traced mean launch
    time of the dominant kernel (`rocprof_avg_launch_us`) and its HBM bytes
    per launch from the FETCH_SIZE / WRITE_SIZE counters
    (`traffic_bytes_per_launch`)."""
    out = {}
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        kv = {}
        for line in open(path):
            line = line.strip()
            if "=" in line and " " not in line:
                k, v = line.split("=", 1)
                kv[k] = v
        if kv.get("config_key") != config_key:
            continue
        h = hashlib.sha256()
        ok = True
        for name in kv.get("kernel_sources", "").split(","):
            src = os.path.join(ROOT, "paper_2309_08864_amd", "csrc", name)
            if not os.path.isfile(src):
                ok = False
                break
            h.update(open(src, "rb").read())
        if not ok or h.hexdigest() != kv.get("kernel_sources_sha256"):
            continue
        for k in ("traffic_bytes_per_launch", "rocprof_avg_launch_us"):
            if k in kv:
                out[k] = float(kv[k])
                out[k + "_source"] = os.path.relpath(path, ROOT)
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2_3d7pt")
    ap.add_argument("--storage", default=None)
    ap.add_argument("--k-on", type=int, default=0)
    ap.add_argument("--tb-depth", type=int, default=0)
    ap.add_argument("--chunks", type=int, default=0)
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--method", default="so2dr", choices=["so2dr", "resreu"],
                    help="resreu: the paper's comparison code (per-step sharing, one-step kernels)")
    ap.add_argument("--rounding", default="every_step", choices=["every_step", "at_store"],
                    help="BF16/F16 storage: round after every step, or only where a launch stores")
    ap.add_argument("--auto", action="store_true",
                    help="let the cost model choose chunks, k_on and slots (the TB depth stays "
                         "the workload's unless --auto-depth)")
    ap.add_argument("--auto-depth", action="store_true", help="with --auto: choose the TB depth too")
    ap.add_argument("--T", type=int, default=0, help="override the workload's number of time steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the BF16/FP16 precision leg of the default workload")
    ap.add_argument("--no-link-probe", action="store_true")
    ap.add_argument("--host-alloc", default="so2dr", choices=["so2dr", "torch"],
                    help="allocator of the pinned host fields")
    ap.add_argument("--copy-engine", default="auto", choices=["auto", "dma", "kernel", "kernel_out"],
                    help="what moves chunks between host and HBM")
    ap.add_argument("--cpu-sample-planes", type=int, default=32)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run plain device copies of 1 GiB (known bytes) so that "
                         "hardware byte counters can be scaled")
    ap.add_argument("--kernel-rates", action="store_true",
                    help="instead of a run: time one launch per fused depth and storage type of "
                         "the workload's stencil on an interior chunk (so2dr_kernel_bench) and "
                         "print one JSON line per kernel")
    ap.add_argument("--grid", default=None,
                    help="with --kernel-rates: override the workload's extents, NXxNY or NXxNYxNZ")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of one run: the workload under every chunk count x TB depth "
                         "of --sweep-chunks / --sweep-depths, one JSON line each")
    ap.add_argument("--link-sweep", action="store_true",
                    help="print one JSON line per copy pattern of the host-link probe (bytes per "
                         "direction x copies queued) and exit")
    ap.add_argument("--sweep-chunks", default="4,8")
    ap.add_argument("--sweep-depths", default="40,80,160,320,640")
    return ap.parse_args()


def weights_for(wl, offs):
    import workloads
    tag = wl.weights.split(":")
    if tag[0] == "const":
        return workloads.const_weights(offs, float(tag[1]))
    if tag[0] == "centre_arm":
        return workloads.centre_arm_weights(offs, float(tag[1]), [float(x) for x in tag[2:]])
    if tag[0] == "random_box":
        return workloads.random_box_weights(offs, wl.seed)
    raise ValueError(wl.weights)


HOST_ALLOC = "so2dr"


def host_empty(shape, dtype):
    """Page-locked host tensor: from the library's allocator (the HIP
    runtime's own, one mapped allocation per field) or, with --host-alloc
    torch, PyTorch's pinned allocator."""
    import torch
    if HOST_ALLOC == "torch":
        return torch.empty(shape, dtype=dtype, pin_memory=True)
    from paper_2309_08864_amd import pinned_empty
    return pinned_empty(shape, dtype)


def draw_into(wl, arr):
    """Fill numpy array `arr` with the workload's initial field (block by
    block from the recipe's seed)."""
    import workloads
    gen = {"uniform": workloads.uniform_into, "fourier": workloads.fourier_modes_into,
           "bump": workloads.gaussian_bump_into}[wl.init]
    gen(arr, wl.seed)
    return arr


def field_shape(wl):
    return (wl.ny, wl.nx) if wl.ndim == 2 else (wl.nz, wl.ny, wl.nx)


def draw_field(wl, dtype):
    """The workload's initial field as a pinned host tensor of `dtype`
    (float32 or float64)."""
    h = host_empty(field_shape(wl), dtype)
    draw_into(wl, h.numpy())
    return h


def fill_rounded(dst, src):
    """dst (pinned tensor) <- src (tensor) rounded to dst's type, block by block."""
    for z0 in range(0, src.shape[0], 64):
        dst[z0:z0 + 64].copy_(src[z0:z0 + 64])


def plan_for(wl, w, storage, args, K, d, k_on=0, slots=0, rounding="every_step"):
    from paper_2309_08864_amd import Plan
    return Plan(ndim=wl.ndim, nx=wl.nx, ny=wl.ny, nz=wl.nz, shape=wl.shape, radius=wl.radius,
                weights=list(w), T=wl.T, tb_depth=K, n_chunks=d, k_on=k_on, n_slots=slots,
                budget=wl.budget, storage=storage, bc=wl.periodic, method=args.method,
                rounding=rounding, copy_engine=args.copy_engine)


# ---------------------------------------------------------------- host link
def link_probe(nbytes=4 << 30, pieces=8, reps=3):
    """Pinned host <-> HBM copies as the executor issues them
    (so2dr_link_probe: hipMemcpyAsync on the library's copy-in and copy-out
    streams, `pieces` copies per direction queued back to back, as a round
    of chunks is): host -> HBM alone, HBM -> host alone, both directions at
    once.  GB/s = bytes moved / wall time, best of `reps`."""
    import ctypes
    import torch
    from paper_2309_08864_amd import _lib, pinned_empty
    from paper_2309_08864_amd.plan import _plan_streams
    n = nbytes // 4
    h_a = pinned_empty((n,), torch.float32).fill_(1.0)
    h_b = pinned_empty((n,), torch.float32)
    d_a = torch.empty(n, dtype=torch.float32, device="cuda")
    d_b = torch.ones(n, dtype=torch.float32, device="cuda")
    s_in, s_out = _plan_streams("cuda", 2)
    g = (ctypes.c_double * 3)()
    _lib.check(_lib.lib().so2dr_link_probe(
        ctypes.c_void_p(h_a.data_ptr()), ctypes.c_void_p(h_b.data_ptr()),
        ctypes.c_void_p(d_a.data_ptr()), ctypes.c_void_p(d_b.data_ptr()), nbytes, pieces,
        ctypes.c_void_p(s_in.cuda_stream), ctypes.c_void_p(s_out.cuda_stream), reps, g))
    del h_a, h_b, d_a, d_b
    return {"h2d_GBps": round(g[0], 2), "d2h_GBps": round(g[1], 2), "duplex_GBps": round(g[2], 2),
            "method": f"so2dr_link_probe: {pieces} hipMemcpyAsync copies of {(nbytes // pieces) >> 20} "
                      f"MiB per direction on the copy-in and copy-out streams, best of {reps}"}


# ---------------------------------------------------------------- CPU oracle
def _cpu_host():
    """CPU model, logical CPUs and NUMA layout of this host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    nodes = []
    for d in sorted(glob.glob("/sys/devices/system/node/node[0-9]*")):
        try:
            nodes.append(f"{os.path.basename(d)}: cpus {open(os.path.join(d, 'cpulist')).read().strip()}")
        except OSError:
            pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "numa": nodes or ["unknown"]}


_CPU_CHILD = r"""
import sys, time, json
sys.path.insert(0, sys.argv[1])
import oracle, workloads
ndim, nx, ny, planes, T, seed = map(int, sys.argv[2:8])
shape, r = sys.argv[8], int(sys.argv[9])
w = json.loads(sys.argv[10]); per = tuple(json.loads(sys.argv[11]))
u = workloads.uniform((planes, ny, nx) if ndim == 3 else (planes, nx), seed=seed)
offs = oracle.stencil_offsets(ndim, shape, r)
t0 = time.perf_counter(); oracle.sweep(u, offs, w, T, per); print(time.perf_counter() - t0)
"""


def cpu_baseline(wl, offs, w, planes):
    """The FP64 oracle (plain C loops, OpenMP over planes) on a bounded
    sample: the full xy plane of the workload, `planes` planes deep, all T
    steps.  Median of three runs on all host threads, plus one run with one
    thread on a slab an eighth as deep (a child process with
    OMP_NUM_THREADS=1).  Reported in GCell-updates/s."""
    import oracle
    import workloads
    oracle.build()
    plane = wl.ny * wl.nx if wl.ndim == 3 else wl.nx
    shp = (planes, wl.ny, wl.nx) if wl.ndim == 3 else (planes, wl.nx)
    u = workloads.uniform(shp, seed=wl.seed)
    per = tuple(wl.periodic)
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.sweep(u, offs, w, wl.T, per)
        times.append(time.perf_counter() - t0)
    dt = statistics.median(times)
    cells = planes * plane
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    res = {"value": cells * wl.T / dt / 1e9, "unit": "GCell-updates/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{planes} planes ({'x'.join(map(str, shp[::-1]))} cells) of the same stencil, "
                     f"weights and T={wl.T} "
                     f"(FP64; median of 3 runs: {', '.join(f'{t:.1f}' for t in times)} s)"}
    p1 = max(1, planes // 8)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", _CPU_CHILD, ROOT, str(wl.ndim), str(wl.nx),
                            str(wl.ny), str(p1),
                            str(wl.T), str(wl.seed), wl.shape, str(wl.radius),
                            json.dumps([float(x) for x in w]), json.dumps(list(per))],
                           env=env, capture_output=True, text=True, timeout=300, check=True)
        t1 = float(r.stdout.strip().splitlines()[-1])
        res["single_thread"] = {"value": p1 * plane * wl.T / t1 / 1e9, "cores": 1,
                                "sample": f"{p1} planes, {t1:.1f} s"}
    except Exception as e:   # reported, not fatal
        res["single_thread"] = {"error": str(e)[-200:]}
    res["host"] = _cpu_host()
    return res


# ---------------------------------------------------------------- precision
def _boxes(wl, n_chunks, rng, size=2, extra=3):
    """Sampled output boxes: the grid's corners, across chunk boundaries and
    at random places."""
    nx, ny, nz = wl.nx, wl.ny, wl.nz
    corners = [(0, 0, 0), (nx - size, ny - size, nz - size), (0, ny - size, nz // 2),
               (nx - size, 0, 0)]
    boxes = list(corners)
    for i in range(1, min(n_chunks, 3)):
        z = nz * i // n_chunks - size // 2
        boxes.append((int(rng.integers(0, nx - size)), int(rng.integers(0, ny - size)), z))
    for _ in range(extra):
        boxes.append(tuple(int(rng.integers(0, n - size + 1)) for n in (nx, ny, nz)))
    return [(b, tuple(v + size for v in b)) for b in boxes]


def _errors(got, refs, boxes):
    """Worst per-box relative L2 and the pooled relative L2 over all boxes."""
    worst, num, den = 0.0, 0.0, 0.0
    for (lo, hi), ref in zip(boxes, refs):
        g = got[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].double().numpy()
        d2 = float(np.sum((g - ref) ** 2))
        r2 = float(np.sum(ref ** 2))
        worst = max(worst, (d2 / r2) ** 0.5 if r2 else 0.0)
        num += d2
        den += r2
    return worst, (num / den) ** 0.5 if den else 0.0


def precision_leg(args, name="c4_3d13pt"):
    """The 13-point radius-2 workload (2048^3, T = 64, K = 8, 32 chunks, 8
    GiB) in FP32, BF16, FP16 and BF16 rounded at store.  The FP32 field (the
    FP64 recipe rounded once) is the input; BF16 / FP16 inputs are its
    roundings.  Per storage type: two timed runs after a small warm-up plan
    of the same stencil and storage and one warm-up round of the plan
    itself; GCell-updates/s of the faster run (both listed); e_total = error
    against the
    FP64 oracle run from the FP32 input, e_arith = against the oracle run
    from the storage-rounded input (sampled light-cone boxes: worst box and
    pooled over the boxes)."""
    import torch
    import oracle
    import workloads
    from paper_2309_08864_amd import Plan, stencil_offsets
    wl = workloads.CONFIGS[name]
    offs = stencil_offsets(3, wl.shape, wl.radius)
    w = workloads.fp32_rounded(weights_for(wl, offs))
    t0 = time.perf_counter()
    master = draw_into(wl, np.empty(field_shape(wl), np.float32))
    tm = torch.from_numpy(master)
    print(f"# precision leg: input ready in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    boxes = _boxes(wl, wl.n_chunks, np.random.default_rng(11))
    refs32 = [oracle.sweep_box_from_field(master, offs, w, wl.T, lo, hi) for lo, hi in boxes]
    out = {"workload": f"{name}: 3D star r=2 {wl.nx}x{wl.ny}x{wl.nz}, T={wl.T}, "
                       f"tb_depth={wl.tb_depth}, {wl.n_chunks} chunks, budget "
                       f"{wl.budget / 2**30:g} GiB; input Gaussian bump + U[-1e-3, 1e-3)",
           "error_metric": "relative L2 on sampled light-cone boxes "
                           f"({len(boxes)} boxes of 2^3 cells: 4 corners, chunk boundaries, random)"}
    refs_own = {}
    for storage, rounding in (("f32", "every_step"), ("bf16", "every_step"), ("f16", "every_step"),
                              ("bf16", "at_store")):
        dt = getattr(torch, TORCH_DT[storage])
        warm = Plan(ndim=3, nx=wl.nx, ny=64, nz=64, shape=wl.shape, radius=wl.radius,
                    weights=list(w), T=wl.T, tb_depth=wl.tb_depth, n_chunks=2,
                    budget=1 << 30, storage=storage, rounding=rounding).bind()
        warm.run(host_empty((64, 64, wl.nx), dt).zero_())
        warm.close()
        h = host_empty(field_shape(wl), dt)
        fill_rounded(h, tm)
        if storage not in refs_own:
            refs_own[storage] = refs32 if storage == "f32" else \
                [oracle.sweep_box_from_field(h, offs, w, wl.T, lo, hi) for lo, hi in boxes]
        p = plan_for(wl, w, storage, args, wl.tb_depth, wl.n_chunks, rounding=rounding).bind()
        info = p.info()
        # warm-up: one round of the same plan on the same host field (the
        # first copies of fresh page-locked memory are slow), then the input
        # again
        p.run_steps(h, h, wl.tb_depth)
        runs = []
        for rep in range(2):
            fill_rounded(h, tm)
            t1 = time.perf_counter()
            st = p.run(h)
            runs.append((time.perf_counter() - t1, st))
            if rep == 0:       # the result is the same bits every run
                e_tot_w, e_tot = _errors(h, refs32, boxes)
                e_ar_w, e_ar = _errors(h, refs_own[storage], boxes)
        p.close()
        el, st = min(runs, key=lambda r: r[0])
        key = storage + ("_round_at_store" if rounding == "at_store" else "")
        out[key] = {"GCells": round(wl.cells * wl.T / el / 1e9, 2),
                    "runs_GCells": [round(wl.cells * wl.T / e / 1e9, 2) for e, _ in runs],
                    "wall_ms": round(st["wall_ms"], 1),
                    "link_GBps": round((st["bytes_h2d"] + st["bytes_d2h"]) / el / 1e9, 2),
                    "e_total_pooled": e_tot, "e_total_worst_box": e_tot_w,
                    "e_arith_pooled": e_ar, "e_arith_worst_box": e_ar_w,
                    "k_on": info["k_on"], "n_slots": info["n_slots"],
                    "copy_engine": {1: "dma", 2: "kernel", 3: "kernel_out"}[info["copy_engine"]]}
        print(f"# precision {key}: {out[key]}", file=sys.stderr, flush=True)
        del h
    for key in ("bf16", "f16", "bf16_round_at_store"):
        out[key]["speedup_vs_f32"] = round(out[key]["GCells"] / out["f32"]["GCells"], 3)
    del tm, master
    return out


# ---------------------------------------------------------------- adjoint
def bench_adjoint(args, wl, w):
    """Times the whole gradient (forward with host checkpoints, loss, reverse
    sweep with recompute, weight gradients) of 1/2 ||u_T - y||^2; the target
    y is the same sweep with perturbed weights.  value = nx ny nz T / wall."""
    import torch
    import workloads
    from paper_2309_08864_amd import Plan
    from paper_2309_08864_amd.plan import adjoint_buffers_needed
    c = wl.extra["ckpt_every"]
    shape = (wl.nz, wl.ny, wl.nx)
    base = dict(ndim=wl.ndim, nx=wl.nx, ny=wl.ny, nz=wl.nz, shape=wl.shape, radius=wl.radius,
                T=wl.T, tb_depth=args.tb_depth or wl.tb_depth, n_chunks=args.chunks or wl.n_chunks,
                k_on=args.k_on, n_slots=args.slots, budget=wl.budget, bc=wl.periodic,
                copy_engine=args.copy_engine)
    u0 = draw_field(wl, torch.float32)
    wt = workloads.fp32_rounded(workloads.perturbed(w, wl.extra["target_seed"]))
    y = host_empty(shape, torch.float32)
    pt = Plan(weights=list(wt), **base).bind()
    t0 = time.perf_counter()
    pt.run_steps(u0, y, wl.T)
    t_fwd = time.perf_counter() - t0
    pt.close()
    plan = Plan(weights=list(w), adjoint=True, **base).bind()
    info = plan.info()
    ckpt = [host_empty(shape, torch.float32)
            for _ in range(adjoint_buffers_needed(wl.T, info["tb_depth"], c))]
    g = host_empty(shape, torch.float32)
    print(f"# adjoint plan {info}; {len(ckpt)} host checkpoint fields; forward {t_fwd:.2f} s",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        plan.adjoint(u0, y, c, ckpt=ckpt, grad_u0=g)
        print(f"# warmup {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    link = 0
    t_start = time.perf_counter()
    for i in range(args.steps):
        loss, _, gw, st = plan.adjoint(u0, y, c, ckpt=ckpt, grad_u0=g)
        link += st["bytes_h2d"] + st["bytes_d2h"]
        print(f"# step {i}: {st['wall_ms']:.1f} ms, loss {loss:.6e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    plan.close()
    value = wl.cells * wl.T * args.steps / elapsed / 1e9
    res = {
        "metric": "GCell-updates/s out-of-core (gradient of the sweep)",
        "value": round(value, 3), "unit": "GCell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": f"{wl.name}: gradient of 1/2||u_T - y||^2 through the {wl.ndim}D "
                        f"{wl.shape} r={wl.radius} sweep, {wl.nx}x{wl.ny}x{wl.nz} f32, T={wl.T}, "
                        f"checkpoints every {c} steps, tb_depth={info['tb_depth']}, "
                        f"{info['n_chunks']} chunks, k_on={info['k_on']}, "
                        f"budget {wl.budget / 2**30:g} GiB",
            "cells": wl.cells, "T": wl.T, "workspace_bytes": info["workspace_bytes"],
            "host_checkpoint_fields": len(ckpt), "host_alloc": args.host_alloc,
            "copy_engine": {1: "dma", 2: "kernel", 3: "kernel_out"}[info["copy_engine"]]},
        "forward_GCells": round(wl.cells * wl.T / t_fwd / 1e9, 3),
        "gradient_over_forward_time": round(elapsed / args.steps / t_fwd, 3),
        "link": {"achieved_GBps": round(link / elapsed / 1e9, 2), "peak_GBps": LINK_PEAK_GBPS},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


# ---------------------------------------------------------------- kernel rates
def kernel_rates(args, wl, offs, w):
    """One JSON line per (storage type, fused depth) of the workload's
    stencil: mean launch time over an interior chunk of 64 output planes plus
    its halo, algorithmic GB/s and output cell-updates/s; and the library's
    device copy kernel over the same planes."""
    import workloads
    from paper_2309_08864_amd import So2drError
    from paper_2309_08864_amd import Plan
    storages = [args.storage] if args.storage else ["f32", "bf16", "f16", "f64"]
    for storage in storages:
        ww = w if storage == "f64" else workloads.fp32_rounded(w)
        try:
            p = Plan(ndim=wl.ndim, nx=wl.nx, ny=wl.ny, nz=wl.nz, shape=wl.shape, radius=wl.radius,
                     weights=list(ww), T=wl.T, tb_depth=wl.T, n_chunks=1, budget=1 << 40,
                     storage=storage, bc=wl.periodic)
        except So2drError as e:
            print(json.dumps({"storage": storage, "error": str(e)}), flush=True)
            continue
        info = p.info()
        esz = {"f32": 4, "f64": 8, "bf16": 2, "f16": 2}[storage]
        pb = info["plane_elems"] * esz
        for L in range(0, info["max_k_on"] + 1):
            own = 64 if wl.ndim == 3 else 1200
            in_planes = own + 2 * L * wl.radius
            ms = p.kernel_ms(L, in_planes, reps=20)
            out_planes = own if L else in_planes
            alg = (in_planes + out_planes) * pb
            line = {"workload": wl.name, "grid": f"{wl.nx}x{wl.ny}x{wl.nz}", "storage": storage,
                    "levels": L,
                    "kernel": "device copy" if L == 0 else "fused stencil",
                    "in_planes": in_planes, "plane_bytes": pb, "ms": round(ms, 4),
                    "alg_GBps": round(alg / ms / 1e6, 1),
                    "hbm_frac": round(alg / ms / 1e6 / HBM_PEAK_GBPS, 4)}
            if L:
                upd = sum(own + 2 * (L - j) * wl.radius for j in range(1, L + 1)) * info["plane_elems"]
                line["G_updates_per_s"] = round(upd / ms / 1e6, 1)
                line["G_output_updates_per_s"] = round(own * info["plane_elems"] * L / ms / 1e6, 1)
            print(json.dumps(line), flush=True)
        p.close()


# ---------------------------------------------------------------- main
def timed_runs(plan, h, steps, warmup, tag=""):
    import torch
    for i in range(warmup):
        st = plan.run(h)
        print(f"# {tag}warmup {i}: {st['wall_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tot = None
    t_start = time.perf_counter()
    for i in range(steps):
        st = plan.run(h)
        if tot is None:
            tot = {k: (list(v) if isinstance(v, list) else v) for k, v in st.items()}
        else:
            for k, v in st.items():
                if isinstance(v, list):
                    tot[k] = [a + b for a, b in zip(tot[k], v)]
                else:
                    tot[k] += v
        print(f"# {tag}step {i}: {st['wall_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return tot, time.perf_counter() - t_start


def roofline_block(tot, config_key):
    """The dominant kernel: the fused depth with the most kernel time."""
    by_ms = tot["kernel_ms_by_levels"]
    L = max(range(8), key=lambda i: by_ms[i]) + 1
    n = tot["launches_by_levels"][L - 1]
    alg = tot["alg_bytes_by_levels"][L - 1] / max(1, n)
    avg_ms = by_ms[L - 1] / max(1, n)
    achieved = alg / (avg_ms / 1e3) / 1e9 if avg_ms else 0.0
    prof = committed_profile(config_key)
    traffic = prof.get("traffic_bytes_per_launch")
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBPS, 4),
           "traffic": round(traffic) if traffic else None,
           "kernel": f"fused {L}-level launches (march3d_kernel for 3D grids, march2d_kernel for 2D)",
           "levels": L, "launches": n, "avg_launch_ms": round(avg_ms, 4),
           "alg_bytes_per_launch": int(alg), "timing": "HIP events on the compute stream",
           "all_launches": {"launches": tot["kernel_launches"],
                            "alg_GBps": round(tot["kernel_alg_bytes"] / (tot["kernel_ms"] / 1e3) / 1e9, 1)
                            if tot["kernel_ms"] else None}}
    if traffic and avg_ms:
        out["traffic_GBps"] = round(traffic / (avg_ms / 1e3) / 1e9, 1)
        out["traffic_source"] = prof["traffic_bytes_per_launch_source"]
    rp = prof.get("rocprof_avg_launch_us")
    if rp:
        out["rocprof_avg_launch_ms"] = round(rp / 1e3, 4)
        out["frac_rocprof"] = round(alg / (rp / 1e6) / 1e9 / HBM_PEAK_GBPS, 4)
        out["event_over_rocprof"] = round(avg_ms / (rp / 1e3), 3)
        out["rocprof_source"] = prof["rocprof_avg_launch_us_source"]
    return out


def sweep(args, wl, w, storage):
    """The workload under each (chunks, TB depth) pair: one warm-up and
    --steps timed runs each, one JSON line per pair (the paper's run-time
    configuration sweep, Sec. V-B)."""
    import torch
    tdt = getattr(torch, TORCH_DT[storage])
    h = draw_field(wl, tdt if storage in ("f32", "f64") else torch.float32)
    for d in [int(x) for x in args.sweep_chunks.split(",")]:
        for K in [int(x) for x in args.sweep_depths.split(",")]:
            try:
                p = plan_for(wl, w, storage, args, K, d, k_on=args.k_on, slots=args.slots).bind()
            except Exception as e:
                print(json.dumps({"workload": wl.name, "chunks": d, "tb_depth": K,
                                  "error": str(e)}), flush=True)
                continue
            info = p.info()
            tot, el = timed_runs(p, h, args.steps, 1, tag=f"d={d} K={K} ")
            p.close()
            value = wl.cells * wl.T * args.steps / el / 1e9
            halo = 2 * wl.radius * info["tb_depth"] / info["max_chunk_planes"]
            print(json.dumps({"workload": wl.name, "chunks": d, "tb_depth": info["tb_depth"],
                              "k_on": info["k_on"], "n_slots": info["n_slots"],
                              "halo_over_chunk": round(halo, 4), "GCells": round(value, 2),
                              "ms_per_run": round(el / args.steps * 1e3, 1),
                              "kernel_ms_per_run": round(tot["kernel_ms"] / args.steps, 1),
                              "redundant_fraction": round(info["redundant_fraction"], 4)}),
                  flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the out-of-core path "
              "shards along the cut axis across GPUs by design but is measured per GPU.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads
    from paper_2309_08864_amd import stencil_offsets
    global HOST_ALLOC
    HOST_ALLOC = args.host_alloc

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = workloads.CONFIGS[args.workload]
    if args.T:
        import dataclasses
        wl = dataclasses.replace(wl, T=args.T)
    if args.grid:
        import dataclasses
        ext = [int(x) for x in args.grid.lower().split("x")]
        wl = dataclasses.replace(wl, nx=ext[0], ny=ext[1], nz=ext[2] if len(ext) > 2 else 1)
    storage = args.storage or wl.dtypes[0]
    offs = stencil_offsets(wl.ndim, wl.shape, wl.radius)
    w = weights_for(wl, offs)
    if args.kernel_rates:
        return kernel_rates(args, wl, offs, w)
    if args.link_sweep:
        for nbytes, pieces in ((1 << 30, 1), (1 << 30, 2), (4 << 30, 8), (4 << 30, 16), (4 << 30, 32),
                               (8 << 30, 16)):
            line = {"MiB_per_direction": nbytes >> 20, "copies": pieces}
            line.update(link_probe(nbytes, pieces))
            print(json.dumps(line), flush=True)
        return
    if storage != "f64":
        w = workloads.fp32_rounded(w)
    if wl.extra.get("ckpt_every"):
        return bench_adjoint(args, wl, w)
    if args.sweep:
        return sweep(args, wl, w, storage)
    K = args.tb_depth or wl.tb_depth
    d = args.chunks or wl.n_chunks
    if args.auto:
        from paper_2309_08864_amd import suggest
        kw, _ = suggest(ndim=wl.ndim, nx=wl.nx, ny=wl.ny, nz=wl.nz, shape=wl.shape,
                        radius=wl.radius, weights=list(w), T=wl.T,
                        tb_depth=0 if args.auto_depth else K, n_chunks=args.chunks,
                        k_on=args.k_on, n_slots=args.slots, budget=wl.budget, storage=storage,
                        bc=wl.periodic, method=args.method, rounding=args.rounding,
                        copy_engine=args.copy_engine)
        K, d, args.k_on, args.slots = kw["tb_depth"], kw["n_chunks"], kw["k_on"], kw["n_slots"]
    plan = plan_for(wl, w, storage, args, K, d, k_on=args.k_on, slots=args.slots,
                    rounding=args.rounding)
    info = plan.info()
    predicted_ms = plan.predict()
    plan.bind()
    plan.set_timing(True)
    tdt = getattr(torch, TORCH_DT[storage])
    t0 = time.perf_counter()
    if tdt in (torch.float32, torch.float64):
        h = draw_field(wl, tdt)
    else:   # reduced storage: the FP32 field rounded once to the storage type
        master = draw_field(wl, torch.float32)
        h = host_empty(master.shape, tdt)
        fill_rounded(h, master)
        del master
    print(f"# input ready in {time.perf_counter() - t0:.1f} s; plan {info}", file=sys.stderr,
          flush=True)
    tot, elapsed = timed_runs(plan, h, args.steps, args.warmup)
    plan.close()
    del h

    cells = wl.cells
    value = cells * wl.T * args.steps / elapsed / 1e9
    link_bytes = tot["bytes_h2d"] + tot["bytes_d2h"]
    config_key = (f"{wl.name}/{storage}/K{info['tb_depth']}/d{info['n_chunks']}/"
                  f"k_on{info['k_on']}/{args.method}")
    bpe = {"f32": 4, "f64": 8, "bf16": 2, "f16": 2}[storage]
    res = {
        "metric": "GCell-updates/s out-of-core",
        "value": round(value, 3),
        "unit": "GCell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": storage,
        "data": "synthetic",
        "config": {
            "workload": f"{wl.name}: {wl.ndim}D {wl.shape} r={wl.radius} "
                        f"{wl.nx}x{wl.ny}x{wl.nz} {storage}, T={wl.T}, tb_depth={info['tb_depth']}, "
                        f"{info['n_chunks']} chunks, {info['n_slots']} slots, k_on={info['k_on']}, "
                        f"budget {wl.budget / 2**30:g} GiB, method {args.method}",
            "cells": cells, "T": wl.T, "tb_depth": info["tb_depth"], "n_chunks": info["n_chunks"],
            "k_on": info["k_on"], "n_slots": info["n_slots"], "budget_bytes": wl.budget,
            "workspace_bytes": info["workspace_bytes"],
            "redundant_fraction": round(info["redundant_fraction"], 4),
            "method": args.method, "lean": info["lean"], "rounding": args.rounding,
            "planned_by": "cost model" if args.auto else "given",
            "host_alloc": args.host_alloc,
            "copy_engine": {1: "dma", 2: "kernel", 3: "kernel_out"}[info["copy_engine"]],
        },
        "roofline": roofline_block(tot, config_key),
        "link": {
            "achieved_GBps": round(link_bytes / elapsed / 1e9, 2),
            "peak_GBps": LINK_PEAK_GBPS,
            "link_bound_GCells": round(LINK_PEAK_GBPS / (2 * bpe) * info["tb_depth"], 1),
            "frac_of_peak": round(link_bytes / elapsed / 1e9 / LINK_PEAK_GBPS, 4),
            "h2d_GBps_while_busy": round(tot["bytes_h2d"] / (tot["h2d_ms"] / 1e3) / 1e9, 2)
            if tot["h2d_ms"] else None,
            "d2h_GBps_while_busy": round(tot["bytes_d2h"] / (tot["d2h_ms"] / 1e3) / 1e9, 2)
            if tot["d2h_ms"] else None,
        },
        "model": {"predicted_ms_per_step": round(predicted_ms, 2)},
        "cpu_baseline": None,
    }
    if not args.no_link_probe:
        probe = link_probe()
        res["link"]["measured"] = probe
        res["link"]["link_bound_GCells_measured"] = round(
            probe["duplex_GBps"] / (2 * bpe) * info["tb_depth"], 1)
        res["link"]["frac_of_measured_duplex"] = round(
            link_bytes / elapsed / 1e9 / probe["duplex_GBps"], 4)
    default_run = (args.workload == "c2_3d7pt" and not args.storage and not args.auto
                   and not args.T and args.method == "so2dr")
    if default_run and not args.no_precision:
        res["precision"] = precision_leg(args)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl, offs, w, args.cpu_sample_planes)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
