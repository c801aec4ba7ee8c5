"""Benchmark: out-of-core 3D 7-point Jacobi sweep on one MI355X.

Workload (default): 2048 x 1024 x 1024 FP32 grid (8 GiB per field) in pinned
host memory, zero Dirichlet boundary, weights 0.4 centre / 0.1 neighbours,
U[0,1) input from seed 2, T = 64 steps, 8 steps per HBM residency, 16 chunks
along z, device budget capped at 4 GiB.  One "step" of this benchmark is one
whole out-of-core run of T time steps over the grid (host -> HBM -> host).

Prints one JSON line with the whole-job GCell-updates/s, the dominant
kernel's HBM roofline position (HIP-event kernel time on the kernel's own
stream) and the FP64 CPU oracle timed on a bounded sample of the same sweep.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, vendor figure
LINK_PEAK_GBPS = 2 * 63.0       # PCIe 5.0 x16, both directions, vendor figure


def measured_traffic(config_key):
    """HBM bytes per launch of the fused kernel, from a committed hardware
    counter summary under profiles/ (FETCH_SIZE and WRITE_SIZE scaled by a
    copy of known size), or None when no summary covers this configuration
    or the kernel sources changed after the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        kv = {}
        for line in open(path):
            line = line.strip()
            if "=" in line and " " not in line:
                k, v = line.split("=", 1)
                kv[k] = v
        if kv.get("config_key") != config_key:
            continue
        h = hashlib.sha256()
        for name in kv.get("kernel_sources", "").split(","):
            src = os.path.join(ROOT, "paper_2309_08864_amd", "csrc", name)
            if not os.path.isfile(src):
                return None
            h.update(open(src, "rb").read())
        if h.hexdigest() != kv.get("kernel_sources_sha256"):
            return None
        return float(kv["traffic_bytes_per_launch"])
    return None


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
    ap.add_argument("--host-alloc", default="so2dr", choices=["so2dr", "torch"],
                    help="allocator of the pinned host fields")
    ap.add_argument("--copy-engine", default="auto", choices=["auto", "dma", "kernel", "kernel_out"],
                    help="what moves chunks between host and HBM")
    ap.add_argument("--cpu-sample-planes", type=int, default=0)
    ap.add_argument("--compare-storage", default=None,
                    help="also run this storage type on the same input and report the "
                         "relative L2 deviation of the main run from it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run plain device copies of 1 GiB (known bytes) so that "
                         "hardware byte counters can be scaled")
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


def draw_field(wl, dtype):
    """The workload's initial field as a pinned host tensor of `dtype`
    (float32 or float64), drawn block by block from the recipe's seed."""
    import torch
    import workloads
    gen = {"uniform": workloads.uniform_into, "fourier": workloads.fourier_modes_into,
           "bump": workloads.gaussian_bump_into}[wl.init]
    shape = (wl.ny, wl.nx) if wl.ndim == 2 else (wl.nz, wl.ny, wl.nx)
    h = host_empty(shape, dtype)
    gen(h.numpy(), wl.seed)
    return h


def rounded_copy(src, dtype):
    """Pinned copy of src rounded (nearest even) to dtype, plane block by block."""
    import torch
    h = host_empty(src.shape, dtype)
    for z0 in range(0, src.shape[0], 64):
        h[z0:z0 + 64].copy_(src[z0:z0 + 64])
    return h


def cpu_baseline(wl, offs, w, planes):
    """The FP64 oracle (plain C loops, OpenMP over planes) on a bounded
    sample: the full xy plane of the workload, `planes` planes deep, all T
    steps.  Reported in GCell-updates/s."""
    import oracle
    import workloads
    oracle.build()
    rng_u = workloads.uniform((planes, wl.ny, wl.nx), seed=wl.seed)
    per = tuple(wl.periodic)
    t0 = time.perf_counter()
    oracle.sweep(rng_u, offs, w, wl.T, per)
    dt = time.perf_counter() - t0
    cells = planes * wl.ny * wl.nx
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": cells * wl.T / dt / 1e9, "unit": "GCell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{wl.nx}x{wl.ny}x{planes} slab of the same stencil, weights and T={wl.T} "
                      f"(FP64, {dt:.1f} s)"}


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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the out-of-core path "
              "shards along the cut axis across GPUs by design but is measured per GPU.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads
    from paper_2309_08864_amd import Plan, stencil_offsets
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
    storage = args.storage or wl.dtypes[0]
    offs = stencil_offsets(wl.ndim, wl.shape, wl.radius)
    w = weights_for(wl, offs)
    if storage != "f64":
        w = workloads.fp32_rounded(w)
    if wl.extra.get("ckpt_every"):
        return bench_adjoint(args, wl, w)
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
    plan = Plan(ndim=wl.ndim, nx=wl.nx, ny=wl.ny, nz=wl.nz, shape=wl.shape, radius=wl.radius,
                weights=list(w), T=wl.T, tb_depth=K, n_chunks=d, k_on=args.k_on,
                n_slots=args.slots, budget=wl.budget, storage=storage, bc=wl.periodic,
                method=args.method, rounding=args.rounding, copy_engine=args.copy_engine)
    info = plan.info()
    predicted_ms = plan.predict()
    plan.bind()
    plan.set_timing(True)
    tdt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16,
           "f16": torch.float16}[storage]
    shape = (wl.ny, wl.nx) if wl.ndim == 2 else (wl.nz, wl.ny, wl.nx)
    t0 = time.perf_counter()
    if tdt in (torch.float32, torch.float64):
        master = draw_field(wl, tdt)
    else:   # reduced storage: the FP32 field rounded once to the storage type
        master = draw_field(wl, torch.float32)
    h = rounded_copy(master, tdt) if args.compare_storage or master.dtype != tdt else master
    print(f"# input ready in {time.perf_counter() - t0:.1f} s; plan {info}", file=sys.stderr,
          flush=True)

    for i in range(args.warmup):
        st = plan.run(h)
        print(f"# warmup {i}: {st['wall_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tot = {"kernel_ms": 0.0, "kernel_alg_bytes": 0, "kernel_launches": 0, "bytes_h2d": 0,
           "bytes_d2h": 0, "h2d_ms": 0.0, "d2h_ms": 0.0, "cell_updates": 0, "cell_updates_done": 0}
    t_start = time.perf_counter()
    for i in range(args.steps):
        st = plan.run(h)
        for k in tot:
            tot[k] += st[k]
        print(f"# step {i}: {st['wall_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    cells = wl.cells
    value = cells * wl.T * args.steps / elapsed / 1e9
    achieved = tot["kernel_alg_bytes"] / (tot["kernel_ms"] / 1e3) / 1e9 if tot["kernel_ms"] else 0.0
    link_bytes = tot["bytes_h2d"] + tot["bytes_d2h"]
    traffic = measured_traffic(f"{wl.name}/{storage}/K{info['tb_depth']}/d{info['n_chunks']}/"
                               f"k_on{info['k_on']}/{args.method}")
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
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": round(traffic) if traffic else None,
            "kernel": "fused-step stencil kernel (march3d_kernel for 3D grids, march2d_kernel for 2D)",
            "launches": tot["kernel_launches"],
            "avg_launch_ms": round(tot["kernel_ms"] / max(1, tot["kernel_launches"]), 4),
            "alg_bytes_per_launch": tot["kernel_alg_bytes"] // max(1, tot["kernel_launches"]),
        },
        "link": {
            "achieved_GBps": round(link_bytes / elapsed / 1e9, 2),
            "peak_GBps": LINK_PEAK_GBPS,
            "h2d_GBps_while_busy": round(tot["bytes_h2d"] / (tot["h2d_ms"] / 1e3) / 1e9, 2)
            if tot["h2d_ms"] else None,
            "d2h_GBps_while_busy": round(tot["bytes_d2h"] / (tot["d2h_ms"] / 1e3) / 1e9, 2)
            if tot["d2h_ms"] else None,
            "link_bound_GCells": round(LINK_PEAK_GBPS * 1e9 / (2 * h.element_size()) * info["tb_depth"] / 1e9, 1),
        },
        "model": {"predicted_ms_per_step": round(predicted_ms, 2)},
        "cpu_baseline": None,
    }
    plan.close()
    if args.compare_storage:
        # the timed runs advanced h by many sweeps: round the input into h
        # again and run one sweep in the bench's storage type, then one in the
        # reference type (in place on the master field when the types agree,
        # so that only two host fields are pinned)
        cdt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16,
               "f16": torch.float16}[args.compare_storage]
        for z0 in range(0, shape[0], 64):
            h[z0:z0 + 64].copy_(master[z0:z0 + 64])
        plan2 = Plan(ndim=wl.ndim, nx=wl.nx, ny=wl.ny, nz=wl.nz, shape=wl.shape, radius=wl.radius,
                     weights=list(w), T=wl.T, tb_depth=K, n_chunks=d, k_on=args.k_on,
                     n_slots=args.slots, budget=wl.budget, storage=storage, bc=wl.periodic,
                     rounding=args.rounding, copy_engine=args.copy_engine).bind()
        plan2.run(h)
        plan2.close()
        hm = h
        wr = weights_for(wl, offs)
        if args.compare_storage != "f64":
            wr = workloads.fp32_rounded(wr)
        ref_plan = Plan(ndim=wl.ndim, nx=wl.nx, ny=wl.ny, nz=wl.nz, shape=wl.shape,
                        radius=wl.radius, weights=list(wr), T=wl.T, tb_depth=K, n_chunks=d,
                        n_slots=args.slots, budget=wl.budget, storage=args.compare_storage,
                        bc=wl.periodic, copy_engine=args.copy_engine).bind()
        hr = master if master.dtype == cdt else rounded_copy(master, cdt)
        t1 = time.perf_counter()
        ref_plan.run(hr)
        t_ref = time.perf_counter() - t1
        ref_plan.close()
        num = den = 0.0
        for z0 in range(0, shape[0], 32):
            a_ = hm[z0:z0 + 32].double()
            b_ = hr[z0:z0 + 32].double()
            num += float(((a_ - b_) ** 2).sum())
            den += float((b_ ** 2).sum())
        res["precision"] = {
            "reference_storage": args.compare_storage,
            "rel_l2_vs_reference": (num / den) ** 0.5 if den else None,
            "reference_GCells": round(wl.cells * wl.T / t_ref / 1e9, 3),   # one run, no warm-up
            "speedup_vs_reference": round(value / (wl.cells * wl.T / t_ref / 1e9), 3),
        }
        del hr, hm
    del h, master
    if not args.no_cpu_baseline:
        planes = args.cpu_sample_planes or 64
        res["cpu_baseline"] = cpu_baseline(wl, offs, w, planes)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
