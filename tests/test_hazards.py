"""Race check of the executor's stream schedule (host-only).

so2dr_plan_get_deps returns, from the code the executor itself runs, the
stream every operation is enqueued on and the earlier operations whose
completion it waits for.  Happens-before is then: list order on one stream,
plus the waits, transitively (vector clocks over the streams).  Every
operation reads and writes known plane ranges: its slot buffer, the
region-sharing buffer, or the host array (in place, as so2dr_run uses it).
Two accesses to one plane where at least one writes, by operations that are
not ordered by happens-before, can run in either order on the GPU: a race.
Replaying the list order (a legal serialisation) and checking every access
against the last write and the reads since then covers every interleaving
the streams allow (read-after-write, write-after-read, write-after-write).
Algorithm 1's "read and then write" of the sharing buffer, slot reuse and
the in-place host array across rounds are among the orderings checked.

A second check replays random topological orders of the same graph, some
holding back one stream as long as possible, and asserts every read sees the
value the list order gives it; and deleting any one class of waits, in a plan
where the others do not imply it, must make the check fail (the rules are
needed and the checker sees it)."""
import random

import numpy as np
import pytest

from paper_2309_08864_amd import Plan

MiB = 1 << 20


def _plan(ndim=3, nx=8, ny=6, nz=48, shape="star", r=1, T=10, K=3, d=4, k_on=0, slots=0,
          budget=1 << 30, method="so2dr", storage="f32"):
    from paper_2309_08864_amd import stencil_offsets
    w = [0.1] * len(stencil_offsets(ndim, shape, r))
    if ndim == 2:   # a 2D grid is cut along y: its rows are the planes
        ny, nz = nz, 1
    return Plan(ndim=ndim, nx=nx, ny=ny, nz=nz, shape=shape, radius=r,
                weights=w, T=T, tb_depth=K, n_chunks=d, k_on=k_on, n_slots=slots, budget=budget,
                method=method, storage=storage)


def footprint(op, n_axis):
    """(reads, writes) of one operation: lists of (region, lo, hi) plane
    ranges.  Regions: ("buf", slot, buffer) indices inside a slot buffer;
    ("pool",) planes of the region-sharing buffer; ("host",) global planes of
    the in-place host array.  A kernel may load any plane of its input's
    valid area inside the grid."""
    k, z0, z1, b0 = op["kind"], op["z0"], op["z1"], op["buf_z0"]
    if k == "H2D":
        return [(("host",), z0, z1)], [(("buf", op["slot"], op["buf_out"]), z0 - b0, z1 - b0)]
    if k == "RS_READ":
        po = op["pool_off"]
        return ([(("pool",), po, po + z1 - z0)],
                [(("buf", op["slot"], op["buf_out"]), z0 - b0, z1 - b0)])
    if k == "RS_WRITE":
        po = op["pool_off"]
        return ([(("buf", op["slot"], op["buf_in"]), z0 - b0, z1 - b0)],
                [(("pool",), po, po + z1 - z0)])
    if k == "KERNEL":
        lo, hi = max(op["in_z0"], 0), min(op["in_z1"], n_axis)
        return ([(("buf", op["slot"], op["buf_in"]), lo - b0, hi - b0)],
                [(("buf", op["slot"], op["buf_out"]), z0 - op["out_z0"], z1 - op["out_z0"])])
    if k == "D2H":
        return [(("buf", op["slot"], op["buf_in"]), z0 - b0, z1 - b0)], [(("host",), z0, z1)]
    raise ValueError(k)


def vector_clocks(stream, waits, ns):
    """pos[k]: index of op k on its stream; vc[k][s]: highest position on
    stream s that happens before (or is) op k."""
    n = len(stream)
    pos = [0] * n
    cnt = [0] * ns
    last = [None] * ns
    vc = []
    for k in range(n):
        s = stream[k]
        pos[k] = cnt[s]
        cnt[s] += 1
        c = list(vc[last[s]]) if last[s] is not None else [-1] * ns
        for w in waits[k]:
            assert 0 <= w < k, f"op {k} waits on op {w}, not an earlier one"
            c = [max(a, b) for a, b in zip(c, vc[w])]
        c[s] = pos[k]
        vc.append(c)
        last[s] = k
    return pos, vc


def find_races(ops, stream, waits, ns, n_axis, limit=5):
    """Unordered conflicting accesses, as (op a, op b, region, plane, kind)."""
    pos, vc = vector_clocks(stream, waits, ns)

    def hb(a, b):
        return a == b or vc[b][stream[a]] >= pos[a]

    last_w, readers, races = {}, {}, []
    for k, op in enumerate(ops):
        reads, writes = footprint(op, n_axis)
        for reg, lo, hi in reads:
            assert lo <= hi
            for p in range(lo, hi):
                w = last_w.get((reg, p))
                if w is not None and not hb(w, k):
                    races.append((w, k, reg, p, "read after write"))
        for reg, lo, hi in writes:
            for p in range(lo, hi):
                key = (reg, p)
                w = last_w.get(key)
                if w is not None and not hb(w, k):
                    races.append((w, k, reg, p, "write after write"))
                for rd in readers.get(key, ()):
                    if not hb(rd, k):
                        races.append((rd, k, reg, p, "write after read"))
        for reg, lo, hi in reads:
            for p in range(lo, hi):
                readers.setdefault((reg, p), []).append(k)
        for reg, lo, hi in writes:
            for p in range(lo, hi):
                last_w[(reg, p)] = k
                readers[(reg, p)] = []
        if len(races) >= limit:
            break
    return races


def replay_values(ops, order, n_axis):
    """Replay `order` (a permutation of the ops) and return, per op, the
    writer each plane it reads holds (a tuple, in footprint order)."""
    cur = {}
    seen = [None] * len(ops)
    for k in order:
        reads, writes = footprint(ops[k], n_axis)
        seen[k] = tuple(cur.get((reg, p)) for reg, lo, hi in reads for p in range(lo, hi))
        for reg, lo, hi in writes:
            for p in range(lo, hi):
                cur[(reg, p)] = k
    return seen


def topo_order(stream, waits, rng, hold=None):
    """A random topological order of the happens-before graph; `hold`: a
    stream whose ops run only when nothing else is ready."""
    n = len(stream)
    succ = [[] for _ in range(n)]
    indeg = [0] * n
    last = {}
    for k in range(n):
        preds = set(waits[k])
        if stream[k] in last:
            preds.add(last[stream[k]])
        last[stream[k]] = k
        for p in preds:
            succ[p].append(k)
            indeg[k] += 1
    ready = [k for k in range(n) if indeg[k] == 0]
    out = []
    while ready:
        pick = [k for k in ready if stream[k] != hold] or ready
        k = pick[rng.randrange(len(pick))]
        ready.remove(k)
        out.append(k)
        for s in succ[k]:
            indeg[s] -= 1
            if indeg[s] == 0:
                ready.append(s)
    assert len(out) == n, "the schedule's waits form a cycle"
    return out


def _check_plan(p, n_streams_list=(1, 2, 3, 4, 5), orders=0):
    info = p.info()
    ops = p.ops()
    assert len(ops) == info["n_ops"]
    for ns in n_streams_list:
        stream, waits = p.deps(ns)
        assert all(0 <= s < ns for s in stream)
        races = find_races(ops, stream, waits, ns, info["n_axis"])
        assert not races, f"{ns} streams: races {races}"
        if orders:
            base = replay_values(ops, range(len(ops)), info["n_axis"])
            rng = random.Random(ns)
            for i in range(orders):
                hold = i % (ns + 1) if i % 2 else None
                order = topo_order(stream, waits, rng, hold=hold)
                assert replay_values(ops, order, info["n_axis"]) == base, (ns, i)


GRID = [
    # ndim, shape, r, T, K, d, k_on, slots
    (3, "star", 1, 10, 3, 4, 2, 0), (3, "star", 1, 10, 3, 4, 2, 1), (3, "star", 1, 10, 3, 4, 2, 2),
    (3, "star", 2, 9, 4, 3, 2, 0), (3, "box", 1, 8, 4, 5, 3, 3), (3, "star", 1, 5, 5, 1, 2, 0),
    (3, "box", 1, 11, 3, 6, 3, 2), (3, "star", 1, 16, 8, 3, 3, 0), (3, "star", 1, 7, 2, 7, 1, 3),
    (2, "star", 1, 16, 4, 4, 4, 0), (2, "box", 2, 7, 3, 3, 2, 1), (2, "box", 4, 6, 2, 3, 1, 2),
]


@pytest.mark.parametrize("ndim,shape,r,T,K,d,k_on,slots", GRID)
@pytest.mark.parametrize("method", ["so2dr", "resreu"])
def test_schedule_race_free(ndim, shape, r, T, K, d, k_on, slots, method):
    p = _plan(ndim=ndim, shape=shape, r=r, T=T, K=K, d=d, k_on=k_on, slots=slots, method=method)
    _check_plan(p, orders=12)
    p.close()


@pytest.mark.parametrize("ndim,shape,r,T,K,d,k_on", [(3, "star", 1, 10, 3, 4, 2),
                                                      (3, "box", 1, 8, 4, 5, 3),
                                                      (2, "box", 2, 7, 3, 3, 2)])
def test_lean_schedule_race_free(ndim, shape, r, T, K, d, k_on):
    """One buffer per slot (kernels in shifted sub-blocks writing below what
    later sub-blocks read), forced by a budget just under two buffers."""
    p0 = _plan(ndim=ndim, shape=shape, r=r, T=T, K=K, d=d, k_on=k_on, slots=1)
    budget = p0.info()["workspace_bytes"] - 1
    p0.close()
    p = _plan(ndim=ndim, shape=shape, r=r, T=T, K=K, d=d, k_on=k_on, slots=1, budget=budget)
    assert p.info()["lean"] == 1
    _check_plan(p, orders=12)
    p.close()


@pytest.mark.parametrize("name,over", [
    ("c2_3d7pt", {}), ("c2_3d7pt", dict(tb_depth=24, n_chunks=16, k_on=3, n_slots=2)),
    ("c3_3d27pt", {}), ("c3_3d27pt", dict(tb_depth=16, n_chunks=29, k_on=2, n_slots=3)),
    ("c4_3d13pt", {}), ("c4_3d13pt", dict(tb_depth=24, n_chunks=19, k_on=2, n_slots=1)),
    ("c1_2d5pt", {})])
def test_workload_plans_race_free(name, over):
    """The workloads' plans at full size, and the cost model's plans, on the
    stream counts the library binds (3) and its neighbours.  Only the cut
    axis matters to the schedule, so the in-plane extents are shrunk."""
    import workloads
    wl = workloads.CONFIGS[name]
    kw = dict(tb_depth=wl.tb_depth, n_chunks=wl.n_chunks, k_on=0, n_slots=0)
    kw.update(over)
    # same chunk geometry and slot count: scale the budget with the plane
    n_axis = wl.nz if wl.ndim == 3 else wl.ny
    real = _plan(ndim=wl.ndim, nx=wl.nx, ny=wl.ny, nz=n_axis, shape=wl.shape, r=wl.radius, T=wl.T,
                 K=kw["tb_depth"], d=kw["n_chunks"], k_on=kw["k_on"], slots=kw["n_slots"],
                 budget=wl.budget)
    ri = real.info()
    real.close()
    small = (8, 4) if wl.ndim == 3 else (8, 1)
    scale = (wl.nx * wl.ny) / (small[0] * small[1]) if wl.ndim == 3 else wl.nx / small[0]
    p = _plan(ndim=wl.ndim, nx=small[0], ny=small[1], nz=n_axis, shape=wl.shape, r=wl.radius, T=wl.T,
              K=ri["tb_depth"], d=ri["n_chunks"], k_on=ri["k_on"], slots=ri["n_slots"],
              budget=int(wl.budget / scale) + (1 << 20))
    pi = p.info()
    for k in ("n_chunks", "tb_depth", "k_on", "n_slots", "lean", "n_ops"):
        assert pi[k] == ri[k], (k, pi[k], ri[k])
    _check_plan(p, n_streams_list=(2, 3, 4))
    p.close()


def _drop(waits, ops, d, n_slots, rule):
    """A copy of waits without one class of dependency."""
    def g(op):
        return op["round"] * d + op["chunk"]

    def cls(a, b):
        if a["kind"].startswith("RS") and b["kind"].startswith("RS") and g(a) != g(b):
            return "rs_chain"
        if a["kind"] == "D2H" and b["kind"] == "H2D":
            return "slot_reuse" if g(a) == g(b) - n_slots else "host_rounds"
        if a["kind"] == "H2D":
            return "copy_in"
        if b["kind"] == "D2H":
            return "copy_out"
        return "other"

    return [[w for w in ws if cls(ops[w], ops[k]) != rule] for k, ws in enumerate(waits)]


@pytest.mark.parametrize("rule,d,slots", [("rs_chain", 6, 2), ("slot_reuse", 6, 2), ("copy_in", 6, 2),
                                           ("copy_out", 6, 2), ("host_rounds", 3, 3)])
def test_every_wait_class_is_needed(rule, d, slots):
    """Without any one class of waits the checker reports a race: the rules
    are all needed, and the checker would notice a missing one.  (With fewer
    slots than chunks, slot reuse and the in-order copy-out stream already
    order the next round's copy-ins after the copy-outs they must follow, so
    the host-array waits are exercised with as many slots as chunks.)"""
    p = _plan(ndim=3, shape="star", r=1, T=12, K=3, d=d, k_on=2, slots=slots)
    info = p.info()
    ops = p.ops()
    ns = 5   # three compute streams: consecutive chunks' sharing copies on different streams
    stream, waits = p.deps(ns)
    assert not find_races(ops, stream, waits, ns, info["n_axis"])
    dropped = _drop(waits, ops, info["n_chunks"], info["n_slots"], rule)
    assert sum(map(len, dropped)) < sum(map(len, waits))
    races = find_races(ops, stream, dropped, ns, info["n_axis"])
    assert races, f"dropping {rule} waits left no race"
    p.close()
