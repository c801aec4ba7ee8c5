"""Python face of the library: build a plan, give it device memory and
streams from PyTorch, run it on pinned host tensors.

PyTorch supplies only the device arena (one uint8 tensor of the plan's
workspace size), the HIP streams and pinned host tensors; the planner,
executor and kernels are the native library's."""
import ctypes

import numpy as np

from . import _lib
from ._lib import COPY_ENGINES, DTYPES, METHODS, OP_KINDS, ROUNDING, SHAPES, check, lib

TORCH_DTYPES = {"f32": "float32", "f64": "float64", "bf16": "bfloat16", "f16": "float16"}


def stencil_offsets(ndim, shape, r):
    """(dz, dy, dx) offsets of a star or box stencil in the lexicographic order
    the weight array uses (2D stencils have dz == 0; their rows are the cut
    axis)."""
    rng = range(-r, r + 1)
    pts = []
    for a in (rng if ndim == 3 else (0,)):
        for b in rng:
            for c in rng:
                if shape == "box" or (a != 0) + (b != 0) + (c != 0) <= 1:
                    pts.append((a, b, c))
    return pts


class Plan:
    """A planned out-of-core sweep.

    Grid extents are (nx, ny, nz) with x contiguous; a 2D grid has nz == 1
    and is cut along y.  ``weights`` follows stencil_offsets' order.
    ``bc`` gives, per axis x, y, z, 0 for zero Dirichlet or 1 for periodic.
    ``rounding`` ("every_step" or "at_store") applies to BF16/F16 storage:
    round after every step, or only where a launch stores to HBM.
    ``copy_engine`` ("auto", "dma" or "kernel") picks what moves the chunks
    between host and HBM: the runtime's DMA engines or copy kernels through
    the host array's device mapping."""

    def __init__(self, *, ndim, nx, ny, nz=1, shape="star", radius=1, weights, T, tb_depth=0,
                 n_chunks=0, k_on=0, n_slots=0, budget, storage="f32", bc=(0, 0, 0),
                 adjoint=False, method="so2dr", rounding="every_step", copy_engine="auto"):
        self.storage = storage
        self.shape3 = (nz, ny, nx)
        self._T = T
        self._nw = len(weights)
        d, self._w = _make_desc(ndim=ndim, nx=nx, ny=ny, nz=nz, shape=shape, radius=radius,
                                weights=weights, T=T, tb_depth=tb_depth, n_chunks=n_chunks,
                                k_on=k_on, n_slots=n_slots, budget=budget, storage=storage,
                                bc=bc, adjoint=adjoint, method=method, rounding=rounding,
                                copy_engine=copy_engine)
        h = ctypes.c_void_p()
        check(lib().so2dr_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._arena = None
        self._streams = None

    # ------------------------------------------------------------ host-only
    def info(self):
        i = _lib.PlanInfo()
        check(lib().so2dr_plan_get_info(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in i._fields_}

    def ops(self):
        n = self.info()["n_ops"]
        arr = (_lib.Op * max(n, 1))()
        check(lib().so2dr_plan_get_ops(self._h, arr, n))
        out = []
        for k in range(n):
            o = arr[k]
            d = {f: getattr(o, f) for f, _ in o._fields_}
            d["kind"] = OP_KINDS[d["kind"]]
            out.append(d)
        return out

    def deps(self, n_streams=3):
        """The executor's schedule on n_streams streams: (stream index per op,
        list of earlier ops each op waits for), as so2dr_plan_get_deps."""
        n = self.info()["n_ops"]
        strm = (ctypes.c_int32 * max(n, 1))()
        w = (ctypes.c_int64 * max(n * _lib.MAX_WAITS, 1))()
        check(lib().so2dr_plan_get_deps(self._h, int(n_streams), strm, w, n))
        waits = [[x for x in w[k * _lib.MAX_WAITS:(k + 1) * _lib.MAX_WAITS] if x >= 0]
                 for k in range(n)]
        return list(strm[:n]), waits

    def machine(self):
        """The built-in machine figures for this plan's stencil and storage."""
        m = _lib.Machine()
        check(lib().so2dr_machine_default(self._h, ctypes.byref(m)))
        return _machine_dict(m)

    def predict(self, steps=0, machine=None):
        """Predicted wall time (ms) of `steps` steps (0 = T) from the cost
        model; `machine` is a dict like machine()'s (None = built-in)."""
        ms = ctypes.c_double()
        mp = ctypes.byref(_machine_struct(machine)) if machine else None
        check(lib().so2dr_plan_predict(self._h, mp, int(steps), ctypes.byref(ms)))
        return ms.value

    # ------------------------------------------------------------ device
    def bind(self, device="cuda", n_streams=None):
        import torch
        ws = self.info()["workspace_bytes"]
        self._arena = torch.empty(max(ws, 256), dtype=torch.uint8, device=device)
        ns = n_streams or 3    # copy-in, copy-out, one compute stream
        self._streams = _plan_streams(device, ns)
        arr = (ctypes.c_void_p * ns)(*[s.cuda_stream for s in self._streams])
        check(lib().so2dr_plan_bind(self._h, ctypes.c_void_p(self._arena.data_ptr()),
                                    self._arena.numel(), arr, ns))
        return self

    def kernel_ms(self, levels, in_planes, reps=20, device="cuda"):
        """Mean time (ms) of one launch of this plan's kernel fusing `levels`
        steps over an interior chunk of `in_planes` planes (levels = 0: the
        library's device copy kernel over those planes), on device buffers
        allocated here (so2dr_kernel_bench)."""
        import torch
        esz = torch.empty((), dtype=getattr(torch, TORCH_DTYPES[self.storage])).element_size()
        n = int(in_planes) * int(self.info()["plane_elems"]) * esz
        src = torch.rand((n + 3) // 4, dtype=torch.float32, device=device)   # timing only
        dst = torch.zeros_like(src)
        s = _plan_streams(device, 3)[2]
        ms = ctypes.c_double()
        check(lib().so2dr_kernel_bench(self._h, int(levels), ctypes.c_void_p(src.data_ptr()),
                                       ctypes.c_void_p(dst.data_ptr()), int(in_planes), int(reps),
                                       ctypes.c_void_p(s.cuda_stream), ctypes.byref(ms)))
        return ms.value

    def set_timing(self, enable=True):
        check(lib().so2dr_plan_set_timing(self._h, 1 if enable else 0))

    def run(self, host_u):
        """In place: host_u (pinned tensor of the storage dtype) u_0 -> u_T."""
        self._check_host(host_u)
        st = _lib.Stats()
        check(lib().so2dr_run(self._h, ctypes.c_void_p(host_u.data_ptr()), ctypes.byref(st)))
        return st.as_dict()

    def run_noalloc(self, host_u, device="cuda", n_streams=3):
        """As run(), in the library's static device workspace
        (so2dr_run_noalloc): no device memory is allocated for the call, and
        the plan need not be bound."""
        self._check_host(host_u)
        streams = _plan_streams(device, n_streams)
        arr = (ctypes.c_void_p * n_streams)(*[s.cuda_stream for s in streams])
        st = _lib.Stats()
        check(lib().so2dr_run_noalloc(self._h, ctypes.c_void_p(host_u.data_ptr()), arr, n_streams,
                                      ctypes.byref(st)))
        return st.as_dict()

    def run_steps(self, host_in, host_out, steps):
        self._check_host(host_in)
        self._check_host(host_out)
        st = _lib.Stats()
        check(lib().so2dr_run_steps(self._h, ctypes.c_void_p(host_in.data_ptr()),
                                    ctypes.c_void_p(host_out.data_ptr()), int(steps),
                                    ctypes.byref(st)))
        return st.as_dict()

    def _check_host(self, t):
        import torch
        if t.dtype != getattr(torch, TORCH_DTYPES[self.storage]):
            raise TypeError(f"host array must be {TORCH_DTYPES[self.storage]}")
        if not t.is_contiguous() or t.numel() != int(np.prod(self.shape3)):
            raise ValueError("host array must be contiguous with nx*ny*nz elements")

    def close(self):
        if getattr(self, "_h", None):
            lib().so2dr_plan_destroy(self._h)
            self._h = None
        self._arena = None
        self._streams = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_STREAMS = {}


def _plan_streams(device, n):
    """The first n of the library's streams on `device`, created once per
    process and shared by every plan.  The runtime spreads streams over a few
    hardware queues; a stream created after others may get a queue that one
    of them already holds, and two of a plan's streams on one queue run one
    after the other (measured on MI355X: a second plan's copy-in and copy-out
    streams on one queue serialised the whole pipeline, 9.6 s instead of
    about 5 s for the gradient workload).  Plans bound in one process
    therefore take turns on the same streams."""
    import torch
    dev = torch.device(device)
    if dev.index is None:
        dev = torch.device(dev.type, torch.cuda.current_device())
    streams = _STREAMS.setdefault(dev, [])
    while len(streams) < n:
        streams.append(torch.cuda.Stream(device=dev))
    return streams[:n]


class _HostBlock:
    """Page-locked bytes from so2dr_host_alloc, released when the last array
    viewing them is collected."""

    def __init__(self, nbytes):
        p = ctypes.c_void_p()
        check(lib().so2dr_host_alloc(nbytes, ctypes.byref(p)))
        self.ptr = p.value
        self.__array_interface__ = {"shape": (nbytes,), "typestr": "|u1",
                                    "data": (self.ptr, False), "version": 3}

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().so2dr_host_free(ctypes.c_void_p(self.ptr))
            self.ptr = None


def pinned_empty(shape, dtype):
    """Uninitialised CPU tensor of `shape` and torch `dtype` in page-locked
    memory from the HIP runtime's own allocator (so2dr_host_alloc): one
    mapped allocation of exactly the tensor's size, released with the last
    tensor that views it."""
    import torch
    shape = tuple(int(n) for n in (shape if isinstance(shape, (tuple, list)) else (shape,)))
    n = int(np.prod(shape)) * torch.empty((), dtype=dtype).element_size()
    if n == 0:
        return torch.empty(shape, dtype=dtype)
    raw = torch.from_numpy(np.asarray(_HostBlock(n)))
    return raw.view(dtype).view(shape)


def _make_desc(*, ndim, nx, ny, nz, shape, radius, weights, T, tb_depth, n_chunks, k_on, n_slots,
               budget, storage, bc, adjoint, method, rounding, copy_engine="auto"):
    w = (ctypes.c_double * len(weights))(*[float(x) for x in weights])
    d = _lib.Desc()
    d.ndim, d.nx, d.ny, d.nz = ndim, nx, ny, nz
    d.shape, d.radius = SHAPES[shape], radius
    d.weights = ctypes.cast(w, ctypes.POINTER(ctypes.c_double))
    d.n_weights = len(weights)
    d.bc = (ctypes.c_int * 3)(*bc)
    d.storage = DTYPES[storage]
    d.T, d.n_chunks, d.tb_depth, d.k_on, d.n_slots = T, n_chunks, tb_depth, k_on, n_slots
    d.device_budget_bytes = int(budget)
    d.adjoint = 1 if adjoint else 0
    d.method = METHODS[method]
    d.rounding = ROUNDING[rounding]
    d.copy_engine = COPY_ENGINES[copy_engine]
    return d, w


def _machine_dict(m):
    out = {k: getattr(m, k) for k, _ in m._fields_ if k != "gupd"}
    out["gupd"] = list(m.gupd)
    return out


def _machine_struct(md):
    m = _lib.Machine()
    for k, v in md.items():
        if k == "gupd":
            m.gupd = (ctypes.c_double * 8)(*(list(v) + [0.0] * (8 - len(v))))
        else:
            setattr(m, k, float(v))
    return m


def suggest(machine=None, **plan_kwargs):
    """Fill the plan parameters left 0 or unset (tb_depth, n_chunks, k_on,
    n_slots) with the combination of least predicted time that fits the
    budget.  Returns (plan keyword arguments, predicted ms)."""
    kw = dict(nz=1, shape="star", radius=1, tb_depth=0, n_chunks=0, k_on=0, n_slots=0,
              storage="f32", bc=(0, 0, 0), adjoint=False, method="so2dr", rounding="every_step",
              copy_engine="auto")
    kw.update(plan_kwargs)
    d, keep = _make_desc(**kw)
    out = _lib.Desc()
    ms = ctypes.c_double()
    mp = ctypes.byref(_machine_struct(machine)) if machine else None
    check(lib().so2dr_plan_suggest(ctypes.byref(d), mp, ctypes.byref(out), ctypes.byref(ms)))
    del keep
    res = dict(kw, tb_depth=out.tb_depth, n_chunks=out.n_chunks, k_on=out.k_on,
               n_slots=out.n_slots)
    return res, ms.value


def adjoint_buffers_needed(T, tb_depth, ckpt_every):
    """Pinned host fields so2dr_adjoint_run needs: one per segment start after
    the first, plus the round starts inside one segment."""
    if T <= 0:
        return 0
    c = min(ckpt_every, T)
    nseg = -(-T // c)
    return max(0, nseg - 1) + max(0, -(-c // tb_depth) - 1)


def _adjoint(self, u0, target, ckpt_every, ckpt=None, grad_u0=None):
    """Gradient of L = 1/2 ||u_T - target||^2.  u0, target: pinned host
    tensors of the storage type (F32 or F64).  Returns (loss, grad_u0,
    grad_w, stats); grad_w is an FP64 numpy array in weight order."""
    import torch
    info = self.info()
    self._check_host(u0)
    self._check_host(target)
    need = adjoint_buffers_needed(self._T, info["tb_depth"], ckpt_every)
    if ckpt is None:
        ckpt = [pinned_empty(u0.shape, u0.dtype) for _ in range(need)]
    if grad_u0 is None:
        grad_u0 = pinned_empty(u0.shape, u0.dtype)
    arr = (ctypes.c_void_p * max(1, len(ckpt)))(*[t.data_ptr() for t in ckpt])
    gw = (ctypes.c_double * self._nw)()
    loss = ctypes.c_double()
    st = _lib.Stats()
    check(lib().so2dr_adjoint_run(self._h, ctypes.c_void_p(u0.data_ptr()),
                                  ctypes.c_void_p(target.data_ptr()),
                                  ctypes.c_void_p(grad_u0.data_ptr()), gw, ctypes.byref(loss),
                                  int(ckpt_every), arr, len(ckpt), ctypes.byref(st)))
    return loss.value, grad_u0, np.array(gw[:]), st.as_dict()


Plan.adjoint = _adjoint
