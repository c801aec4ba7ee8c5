"""Shared test helpers: run a plan on pinned tensors and compare with the
oracle.  The oracle is imported only here in tests, never by the library."""
import numpy as np

STENCIL_CASES = [
    # (ndim, shape, r)
    (2, "star", 1), (2, "box", 1), (2, "box", 2), (2, "box", 3), (2, "box", 4),
    (3, "star", 1), (3, "star", 2), (3, "box", 1),
]


def grid_dims(ndim, nx, ny, nz):
    return (nx, ny, 1) if ndim == 2 else (nx, ny, nz)


def np_shape(ndim, nx, ny, nz):
    return (ny, nx) if ndim == 2 else (nz, ny, nx)


def torch_dtype(storage):
    import torch
    return {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16,
            "f16": torch.float16}[storage]


def to_storage(u64, storage):
    """The FP64 field rounded (to nearest even) to the storage type, as a
    torch CPU tensor."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(u64)).to(torch_dtype(storage))


def pinned_copy(t):
    import torch
    p = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
    p.copy_(t)
    return p


def gpu_run(plan_kwargs, u_storage, steps=None, bind_streams=None):
    """Run a plan on a pinned copy of u_storage; returns (result tensor, stats, info)."""
    from paper_2309_08864_amd import Plan
    p = Plan(**plan_kwargs)
    p.bind(n_streams=bind_streams)
    h = pinned_copy(u_storage)
    if steps is None:
        st = p.run(h)
        out = h
    else:
        out = pinned_copy(u_storage)
        st = p.run_steps(h, out, steps)
    info = p.info()
    p.close()
    return out.clone(), st, info


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def fp32_weights(w):
    return np.asarray(w, dtype=np.float64).astype(np.float32).astype(np.float64)


def store_steps(T, K, k_on):
    """Step counts after which a plan stores the field to HBM: rounds of K
    steps (the last one shorter), and inside a round one store per launch of
    k_on steps plus one for the remainder -- the documented schedule of
    round-at-store BF16/F16 plans."""
    out = set()
    t0 = 0
    while t0 < T:
        kp = min(K, T - t0)
        t = t0
        while t < t0 + kp:
            t = min(t + k_on, t0 + kp)
            out.add(t)
        t0 += kp
    return out
