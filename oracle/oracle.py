"""ctypes wrapper around the C oracle plus the stencil point sets.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Stencil point sets (paper Sec. II-A, Fig. 1a; Table III for the box family):
  * star, radius r: the centre plus the points at distance 1..r along each
    axis in both directions (1 + 2*dim*r points);
  * box, radius r: every point of the (2r+1)^dim cube.
Offsets are (dz, dy, dx) triples; a 2D stencil has dz == 0 and acts on a grid
with nz == 1, its second axis (y) being the one the grid is cut along.  The
weight array that goes with a point set is listed in lexicographic order of
the (dz, dy, dx) triples.
"""
import ctypes
import os
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib_path() -> str:
    return os.path.join(_HERE, "libso2dr_oracle.so")


def build() -> str:
    from .build import build as _b
    return _b()


def _lib():
    global _LIB
    if _LIB is None:
        p = lib_path()
        srcs = [os.path.join(_HERE, f) for f in ("so2dr_oracle.c", "emulator_bits.c")]
        if not os.path.exists(p) or os.path.getmtime(p) < max(os.path.getmtime(s) for s in srcs):
            build()
        L = ctypes.CDLL(p)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.oracle_sweep.argtypes = [i64, i64, i64, vp, i32, vp, vp, i32, vp, vp]
        L.oracle_transpose_step.argtypes = [i64, i64, i64, vp, i32, vp, vp, vp, vp]
        L.oracle_adjoint.argtypes = [i64, i64, i64, vp, i32, vp, vp, i32, vp, vp, i32,
                                     vp, vp, vp, vp]
        L.oracle_sweep_box.argtypes = [i64, i64, i64, vp, i32, vp, vp, i32, vp, vp, vp, vp]
        L.oracle_sweep_box_win.argtypes = [i64, i64, i64, vp, i32, vp, vp, i32, vp, vp, vp, vp]
        L.emu_sweep.argtypes = [i64, i64, i64, vp, i32, vp, vp, i32, i32, vp, vp, vp]
        L.emu_sweep_box_win.argtypes = [i64, i64, i64, vp, i32, vp, vp, i32, i32, vp, vp, vp, vp,
                                        vp]
        for f in (L.oracle_sweep, L.oracle_transpose_step, L.oracle_adjoint, L.oracle_sweep_box,
                  L.oracle_sweep_box_win, L.emu_sweep, L.emu_sweep_box_win):
            f.restype = i32
        _LIB = L
    return _LIB


def stencil_offsets(ndim: int, shape: str, r: int):
    """List of (dz, dy, dx) offsets of a star or box stencil of radius r, in
    lexicographic order."""
    if ndim not in (2, 3) or r < 1:
        raise ValueError("ndim must be 2 or 3 and r >= 1")
    rng = range(-r, r + 1)
    pts = []
    for dz in (rng if ndim == 3 else [0]):
        for dy in rng:
            for dx in rng:
                nz = (dz != 0) + (dy != 0) + (dx != 0)
                if shape == "box" or nz <= 1:
                    pts.append((dz, dy, dx))
    if shape not in ("star", "box"):
        raise ValueError(shape)
    return sorted(pts)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _prep(u, offsets, weights, periodic):
    u = np.ascontiguousarray(u, dtype=np.float64)
    if u.ndim == 2:
        nz, (ny, nx) = 1, u.shape
    elif u.ndim == 3:
        nz, ny, nx = u.shape
    else:
        raise ValueError("field must be (ny, nx) or (nz, ny, nx)")
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 3))
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
    if off.shape[0] != w.shape[0]:
        raise ValueError("one weight per offset")
    per = np.ascontiguousarray(np.asarray(periodic, dtype=np.int32).reshape(3))
    return u, nx, ny, nz, off, w, per


def sweep(u0, offsets, weights, T, periodic=(0, 0, 0)):
    """u_T after T Jacobi steps from u0 (FP64). periodic is per axis (x, y, z)."""
    u, nx, ny, nz, off, w, per = _prep(u0, offsets, weights, periodic)
    out = np.empty_like(u)
    rc = _lib().oracle_sweep(nx, ny, nz, _ptr(per), len(w), _ptr(off), _ptr(w), int(T),
                             _ptr(u), _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_sweep failed ({rc})")
    return out


def transpose_step(lam, offsets, weights, periodic=(0, 0, 0)):
    """One step of the transpose map: out(x) = sum_k w_k ext(lam, x - o_k)."""
    u, nx, ny, nz, off, w, per = _prep(lam, offsets, weights, periodic)
    out = np.empty_like(u)
    rc = _lib().oracle_transpose_step(nx, ny, nz, _ptr(per), len(w), _ptr(off), _ptr(w),
                                      _ptr(u), _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_transpose_step failed ({rc})")
    return out


def adjoint(u0, target, offsets, weights, T, periodic=(0, 0, 0), ckpt=0):
    """(loss, grad_u0, grad_w, u_T) for L = 1/2 ||u_T - target||^2."""
    u, nx, ny, nz, off, w, per = _prep(u0, offsets, weights, periodic)
    y = np.ascontiguousarray(target, dtype=np.float64)
    if y.shape != u.shape:
        raise ValueError("target shape")
    loss = np.zeros(1)
    gu = np.empty_like(u)
    gw = np.empty(len(w))
    uT = np.empty_like(u)
    rc = _lib().oracle_adjoint(nx, ny, nz, _ptr(per), len(w), _ptr(off), _ptr(w), int(T),
                               _ptr(u), _ptr(y), int(ckpt), _ptr(loss), _ptr(gu), _ptr(gw),
                               _ptr(uT))
    if rc:
        raise RuntimeError(f"oracle_adjoint failed ({rc})")
    return float(loss[0]), gu, gw, uT


def sweep_box(u0, offsets, weights, T, box_lo, box_hi, periodic=(0, 0, 0)):
    """u_T restricted to the sub-box [box_lo, box_hi) given as (x, y, z)
    triples, computed from the dependency cone of the box only.  Returns an
    array shaped (z, y, x) (or (y, x) for a 2D field)."""
    u, nx, ny, nz, off, w, per = _prep(u0, offsets, weights, periodic)
    lo = np.ascontiguousarray(np.asarray(box_lo, dtype=np.int64).reshape(3))
    hi = np.ascontiguousarray(np.asarray(box_hi, dtype=np.int64).reshape(3))
    ext = hi - lo
    out = np.empty((ext[2], ext[1], ext[0]))
    rc = _lib().oracle_sweep_box(nx, ny, nz, _ptr(per), len(w), _ptr(off), _ptr(w), int(T),
                                 _ptr(u), _ptr(lo), _ptr(hi), _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_sweep_box failed ({rc})")
    return out[0] if np.asarray(u0).ndim == 2 else out


def reach_of(offsets):
    """Largest |offset| per axis (x, y, z)."""
    off = np.asarray(offsets).reshape(-1, 3)
    return tuple(int(np.abs(off[:, a]).max()) for a in (2, 1, 0))


def extract_window(u, lo, hi, periodic):
    """Values of field u (array (z, y, x), any float dtype, may be a view of a
    huge array) at unreduced coordinates [lo, hi) per axis (x, y, z): wrapped
    on periodic axes, zero outside the grid on Dirichlet axes.  FP64 result
    shaped (z, y, x)."""
    shape = tuple(u.shape) if u.ndim == 3 else (1,) + tuple(u.shape)
    n = (shape[2], shape[1], shape[0])
    idx, ok = [], []
    for a in range(3):
        c = np.arange(lo[a], hi[a])
        if periodic[a]:
            idx.append(np.mod(c, n[a]))
            ok.append(np.ones(len(c), bool))
        else:
            inside = (c >= 0) & (c < n[a])
            idx.append(np.clip(c, 0, n[a] - 1))
            ok.append(inside)
    u3 = u if u.ndim == 3 else u[None]
    if hasattr(u3, "index_select"):   # a torch tensor (e.g. bfloat16 storage)
        import torch
        g = u3.index_select(0, torch.from_numpy(idx[2]))
        g = g.index_select(1, torch.from_numpy(idx[1]))
        g = g.index_select(2, torch.from_numpy(idx[0]))
        win = g.double().numpy()
    else:
        win = np.asarray(u3[np.ix_(idx[2], idx[1], idx[0])], dtype=np.float64)
    mask = ok[2][:, None, None] & ok[1][None, :, None] & ok[0][None, None, :]
    win[~mask] = 0.0
    return np.ascontiguousarray(win)


def sweep_box_from_field(u0, offsets, weights, T, box_lo, box_hi, periodic=(0, 0, 0)):
    """u_T on the sub-box [box_lo, box_hi) of a field of any size (only the
    box's dependency cone is read).  Returns (z, y, x) FP64."""
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 3))
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
    per = np.ascontiguousarray(np.asarray(periodic, dtype=np.int32).reshape(3))
    shape = tuple(u0.shape) if u0.ndim == 3 else (1,) + tuple(u0.shape)
    nx, ny, nz = shape[2], shape[1], shape[0]
    reach = reach_of(off)
    lo = np.asarray(box_lo, dtype=np.int64).reshape(3)
    hi = np.asarray(box_hi, dtype=np.int64).reshape(3)
    wlo = lo - T * np.asarray(reach)
    whi = hi + T * np.asarray(reach)
    win = extract_window(u0, wlo, whi, per)
    return sweep_box_window(win, (nx, ny, nz), off, w, T, lo, hi, per)


def sweep_box_window(win, grid, offsets, weights, T, box_lo, box_hi, periodic=(0, 0, 0)):
    """u_T on [box_lo, box_hi) from a level-0 window covering the box dilated
    by T*reach (see extract_window)."""
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 3))
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
    per = np.ascontiguousarray(np.asarray(periodic, dtype=np.int32).reshape(3))
    lo = np.ascontiguousarray(np.asarray(box_lo, dtype=np.int64).reshape(3))
    hi = np.ascontiguousarray(np.asarray(box_hi, dtype=np.int64).reshape(3))
    reach = reach_of(off)
    ext = [int(hi[a] - lo[a] + 2 * T * reach[a]) for a in range(3)]
    win = np.ascontiguousarray(win, dtype=np.float64)
    if win.shape != (ext[2], ext[1], ext[0]):
        raise ValueError(f"window shape {win.shape} != {(ext[2], ext[1], ext[0])}")
    e = hi - lo
    out = np.empty((e[2], e[1], e[0]))
    nx, ny, nz = grid
    rc = _lib().oracle_sweep_box_win(nx, ny, nz, _ptr(per), len(w), _ptr(off), _ptr(w), int(T),
                                     _ptr(win), _ptr(lo), _ptr(hi), _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_sweep_box_win failed ({rc})")
    return out
