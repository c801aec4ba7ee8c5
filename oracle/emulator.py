"""Bit-exact CPU model of the library's reduced-precision arithmetic.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  The C interface
promises a specific arithmetic: every cell's sum is a chain of fused
multiply-adds in FP32, starting from +0 and running over the stencil points
in lexicographic (dz, dy, dx) order, with FP32-rounded weights; BF16 / FP16
storage rounds the sum to nearest-even after every step.  This module models
exactly that in NumPy, so GPU results can be compared bit for bit.  It shares
nothing with the HIP code: it is written from the interface's description.

FP32 fused multiply-add, exactly: for float32 a, b, c the product a*b is
exact in float64 (48 significant bits); TwoSum gives s + e == a*b + c exactly
with s, e float64; rounding s to float32 gives the correct result unless s is
exactly halfway between two float32 values and e != 0, in which case the
exact value lies on e's side of the midpoint.
"""
import numpy as np


def _two_sum(a, b):
    s = a + b
    bp = s - a
    ap = s - bp
    return s, (a - ap) + (b - bp)


def fma32(a, b, c):
    """Correctly rounded float32 fma(a, b, c), elementwise."""
    a = np.asarray(a, np.float32).astype(np.float64)
    b = np.asarray(b, np.float32).astype(np.float64)
    c = np.asarray(c, np.float32).astype(np.float64)
    p = a * b
    s, e = _two_sum(p, c)
    r = s.astype(np.float32)
    # s is an exact float32 midpoint iff it is not a float32 but s +- half an
    # ulp are; detect it as: rounding down and up of s straddle it equally
    lo = np.nextafter(r, np.float32(-np.inf)).astype(np.float64)
    hi = np.nextafter(r, np.float32(np.inf)).astype(np.float64)
    r64 = r.astype(np.float64)
    mid_lo = (r64 + lo) / 2.0      # exact in float64
    mid_hi = (r64 + hi) / 2.0
    at_lo = (s == mid_lo) & (e != 0)
    at_hi = (s == mid_hi) & (e != 0)
    out = r.copy()
    # s halfway below r (r was chosen by ties-to-even): exact value is below s
    # when e < 0, so the right answer is the lower neighbour
    out = np.where(at_lo & (e < 0), lo.astype(np.float32), out)
    out = np.where(at_hi & (e > 0), hi.astype(np.float32), out)
    # s halfway and r rounded away from the exact side: when s == mid_lo and
    # e > 0 the exact value is above the midpoint, so r (above) is right; when
    # s == mid_hi and e < 0, r (below) is right
    return out


def round_bf16(x):
    """float32 -> nearest-even bfloat16, returned as float32 values."""
    x = np.ascontiguousarray(x, np.float32)
    bits = x.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rb = ((bits + 0x7FFF + lsb) >> 16) << 16
    return rb.astype(np.uint32).view(np.float32)


def round_f16(x):
    """float32 -> nearest-even float16, returned as float32 values."""
    return np.asarray(x, np.float32).astype(np.float16).astype(np.float32)


_ROUND = {"f32": lambda v: v, "bf16": round_bf16, "f16": round_f16}


def _shifted(u, o, periodic):
    """v(x) = u(x + o) with zero (Dirichlet) or wrapped (periodic) ghosts;
    u is (z, y, x), o is (dz, dy, dx), periodic is per axis (x, y, z)."""
    v = u
    for axis, d in enumerate(o):
        if d == 0:
            continue
        if periodic[2 - axis]:
            v = np.roll(v, -d, axis=axis)
        else:
            n = v.shape[axis]
            w = np.zeros_like(v)
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            if abs(d) < n:
                if d > 0:
                    src[axis], dst[axis] = slice(d, n), slice(0, n - d)
                else:
                    src[axis], dst[axis] = slice(0, n + d), slice(-d, n)
                w[tuple(dst)] = v[tuple(src)]
            v = w
    return v


def sweep_bits(u0, offsets, weights, T, storage="f32", periodic=(0, 0, 0), round_after=None):
    """T steps of the FP32-FMA sweep with rounding to `storage` (f32, bf16 or
    f16).  u0 holds values already representable in the storage type;
    returns float32 values.  offsets: (dz, dy, dx) in the order the sums run
    (lexicographic); a 2D field is (y, x) with dz == 0.  round_after: the
    step counts t (1..T) after which the field is rounded to storage; None
    rounds after every step.  Between roundings the field stays FP32."""
    two_d = np.asarray(u0).ndim == 2
    u = np.asarray(u0, np.float32)
    u = u[None] if two_d else u
    w32 = np.asarray(weights, np.float64).astype(np.float32)
    rnd = _ROUND[storage]
    for t in range(1, T + 1):
        acc = np.zeros_like(u)           # +0
        for o, wk in zip(offsets, w32):
            acc = fma32(wk, _shifted(u, o, periodic), acc)
        u = rnd(acc) if round_after is None or t in round_after else acc
    return u[0] if two_d else u


# ---------------------------------------------------------------- C model
# emulator_bits.c computes the same arithmetic with the C library's correctly
# rounded fmaf, fast enough for grids of tens of millions of cells; it is
# checked against sweep_bits above in the tests.

_STORAGE_CODE = {"f32": 0, "bf16": 2, "f16": 3}


def _c_args(offsets, weights, periodic, T, round_after):
    import ctypes
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 3))
    w32 = np.ascontiguousarray(np.asarray(weights, np.float64).astype(np.float32).reshape(-1))
    per = np.ascontiguousarray(np.asarray(periodic, dtype=np.int32).reshape(3))
    flags = None
    if round_after is not None:
        flags = np.zeros(T + 1, np.uint8)
        for t in round_after:
            if 1 <= t <= T:
                flags[t] = 1
    ptr = (lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None)
    return off, w32, per, flags, ptr


def sweep_bits_c(u0, offsets, weights, T, storage="f32", periodic=(0, 0, 0), round_after=None):
    """sweep_bits computed by the C model (same arguments and result)."""
    from .oracle import _lib
    two_d = np.asarray(u0).ndim == 2
    u = np.ascontiguousarray(np.asarray(u0, np.float32))
    u3 = u[None] if two_d else u
    nz, ny, nx = u3.shape
    off, w32, per, flags, ptr = _c_args(offsets, weights, periodic, T, round_after)
    out = np.empty_like(u3)
    rc = _lib().emu_sweep(nx, ny, nz, ptr(per), len(w32), ptr(off), ptr(w32), int(T),
                          _STORAGE_CODE[storage], ptr(flags), ptr(u3), ptr(out))
    if rc:
        raise RuntimeError(f"emu_sweep failed ({rc})")
    return out[0] if two_d else out


def sweep_bits_box_from_field(u0, offsets, weights, T, box_lo, box_hi, storage="f32",
                              periodic=(0, 0, 0), round_after=None):
    """sweep_bits restricted to the sub-box [box_lo, box_hi) ((x, y, z)
    triples) of a field of any size (numpy array or torch CPU tensor of the
    storage type, (z, y, x)); only the box's dependency cone is read.
    Returns FP32 values shaped (z, y, x)."""
    from .oracle import _lib, extract_window, reach_of
    shape = tuple(u0.shape) if len(u0.shape) == 3 else (1,) + tuple(u0.shape)
    nx, ny, nz = shape[2], shape[1], shape[0]
    off, w32, per, flags, ptr = _c_args(offsets, weights, periodic, T, round_after)
    reach = np.asarray(reach_of(off))
    lo = np.ascontiguousarray(np.asarray(box_lo, dtype=np.int64).reshape(3))
    hi = np.ascontiguousarray(np.asarray(box_hi, dtype=np.int64).reshape(3))
    win = np.ascontiguousarray(extract_window(u0, lo - T * reach, hi + T * reach, per)
                               .astype(np.float32))
    e = hi - lo
    out = np.empty((e[2], e[1], e[0]), np.float32)
    rc = _lib().emu_sweep_box_win(nx, ny, nz, ptr(per), len(w32), ptr(off), ptr(w32), int(T),
                                  _STORAGE_CODE[storage], ptr(flags), ptr(win), ptr(lo),
                                  ptr(hi), ptr(out))
    if rc:
        raise RuntimeError(f"emu_sweep_box_win failed ({rc})")
    return out
