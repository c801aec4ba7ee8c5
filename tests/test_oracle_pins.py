"""Pins for the FP64 oracle.

Every test checks the oracle against something that does not run through its
own code: exact rational arithmetic, library correlation / convolution
routines, closed-form Fourier eigenvalues, conservation laws, the light cone
of the update, the adjoint dot-product identity, finite differences and
PyTorch autograd.  Each is chosen so that a plausible slip in the oracle (a
dropped term, a flipped offset sign, a transposed axis, a wrong boundary rule,
a wrong adjoint) fails at least one of them.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.signal as sig

import oracle
from oracle import adjoint, stencil_offsets, sweep, sweep_box, transpose_step

HERE = os.path.dirname(os.path.abspath(__file__))
STENCILS = [(2, "star", 1), (2, "box", 1), (2, "box", 2), (3, "star", 1), (3, "star", 2),
            (3, "box", 1)]
BCS = [(0, 0, 0), (1, 1, 1), (1, 1, 0), (1, 0, 0)]


def _shape(ndim):
    # deliberately non-cubic, so a transposed axis changes the answer
    return (7, 6) if ndim == 2 else (5, 6, 7)


def _bc_for(ndim, bc):
    return (bc[0], bc[1], 0) if ndim == 2 else bc


def _as3(u):
    return u[None] if u.ndim == 2 else u


# ---------------------------------------------------------------- P1 exact
def _shift_exact(u, o, periodic):
    """v(x) = u(x + o) under the boundary rule, by whole-array shifting."""
    v = u
    for axis, d in enumerate(o):          # array axes are (z, y, x); o is (dz, dy, dx)
        if d == 0:
            continue
        per = periodic[2 - axis]
        if per:
            v = np.roll(v, -d, axis=axis)
        else:
            n = v.shape[axis]
            w = np.empty_like(v)
            w[...] = Fraction(0)
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


@pytest.mark.parametrize("ndim,shape,r", STENCILS)
@pytest.mark.parametrize("bc", BCS)
def test_p1_exact_rational(ndim, shape, r, bc):
    """Dyadic weights and inputs: FP64 is exact, so the oracle must equal the
    rational-arithmetic answer bit for bit."""
    rng = np.random.default_rng(100 + 7 * r + ndim)
    offs = stencil_offsets(ndim, shape, r)
    wn = rng.integers(-4, 5, len(offs))
    u0n = rng.integers(-512, 513, _shape(ndim))
    per = _bc_for(ndim, bc)
    T = 3
    w = [Fraction(int(k), 8) for k in wn]
    u = _as3(np.vectorize(lambda k: Fraction(int(k), 1024), otypes=[object])(u0n))
    for _ in range(T):
        acc = np.empty_like(u)
        acc[...] = Fraction(0)
        for o, wk in zip(offs, w):
            acc = acc + wk * _shift_exact(u, o, per)
        u = acc
    exact = np.vectorize(float)(u).reshape(_shape(ndim))
    got = sweep(u0n / 1024.0, offs, wn / 8.0, T, per)
    assert np.array_equal(got, exact)


# ---------------------------------------------------------------- P2 libraries
def _weights_cube(offs, w, r):
    W = np.zeros((2 * r + 1,) * 3)
    for o, wk in zip(offs, w):
        W[o[0] + r, o[1] + r, o[2] + r] = wk
    return W


def _lib_step(u3, W, r, per):
    p = u3
    for axis in range(3):
        pad = [(0, 0)] * 3
        pad[axis] = (r, r)
        p = np.pad(p, pad, mode="wrap" if per[2 - axis] else "constant")
    return sig.correlate(p, W, mode="valid", method="direct")


@pytest.mark.parametrize("ndim,shape,r", STENCILS)
@pytest.mark.parametrize("bc", BCS)
def test_p2_scipy_correlate(ndim, shape, r, bc):
    rng = np.random.default_rng(200 + r)
    offs = stencil_offsets(ndim, shape, r)
    w = rng.uniform(-1, 1, len(offs))
    per = _bc_for(ndim, bc)
    u0 = rng.random(_shape(ndim))
    W = _weights_cube(offs, w, r)
    ref = _as3(u0)
    for _ in range(2):
        ref = _lib_step(ref, W, r, per)
    got = _as3(sweep(u0, offs, w, 2, per))
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)
    if per in ((0, 0, 0), (1, 1, 1)):   # uniform modes also go through ndimage
        mode = "wrap" if per[0] else "constant"
        one = ndi.correlate(_as3(u0), W, mode=mode, cval=0.0)
        if ndim == 2:   # the stencil has no dz extent; ndimage would wrap z
            one = _lib_step(_as3(u0), W, r, per)
        assert np.allclose(_as3(sweep(u0, offs, w, 1, per)), one, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("ndim,shape,r", STENCILS)
def test_p2_torch_conv(ndim, shape, r):
    """torch's convNd is a cross-correlation, i.e. the same operation."""
    torch = pytest.importorskip("torch")
    import torch.nn.functional as F
    rng = np.random.default_rng(300 + r)
    offs = stencil_offsets(ndim, shape, r)
    w = rng.uniform(-1, 1, len(offs))
    u0 = rng.random(_shape(ndim))
    W = _weights_cube(offs, w, r)
    x = torch.from_numpy(_as3(u0))[None, None]
    k = torch.from_numpy(W)[None, None]
    for bc in ((0, 0, 0), (1, 1, 1)):
        per = _bc_for(ndim, bc)
        y = x
        for _ in range(3):
            if per[0]:
                if ndim == 2:
                    yp = F.pad(y[:, :, 0], (r, r, r, r), mode="circular")[:, :, None]
                    yp = F.pad(yp, (0, 0, 0, 0, r, r))
                else:
                    yp = F.pad(y, (r,) * 6, mode="circular")
                y = F.conv3d(yp, k)
            else:
                y = F.conv3d(y, k, padding=r)
        got = _as3(sweep(u0, offs, w, 3, per))
        assert np.allclose(got, y[0, 0].numpy(), rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- P3 constants
@pytest.mark.parametrize("ndim,shape,r", STENCILS)
def test_p3_constant_preserved(ndim, shape, r):
    rng = np.random.default_rng(400 + r)
    offs = stencil_offsets(ndim, shape, r)
    # dyadic weights summing to exactly 1: k_i / 2^m with sum k_i = 2^m
    m = 10
    k = rng.integers(1, 16, len(offs))
    k[0] += (1 << m) - k.sum()
    w = k / float(1 << m)
    assert w.sum() == 1.0
    c = 0.625
    u = np.full(_shape(ndim), c)
    per = _bc_for(ndim, (1, 1, 1))
    assert np.array_equal(sweep(u, offs, w, 6, per), u)
    # non-dyadic weights summing to 1 in exact arithmetic: within T*P ulps
    w2 = np.full(len(offs), 1.0 / len(offs))
    got = sweep(u, offs, w2, 6, per)
    assert np.max(np.abs(got - c)) <= 6 * len(offs) * np.finfo(float).eps * c * 4
    # Dirichlet: cells farther than T*r from every boundary keep the constant
    big = (16, 17) if ndim == 2 else (12, 13, 14)
    T = 2
    got = sweep(np.full(big, c), offs, w, T, (0, 0, 0))
    s = T * r
    inner = got[s:-s, s:-s] if ndim == 2 else got[s:-s, s:-s, s:-s]
    assert np.array_equal(inner, np.full(inner.shape, c))
    edge = got[0, 0] if ndim == 2 else got[0, 0, 0]
    assert edge < c


# ---------------------------------------------------------------- P4 Fourier
@pytest.mark.parametrize("ndim,shape,r", STENCILS)
def test_p4_fourier_periodic(ndim, shape, r):
    """On a periodic grid exp(2 pi i k.x/n) is an eigenvector with eigenvalue
    sum_o w_o exp(2 pi i k.o/n); holds for non-symmetric weights too."""
    rng = np.random.default_rng(500 + r)
    offs = stencil_offsets(ndim, shape, r)
    w = rng.uniform(0, 1, len(offs))
    w /= w.sum()
    shp = (12, 10) if ndim == 2 else (8, 10, 12)
    kvec = (0, 2, 3) if ndim == 2 else (1, 2, 3)   # (kz, ky, kx)
    ns = (1,) + shp if ndim == 2 else shp
    grids = np.meshgrid(*[np.arange(n) for n in ns], indexing="ij")
    phase = sum(2 * np.pi * kvec[a] * grids[a] / ns[a] for a in range(3)) + 0.3
    lam = sum(wk * np.exp(2j * np.pi * sum(kvec[a] * o[a] / ns[a] for a in range(3)))
              for o, wk in zip(offs, w))
    T = 7
    u0 = np.cos(phase).reshape(shp)
    ref = np.real(lam ** T * np.exp(1j * phase)).reshape(shp)
    got = sweep(u0, offs, w, T, (1, 1, 1))
    assert np.allclose(got, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("shape", ["star", "box"])
def test_p4_fourier_mixed_bc(shape):
    """Periodic x/y, Dirichlet z, radius 1 with weights symmetric in dz: the
    mode cos(2 pi (kx x/nx + ky y/ny) + phi) sin(pi m (z+1)/(nz+1)) is an
    eigenvector (the zero ghost planes coincide with the sine's zeros)."""
    rng = np.random.default_rng(550)
    offs = stencil_offsets(3, shape, 1)
    base = {}
    w = []
    for o in offs:
        key = (abs(o[0]), o[1], o[2])
        if key not in base:
            base[key] = rng.uniform(0, 1)
        w.append(base[key])
    w = np.array(w) / np.sum(w)
    nz, ny, nx = 9, 8, 10
    kx, ky, m, phi = 3, 2, 4, 0.7
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ang = 2 * np.pi * (kx * x / nx + ky * y / ny) + phi
    s = np.sin(np.pi * m * (z + 1) / (nz + 1))
    lam = sum(wk * np.exp(2j * np.pi * (kx * o[2] / nx + ky * o[1] / ny))
              * np.cos(np.pi * m * o[0] / (nz + 1)) for o, wk in zip(offs, w))
    T = 9
    got = sweep(np.cos(ang) * s, offs, w, T, (1, 1, 0))
    ref = np.real(lam ** T * np.exp(1j * ang)) * s
    assert np.allclose(got, ref, rtol=0, atol=1e-13)


def test_p4_fourier_dirichlet_sine():
    """Zero Dirichlet on every axis, symmetric radius-1 star: a product of
    sines is an eigenvector with eigenvalue w_c + sum_a 2 w_a cos(theta_a)."""
    offs = stencil_offsets(3, "star", 1)
    wa = {0: 0.11, 1: 0.13, 2: 0.07}    # per array axis (z, y, x)
    wc = 1 - 2 * sum(wa.values())
    w = []
    for o in offs:
        nzax = [a for a in range(3) if o[a] != 0]
        w.append(wc if not nzax else wa[nzax[0]])
    shp = (7, 9, 11)
    ms = (2, 3, 5)
    grids = np.meshgrid(*[np.arange(n) for n in shp], indexing="ij")
    u0 = np.ones(shp)
    lam = wc
    for a in range(3):
        th = np.pi * ms[a] / (shp[a] + 1)
        u0 = u0 * np.sin(th * (grids[a] + 1))
        lam += 2 * wa[a] * np.cos(th)
    got = sweep(u0, offs, w, 12, (0, 0, 0))
    assert np.allclose(got, lam ** 12 * u0, rtol=0, atol=1e-13)


# ---------------------------------------------------------------- P5 invariants
@pytest.mark.parametrize("ndim,shape,r", STENCILS)
def test_p5_linearity_mass_maxprinciple(ndim, shape, r):
    rng = np.random.default_rng(600 + r)
    offs = stencil_offsets(ndim, shape, r)
    w = rng.uniform(-0.5, 1, len(offs))
    a, b = rng.random(_shape(ndim)), rng.random(_shape(ndim))
    per = _bc_for(ndim, (0, 0, 0))
    lhs = sweep(2.5 * a - 0.75 * b, offs, w, 4, per)
    rhs = 2.5 * sweep(a, offs, w, 4, per) - 0.75 * sweep(b, offs, w, 4, per)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)
    # mass: on a fully periodic grid sum(u_{t+1}) = (sum w) sum(u_t)
    perp = _bc_for(ndim, (1, 1, 1))
    u1 = sweep(a, offs, w, 1, perp)
    assert np.isclose(u1.sum(), w.sum() * a.sum(), rtol=1e-13)
    # discrete maximum principle: w >= 0, sum w = 1, zero Dirichlet
    wp = rng.uniform(0, 1, len(offs))
    wp /= wp.sum()
    u = rng.uniform(-1, 2, _shape(ndim))
    lo, hi = min(0.0, u.min()), max(0.0, u.max())
    for T in (1, 3, 8):
        g = sweep(u, offs, wp, T, per)
        assert g.min() >= lo - 1e-14 and g.max() <= hi + 1e-14


# ---------------------------------------------------------------- P6 light cone
@pytest.mark.parametrize("ndim,shape,r", STENCILS)
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0), (1, 1, 1)])
def test_p6_subbox_matches_full(ndim, shape, r, bc):
    rng = np.random.default_rng(700 + r + ndim)
    offs = stencil_offsets(ndim, shape, r)
    w = rng.uniform(-0.3, 1, len(offs))
    shp = (20, 17) if ndim == 2 else (11, 12, 13)
    per = _bc_for(ndim, bc)
    u0 = rng.random(shp)
    T = 4
    full = sweep(u0, offs, w, T, per)
    full3 = _as3(full)
    ns = full3.shape[::-1]   # (nx, ny, nz)
    for _ in range(3):
        lo = [int(rng.integers(0, n)) for n in ns]
        hi = [min(n, l + int(rng.integers(1, 5))) for l, n in zip(lo, ns)]
        got = _as3(sweep_box(u0, offs, w, T, lo, hi, per))
        ref = full3[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("ndim,shape,r", [(3, "star", 2), (3, "box", 1), (2, "box", 3)])
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0)])
def test_p6_window_sweep_matches_full(ndim, shape, r, bc):
    """The window form (level 0 extracted with the boundary rule, used for
    grids too large to convert whole) equals the full sweep, on float32
    input as the large workloads store it."""
    rng = np.random.default_rng(750 + r)
    offs = stencil_offsets(ndim, shape, r)
    w = rng.uniform(0, 1, len(offs))
    shp = (23, 19) if ndim == 2 else (13, 12, 11)
    per = _bc_for(ndim, bc)
    u0 = rng.random(shp).astype(np.float32)
    T = 3
    full = _as3(sweep(u0.astype(np.float64), offs, w, T, per))
    ns = full.shape[::-1]
    for _ in range(3):
        lo = [int(rng.integers(0, n)) for n in ns]
        hi = [min(n, l + int(rng.integers(1, 4))) for l, n in zip(lo, ns)]
        got = oracle.sweep_box_from_field(u0, offs, w, T, lo, hi, per)
        assert np.array_equal(got, full[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]])


@pytest.mark.parametrize("shape", ["star", "box"])
def test_p6_impulse_support(shape):
    offs = stencil_offsets(3, shape, 1)
    w = np.full(len(offs), 1.0 / len(offs))
    n = 15
    u0 = np.zeros((n, n, n))
    c = n // 2
    u0[c, c, c] = 1.0
    T = 3
    g = sweep(u0, offs, w, T, (0, 0, 0))
    z, y, x = np.meshgrid(*(np.arange(n) - c,) * 3, indexing="ij")
    dist = (abs(x) + abs(y) + abs(z)) if shape == "star" else np.maximum(np.maximum(abs(x), abs(y)), abs(z))
    assert np.all(g[dist > T] == 0)
    assert np.all(g[dist == T] > 0)


# ---------------------------------------------------------------- P7 adjoint
@pytest.mark.parametrize("ndim,shape,r", STENCILS)
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0), (1, 1, 1)])
def test_p7_transpose_identity(ndim, shape, r, bc):
    rng = np.random.default_rng(800 + r)
    offs = stencil_offsets(ndim, shape, r)
    w = rng.uniform(-1, 1, len(offs))
    per = _bc_for(ndim, bc)
    u, v = rng.standard_normal(_shape(ndim)), rng.standard_normal(_shape(ndim))
    lhs = np.vdot(sweep(u, offs, w, 1, per), v)
    rhs = np.vdot(u, transpose_step(v, offs, w, per))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


# ---------------------------------------------------------------- P8 gradients
def _loss(u0, y, offs, w, T, per):
    d = sweep(u0, offs, w, T, per) - y
    return 0.5 * float(np.sum(d * d))


@pytest.mark.parametrize("ndim,shape,r", [(3, "star", 1), (3, "box", 1), (2, "box", 2), (3, "star", 2)])
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0)])
def test_p8_directional_fd_u0(ndim, shape, r, bc):
    """L is quadratic in u0, so the central difference with step 1 is exact."""
    rng = np.random.default_rng(900 + r)
    offs = stencil_offsets(ndim, shape, r)
    w = rng.uniform(0, 0.3, len(offs))
    per = _bc_for(ndim, bc)
    u0, y, v = (rng.standard_normal(_shape(ndim)) for _ in range(3))
    T = 5
    loss, gu, gw, uT = adjoint(u0, y, offs, w, T, per)
    assert np.isclose(loss, _loss(u0, y, offs, w, T, per), rtol=1e-14)
    fd = (_loss(u0 + v, y, offs, w, T, per) - _loss(u0 - v, y, offs, w, T, per)) / 2.0
    assert abs(fd - np.vdot(gu, v)) <= 1e-11 * max(1.0, abs(fd))


def test_p8_central_fd_weights_c5_shape():
    """Central differences in every weight on the 32^3, T=128 instance of the
    7-point adjoint workload (O(h^2) error)."""
    offs = stencil_offsets(3, "star", 1)
    import workloads
    w = workloads.centre_arm_weights(offs, 0.4, [0.1])
    rng = np.random.default_rng(5)
    u0 = rng.random((32, 32, 32))
    y = sweep(u0, offs, workloads.perturbed(w, 50), 128, (0, 0, 0))
    T = 128
    loss, gu, gw, _ = adjoint(u0, y, offs, w, T, (0, 0, 0), ckpt=16)
    for k in range(len(w)):
        h = 1e-6 * abs(w[k])
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (_loss(u0, y, offs, wp, T, (0, 0, 0)) - _loss(u0, y, offs, wm, T, (0, 0, 0))) / (2 * h)
        assert abs(fd - gw[k]) <= 1e-6 * max(abs(gw).max(), 1e-30)


@pytest.mark.parametrize("ndim,shape,r", [(3, "star", 1), (3, "box", 1), (2, "box", 1), (3, "star", 2)])
@pytest.mark.parametrize("periodic", [False, True])
def test_p8_torch_autograd(ndim, shape, r, periodic):
    """Independent library reference: autograd through FP64 CPU conv3d."""
    torch = pytest.importorskip("torch")
    import torch.nn.functional as F
    rng = np.random.default_rng(950 + r)
    offs = stencil_offsets(ndim, shape, r)
    w = rng.uniform(0, 0.3, len(offs))
    shp = _shape(ndim)
    u0, y = rng.standard_normal(shp), rng.standard_normal(shp)
    T = 4
    per = _bc_for(ndim, (1, 1, 1) if periodic else (0, 0, 0))
    loss, gu, gw, _ = adjoint(u0, y, offs, w, T, per)
    wt = torch.tensor(w, requires_grad=True)
    ut = torch.tensor(_as3(u0), requires_grad=True)
    idx = [(o[0] + r) * (2 * r + 1) ** 2 + (o[1] + r) * (2 * r + 1) + (o[2] + r) for o in offs]
    K = torch.zeros((2 * r + 1) ** 3, dtype=torch.float64).index_put((torch.tensor(idx),), wt)
    K = K.reshape(1, 1, 2 * r + 1, 2 * r + 1, 2 * r + 1)
    x = ut[None, None]
    for _ in range(T):
        if periodic:
            if ndim == 2:
                xp = F.pad(x[:, :, 0], (r, r, r, r), mode="circular")[:, :, None]
                xp = F.pad(xp, (0, 0, 0, 0, r, r))
            else:
                xp = F.pad(x, (r,) * 6, mode="circular")
            x = F.conv3d(xp, K)
        else:
            x = F.conv3d(x, K, padding=r)
    L = 0.5 * ((x[0, 0] - torch.from_numpy(_as3(y))) ** 2).sum()
    L.backward()
    assert np.isclose(loss, L.item(), rtol=1e-13)
    assert np.allclose(_as3(gu), ut.grad.numpy(), rtol=1e-11, atol=1e-12)
    assert np.allclose(gw, wt.grad.numpy(), rtol=1e-11, atol=1e-12)


def test_p8_symmetric_special_case_and_checkpoints():
    """Symmetric weights under zero Dirichlet make the step matrix symmetric,
    so grad_u0 = A^T (A u0 - y) with A^T = A; and the checkpoint interval must
    not change any result."""
    offs = stencil_offsets(3, "star", 1)
    import workloads
    w = workloads.centre_arm_weights(offs, 0.4, [0.1])
    rng = np.random.default_rng(12)
    u0, y = rng.random((9, 10, 11)), rng.random((9, 10, 11))
    T = 10
    base = adjoint(u0, y, offs, w, T, (0, 0, 0), ckpt=0)
    ref = sweep(sweep(u0, offs, w, T) - y, offs, w, T)
    assert np.allclose(base[1], ref, rtol=1e-13, atol=1e-13)
    for c in (1, 3, 4, 10):
        other = adjoint(u0, y, offs, w, T, (0, 0, 0), ckpt=c)
        assert other[0] == base[0]
        assert np.array_equal(other[1], base[1])
        assert np.array_equal(other[2], base[2])


# ---------------------------------------------------------------- golden
def test_table3_point_counts():
    """Point counts and flops per element of the paper's benchmarks."""
    g = json.load(open(os.path.join(HERE, "golden", "table3_benchmarks.json")))
    for row in g["box2d"]:
        offs = stencil_offsets(2, "box", row["radius"])
        assert len(offs) == row["points"]
        assert 2 * len(offs) - 1 == row["flops_per_element"]
    assert len(stencil_offsets(2, "star", 1)) == g["gradient2d"]["points"]
    # the stated in-core / out-of-core sizes are two FP32 arrays, in GiB
    for key, gb in (("in_core", "in_core_total_GB"), ("out_of_core", "out_of_core_total_GB")):
        n = g["sizes"][key][0]
        assert round(2 * n * n * 4 / 2 ** 30, 1) == g["sizes"][gb]
