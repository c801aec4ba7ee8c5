"""Pins for the bit-exact arithmetic model (oracle/emulator.py): its fused
multiply-add against exact rational rounding (including operands built so the
float64 sum lands exactly on a float32 midpoint), its BF16/FP16 rounding
against torch's conversions, and its sweep against the FP64 oracle."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import emulator as em


def _round_f32_exact(q):
    """Nearest-even float32 of the rational q."""
    f = np.float32(float(q))
    cands = [np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))]
    best = None
    for c in cands:
        d = abs(Fraction(float(c)) - q)
        key = (d, int(np.array(c, np.float32).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, c)
    return np.float32(best[1])


def test_fma32_random_and_midpoints():
    rng = np.random.default_rng(0)
    a = rng.standard_normal(3000).astype(np.float32)
    b = rng.standard_normal(3000).astype(np.float32)
    c = (rng.standard_normal(3000) * np.exp2(rng.integers(-30, 5, 3000))).astype(np.float32)
    # midpoint constructions: (1 + 2^-12)^2 = 1 + 2^-11 + 2^-24 sits halfway
    # between two float32 values; a tiny c decides the direction
    ma = np.float32(1 + 2.0 ** -12)
    extra_a = np.array([ma] * 4, np.float32)
    extra_b = np.array([ma] * 4, np.float32)
    extra_c = np.array([2.0 ** -60, -2.0 ** -60, 0.0, 2.0 ** -100], np.float32)
    a = np.concatenate([a, extra_a, -extra_a])
    b = np.concatenate([b, extra_b, extra_b])
    c = np.concatenate([c, extra_c, -extra_c])
    got = em.fma32(a, b, c)
    for i in range(len(a)):
        exact = Fraction(float(a[i])) * Fraction(float(b[i])) + Fraction(float(c[i]))
        want = _round_f32_exact(exact)
        assert got[i].view(np.uint32) == want.view(np.uint32) or (got[i] == 0 and want == 0), i
    # the constructed cases really are midpoint cases that plain double
    # rounding gets wrong for one direction
    naive = (extra_a.astype(np.float64) * extra_b + extra_c.astype(np.float64)).astype(np.float32)
    assert naive[0] != em.fma32(extra_a[:1], extra_b[:1], extra_c[:1])[0]


def test_storage_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(200000) * np.exp2(rng.integers(-20, 20, 200000))).astype(np.float32)
    # include exact ties of both kinds
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11], np.float32)
    x = np.concatenate([x, ties, -ties])
    tb = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    th = torch.from_numpy(x).to(torch.float16).float().numpy()
    assert np.array_equal(em.round_bf16(x).view(np.uint32), tb.view(np.uint32))
    assert np.array_equal(em.round_f16(x).view(np.uint32), th.view(np.uint32))


@pytest.mark.parametrize("ndim,shape,r", [(3, "star", 1), (3, "box", 1), (2, "box", 2), (3, "star", 2)])
def test_sweep_bits_vs_oracle(ndim, shape, r):
    rng = np.random.default_rng(2 + r)
    offs = oracle.stencil_offsets(ndim, shape, r)
    w = rng.uniform(0.1, 1, len(offs))
    w /= w.sum()
    w32 = w.astype(np.float32).astype(np.float64)
    shp = (9, 8, 7) if ndim == 3 else (11, 10)
    u0 = rng.random(shp).astype(np.float32)
    T = 5
    got = em.sweep_bits(u0, offs, w32, T)
    ref = oracle.sweep(u0.astype(np.float64), offs, w32, T)
    assert np.max(np.abs(got - ref)) <= T * len(offs) * 2.0 ** -24 * 2
    # dyadic weights and inputs: FP32 is exact, so the bits equal the oracle's
    wd = rng.integers(1, 8, len(offs)) / 64.0
    ud = (rng.integers(0, 256, shp) / 256.0).astype(np.float32)
    got = em.sweep_bits(ud, offs, wd, 2)
    ref = oracle.sweep(ud.astype(np.float64), offs, wd, 2)
    assert np.array_equal(got.astype(np.float64), ref)
    # bf16: every stored value is a bf16 value
    ub = em.round_bf16(u0)
    gb = em.sweep_bits(ub, offs, w32, T, "bf16")
    assert np.array_equal(gb, em.round_bf16(gb))


def test_round_after_schedule_semantics():
    """round_after: no rounding equals the FP32 sweep; rounding only after the
    last step equals the rounded FP32 sweep; a schedule {2, T} equals two
    FP32 sweeps with a rounding after each; every step equals the default."""
    rng = np.random.default_rng(9)
    offs = oracle.stencil_offsets(3, "star", 1)
    w = rng.uniform(0.1, 1, len(offs))
    w32 = (w / w.sum()).astype(np.float32).astype(np.float64)
    u0 = em.round_bf16(rng.random((6, 7, 8)).astype(np.float32))
    T = 4
    f32 = em.sweep_bits(u0, offs, w32, T, "f32")
    assert np.array_equal(em.sweep_bits(u0, offs, w32, T, "bf16", round_after=set()), f32)
    assert np.array_equal(em.sweep_bits(u0, offs, w32, T, "bf16", round_after={T}), em.round_bf16(f32))
    half = em.round_bf16(em.sweep_bits(u0, offs, w32, 2, "f32"))
    two = em.round_bf16(em.sweep_bits(half, offs, w32, 2, "f32"))
    assert np.array_equal(em.sweep_bits(u0, offs, w32, T, "bf16", round_after={2, T}), two)
    assert np.array_equal(em.sweep_bits(u0, offs, w32, T, "bf16", round_after=set(range(1, T + 1))),
                          em.sweep_bits(u0, offs, w32, T, "bf16"))


def test_store_steps_schedule():
    """The documented store schedule: one store per launch of k_on steps inside
    each round of K steps, one for a round's remainder (hand-worked cases)."""
    from helpers import store_steps
    assert store_steps(10, 4, 2) == {2, 4, 6, 8, 10}
    assert store_steps(10, 4, 3) == {3, 4, 7, 8, 10}
    assert store_steps(7, 3, 3) == {3, 6, 7}
    assert store_steps(5, 8, 2) == {2, 4, 5}
    assert store_steps(6, 6, 1) == {1, 2, 3, 4, 5, 6}


# ------------------------------------------------- C model (emulator_bits.c)

def _fma_through_c(a, b, c):
    """fma(a, b, c) per element through the C model: a 1D grid holding c_i,
    b_i in cells 2i, 2i+1 and the stencil {dx = -1: weight 1, dx = 0: weight
    a} gives cell 2i + 1 the chain fma(a, b_i, fma(1, c_i, +0)) =
    fma(a, b_i, c_i)."""
    n = len(b)
    u = np.empty(2 * n, np.float32)
    u[0::2], u[1::2] = c, b
    out = em.sweep_bits_c(u.reshape(1, 1, -1), [(0, 0, -1), (0, 0, 0)], [1.0, float(a)], 1)
    return out.reshape(-1)[1::2]


def test_c_model_fma_against_exact_rationals():
    rng = np.random.default_rng(20)
    for a in (np.float32(1 + 2.0 ** -12), np.float32(-0.3712), np.float32(3.0e-5)):
        b = rng.standard_normal(1500).astype(np.float32)
        c = (rng.standard_normal(1500) * np.exp2(rng.integers(-30, 5, 1500))).astype(np.float32)
        if a == np.float32(1 + 2.0 ** -12):   # the float64 sum lands on a float32 midpoint
            b[:4] = a
            c[:4] = np.array([2.0 ** -60, -2.0 ** -60, 0.0, 2.0 ** -100], np.float32)
        got = _fma_through_c(a, b, c)
        for i in range(len(b)):
            exact = Fraction(float(a)) * Fraction(float(b[i])) + Fraction(float(c[i]))
            want = _round_f32_exact(exact)
            assert got[i].view(np.uint32) == want.view(np.uint32) or (got[i] == 0 and want == 0), (a, i)


def test_c_model_storage_rounding_matches_torch():
    """One step of the identity stencil rounds every value to storage: the C
    model's BF16 and FP16 rounding against torch's conversions, over normal,
    subnormal, tie and overflowing values."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(21)
    x = (rng.standard_normal(100000) * np.exp2(rng.integers(-30, 20, 100000))).astype(np.float32)
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11,
                     65504.0, 65519.0, 65520.0, 70000.0, 2.0 ** -24, 1.5 * 2.0 ** -24,
                     2.0 ** -25, 3 * 2.0 ** -26, 2.0 ** -14 * (1 - 2.0 ** -11)], np.float32)
    x = np.concatenate([x, ties, -ties, np.zeros(1, np.float32)])
    for storage, tdt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        got = em.sweep_bits_c(x.reshape(1, 1, -1), [(0, 0, 0)], [1.0], 1, storage)
        want = torch.from_numpy(x).to(tdt).float().numpy()
        assert np.array_equal(got.reshape(-1).view(np.uint32), want.view(np.uint32)), storage


@pytest.mark.parametrize("ndim,shape,r", [(3, "star", 1), (3, "star", 2), (3, "box", 1),
                                          (2, "star", 1), (2, "box", 2), (2, "box", 4)])
def test_c_model_equals_numpy_model(ndim, shape, r):
    """The C model's bits equal the NumPy model's (which the exact-rational
    pins above fix) for every storage type, boundary mix and rounding
    schedule, with signed weights."""
    rng = np.random.default_rng(30 + 3 * r + ndim)
    offs = oracle.stencil_offsets(ndim, shape, r)
    w = rng.uniform(-1, 1, len(offs))
    w = (w / np.abs(w).sum()).astype(np.float32).astype(np.float64)
    shp = (7, 9, 11) if ndim == 3 else (13, 12)
    for storage in ("f32", "bf16", "f16"):
        u0 = em._ROUND[storage](rng.standard_normal(shp).astype(np.float32))
        for per in ((0, 0, 0), (1, 1, 0), (1, 0, 1)):
            for ra in (None, {2, 5}):
                a = em.sweep_bits(u0, offs, w, 5, storage, per, round_after=ra)
                b = em.sweep_bits_c(u0, offs, w, 5, storage, per, round_after=ra)
                assert a.shape == b.shape
                assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (storage, per, ra)


@pytest.mark.parametrize("shape,r,per", [("star", 1, (0, 0, 0)), ("star", 2, (1, 1, 0)),
                                         ("box", 1, (1, 0, 0))])
def test_c_model_box_equals_whole_grid(shape, r, per):
    """Light cone: the sub-box model equals the whole-grid model on boxes at
    corners, edges and inside, for FP32 and BF16."""
    rng = np.random.default_rng(40 + r)
    offs = oracle.stencil_offsets(3, shape, r)
    w = rng.uniform(0.1, 1, len(offs))
    w = (w / w.sum()).astype(np.float32).astype(np.float64)
    shp = (23, 19, 29)
    T = 4
    for storage in ("f32", "bf16"):
        u0 = em._ROUND[storage](rng.random(shp).astype(np.float32))
        full = em.sweep_bits_c(u0, offs, w, T, storage, per)
        for lo in ((0, 0, 0), (26, 16, 20), (10, 0, 9), (5, 7, 11)):
            hi = tuple(min(a + 3, n) for a, n in zip(lo, (29, 19, 23)))
            box = em.sweep_bits_box_from_field(u0, offs, w, T, lo, hi, storage, per)
            want = full[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
            assert np.array_equal(box.view(np.uint32), want.view(np.uint32)), (storage, lo)
