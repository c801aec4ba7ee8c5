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
