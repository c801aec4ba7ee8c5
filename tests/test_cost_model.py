"""The cost model and the model-driven planner (so2dr_plan_predict,
so2dr_plan_suggest): bounds every schedule must respect, monotonicity in the
machine figures, and the planner's contract (fixed fields kept, budget
respected, never worse than a given plan).  Host-only."""
import math

import pytest

from paper_2309_08864_amd import Plan, So2drError, stencil_offsets, suggest

GiB = 1 << 30


def _base(**kw):
    offs = stencil_offsets(3, "star", 1)
    b = dict(ndim=3, nx=2048, ny=1024, nz=1024, shape="star", radius=1,
             weights=[1.0 / len(offs)] * len(offs), T=64, budget=4 * GiB)
    b.update(kw)
    return b


def _bounds(p, m):
    """Link-only lower bound and fully serial upper bound of a plan's run."""
    info = p.info()
    pb = info["plane_elems"] * 4
    h2d = d2h = kern = d2d = 0.0
    for op in p.ops():
        n = (op["z1"] - op["z0"]) * pb
        if op["kind"] == "H2D":
            h2d += n
        elif op["kind"] == "D2H":
            d2h += n
        elif op["kind"] == "KERNEL":
            kern += m["launch_us"] * 1e-6 + (op["z1"] - op["z0"]) * info["plane_elems"] * op["levels"] / (
                m["gupd"][op["levels"] - 1] * 1e9)
        else:
            d2d += 2 * n / (m["d2d_gbps"] * 1e9) + m["launch_us"] * 1e-6
    lower = max((h2d + d2h) / (m["duplex_gbps"] * 1e9), h2d / (m["h2d_gbps"] * 1e9),
                d2h / (m["d2h_gbps"] * 1e9), kern)
    upper = h2d / (0.5 * m["duplex_gbps"] * 1e9) + d2h / (0.5 * m["duplex_gbps"] * 1e9) + kern + d2d
    return 1e3 * lower, 1e3 * upper


@pytest.mark.parametrize("K,d,k_on", [(8, 16, 3), (8, 16, 1), (4, 32, 2), (16, 8, 4), (64, 1, 3)])
def test_prediction_between_link_and_serial_bounds(K, d, k_on):
    p = Plan(tb_depth=K, n_chunks=d, k_on=k_on, **_base(budget=24 * GiB))
    m = p.machine()
    lo, hi = _bounds(p, m)
    t = p.predict()
    assert lo * (1 - 1e-9) <= t <= hi * (1 + 1e-9), (lo, t, hi)


def test_prediction_monotone_in_machine_figures():
    p = Plan(tb_depth=8, n_chunks=16, **_base())
    m = p.machine()
    t = p.predict()
    fast_link = dict(m, h2d_gbps=2 * m["h2d_gbps"], d2h_gbps=2 * m["d2h_gbps"],
                     duplex_gbps=2 * m["duplex_gbps"])
    slow_kern = dict(m, gupd=[g / 10 for g in m["gupd"]])
    assert p.predict(machine=fast_link) < t < p.predict(machine=slow_kern)
    # this plan is link-bound: the link-only bound is within 5 %
    lo, _ = _bounds(p, m)
    assert t <= 1.05 * lo


def test_suggest_keeps_fixed_fields_and_fits_the_budget():
    kw, ms = suggest(**_base(tb_depth=8))
    assert kw["tb_depth"] == 8 and kw["n_chunks"] >= 1 and kw["k_on"] >= 1
    p = Plan(**kw)
    assert p.info()["workspace_bytes"] <= 4 * GiB
    assert math.isclose(p.predict(), ms, rel_tol=1e-9)
    hand = Plan(tb_depth=8, n_chunks=16, **_base()).predict()
    assert ms <= hand * 1.01   # the search keeps fewer chunks or levels on a 1 % tie


def test_suggest_free_depth_beats_fixed_depth_when_link_bound():
    """With K free the planner trades redundant halo work for fewer round
    trips over the link (the S_TB trade-off of Sec. V-B)."""
    kw8, ms8 = suggest(**_base(tb_depth=8))
    kw, ms = suggest(**_base())
    assert ms <= ms8 and kw["tb_depth"] >= 8


def test_suggest_fuses_when_kernels_bind():
    b = _base()
    m = Plan(tb_depth=8, n_chunks=16, **b).machine()
    slow = dict(m, gupd=[g / 50 for g in m["gupd"]])   # kernels far slower than the link
    kw, _ = suggest(machine=slow, **dict(b, tb_depth=8, n_chunks=16))
    assert kw["k_on"] >= 3
    resreu, _ = suggest(machine=slow, **dict(b, tb_depth=8, n_chunks=16, method="resreu"))
    assert resreu["k_on"] == 1


def test_suggest_reports_budget_failure():
    with pytest.raises(So2drError) as e:
        suggest(**_base(budget=1 << 20))
    assert "E_BUDGET" in str(e.value)
