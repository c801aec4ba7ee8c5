"""Bit-for-bit parity of every fused-kernel shape the launcher picks, on
grids large enough that most workgroups take the kernels' interior path.

The march kernels run a second copy of their loop, without ghost handling,
in every workgroup whose tile and plane segment touch no Dirichlet boundary;
at the workloads' sizes that copy computes almost every cell.  These grids
have at least three fully interior tiles along each in-plane axis for every
tile shape (3D: 1032 x 160 with 224-, 240-, 248- or 120-column and 26- to
42-row output tiles; 2D: 4100-cell rows with 248- or 240-cell tiles) and chunks long enough
to be cut into several plane segments, so the interior copy, the boundary
copy and their seams are all exercised.  The launcher's choice per fused
depth (launch_any): 3D single steps (16 waves, 2 rows, 4 cells per lane);
two fused steps of the 7-point star (8, 4, 4); three of the 7-point star and
two of the 13-point star (8, 6, 2); the other depths and the 27-point box
(8, 4, 2); 2D rows with unrolled sums, and with shifted sums for the widest
boxes (radius 4, and radius 3 at two levels).  Each case runs out of core
(two chunks, two rounds of k_on steps) and is compared with the C model of
the documented arithmetic (oracle/emulator_bits.c) bit for bit, for 16-bit
storage also with rounding only where a launch stores; FP64 storage,
which that model does not cover, against the FP64 oracle and bit for bit
against its own in-core run."""
import numpy as np
import pytest

import oracle
import torch

from helpers import fp32_weights, gpu_run, np_shape, rel_l2, to_storage

pytestmark = pytest.mark.gpu

CASES_3D = [("star", 1, 1), ("star", 1, 2), ("star", 1, 3), ("star", 1, 4), ("star", 2, 1),
            ("star", 2, 2), ("box", 1, 1), ("box", 1, 2), ("box", 1, 3)]
CASES_2D = [("star", 1, 4), ("star", 1, 8), ("box", 1, 4), ("box", 2, 2), ("box", 3, 1),
            ("box", 3, 2), ("box", 4, 1)]


def _run_case(ndim, shape, r, k_on, storage, bc=(0, 0, 0), rounding="every_step"):
    from oracle import emulator
    from paper_2309_08864_amd import Plan, So2drError
    nx, ny, nz = (1032, 160, 120) if ndim == 3 else (4100, 200, 1)
    rng = np.random.default_rng(1000 + 100 * ndim + 10 * r + k_on)
    offs = oracle.stencil_offsets(ndim, shape, r)
    w = rng.uniform(-1.0, 1.0, len(offs))
    w = fp32_weights(w / np.abs(w).sum())
    u0 = rng.standard_normal(np_shape(ndim, nx, ny, nz))
    us = to_storage(u0, storage)
    T = 2 * k_on
    kw = dict(ndim=ndim, nx=nx, ny=ny, nz=nz, shape=shape, radius=r, weights=list(w), T=T,
              tb_depth=k_on, n_chunks=2, k_on=k_on, budget=1 << 30, storage=storage, bc=bc,
              rounding=rounding)
    try:
        Plan(**kw).close()
    except So2drError as e:
        if "E_UNSUPPORTED" in str(e):
            pytest.skip(f"{storage} not built for the {ndim}D {shape} r={r} stencil at depth {k_on}")
        raise
    print(f"[{storage} {rounding} {ndim}D {shape} r={r} k_on={k_on} bc={bc}] {nx}x{ny}x{nz}", flush=True)
    got, st, info = gpu_run(kw, us)
    assert info["k_on"] == k_on and info["n_chunks"] == 2
    assert st["kernel_launches"] == 4
    ra = None
    if rounding == "at_store":
        from helpers import store_steps
        ra = store_steps(T, k_on, k_on)
    model = emulator.sweep_bits_c(us.float().numpy(), offs, w, T, storage, bc, round_after=ra)
    g = np.ascontiguousarray(got.float().numpy())
    diff = int(np.sum(g.view(np.uint32) != model.view(np.uint32)))
    print(f"    cells differing from the model: {diff} of {g.size}", flush=True)
    assert diff == 0


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("shape,r,k_on", CASES_3D)
def test_interior_tiles_3d_bit_exact(shape, r, k_on, storage):
    _run_case(3, shape, r, k_on, storage)


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("shape,r,k_on", CASES_2D)
def test_interior_tiles_2d_bit_exact(shape, r, k_on, storage):
    _run_case(2, shape, r, k_on, storage)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("shape,r,k_on", [("box", 1, 2), ("star", 1, 3), ("star", 2, 2)])
def test_interior_tiles_periodic_xy_bit_exact(shape, r, k_on, storage):
    """Periodic in-plane axes: edge tiles read wrapped columns and rows but
    hold no ghosts, so every workgroup away from the cut axis's ends runs
    the interior copy."""
    _run_case(3, shape, r, k_on, storage, bc=(1, 1, 0))


@pytest.mark.parametrize("shape,r,k_on", [("star", 1, 1), ("star", 1, 2), ("star", 2, 1), ("star", 2, 2),
                                          ("box", 1, 1), ("box", 1, 2)])
def test_interior_tiles_3d_f64(shape, r, k_on):
    """FP64 storage and sums (single steps in the 2 KiB-row tiles with a
    64-byte x halo, two steps in the 4-row tiles): out of core equals in
    core bit for bit, and both are within FP64 rounding of the oracle."""
    nx, ny, nz = 1032, 160, 120
    rng = np.random.default_rng(2000 + 10 * r + k_on)
    offs = oracle.stencil_offsets(3, shape, r)
    w = rng.uniform(-1.0, 1.0, len(offs))
    w = w / np.abs(w).sum()
    u0 = rng.standard_normal((nz, ny, nx))
    us = to_storage(u0, "f64")
    T = 2 * k_on
    kw = dict(ndim=3, nx=nx, ny=ny, nz=nz, shape=shape, radius=r, weights=list(w), T=T,
              tb_depth=k_on, n_chunks=2, k_on=k_on, budget=1 << 30, storage="f64")
    print(f"[f64 3D {shape} r={r} k_on={k_on}] {nx}x{ny}x{nz}", flush=True)
    got, st, info = gpu_run(kw, us)
    assert info["k_on"] == k_on and info["n_chunks"] == 2 and st["kernel_launches"] == 4
    incore, _, _ = gpu_run(dict(kw, tb_depth=T, n_chunks=1, k_on=k_on), us)
    assert torch.equal(got, incore)
    ref = oracle.sweep(u0, offs, w, T)
    assert rel_l2(got.numpy(), ref) <= 1e-13


@pytest.mark.parametrize("storage", ["bf16", "f16"])
@pytest.mark.parametrize("ndim,shape,r,k_on", [(3, "star", 1, 2), (3, "star", 1, 3), (3, "star", 2, 2),
                                               (3, "box", 1, 2), (2, "star", 1, 4), (2, "box", 2, 2)])
def test_interior_tiles_round_at_store(ndim, shape, r, k_on, storage):
    """16-bit storage rounded only where a launch stores (the levels inside a
    launch keep FP32 sums): bit for bit against the C model run with the
    same store schedule, on the interior-tile grids."""
    _run_case(ndim, shape, r, k_on, storage, rounding="at_store")
