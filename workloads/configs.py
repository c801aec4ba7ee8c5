"""The five workloads the library is measured and checked on.  Shapes are
(nx, ny, nz) with x contiguous and the last axis cut into chunks; a 2D grid has
nz = 1 and is cut along y.  Budgets are in bytes (GiB = 2^30)."""
from dataclasses import dataclass, field as _dc_field

MiB = 1 << 20
GiB = 1 << 30


@dataclass(frozen=True)
class Workload:
    name: str
    ndim: int
    nx: int
    ny: int
    nz: int
    shape: str            # "star" | "box"
    radius: int
    T: int
    tb_depth: int         # steps per HBM residency
    n_chunks: int
    budget: int           # device bytes
    periodic: tuple = (0, 0, 0)   # per axis x, y, z
    seed: int = 0
    init: str = "uniform"         # initial field recipe: uniform | fourier | bump
    weights: str = ""             # recipe tag, see describe()
    dtypes: tuple = ("f32",)
    notes: str = ""
    extra: dict = _dc_field(default_factory=dict)

    @property
    def cells(self):
        return self.nx * self.ny * self.nz


CONFIGS = {
    "c1_2d5pt": Workload(
        "c1_2d5pt", 2, 1024, 1024, 1, "star", 1, T=16, tb_depth=4, n_chunks=4,
        budget=4 * MiB, seed=1, init="uniform", weights="const:0.2",
        dtypes=("f32", "f64"),
        notes="2D 5-point Jacobi, zero Dirichlet, 4 row chunks, TB depth 4, 4 MiB budget"),
    "c2_3d7pt": Workload(
        "c2_3d7pt", 3, 2048, 1024, 1024, "star", 1, T=64, tb_depth=8, n_chunks=16,
        budget=4 * GiB, seed=2, init="uniform", weights="centre_arm:0.4:0.1",
        notes="3D 7-point star, zero Dirichlet, 8 GiB per FP32 buffer, 4 GiB budget"),
    "c3_3d27pt": Workload(
        "c3_3d27pt", 3, 2048, 1024, 1024, "box", 1, T=32, tb_depth=4, n_chunks=16,
        budget=4 * GiB, periodic=(1, 1, 0), seed=3, init="fourier", weights="random_box",
        notes="3D 27-point box, random positive weights summing to 1, periodic x/y"),
    "c4_3d13pt": Workload(
        "c4_3d13pt", 3, 2048, 2048, 2048, "star", 2, T=64, tb_depth=8, n_chunks=32,
        budget=8 * GiB, seed=4, init="bump", weights="centre_arm:0.28:0.1:0.02",
        dtypes=("f32", "bf16", "f16"),
        notes="3D 13-point radius-2 star; BF16/FP16 storage vs FP32"),
    "c5_adjoint": Workload(
        "c5_adjoint", 3, 1024, 1024, 1024, "star", 1, T=128, tb_depth=8, n_chunks=0,
        budget=2 * GiB, seed=5, init="uniform", weights="centre_arm:0.4:0.1",
        notes="adjoint of the 7-point sweep, checkpoints every 16 steps",
        extra={"ckpt_every": 16, "target_seed": 50}),
}


# The paper's benchmark family (Table III): box2d{x}r, x = 1..4, FP32, out of
# core at 38400^2 (two arrays = 11.0 GB), 640 steps, 4 chunks, S_TB chosen per
# radius as in Sec. V-B (160, 160, 80, 40), on a 10 GB device.  The stencil
# coefficients of the paper's generator are not given, so the weights are
# random positive values normalised to 1 (seeded); input U[0, 1).
PAPER_S_TB = {1: 160, 2: 160, 3: 80, 4: 40}
for _r in (1, 2, 3, 4):
    CONFIGS[f"paper_box2d{_r}r"] = Workload(
        f"paper_box2d{_r}r", 2, 38400, 38400, 1, "box", _r, T=640, tb_depth=PAPER_S_TB[_r],
        n_chunks=4, budget=10 * 10 ** 9, seed=100 + _r, init="uniform", weights="random_box",
        notes="paper out-of-core dataset (Table III), S_TB as in Sec. V-B")
    CONFIGS[f"paper_box2d{_r}r_incore"] = Workload(
        f"paper_box2d{_r}r_incore", 2, 12800, 12800, 1, "box", _r, T=640, tb_depth=PAPER_S_TB[_r],
        n_chunks=4, budget=10 * 10 ** 9, seed=200 + _r, init="uniform", weights="random_box",
        notes="paper in-core dataset (Table III), chunked like the out-of-core runs")
