"""ctypes view of the C interface declared in include/so2dr.h.

Argument marshalling only: every step of the sweep runs inside libso2dr.so.
Loading fails loudly when the library has not been built."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libso2dr.so")

OK, E_INVALID, E_BUDGET, E_UNSUPPORTED, E_NOT_PINNED, E_HIP, E_UNBOUND = 0, -1, -2, -3, -4, -5, -6
ERROR_NAMES = {E_INVALID: "E_INVALID", E_BUDGET: "E_BUDGET", E_UNSUPPORTED: "E_UNSUPPORTED",
               E_NOT_PINNED: "E_NOT_PINNED", E_HIP: "E_HIP", E_UNBOUND: "E_UNBOUND"}
DTYPES = {"f32": 0, "f64": 1, "bf16": 2, "f16": 3}
SHAPES = {"star": 0, "box": 1}
METHODS = {"so2dr": 0, "resreu": 1}
ROUNDING = {"every_step": 0, "at_store": 1}
COPY_ENGINES = {"auto": 0, "dma": 1, "kernel": 2, "kernel_out": 3}
OP_KINDS = {0: "H2D", 1: "RS_READ", 2: "RS_WRITE", 3: "KERNEL", 4: "D2H"}

# Symbols the header declares; the CPU test checks each is exported.
EXPORTS = ["so2dr_plan_create", "so2dr_plan_destroy", "so2dr_plan_get_info",
           "so2dr_plan_workspace_bytes", "so2dr_plan_get_ops", "so2dr_plan_bind",
           "so2dr_plan_set_timing", "so2dr_run", "so2dr_run_steps", "so2dr_adjoint_run",
           "so2dr_last_error", "so2dr_version", "so2dr_machine_default", "so2dr_plan_predict",
           "so2dr_plan_suggest", "so2dr_host_alloc", "so2dr_host_free", "so2dr_run_noalloc",
           "so2dr_plan_get_deps", "so2dr_kernel_bench", "so2dr_plan_set_fail_after",
           "so2dr_link_probe"]

MAX_WAITS = 4   # SO2DR_MAX_WAITS

# SO2DR_NOALLOC_MAX_BYTES: the static device workspace of so2dr_run_noalloc.
NOALLOC_MAX_BYTES = 128 << 20


class Desc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("nz", ctypes.c_int64), ("shape", ctypes.c_int), ("radius", ctypes.c_int),
                ("weights", ctypes.POINTER(ctypes.c_double)), ("n_weights", ctypes.c_int),
                ("bc", ctypes.c_int * 3), ("storage", ctypes.c_int), ("T", ctypes.c_int),
                ("n_chunks", ctypes.c_int), ("tb_depth", ctypes.c_int), ("k_on", ctypes.c_int),
                ("n_slots", ctypes.c_int), ("device_budget_bytes", ctypes.c_size_t),
                ("adjoint", ctypes.c_int), ("method", ctypes.c_int), ("rounding", ctypes.c_int),
                ("copy_engine", ctypes.c_int)]


class Machine(ctypes.Structure):
    _fields_ = [("h2d_gbps", ctypes.c_double), ("d2h_gbps", ctypes.c_double),
                ("duplex_gbps", ctypes.c_double), ("d2d_gbps", ctypes.c_double),
                ("launch_us", ctypes.c_double), ("gupd", ctypes.c_double * 8),
                ("kcopy_gbps", ctypes.c_double), ("kcopy_out_gbps", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_axis", ctypes.c_int64), ("plane_elems", ctypes.c_int64),
                ("n_chunks", ctypes.c_int), ("tb_depth", ctypes.c_int), ("k_on", ctypes.c_int),
                ("n_slots", ctypes.c_int), ("n_rounds", ctypes.c_int),
                ("max_chunk_planes", ctypes.c_int), ("slot_planes", ctypes.c_int),
                ("max_k_on", ctypes.c_int), ("workspace_bytes", ctypes.c_size_t),
                ("slot_bytes", ctypes.c_size_t), ("rs_bytes", ctypes.c_size_t),
                ("scratch_bytes", ctypes.c_size_t), ("lean", ctypes.c_int),
                ("lean_block", ctypes.c_int), ("method", ctypes.c_int),
                ("redundant_fraction", ctypes.c_double),
                ("n_ops", ctypes.c_int64), ("rounding", ctypes.c_int), ("copy_engine", ctypes.c_int)]


class Op(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("round", ctypes.c_int), ("chunk", ctypes.c_int),
                ("slot", ctypes.c_int), ("z0", ctypes.c_int64), ("z1", ctypes.c_int64),
                ("in_z0", ctypes.c_int64), ("in_z1", ctypes.c_int64), ("level_in", ctypes.c_int),
                ("levels", ctypes.c_int), ("buf_in", ctypes.c_int), ("buf_out", ctypes.c_int),
                ("buf_z0", ctypes.c_int64), ("out_z0", ctypes.c_int64),
                ("pool_off", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("wall_ms", ctypes.c_double), ("h2d_ms", ctypes.c_double),
                ("d2h_ms", ctypes.c_double), ("d2d_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("bytes_h2d", ctypes.c_uint64),
                ("bytes_d2h", ctypes.c_uint64), ("bytes_d2d", ctypes.c_uint64),
                ("kernel_launches", ctypes.c_uint64), ("cell_updates", ctypes.c_uint64),
                ("cell_updates_done", ctypes.c_uint64), ("kernel_alg_bytes", ctypes.c_uint64),
                ("rounds_done", ctypes.c_int), ("kernel_ms_by_levels", ctypes.c_double * 8),
                ("launches_by_levels", ctypes.c_uint64 * 8),
                ("alg_bytes_by_levels", ctypes.c_uint64 * 8)]

    def as_dict(self):
        return {k: (list(getattr(self, k)) if k.endswith("_by_levels") else getattr(self, k))
                for k, _ in self._fields_}


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2309_08864_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        L.so2dr_plan_create.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(vp)]
        L.so2dr_plan_destroy.argtypes = [vp]
        L.so2dr_plan_destroy.restype = None
        L.so2dr_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.so2dr_plan_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.so2dr_plan_get_ops.argtypes = [vp, ctypes.POINTER(Op), i64]
        L.so2dr_plan_get_deps.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(i64), i64]
        L.so2dr_kernel_bench.argtypes = [vp, i32, vp, vp, i64, i32, vp,
                                         ctypes.POINTER(ctypes.c_double)]
        L.so2dr_plan_bind.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(vp), i32]
        L.so2dr_plan_set_timing.argtypes = [vp, i32]
        L.so2dr_plan_set_fail_after.argtypes = [vp, i64]
        L.so2dr_link_probe.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, i32, vp, vp, i32,
                                       ctypes.POINTER(ctypes.c_double)]
        L.so2dr_run.argtypes = [vp, vp, ctypes.POINTER(Stats)]
        L.so2dr_run_noalloc.argtypes = [vp, vp, ctypes.POINTER(vp), i32, ctypes.POINTER(Stats)]
        L.so2dr_run_steps.argtypes = [vp, vp, vp, i32, ctypes.POINTER(Stats)]
        L.so2dr_adjoint_run.argtypes = [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(vp),
                                        i32, ctypes.POINTER(Stats)]
        L.so2dr_machine_default.argtypes = [vp, ctypes.POINTER(Machine)]
        L.so2dr_plan_predict.argtypes = [vp, ctypes.POINTER(Machine), i32,
                                         ctypes.POINTER(ctypes.c_double)]
        L.so2dr_plan_suggest.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(Machine),
                                         ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_double)]
        L.so2dr_host_alloc.argtypes = [ctypes.c_size_t, ctypes.POINTER(vp)]
        L.so2dr_host_free.argtypes = [vp]
        L.so2dr_last_error.restype = ctypes.c_char_p
        L.so2dr_version.restype = ctypes.c_char_p
        for f in ("so2dr_plan_create", "so2dr_plan_get_info", "so2dr_plan_workspace_bytes",
                  "so2dr_plan_get_ops", "so2dr_plan_bind", "so2dr_plan_set_timing", "so2dr_run",
                  "so2dr_run_steps", "so2dr_adjoint_run", "so2dr_machine_default",
                  "so2dr_plan_predict", "so2dr_plan_suggest", "so2dr_host_alloc",
                  "so2dr_host_free", "so2dr_run_noalloc", "so2dr_plan_get_deps",
                  "so2dr_kernel_bench", "so2dr_plan_set_fail_after", "so2dr_link_probe"):
            getattr(L, f).restype = i32
        _LIB = L
    return _LIB


class So2drError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(rc):
    if rc != 0:
        raise So2drError(rc, lib().so2dr_last_error().decode())
    return rc
