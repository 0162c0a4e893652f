"""ctypes binding of ``libstencil.so`` (C ABI in ``include/stencil.h``).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library. Functions keep the C names; ``Plan`` and ``run`` are
thin conveniences over them for torch tensors (device memory and streams come
from PyTorch). Importing this module does not load the library; the first call
does, and raises ``StencilLibraryMissing`` when it has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstencil.so")

STENCIL_OK = 0
STENCIL_ERR_INVALID = -1
STENCIL_ERR_UNSUPPORTED = -2
STENCIL_ERR_ALIAS = -3
STENCIL_ERR_NOMEM = -4
STENCIL_ERR_DEVICE = -5
STENCIL_ERR_BUDGET = -6
STENCIL_ERR_TIMEOUT = -7

STENCIL_F32 = 0
STENCIL_F64 = 1

STENCIL_FLAG_NAIVE = 1
STENCIL_FLAG_NO_CACHE = 2
STENCIL_FLAG_PERSISTENT = 4
STENCIL_FLAG_UNIFORM_TILES = 8
STENCIL_FLAG_DEVICE_TILING = 16
STENCIL_FLAG_OVERLAPPED_TILING = 32

STENCIL_TUNE_BATCH = 1
STENCIL_TUNE_FORCE = 2

TUNE_CACHE_PATH = os.path.join(HERE, "tune_cache.json")

SCHEME_NAMES = {0: "copy", 1: "naive", 2: "blocked_2d", 3: "blocked_3d", 4: "device_3d"}
PATTERN_NAMES = {0: "star", 1: "box", 2: "general"}

STATUS_NAMES = {
    0: "STENCIL_OK", -1: "STENCIL_ERR_INVALID", -2: "STENCIL_ERR_UNSUPPORTED",
    -3: "STENCIL_ERR_ALIAS", -4: "STENCIL_ERR_NOMEM", -5: "STENCIL_ERR_DEVICE",
    -6: "STENCIL_ERR_BUDGET", -7: "STENCIL_ERR_TIMEOUT",
}


class StencilLibraryMissing(RuntimeError):
    pass


class StencilError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class stencil_shape(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int64 * 3)]


class stencil_tuning(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32 * 3), ("depth", ctypes.c_int32), ("flags", ctypes.c_int32)]


class stencil_plan_info(ctypes.Structure):
    _fields_ = [
        ("scheme", ctypes.c_int32), ("pattern", ctypes.c_int32), ("points", ctypes.c_int32),
        ("depth", ctypes.c_int32), ("passes", ctypes.c_int64), ("tiles", ctypes.c_int32),
        ("strips", ctypes.c_int32), ("seg_len", ctypes.c_int32), ("cols_per_lane", ctypes.c_int32),
        ("redundant_lanes", ctypes.c_int32),
        ("grid", ctypes.c_int32), ("block", ctypes.c_int32), ("cells", ctypes.c_int64),
        ("padded_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
        ("edge_seg_len", ctypes.c_int32), ("edge_tiles", ctypes.c_int32),
        ("model_cells_per_s", ctypes.c_double),
    ]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["scheme_name"] = SCHEME_NAMES.get(self.scheme, str(self.scheme))
        d["pattern_name"] = PATTERN_NAMES.get(self.pattern, str(self.pattern))
        return d


class stencil_machine(ctypes.Structure):
    _fields_ = [("hbm_bytes_per_s", ctypes.c_double), ("lds_bytes_per_s", ctypes.c_double),
                ("fp64_flops", ctypes.c_double), ("fp32_flops", ctypes.c_double),
                ("grid_sync_s", ctypes.c_double), ("neighbor_sync_s", ctypes.c_double),
                ("hbm_latency_s", ctypes.c_double), ("lds_latency_s", ctypes.c_double),
                ("fma_latency_s", ctypes.c_double), ("cus", ctypes.c_int32)]


class stencil_job(ctypes.Structure):
    _fields_ = [("coeffs", ctypes.POINTER(ctypes.c_double)), ("radius", ctypes.c_int32),
                ("shape", stencil_shape), ("dtype", ctypes.c_int), ("T", ctypes.c_int64),
                ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p), ("tag", ctypes.c_uint64),
                ("depth", ctypes.c_int32)]


class stencil_model_params(ctypes.Structure):
    _fields_ = [("B_gm", ctypes.c_double), ("B_sm", ctypes.c_double), ("thr_cmp", ctypes.c_double),
                ("cell_bytes", ctypes.c_double), ("a_gm", ctypes.c_double),
                ("a_sm", ctypes.c_double), ("a_cmp", ctypes.c_double), ("D_gm", ctypes.c_double),
                ("D_sm", ctypes.c_double), ("D_cmp", ctypes.c_double), ("D_all", ctypes.c_double),
                ("t", ctypes.c_double), ("tiling", ctypes.c_int32), ("tiled_dims", ctypes.c_int32),
                ("tile", ctypes.c_double * 2), ("rad", ctypes.c_double), ("t_dsync", ctypes.c_double),
                ("n_sync", ctypes.c_double)]


class stencil_model_result(ctypes.Structure):
    _fields_ = [("T_gm", ctypes.c_double), ("T_sm", ctypes.c_double), ("T_cmp", ctypes.c_double),
                ("T_stencil", ctypes.c_double), ("P", ctypes.c_double), ("V", ctypes.c_double),
                ("PP", ctypes.c_double), ("t_desired", ctypes.c_double),
                ("min_tile", ctypes.c_double), ("bottleneck", ctypes.c_int32)]


class stencil_tune_result(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("seg_len", ctypes.c_int32),
                ("seconds_per_step", ctypes.c_double), ("model_cells_per_s", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("flags", ctypes.c_int32)]


class stencil_server_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_slots", ctypes.c_int32),
                ("quantum_passes", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_uint64),
                ("round_target_s", ctypes.c_double), ("rounds_in_flight", ctypes.c_int32)]


class stencil_server_statistics(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
                ("active", ctypes.c_int32), ("queued", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("hbm_in_use", ctypes.c_uint64), ("hbm_peak", ctypes.c_uint64),
                ("cell_updates", ctypes.c_double), ("busy_s", ctypes.c_double), ("wall_s", ctypes.c_double),
                ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double), ("mean_s", ctypes.c_double),
                ("max_s", ctypes.c_double)]


MODEL_NO_TILING, MODEL_SM_TILING, MODEL_DEVICE_TILING = 0, 1, 2

_P = ctypes.c_void_p
_DBL = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes); the same names as include/stencil.h
_SIGNATURES = {
    "stencil_plan": (ctypes.c_int, [ctypes.POINTER(_P), _DBL, ctypes.c_int32,
                                     ctypes.POINTER(stencil_shape), ctypes.c_int, ctypes.c_int64,
                                     ctypes.POINTER(stencil_tuning)]),
    "stencil_plan_workspace": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "stencil_plan_describe": (ctypes.c_int, [_P, ctypes.POINTER(stencil_plan_info)]),
    "stencil_execute": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "stencil_plan_destroy": (ctypes.c_int, [_P]),
    "stencil_run": (ctypes.c_int, [_DBL, ctypes.c_int32, ctypes.POINTER(stencil_shape),
                                    ctypes.c_int, ctypes.c_int64, _P, _P, _P]),
    "stencil_run_noalloc": (ctypes.c_int, [_DBL, ctypes.c_int32, ctypes.POINTER(stencil_shape),
                                            ctypes.c_int, ctypes.c_int64, _P, _P, _P]),
    "stencil_batch_submit": (ctypes.c_int, [ctypes.POINTER(stencil_job), ctypes.c_int32, _P,
                                             ctypes.POINTER(ctypes.c_int)]),
    "stencil_batch_describe": (ctypes.c_int, [ctypes.POINTER(stencil_job), ctypes.POINTER(stencil_plan_info)]),
    "stencil_sync": (ctypes.c_int, [_P]),
    "stencil_probe_grid_sync": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_double)]),
    "stencil_probe_copy": (ctypes.c_int, [ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_double)]),
    "stencil_probe_latency": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_double)]),
    "stencil_probe_lds_bandwidth": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "stencil_probe_neighbor_sync": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P,
                                                    ctypes.POINTER(ctypes.c_double),
                                                    ctypes.POINTER(ctypes.c_uint64)]),
    "stencil_model_eval": (ctypes.c_int, [ctypes.POINTER(stencil_model_params),
                                           ctypes.POINTER(stencil_model_result)]),
    "stencil_machine_get": (ctypes.c_int, [ctypes.POINTER(stencil_machine)]),
    "stencil_machine_set": (ctypes.c_int, [ctypes.POINTER(stencil_machine)]),
    "stencil_machine_calibrate": (ctypes.c_int, [_P, ctypes.POINTER(stencil_machine)]),
    "stencil_tune": (ctypes.c_int, [_DBL, ctypes.c_int32, ctypes.POINTER(stencil_shape), ctypes.c_int,
                                     ctypes.c_int32, _P, ctypes.POINTER(stencil_tune_result)]),
    "stencil_tune_lookup": (ctypes.c_int, [_DBL, ctypes.c_int32, ctypes.POINTER(stencil_shape),
                                            ctypes.c_int, ctypes.c_int32, ctypes.POINTER(stencil_tuning),
                                            ctypes.POINTER(ctypes.c_int32)]),
    "stencil_tune_cache_key": (ctypes.c_int, [_DBL, ctypes.c_int32, ctypes.POINTER(stencil_shape),
                                               ctypes.c_int, ctypes.c_int32, ctypes.c_char_p,
                                               ctypes.c_size_t]),
    "stencil_tune_cache_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]),
    "stencil_tune_cache_save": (ctypes.c_int, [ctypes.c_char_p]),
    "stencil_tune_cache_clear": (ctypes.c_int, []),
    "stencil_server_create": (ctypes.c_int, [ctypes.POINTER(stencil_server_config), ctypes.POINTER(_P)]),
    "stencil_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(stencil_job), _P,
                                              ctypes.POINTER(ctypes.c_uint64)]),
    "stencil_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, _P, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_double)]),
    "stencil_server_wait": (ctypes.c_int, [_P, ctypes.c_uint64, _P, ctypes.POINTER(ctypes.c_double)]),
    "stencil_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(stencil_server_statistics)]),
    "stencil_server_destroy": (ctypes.c_int, [_P]),
    "stencil_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load_library(path: str | None = None):
    """Load the HIP library; raises StencilLibraryMissing if it was not built.
    The path is `path`, else $STENCIL_LIBRARY (another build of the same
    library, e.g. an ablation variant), else the in-tree build."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("STENCIL_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise StencilLibraryMissing(
            f"{path} not found: build it with `python -m paper_2305_07390_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname as the system's.
    # Loading torch first makes the library bind to that one; loading the
    # library first would bring a second HIP/HSA runtime into the process,
    # and the second to initialise finds no GPU.
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover - the library works without torch
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGNATURES)


def stencil_last_error() -> str:
    return load_library().stencil_last_error().decode()


def _check(status: int):
    if status != STENCIL_OK:
        raise StencilError(status, stencil_last_error())


def _shape(interior) -> stencil_shape:
    s = stencil_shape()
    s.ndim = len(interior)
    for i, v in enumerate(interior[:3]):
        s.n[i] = int(v)
    return s


def _coeff_ptr(coeffs: np.ndarray):
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    return c, c.ctypes.data_as(_DBL)


def _dtype_code(dtype) -> int:
    name = str(dtype)
    if "float64" in name or name in ("f64", "double"):
        return STENCIL_F64
    if "float32" in name or name in ("f32", "float"):
        return STENCIL_F32
    raise ValueError(f"unsupported dtype {dtype}")


def padded_nbytes(interior, radius: int, dtype) -> int:
    """Bytes of one padded array (interior + 2r per axis) of `dtype`."""
    n = 1
    for v in interior:
        n *= int(v) + 2 * int(radius)
    return n * (8 if _dtype_code(dtype) == STENCIL_F64 else 4)


def _check_tensor(name: str, x, dtype_code: int, nbytes: int):
    """A device tensor handed to the library must be contiguous, of the plan's
    dtype and exactly one padded array long: the kernels address it from the
    plan's geometry, so anything smaller would be read or written out of
    bounds."""
    if not x.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if _dtype_code(x.dtype) != dtype_code:
        raise ValueError(f"{name}: dtype {x.dtype} does not match the plan's "
                         f"{'float64' if dtype_code == STENCIL_F64 else 'float32'}")
    got = x.numel() * x.element_size()
    if got != nbytes:
        raise ValueError(f"{name}: {got} bytes, the plan needs one padded array of {nbytes} bytes")


def _check_on_gpu(*named):
    for name, x in named:
        if x.device.type != "cuda":
            raise ValueError(f"{name}: tensor must be on a GPU device")


def _check_host(name: str, a: np.ndarray, dtype_code: int, nbytes: int, writable: bool = False):
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError(f"{name}: array must be C-contiguous")
    if _dtype_code(a.dtype) != dtype_code:
        raise ValueError(f"{name}: dtype {a.dtype} does not match the request's")
    if a.nbytes != nbytes:
        raise ValueError(f"{name}: {a.nbytes} bytes, the request needs one padded array of {nbytes} bytes")
    if writable and not a.flags["WRITEABLE"]:
        raise ValueError(f"{name}: array must be writable")


def stencil_plan(coeffs, radius: int, interior, dtype, T: int, depth: int = 0, seg_len: int = 0,
                 flags: int = 0):
    """Create a plan; returns an opaque handle (int). Raises StencilError."""
    lib = load_library()
    c, cp = _coeff_ptr(coeffs)
    shp = _shape(interior)
    tun = stencil_tuning()
    tun.depth = int(depth)
    tun.tile[0] = int(seg_len)
    tun.flags = int(flags)
    h = _P()
    _check(lib.stencil_plan(ctypes.byref(h), cp, int(radius), ctypes.byref(shp), _dtype_code(dtype),
                            int(T), ctypes.byref(tun)))
    return h.value


def stencil_plan_workspace(plan) -> int:
    n = ctypes.c_size_t()
    _check(load_library().stencil_plan_workspace(plan, ctypes.byref(n)))
    return n.value


def stencil_plan_describe(plan) -> dict:
    info = stencil_plan_info()
    _check(load_library().stencil_plan_describe(plan, ctypes.byref(info)))
    return info.as_dict()


def stencil_execute(plan, in_ptr: int, out_ptr: int, ws_ptr: int, stream: int = 0):
    _check(load_library().stencil_execute(plan, in_ptr, out_ptr, ws_ptr or None, stream or None))


def stencil_plan_destroy(plan):
    _check(load_library().stencil_plan_destroy(plan))


def stencil_batch_submit(specs, stream: int = 0):
    """Submit a batch. `specs` is a list of dicts with keys coeffs, radius,
    interior, dtype, T, in_ptr, out_ptr and optional tag, depth. Returns the
    per-job status list; raises StencilError if the call itself fails."""
    lib = load_library()
    n = len(specs)
    arr = (stencil_job * n)()
    keep = []
    for i, sp in enumerate(specs):
        c, cp = _coeff_ptr(sp["coeffs"])
        keep.append(c)
        arr[i].coeffs = cp
        arr[i].radius = int(sp["radius"])
        arr[i].shape = _shape(sp["interior"])
        arr[i].dtype = _dtype_code(sp["dtype"])
        arr[i].T = int(sp["T"])
        arr[i].in_ = sp["in_ptr"]
        arr[i].out = sp["out_ptr"]
        arr[i].tag = int(sp.get("tag", i))
        arr[i].depth = int(sp.get("depth", 0))
    st = (ctypes.c_int * n)()
    _check(lib.stencil_batch_submit(arr, n, stream or None, st))
    return list(st)


def stencil_batch_describe(coeffs, radius: int, interior, dtype, T: int, depth: int = 0) -> dict:
    """The plan stencil_batch_submit would run this job with (host only)."""
    lib = load_library()
    job = stencil_job()
    c, job.coeffs = _coeff_ptr(coeffs)
    job.radius = int(radius)
    job.shape = _shape(interior)
    job.dtype = _dtype_code(dtype)
    job.T = int(T)
    job.depth = int(depth)
    info = stencil_plan_info()
    _check(lib.stencil_batch_describe(ctypes.byref(job), ctypes.byref(info)))
    return info.as_dict()


def stencil_probe_grid_sync(rounds: int = 1000, stream: int = 0) -> float:
    """Seconds per device-wide synchronisation (one workgroup per CU)."""
    out = ctypes.c_double()
    _check(load_library().stencil_probe_grid_sync(int(rounds), stream or None, ctypes.byref(out)))
    return out.value


STENCIL_PROBE_HBM_LATENCY, STENCIL_PROBE_LDS_LATENCY, STENCIL_PROBE_FMA64_LATENCY = 0, 1, 2
PROBE_HBM_LATENCY, PROBE_LDS_LATENCY, PROBE_FMA64_LATENCY = 0, 1, 2


def stencil_probe_copy(nbytes: int = 2 << 30, stream: int = 0) -> float:
    """Reachable HBM bandwidth (read + write bytes per second) of a streaming copy."""
    out = ctypes.c_double()
    _check(load_library().stencil_probe_copy(int(nbytes), stream or None, ctypes.byref(out)))
    return out.value


def stencil_probe_latency(kind: int, stream: int = 0) -> float:
    """Seconds per link of a dependent chain (PROBE_* kinds)."""
    out = ctypes.c_double()
    _check(load_library().stencil_probe_latency(int(kind), stream or None, ctypes.byref(out)))
    return out.value


def stencil_probe_lds_bandwidth(stream: int = 0) -> float:
    out = ctypes.c_double()
    _check(load_library().stencil_probe_lds_bandwidth(stream or None, ctypes.byref(out)))
    return out.value


def stencil_probe_neighbor_sync(mode: int, rounds: int = 2000, payload_bytes: int = 0, stream: int = 0):
    """(seconds per round, payload words that did not carry their round's value)."""
    t = ctypes.c_double()
    bad = ctypes.c_uint64()
    _check(load_library().stencil_probe_neighbor_sync(int(mode), int(rounds), int(payload_bytes), stream or None,
                                                      ctypes.byref(t), ctypes.byref(bad)))
    return t.value, bad.value


def stencil_sync(stream: int = 0):
    _check(load_library().stencil_sync(stream or None))


def stencil_tune(coeffs, radius: int, interior, dtype, flags: int = 0, stream: int = 0) -> dict:
    """Autotune (depth, segment) for this stencil class and size; see the header."""
    c, cp = _coeff_ptr(coeffs)
    shp = _shape(interior)
    r = stencil_tune_result()
    _check(load_library().stencil_tune(cp, int(radius), ctypes.byref(shp), _dtype_code(dtype),
                                       int(flags), stream or None, ctypes.byref(r)))
    return {name: getattr(r, name) for name, _ in r._fields_}


def stencil_tune_lookup(coeffs, radius: int, interior, dtype, flags: int = 0):
    """Cached (depth, seg_len) for this request, or None."""
    c, cp = _coeff_ptr(coeffs)
    shp = _shape(interior)
    out = stencil_tuning()
    found = ctypes.c_int32()
    _check(load_library().stencil_tune_lookup(cp, int(radius), ctypes.byref(shp), _dtype_code(dtype),
                                              int(flags), ctypes.byref(out), ctypes.byref(found)))
    return (out.depth, out.tile[0]) if found.value else None


def stencil_tune_cache_key(coeffs, radius: int, interior, dtype, flags: int = 0) -> str:
    c, cp = _coeff_ptr(coeffs)
    shp = _shape(interior)
    buf = ctypes.create_string_buffer(256)
    _check(load_library().stencil_tune_cache_key(cp, int(radius), ctypes.byref(shp),
                                                 _dtype_code(dtype), int(flags), buf, 256))
    return buf.value.decode()


def stencil_tune_cache_load(path: str = TUNE_CACHE_PATH) -> int:
    n = ctypes.c_int32()
    _check(load_library().stencil_tune_cache_load(path.encode(), ctypes.byref(n)))
    return n.value


def stencil_tune_cache_save(path: str = TUNE_CACHE_PATH):
    _check(load_library().stencil_tune_cache_save(path.encode()))


def stencil_tune_cache_clear():
    _check(load_library().stencil_tune_cache_clear())


def use_tuned_defaults(path: str = TUNE_CACHE_PATH) -> int:
    """Merge the packaged tuning cache (measured on MI355X) into the library's
    cache, so that plans without hints use the tuned depths; returns the
    number of entries (0 if the file is absent)."""
    if not os.path.exists(path):
        return 0
    return stencil_tune_cache_load(path)


def stencil_server_create(hbm_budget_bytes: int, max_slots: int, quantum_passes: int = 0,
                          device: int = 0, round_target_s: float = 0.0, rounds_in_flight: int = 0):
    cfg = stencil_server_config()
    cfg.round_target_s = float(round_target_s)
    cfg.rounds_in_flight = int(rounds_in_flight)
    cfg.device = int(device)
    cfg.max_slots = int(max_slots)
    cfg.quantum_passes = int(quantum_passes)
    cfg.hbm_budget_bytes = int(hbm_budget_bytes)
    h = _P()
    _check(load_library().stencil_server_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def _job_struct(coeffs, radius, interior, dtype, T):
    c, cp = _coeff_ptr(coeffs)
    j = stencil_job()
    j.coeffs = cp
    j.radius = int(radius)
    j.shape = _shape(interior)
    j.dtype = _dtype_code(dtype)
    j.T = int(T)
    return j, c


# (server, ticket) -> (dtype code, padded bytes) of requests not yet collected,
# so that a result is only ever copied into a host array of the right size
_tickets = {}
_tickets_lock = __import__("threading").Lock()


def stencil_server_submit(server, coeffs, radius: int, interior, T: int, host_in: np.ndarray) -> int:
    """Submit one request; `host_in` is the padded input (its dtype is the
    request's). Returns the ticket."""
    a = np.ascontiguousarray(host_in)
    code = _dtype_code(a.dtype)
    nbytes = padded_nbytes(interior, radius, a.dtype)
    _check_host("host_in", a, code, nbytes)
    j, keep = _job_struct(coeffs, radius, interior, a.dtype, T)
    t = ctypes.c_uint64()
    _check(load_library().stencil_server_submit(server, ctypes.byref(j), a.ctypes.data, ctypes.byref(t)))
    with _tickets_lock:
        _tickets[(server, t.value)] = (code, nbytes)
    return t.value


def _out_ptr(server, ticket: int, host_out):
    if host_out is None:
        return None
    with _tickets_lock:
        meta = _tickets.get((server, int(ticket)))
    if meta is None:
        raise ValueError(f"unknown ticket {ticket}")
    _check_host("host_out", host_out, meta[0], meta[1], writable=True)
    return host_out.ctypes.data


def _retire(server, ticket: int):
    with _tickets_lock:
        _tickets.pop((server, int(ticket)), None)


def stencil_server_poll(server, ticket: int, host_out: np.ndarray | None = None):
    """(done, latency_s); when done the result is in host_out and the ticket is retired."""
    done = ctypes.c_int32()
    lat = ctypes.c_double()
    ptr = _out_ptr(server, ticket, host_out)
    status = load_library().stencil_server_poll(server, int(ticket), ptr, ctypes.byref(done), ctypes.byref(lat))
    if done.value or status != STENCIL_OK:
        _retire(server, ticket)
    _check(status)
    return bool(done.value), lat.value


def stencil_server_wait(server, ticket: int, host_out: np.ndarray | None = None) -> float:
    lat = ctypes.c_double()
    ptr = _out_ptr(server, ticket, host_out)
    status = load_library().stencil_server_wait(server, int(ticket), ptr, ctypes.byref(lat))
    _retire(server, ticket)
    _check(status)
    return lat.value


def stencil_server_stats(server) -> dict:
    s = stencil_server_statistics()
    _check(load_library().stencil_server_stats(server, ctypes.byref(s)))
    return {name: getattr(s, name) for name, _ in s._fields_}


def stencil_server_destroy(server):
    _check(load_library().stencil_server_destroy(server))


def run_batch(problems, xs, ys, stream=None, depth=0):
    """Submit torch tensors (lists of inputs and outputs) as one batch on
    `stream`; `problems` provide coefficients, radius and T."""
    specs = []
    for k, (prob, x, y) in enumerate(zip(problems, xs, ys)):
        code = _dtype_code(x.dtype)
        nbytes = padded_nbytes(prob.interior, prob.spec.r, x.dtype)
        _check_tensor(f"job {k} input", x, code, nbytes)
        _check_tensor(f"job {k} output", y, code, nbytes)
        _check_on_gpu((f"job {k} input", x), (f"job {k} output", y))
        specs.append(dict(coeffs=prob.coeffs, radius=prob.spec.r, interior=prob.interior,
                          dtype=x.dtype, T=prob.T, in_ptr=x.data_ptr(), out_ptr=y.data_ptr(),
                          tag=getattr(prob, "tag", k), depth=depth))
    return stencil_batch_submit(specs, _stream_handle(stream))


def stencil_model_eval(**kw) -> dict:
    """Evaluate the attainable-performance model; keyword names as in the C struct
    (``tile`` may be a pair)."""
    p = stencil_model_params()
    for k, v in kw.items():
        if k == "tile":
            p.tile[0], p.tile[1] = (list(v) + [0.0, 0.0])[:2]
        else:
            setattr(p, k, v)
    r = stencil_model_result()
    _check(load_library().stencil_model_eval(ctypes.byref(p), ctypes.byref(r)))
    return {name: getattr(r, name) for name, _ in r._fields_}


def stencil_machine_get() -> dict:
    m = stencil_machine()
    _check(load_library().stencil_machine_get(ctypes.byref(m)))
    return {name: getattr(m, name) for name, _ in m._fields_}


def stencil_machine_set(params=None, **overrides):
    """Replace the model's machine parameters (None and no overrides: the
    defaults); keyword overrides apply on top of the current set."""
    lib = load_library()
    if params is None and not overrides:
        _check(lib.stencil_machine_set(None))
        return stencil_machine_get()
    cur = dict(stencil_machine_get() if params is None else params)
    cur.update(overrides)
    m = stencil_machine(**cur)
    _check(lib.stencil_machine_set(ctypes.byref(m)))
    return stencil_machine_get()


def stencil_machine_calibrate(stream: int = 0) -> dict:
    m = stencil_machine()
    _check(load_library().stencil_machine_calibrate(stream or None, ctypes.byref(m)))
    return {name: getattr(m, name) for name, _ in m._fields_}


def stencil_run(coeffs, radius: int, interior, dtype, T: int, in_ptr: int, out_ptr: int,
                stream: int = 0):
    lib = load_library()
    c, cp = _coeff_ptr(coeffs)
    shp = _shape(interior)
    _check(lib.stencil_run(cp, int(radius), ctypes.byref(shp), _dtype_code(dtype), int(T), in_ptr,
                           out_ptr, stream or None))


def stencil_run_noalloc(coeffs, radius: int, interior, dtype, T: int, in_ptr: int, out_ptr: int,
                        stream: int = 0):
    lib = load_library()
    c, cp = _coeff_ptr(coeffs)
    shp = _shape(interior)
    _check(lib.stencil_run_noalloc(cp, int(radius), ctypes.byref(shp), _dtype_code(dtype), int(T), in_ptr,
                                   out_ptr, stream or None))


# Workspace limit of stencil_run_noalloc (include/stencil.h).
NOALLOC_SCRATCH_BYTES = 64 << 20


# --- torch conveniences -------------------------------------------------------

def _stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def interior_of(x, radius: int):
    return tuple(int(s) - 2 * radius for s in x.shape)


class Plan:
    """A plan bound to a coefficient box, radius, interior shape, dtype and T."""

    def __init__(self, coeffs, radius, interior, dtype, T, depth=0, seg_len=0, flags=0):
        self.handle = stencil_plan(coeffs, radius, interior, dtype, T, depth, seg_len, flags)
        self.dtype_code = _dtype_code(dtype)
        self.radius = radius
        self.flags = int(flags)
        self.interior = tuple(interior)
        self.T = T
        self.info = stencil_plan_describe(self.handle)
        self.workspace_bytes = stencil_plan_workspace(self.handle)
        self._ws = None

    def workspace(self, device):
        import torch
        if self.workspace_bytes == 0:
            return None
        if self._ws is None or self._ws.device != device:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)
        return self._ws

    @property
    def persistent(self) -> bool:
        return bool(self.flags & STENCIL_FLAG_PERSISTENT)

    def execute(self, x_in, x_out, stream=None):
        """Run on torch device tensors (padded, contiguous, of the plan's dtype
        and size). Enqueues on `stream`. A persistent plan's passes, and a
        device-tiled plan's tiles, wait on each other inside a launch; for
        them the call also waits for the stream (stencil_sync), so that an
        expired bounded wait raises StencilError(STENCIL_ERR_TIMEOUT) here
        instead of going unnoticed."""
        nbytes = self.info["padded_bytes"]
        _check_tensor("input", x_in, self.dtype_code, nbytes)
        _check_tensor("output", x_out, self.dtype_code, nbytes)
        _check_on_gpu(("input", x_in), ("output", x_out))
        ws = self.workspace(x_in.device)
        sh = _stream_handle(stream)
        stencil_execute(self.handle, x_in.data_ptr(), x_out.data_ptr(),
                        ws.data_ptr() if ws is not None else 0, sh)
        if (self.persistent and self.info["scheme_name"] in ("blocked_2d", "blocked_3d")) or \
                self.info["scheme_name"] == "device_3d":
            stencil_sync(sh)
        return x_out

    def close(self):
        if self.handle:
            stencil_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run(coeffs, radius: int, x_in, T: int, x_out=None, stream=None):
    """One-shot stencil_run on torch device tensors; returns x_out."""
    import torch
    if x_out is None:
        x_out = torch.empty_like(x_in)
    code = _dtype_code(x_in.dtype)
    nbytes = padded_nbytes(interior_of(x_in, radius), radius, x_in.dtype)
    _check_tensor("input", x_in, code, nbytes)
    _check_tensor("output", x_out, code, nbytes)
    _check_on_gpu(("input", x_in), ("output", x_out))
    stencil_run(coeffs, radius, interior_of(x_in, radius), x_in.dtype, T, x_in.data_ptr(),
                x_out.data_ptr(), _stream_handle(stream))
    return x_out
