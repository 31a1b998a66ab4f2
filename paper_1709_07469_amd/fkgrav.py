"""ctypes binding of libfkgrav.so (include/fkgrav.h).

The functions named like the C entry points only marshal arguments: torch
tensors become device pointers, the current torch stream becomes the HIP
stream, and a non-zero status raises FkError with the library's message.
Every step of a solve runs in the library's HIP kernels; nothing here falls
back to another implementation -- without the built library on a GPU the
calls raise.

``solve(problem, kind)`` is a convenience wrapper that uploads a
``workloads.Problem``, allocates the output and workspace, runs one solve and
returns the per-station statistics as numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfkgrav.so")

FK_OK, FK_EINVAL, FK_EDOMAIN, FK_EWORKSPACE, FK_EDEVICE, FK_ETRUNC, FK_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FK_ENONFINITE = -7
FK_FLAG_TRUNCATED, FK_FLAG_NONFINITE, FK_FLAG_STRICT = 1, 2, 256
FK_F64, FK_MIXED_F64ACC, FK_MIXED_KAHAN = 0, 1, 2
FK_EXIT_OVERSHOOT, FK_EXIT_INTERSECT, FK_EXIT_BRIDGE = 0, 1, 2
FK_DOMAIN_BOX, FK_DOMAIN_BALL = 0, 1
FK_BC_ZERO, FK_BC_QUADRATIC, FK_BC_POINT_MASSES, FK_BC_PRISMS, FK_BC_FACE_GRID = 0, 1, 2, 3, 4
FK_PAIR_CRN, FK_PAIR_INDEPENDENT = 0, 1
FK_MAX_PRISMS = FK_MAX_SPHERES = FK_MAX_BC_ITEMS = 16
FK_MAX_BATCH = 256
CAP_FLAG = 0x80000000


class FkError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"fkgrav status {status}: {message}")
        self.status = status


class fk_box(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class fk_source(C.Structure):
    _fields_ = [("rho", C.c_void_p), ("n", C.c_int32 * 3), ("pad0", C.c_int32), ("origin", C.c_double * 3),
                ("spacing", C.c_double * 3), ("prisms", C.c_void_p), ("n_prisms", C.c_int32), ("pad1", C.c_int32),
                ("spheres", C.c_void_p), ("n_spheres", C.c_int32), ("pad2", C.c_int32),
                ("rho_index", C.c_void_p), ("rho_levels", C.c_void_p)]


class fk_boundary(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad0", C.c_int32), ("data", C.c_void_p), ("n_items", C.c_int64),
                ("face_n", (C.c_int32 * 2) * 6)]


class fk_params(C.Structure):
    _fields_ = [("paths_per_station", C.c_int64), ("dt", C.c_double), ("seed", C.c_uint64), ("G", C.c_double),
                ("h", C.c_double), ("precision", C.c_int32), ("exit_rule", C.c_int32), ("pairing", C.c_int32),
                ("strict", C.c_int32), ("max_steps", C.c_int64), ("problem_id", C.c_uint32), ("domain", C.c_int32),
                ("path_offset", C.c_int64), ("slice_walks", C.c_int64)]


class fk_stat(C.Structure):
    _fields_ = [("mean", C.c_double), ("var", C.c_double), ("se", C.c_double), ("n", C.c_int64),
                ("sum_steps", C.c_int64), ("max_steps", C.c_int64), ("n_trunc", C.c_int64),
                ("mean_steps", C.c_double)]


class fk_launch(C.Structure):
    _fields_ = [("block", C.c_int32), ("blocks_per_cu", C.c_int32), ("grab", C.c_int32),
                ("adjoint_table", C.c_int32), ("stripes", C.c_int32), ("refill_cost", C.c_int32)]


class fk_problem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad0", C.c_int32), ("stations", C.c_void_p), ("n_stations", C.c_int64),
                ("box", fk_box), ("source", fk_source), ("bc", fk_boundary), ("params", fk_params),
                ("out_offset", C.c_int64)]


STAT_DTYPE = np.dtype([("mean", "<f8"), ("var", "<f8"), ("se", "<f8"), ("n", "<i8"), ("sum_steps", "<i8"),
                       ("max_steps", "<i8"), ("n_trunc", "<i8"), ("mean_steps", "<f8")])
assert STAT_DTYPE.itemsize == C.sizeof(fk_stat) == 64

_lock = threading.Lock()
_lib = None


def lib():
    """Loads libfkgrav.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1709_07469_amd.build.build()")
            L = C.CDLL(LIB_PATH)
            p, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
            L.fk_workspace_bytes.argtypes = [i32, i64, p]
            L.fk_workspace_bytes.restype = sz
            L.fk_workspace_layout.argtypes = [i32, i64, p, p, p, p]
            L.fk_workspace_layout.restype = i32
            L.fk_workspace_status.argtypes = [p, p, p]
            L.fk_workspace_status.restype = i32
            L.fk_check_stations.argtypes = [p, i64, p, i32, p]
            L.fk_check_stations.restype = i32
            for nm in ("fk_solve_potential", "fk_solve_gz"):
                getattr(L, nm).argtypes = [p, i64, p, p, p, p, p, p, sz, p]
                getattr(L, nm).restype = i32
            L.fk_solve_static.argtypes = [i32, p, i64, p, p, p, p, p, p]
            L.fk_solve_static.restype = i32
            L.fk_batch_workspace_bytes.argtypes = [p, i32]
            L.fk_batch_workspace_bytes.restype = sz
            L.fk_batch_layout.argtypes = [p, i32, i32, p, p]
            L.fk_batch_layout.restype = i32
            L.fk_solve_batch.argtypes = [p, i32, p, p, sz, p]
            L.fk_solve_batch.restype = i32
            L.fk_adjoint_workspace_bytes.argtypes = [i64, p]
            L.fk_adjoint_workspace_bytes.restype = sz
            for nm in ("fk_potential_adjoint", "fk_gz_adjoint"):
                getattr(L, nm).argtypes = [p, i64, p, p, p, p, p, p, sz, p, p, p, sz, p]
                getattr(L, nm).restype = i32
            L.fk_stream_blocks.argtypes = [p, i64, C.c_uint64, p, p, p, p]
            L.fk_stream_blocks.restype = i32
            L.fk_autotune.argtypes = [i32, p, i64, p, p, p, p, p, p, sz, p, p, p]
            L.fk_autotune.restype = i32
            L.fk_merge_stats.argtypes = [p, p, i64, p]
            L.fk_merge_stats.restype = i32
            L.fk_moving_average.argtypes = [p, p, i64, i32, p, p]
            L.fk_moving_average.restype = i32
            L.fk_set_launch.argtypes = [i32, p]
            L.fk_set_launch.restype = i32
            L.fk_get_launch.argtypes = [i32, p]
            L.fk_get_launch.restype = i32
            L.fk_timing_enable.argtypes = [i32]
            L.fk_timing_enable.restype = i32
            L.fk_timing_read.argtypes = [p, i32, p]
            L.fk_timing_read.restype = i32
            L.fk_status_string.argtypes = [i32]
            L.fk_status_string.restype = C.c_char_p
            L.fk_last_error.restype = C.c_char_p
            L.fk_version.restype = i32
            _lib = L
    return _lib


def _check(status):
    if status != FK_OK:
        raise FkError(status, lib().fk_last_error().decode())


def _ptr(t):
    """Device (torch) or host (numpy) pointer, None for None."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return C.c_void_p(t.data_ptr())
    return t.ctypes.data_as(C.c_void_p)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# --------------------------------------------------------------------------
# Mirrors of the C entry points.
# --------------------------------------------------------------------------

def fk_workspace_bytes(kind: int, n_stations: int, params: fk_params) -> int:
    return int(lib().fk_workspace_bytes(int(kind), int(n_stations), C.byref(params)))


def fk_workspace_layout(kind: int, n_stations: int, params: fk_params):
    v, s, t = C.c_size_t(), C.c_size_t(), C.c_size_t()
    _check(lib().fk_workspace_layout(int(kind), int(n_stations), C.byref(params), C.byref(v), C.byref(s),
                                     C.byref(t)))
    return v.value, s.value, t.value


def fk_workspace_status(workspace, stream=None):
    """Waits for the stream and returns (status, flags) of the last solve run
    in the workspace: status FK_OK, FK_ETRUNC (strict solve with capped
    walks) or FK_ENONFINITE, flags the FK_FLAG_* bits.  Does not raise on
    those two statuses."""
    f = C.c_uint32()
    st = lib().fk_workspace_status(_ptr(workspace), C.byref(f), _stream_handle(stream))
    if st not in (FK_OK, FK_ETRUNC, FK_ENONFINITE):
        _check(st)
    return int(st), int(f.value)


def fk_check_stations(stations_host: np.ndarray, box: fk_box, kind: int, params: fk_params) -> None:
    st = np.ascontiguousarray(stations_host, dtype=np.float64).reshape(-1, 3)
    _check(lib().fk_check_stations(_ptr(st), len(st), C.byref(box), int(kind), C.byref(params)))


def _solve_call(name, stations, box, source, bc, params, out, workspace, stream):
    n = int(stations.shape[0]) if stations is not None else 0
    _check(getattr(lib(), name)(_ptr(stations), n, C.byref(box), C.byref(source), C.byref(bc), C.byref(params),
                                _ptr(out), _ptr(workspace), int(workspace.numel()) if workspace is not None else 0,
                                _stream_handle(stream)))


def fk_solve_potential(stations, box, source, bc, params, out, workspace, stream=None) -> None:
    """stations: cuda float64 (S, 3); out: cuda tensor of S fk_stat (64 B
    each); workspace: cuda uint8 tensor, 256-byte aligned."""
    _solve_call("fk_solve_potential", stations, box, source, bc, params, out, workspace, stream)


def fk_solve_gz(stations, box, source, bc, params, out, workspace, stream=None) -> None:
    _solve_call("fk_solve_gz", stations, box, source, bc, params, out, workspace, stream)


def fk_solve_static(kind, stations, box, source, bc, params, out, stream=None) -> None:
    """fk_solve_potential (kind 0) / fk_solve_gz (kind 1) without a workspace:
    the library's per-GPU scratch array serves instead (no allocation)."""
    n = int(stations.shape[0]) if stations is not None else 0
    _check(lib().fk_solve_static(int(kind), _ptr(stations), n, C.byref(box), C.byref(source), C.byref(bc),
                                 C.byref(params), _ptr(out), _stream_handle(stream)))


def fk_batch_workspace_bytes(problems) -> int:
    return int(lib().fk_batch_workspace_bytes(problems, len(problems)))


def fk_batch_layout(problems, m: int):
    v, s = C.c_size_t(), C.c_size_t()
    _check(lib().fk_batch_layout(problems, len(problems), int(m), C.byref(v), C.byref(s)))
    return v.value, s.value


def fk_solve_batch(problems, out, workspace, stream=None) -> None:
    """problems: ctypes array of fk_problem (host); out: cuda tensor of fk_stat
    rows covering every problem's out_offset range; workspace: cuda uint8."""
    _check(lib().fk_solve_batch(problems, len(problems), _ptr(out), _ptr(workspace), int(workspace.numel()),
                                _stream_handle(stream)))


def fk_adjoint_workspace_bytes(n_stations: int, source: fk_source) -> int:
    return int(lib().fk_adjoint_workspace_bytes(int(n_stations), C.byref(source)))


def _adjoint_call(name, stations, box, source, bc, params, fwd_out, fwd_workspace, grad_out, grad_rho, workspace,
                  stream):
    n = int(stations.shape[0])
    _check(getattr(lib(), name)(_ptr(stations), n, C.byref(box), C.byref(source), C.byref(bc), C.byref(params),
                                _ptr(fwd_out), _ptr(fwd_workspace), int(fwd_workspace.numel()), _ptr(grad_out),
                                _ptr(grad_rho), _ptr(workspace), int(workspace.numel()), _stream_handle(stream)))


def fk_potential_adjoint(stations, box, source, bc, params, fwd_out, fwd_workspace, grad_out, grad_rho, workspace,
                         stream=None) -> None:
    """grad_rho (cuda float64, one per voxel) <- sum_s grad_out[s] d u_s / d rho."""
    _adjoint_call("fk_potential_adjoint", stations, box, source, bc, params, fwd_out, fwd_workspace, grad_out,
                  grad_rho, workspace, stream)


def fk_gz_adjoint(stations, box, source, bc, params, fwd_out, fwd_workspace, grad_out, grad_rho, workspace,
                  stream=None) -> None:
    """grad_rho (cuda float64, one per voxel) <- sum_s grad_out[s] d g_z,s / d rho."""
    _adjoint_call("fk_gz_adjoint", stations, box, source, bc, params, fwd_out, fwd_workspace, grad_out,
                  grad_rho, workspace, stream)


def fk_stream_blocks(counters, seed: int, words=None, normals_f64=None, normals_f32=None, stream=None) -> None:
    """counters: cuda int32/uint32 tensor (n, 4); outputs cuda tensors or None."""
    _check(lib().fk_stream_blocks(_ptr(counters), int(counters.shape[0]), int(seed), _ptr(words), _ptr(normals_f64),
                                  _ptr(normals_f32), _stream_handle(stream)))


def fk_autotune(kind, stations, box, source, bc, params, out, workspace, stream=None):
    """Runs the library's launch-setting sweep; returns ({block,
    blocks_per_cu, grab}, milliseconds)."""
    best = fk_launch()
    ms = C.c_double()
    _check(lib().fk_autotune(int(kind), _ptr(stations), int(stations.shape[0]), C.byref(box), C.byref(source),
                             C.byref(bc), C.byref(params), _ptr(out), _ptr(workspace), int(workspace.numel()),
                             _stream_handle(stream), C.byref(best), C.byref(ms)))
    return {"block": best.block, "blocks_per_cu": best.blocks_per_cu, "grab": best.grab}, ms.value


def fk_merge_stats(a, b):
    """Merges two structured arrays of station statistics (STAT_DTYPE) from
    disjoint walk ranges of the same stations (host)."""
    a = np.ascontiguousarray(a, dtype=STAT_DTYPE)
    b = np.ascontiguousarray(b, dtype=STAT_DTYPE)
    if a.shape != b.shape:
        raise ValueError("statistics of different station counts")
    out = np.empty_like(a)
    _check(lib().fk_merge_stats(_ptr(a), _ptr(b), len(a), _ptr(out)))
    return out


def fk_moving_average(values, se=None, span: int = 5):
    """Centred moving average of a station profile (host); returns
    (smoothed values, their standard errors or None)."""
    v = np.ascontiguousarray(values, dtype=np.float64).ravel()
    e = None if se is None else np.ascontiguousarray(se, dtype=np.float64).ravel()
    ov = np.empty_like(v)
    oe = None if e is None else np.empty_like(e)
    _check(lib().fk_moving_average(_ptr(v), _ptr(e), len(v), int(span), _ptr(ov), _ptr(oe)))
    return ov, oe


LAUNCH_KEYS = ("block", "blocks_per_cu", "grab", "adjoint_table", "stripes", "refill_cost")


def fk_set_launch(precision: int, block: int, blocks_per_cu: int = 0, grab: int = 32, adjoint_table: int = 0,
                  stripes: int = 0, refill_cost: int = 0) -> None:
    _check(lib().fk_set_launch(int(precision), C.byref(fk_launch(block, blocks_per_cu, grab, adjoint_table, stripes,
                                                                 refill_cost))))


def fk_set_launch_dict(precision: int, d: dict) -> None:
    """fk_set_launch from a dict of launch settings (missing keys: 0, the
    defaults, except block 256 and grab 32)."""
    fk_set_launch(precision, d.get("block", 256), d.get("blocks_per_cu", 0), d.get("grab", 32),
                  d.get("adjoint_table", 0), d.get("stripes", 0), d.get("refill_cost", 0))


def fk_get_launch(precision: int):
    l = fk_launch()
    _check(lib().fk_get_launch(int(precision), C.byref(l)))
    return {k: getattr(l, k) for k in LAUNCH_KEYS}


def fk_timing_enable(on: bool) -> None:
    _check(lib().fk_timing_enable(1 if on else 0))


def fk_timing_read(max_n: int = 256) -> list:
    buf = (C.c_double * max_n)()
    n = C.c_int32()
    _check(lib().fk_timing_read(buf, int(max_n), C.byref(n)))
    return [buf[i] for i in range(n.value)]


def fk_status_string(status: int) -> str:
    return lib().fk_status_string(int(status)).decode()


def fk_version() -> int:
    return int(lib().fk_version())


# --------------------------------------------------------------------------
# Problem marshalling.
# --------------------------------------------------------------------------

def grid_levels(rho):
    """An FP32 density grid as levels: (index, levels), index a uint8 array
    of rho's shape and levels 256 float32 values with levels[index] == rho
    element for element (unused entries NaN).  Raises ValueError for a grid
    of more than 256 distinct values."""
    rho = np.ascontiguousarray(np.asarray(rho, dtype=np.float32))
    values, inverse = np.unique(rho.view(np.uint32), return_inverse=True)
    if values.size > 256:
        raise ValueError(f"the grid has {values.size} distinct densities; levels hold at most 256")
    levels = np.full(256, np.nan, dtype=np.float32)
    levels[:values.size] = values.view(np.float32)
    index = inverse.reshape(rho.shape).astype(np.uint8)
    return index, levels


class Prepared:
    """Device copies and ctypes descriptors of one problem."""

    def __init__(self, prob, device="cuda"):
        import torch
        self.keep = []
        self.prob = prob
        self.box = fk_box((C.c_double * 3)(*np.asarray(prob.box_lo, float)),
                          (C.c_double * 3)(*np.asarray(prob.box_hi, float)))
        self.stations_host = np.ascontiguousarray(np.asarray(prob.stations, dtype=np.float64).reshape(-1, 3))
        self.stations = torch.from_numpy(self.stations_host).to(device)
        src = fk_source()
        if prob.rho is not None and np.asarray(prob.rho).size > 0:
            rho = np.ascontiguousarray(np.asarray(prob.rho, dtype=np.float32))
            nz, ny, nx = rho.shape
            if getattr(prob, "grid_levels", False):
                index, levels = grid_levels(rho)
                self.rho_index = torch.from_numpy(index).to(device)
                self.rho_levels = torch.from_numpy(levels).to(device)
                src.rho_index = self.rho_index.data_ptr()
                src.rho_levels = self.rho_levels.data_ptr()
            else:
                self.rho = torch.from_numpy(rho).to(device)
                src.rho = self.rho.data_ptr()
            src.n = (C.c_int32 * 3)(nx, ny, nz)
            src.origin = (C.c_double * 3)(*np.asarray(prob.grid_origin, float))
            src.spacing = (C.c_double * 3)(*np.asarray(prob.grid_spacing, float))
        pr = np.ascontiguousarray(np.asarray(prob.prisms, dtype=np.float64).reshape(-1, 7))
        sp = np.ascontiguousarray(np.asarray(prob.spheres, dtype=np.float64).reshape(-1, 5))
        self.keep += [pr, sp]
        src.prisms = pr.ctypes.data if len(pr) else None
        src.n_prisms = len(pr)
        src.spheres = sp.ctypes.data if len(sp) else None
        src.n_spheres = len(sp)
        self.source = src
        bc = fk_boundary()
        bc.kind = int(prob.bc_kind)
        data = np.ascontiguousarray(np.asarray(prob.bc_data, dtype=np.float64).ravel())
        if bc.kind == FK_BC_FACE_GRID:
            self.face = torch.from_numpy(data).to(device)
            bc.data = self.face.data_ptr()
            fn = np.asarray(prob.face_n, dtype=np.int32).reshape(6, 2)
            for f in range(6):
                bc.face_n[f][0] = int(fn[f, 0])
                bc.face_n[f][1] = int(fn[f, 1])
        elif data.size:
            self.keep.append(data)
            bc.data = data.ctypes.data
        bc.n_items = int(prob.bc_n_items)
        self.bc = bc
        self.params = make_params(prob)


def make_params(prob, **over) -> fk_params:
    g = lambda k, d=None: over.get(k, getattr(prob, k, d))
    p = fk_params()
    p.paths_per_station = int(g("paths_per_station"))
    p.dt = float(g("dt"))
    p.seed = int(g("seed", 0))
    p.G = float(g("G", 1.0))
    p.h = float(g("h", 0.0))
    p.precision = int(g("precision", 0))
    p.exit_rule = int(g("exit_rule", 0))
    p.pairing = int(g("pairing", 0))
    p.strict = int(g("strict", 0))
    p.max_steps = int(g("max_steps", (1 << 31) - 1))
    p.problem_id = int(g("problem_id", 0))
    p.domain = int(g("domain", 0))
    p.path_offset = int(g("path_offset", 0))
    p.slice_walks = int(g("slice_walks", 0))
    return p


def alloc_workspace(nbytes: int, device="cuda"):
    import torch
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


def alloc_stats(n_stations: int, device="cuda"):
    import torch
    return torch.empty((max(int(n_stations), 1), 8), dtype=torch.int64, device=device)


def stats_to_device(stats: np.ndarray, device="cuda"):
    """A device fk_stat array holding the given structured rows."""
    import torch
    out = alloc_stats(len(stats), device)
    raw = torch.from_numpy(np.ascontiguousarray(stats).view(np.int64).reshape(-1, 8).copy())
    out[: len(stats)].copy_(raw.to(device))
    return out


def stats_to_numpy(out) -> np.ndarray:
    return out.cpu().numpy().view(STAT_DTYPE).reshape(-1)


def solve(prob, kind: int = 0, prepared: Prepared | None = None, workspace=None, stream=None, **over):
    """One solve of a workloads.Problem; returns (stats structured array,
    workspace tensor, prepared problem).  kind 0 = potential, 1 = g_z."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("fkgrav needs a ROCm GPU")
    P = prepared or Prepared(prob)
    params = make_params(prob, **over) if over else P.params
    nb = fk_workspace_bytes(kind, len(P.stations_host), params)
    if nb == 0:
        _check(lib().fk_workspace_layout(int(kind), len(P.stations_host), C.byref(params), None, None, None))
    if workspace is None or workspace.numel() < nb:
        workspace = alloc_workspace(nb)
    out = alloc_stats(len(P.stations_host))
    fn = fk_solve_gz if kind == 1 else fk_solve_potential
    fn(P.stations, P.box, P.source, P.bc, params, out, workspace, stream)
    torch.cuda.synchronize()
    return stats_to_numpy(out)[: len(P.stations_host)], workspace, P


def path_samples(workspace, kind: int, n_stations: int, params: fk_params):
    """The per-walk values and step counts a solve left in its workspace, as
    numpy arrays (potential: [S, N]; g_z: [S, N, 2] for the +h and -h walks)."""
    v_off, s_off, _ = fk_workspace_layout(kind, n_stations, params)
    N = int(params.paths_per_station)
    T = n_stations * N * (2 if kind == 1 else 1)
    vals = workspace[v_off:v_off + 8 * T].view(dtype=__import__("torch").float64).cpu().numpy()
    steps = workspace[s_off:s_off + 4 * T].view(dtype=__import__("torch").int32).cpu().numpy().view(np.uint32)
    shape = (n_stations, N, 2) if kind == 1 else (n_stations, N)
    return vals.reshape(shape), steps.reshape(shape)


class PreparedBatch:
    """Device copies of several problems and the fk_problem array of a batch.
    kinds[m] = 0 (potential) or 1 (g_z); results of problem m are the rows
    offsets[m] .. offsets[m] + n_stations - 1 of the output."""

    def __init__(self, probs, kinds):
        self.items = [Prepared(p) for p in probs]
        self.kinds = list(kinds)
        arr = (fk_problem * len(probs))()
        off = 0
        self.offsets = []
        for m, (P, k) in enumerate(zip(self.items, self.kinds)):
            q = arr[m]
            q.kind = int(k)
            q.stations = P.stations.data_ptr()
            q.n_stations = len(P.stations_host)
            q.box = P.box
            q.source = P.source
            q.bc = P.bc
            q.params = P.params
            q.out_offset = off
            self.offsets.append(off)
            off += len(P.stations_host)
        self.problems = arr
        self.n_out = off


def solve_batch(probs, kinds, prepared: PreparedBatch | None = None, workspace=None, stream=None, sync=True):
    """One batched solve; returns (list of per-problem stats arrays, workspace,
    prepared batch, raw output tensor)."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("fkgrav needs a ROCm GPU")
    PB = prepared or PreparedBatch(probs, kinds)
    nb = fk_batch_workspace_bytes(PB.problems)
    if nb == 0:
        _check(lib().fk_batch_layout(PB.problems, len(PB.problems), 0, None, None))
    if workspace is None or workspace.numel() < nb:
        workspace = alloc_workspace(nb)
    out = alloc_stats(PB.n_out)
    fk_solve_batch(PB.problems, out, workspace, stream)
    if sync:
        torch.cuda.synchronize()
    st = stats_to_numpy(out)
    res = [st[o:o + len(P.stations_host)] for o, P in zip(PB.offsets, PB.items)]
    return res, workspace, PB, out


def batch_path_samples(workspace, PB: PreparedBatch, m: int):
    """Per-walk values and step counts of problem m after a batched solve."""
    import torch
    v_off, s_off = fk_batch_layout(PB.problems, m)
    P = PB.items[m]
    kind = PB.kinds[m]
    S, N = len(P.stations_host), int(P.params.paths_per_station)
    T = S * N * (2 if kind == 1 else 1)
    vals = workspace[v_off:v_off + 8 * T].view(dtype=torch.float64).cpu().numpy()
    steps = workspace[s_off:s_off + 4 * T].view(dtype=torch.int32).cpu().numpy().view(np.uint32)
    shape = (S, N, 2) if kind == 1 else (S, N)
    return vals.reshape(shape), steps.reshape(shape)


def _gradient_function():
    import torch

    class GzFunction(torch.autograd.Function):
        """Station means of a potential (kind 0) or g_z (kind 1) solve as a
        differentiable function of the voxel densities rho (cuda float32,
        shape (nz, ny, nx)).  backward runs the library's adjoint, which
        replays the forward walks; the random streams are fixed by the
        problem's seed, so the forward is an affine function of rho and the
        adjoint is its exact derivative."""

        @staticmethod
        def forward(ctx, rho, prepared, kind):
            P = prepared
            rho_c = rho.detach().contiguous()
            if rho_c.dtype != torch.float32 or not rho_c.is_cuda:
                raise TypeError("rho must be a cuda float32 tensor")
            src = fk_source.from_buffer_copy(P.source)
            src.rho = rho_c.data_ptr()
            src.rho_index = None          # the differentiable densities replace any levels
            src.rho_levels = None
            nz, ny, nx = rho_c.shape
            src.n = (C.c_int32 * 3)(nx, ny, nz)
            nb = fk_workspace_bytes(kind, len(P.stations_host), P.params)
            ws = alloc_workspace(nb)
            out = alloc_stats(len(P.stations_host))
            fn = fk_solve_gz if kind == 1 else fk_solve_potential
            fn(P.stations, P.box, src, P.bc, P.params, out, ws)
            ctx.save_for_backward(rho_c)
            ctx.state = (P, src, kind, ws, out)
            means = out[: len(P.stations_host)].view(torch.float64)[:, 0].clone()
            return means

        @staticmethod
        def backward(ctx, grad_means):
            (rho_c,) = ctx.saved_tensors
            P, src, kind, ws, out = ctx.state
            g = grad_means.detach().to(torch.float64).contiguous()
            grad_rho = torch.empty(rho_c.numel(), dtype=torch.float64, device=rho_c.device)
            aws = alloc_workspace(fk_adjoint_workspace_bytes(len(P.stations_host), src))
            fn = fk_gz_adjoint if kind == 1 else fk_potential_adjoint
            fn(P.stations, P.box, src, P.bc, P.params, out, ws, g, grad_rho, aws)
            return grad_rho.view(rho_c.shape).to(rho_c.dtype), None, None

    return GzFunction


_GZ = None


def gz_function():
    """The torch.autograd.Function class (created on first use, so importing
    this module does not import torch)."""
    global _GZ
    if _GZ is None:
        _GZ = _gradient_function()
    return _GZ


def adjoint(prob, kind: int, grad_out, prepared: Prepared | None = None, stream=None):
    """Forward solve plus the adjoint of a workloads.Problem; returns (stats,
    grad_rho as a float64 numpy array shaped like prob.rho)."""
    import torch
    P = prepared or Prepared(prob)
    stats, ws, P = solve(prob, kind, prepared=P)
    out = stats_to_device(stats, P.stations.device)
    g = torch.as_tensor(np.asarray(grad_out, dtype=np.float64), device=P.stations.device)
    grad_rho = torch.empty(int(np.asarray(prob.rho).size), dtype=torch.float64, device=P.stations.device)
    aws = alloc_workspace(fk_adjoint_workspace_bytes(len(P.stations_host), P.source))
    fn = fk_gz_adjoint if kind == 1 else fk_potential_adjoint
    fn(P.stations, P.box, P.source, P.bc, P.params, out, ws, g, grad_rho, aws, stream)
    torch.cuda.synchronize()
    return stats, grad_rho.cpu().numpy().reshape(np.asarray(prob.rho).shape)
