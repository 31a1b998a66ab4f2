"""The oracle: a plain FP64 CPU implementation of the Monte Carlo Feynman-Kac
gravity estimator (arXiv:1709.07469, section 2), written in C in
``fk_oracle.c`` and loaded here with ctypes.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It never imports the
product package and the product never imports it; the two meet only through
the seeded problem descriptions the tests build (any object carrying the
attributes listed in ``_marshal``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fk_oracle.c")
_LIB = os.path.join(_HERE, "libfk_oracle.so")
_lock = threading.Lock()
_lib = None

TRUNC_FLAG = 0x80000000
STREAM_F64, STREAM_F32 = 0, 1


def build(force: bool = False) -> str:
    """Compiles fk_oracle.c with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class Box(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class Source(C.Structure):
    _fields_ = [("rho", C.c_void_p), ("n", C.c_int32 * 3), ("origin", C.c_double * 3),
                ("spacing", C.c_double * 3), ("prisms", C.c_void_p), ("n_prisms", C.c_int32),
                ("spheres", C.c_void_p), ("n_spheres", C.c_int32)]


class BC(C.Structure):
    _fields_ = [("kind", C.c_int32), ("data", C.c_void_p), ("n_items", C.c_int64),
                ("face_n", (C.c_int32 * 2) * 6)]


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("seed", C.c_uint64), ("G", C.c_double), ("h", C.c_double),
                ("stream", C.c_int32), ("exit_rule", C.c_int32), ("pairing", C.c_int32),
                ("domain", C.c_int32), ("max_steps", C.c_int64), ("problem_id", C.c_uint32),
                ("pad2_", C.c_uint32), ("path_offset", C.c_int64)]


class Stat(C.Structure):
    _fields_ = [("mean", C.c_double), ("var", C.c_double), ("se", C.c_double), ("n", C.c_int64),
                ("mean_steps", C.c_double), ("max_steps", C.c_int64), ("n_trunc", C.c_int64)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB)
            d, p, i32, i64, u32, u64 = C.c_double, C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
            L.fko_philox4x32_10.argtypes = [p, p, p]
            L.fko_normal.argtypes = [i32, u64, u32, u32, u32, i64]
            L.fko_normal.restype = d
            L.fko_bridge_uniform.argtypes = [i32, u64, u32, u32, u32, i64]
            L.fko_bridge_uniform.restype = d
            L.fko_rho.argtypes = [p, p]
            L.fko_rho.restype = d
            L.fko_voxel_index.argtypes = [p, p]
            L.fko_voxel_index.restype = i64
            L.fko_bc_value.argtypes = [p, p, d, p]
            L.fko_bc_value.restype = d
            for nm in ("fko_prism_potential", "fko_prism_gz"):
                getattr(L, nm).argtypes = [p, p, d, d, p]
                getattr(L, nm).restype = d
            L.fko_prism_newton.argtypes = [p, p, p]
            L.fko_prism_newton.restype = d
            for nm in ("fko_sphere_potential", "fko_sphere_gz"):
                getattr(L, nm).argtypes = [p, d, d, d, p]
                getattr(L, nm).restype = d
            L.fko_run_paths.argtypes = [i32, p, i64, p, p, p, p, p, i64, p, p, p, p, i32]
            L.fko_run_paths.restype = i32
            L.fko_station_stats.argtypes = [p, p, i64, p]
            L.fko_occupation.argtypes = [i32, p, i64, p, p, p, p, i64, i64, p, p, i32]
            L.fko_occupation.restype = i32
            L.fko_max_threads.restype = i32
            L.fko_moving_average.argtypes = [p, p, i64, i32, p, p]
            L.fko_moving_average.restype = i32
            _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


class _Marshalled:
    """Holds the ctypes structures and the numpy buffers they point into."""

    def __init__(self, prob, stream=None, **overrides):
        g = lambda k, dflt=None: overrides.get(k, getattr(prob, k, dflt))
        self.keep = []
        self.box = Box((C.c_double * 3)(*_f64(g("box_lo"))), (C.c_double * 3)(*_f64(g("box_hi"))))
        rho = g("rho")
        src = Source()
        if rho is not None and np.asarray(rho).size > 0:
            rho = np.ascontiguousarray(np.asarray(rho, dtype=np.float32))
            self.keep.append(rho)
            nz, ny, nx = rho.shape
            src.rho = rho.ctypes.data
            src.n = (C.c_int32 * 3)(nx, ny, nz)
            src.origin = (C.c_double * 3)(*_f64(g("grid_origin")))
            src.spacing = (C.c_double * 3)(*_f64(g("grid_spacing")))
        prisms = _f64(g("prisms", np.zeros((0, 7))), (-1, 7))
        spheres = _f64(g("spheres", np.zeros((0, 5))), (-1, 5))
        self.keep += [prisms, spheres]
        src.prisms = prisms.ctypes.data if len(prisms) else None
        src.n_prisms = len(prisms)
        src.spheres = spheres.ctypes.data if len(spheres) else None
        src.n_spheres = len(spheres)
        self.src = src
        bc = BC()
        bc.kind = int(g("bc_kind", 0))
        bcd = _f64(g("bc_data", np.zeros(0)))
        self.keep.append(bcd)
        bc.data = bcd.ctypes.data if bcd.size else None
        bc.n_items = int(g("bc_n_items", 0))
        fn = np.asarray(g("face_n", np.zeros((6, 2), dtype=np.int32)), dtype=np.int32).reshape(6, 2)
        for f in range(6):
            bc.face_n[f][0] = int(fn[f, 0])
            bc.face_n[f][1] = int(fn[f, 1])
        self.bc = bc
        prm = Params()
        prm.dt = float(g("dt"))
        prm.seed = int(g("seed", 0))
        prm.G = float(g("G", 1.0))
        prm.h = float(g("h", 0.0))
        if stream is None:
            stream = STREAM_F64 if int(g("precision", 0)) == 0 else STREAM_F32
        prm.stream = int(stream)
        prm.exit_rule = int(g("exit_rule", 0))
        prm.pairing = int(g("pairing", 0))
        prm.domain = int(g("domain", 0))
        prm.max_steps = int(g("max_steps", 1 << 30))
        prm.problem_id = int(g("problem_id", 0))
        prm.path_offset = int(g("path_offset", 0))
        self.prm = prm
        self.stations = _f64(g("stations"), (-1, 3))
        self.keep.append(self.stations)


def philox4x32_10(counter, key):
    """The oracle's Philox4x32-10 block for a 4-word counter and 2-word key."""
    c = np.asarray(counter, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().fko_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def normal(stream, seed, m, s, p, j):
    return lib().fko_normal(int(stream), int(seed), int(m), int(s), int(p), int(j))


def bridge_uniform(stream, seed, m, s, p, n):
    return lib().fko_bridge_uniform(int(stream), int(seed), int(m), int(s), int(p), int(n))


def rho_at(prob, x):
    M = _Marshalled(prob)
    x = _f64(x)
    return lib().fko_rho(C.byref(M.src), _ptr(x))


def voxel_index(prob, x):
    M = _Marshalled(prob)
    x = _f64(x)
    return lib().fko_voxel_index(C.byref(M.src), _ptr(x))


def bc_value(prob, x):
    M = _Marshalled(prob)
    x = _f64(x)
    return lib().fko_bc_value(C.byref(M.bc), C.byref(M.box), M.prm.G, _ptr(x))


def prism_potential(lo, hi, rho, G, P):
    return lib().fko_prism_potential(_ptr(_f64(lo)), _ptr(_f64(hi)), float(rho), float(G), _ptr(_f64(P)))


def prism_newton(lo, hi, P):
    return lib().fko_prism_newton(_ptr(_f64(lo)), _ptr(_f64(hi)), _ptr(_f64(P)))


def prism_gz(lo, hi, rho, G, P):
    return lib().fko_prism_gz(_ptr(_f64(lo)), _ptr(_f64(hi)), float(rho), float(G), _ptr(_f64(P)))


def sphere_potential(c, a, rho, G, P):
    return lib().fko_sphere_potential(_ptr(_f64(c)), float(a), float(rho), float(G), _ptr(_f64(P)))


def sphere_gz(c, a, rho, G, P):
    return lib().fko_sphere_gz(_ptr(_f64(c)), float(a), float(rho), float(G), _ptr(_f64(P)))


def exact_potential(prob, P):
    """Sum of the closed-form potentials of the problem's analytic bodies
    (prisms and spheres) at P; voxel grids are not included."""
    G = float(prob.G)
    v = 0.0
    for q in np.asarray(getattr(prob, "prisms", np.zeros((0, 7)))).reshape(-1, 7):
        v += prism_potential(q[:3], q[3:6], q[6], G, P)
    for q in np.asarray(getattr(prob, "spheres", np.zeros((0, 5)))).reshape(-1, 5):
        v += sphere_potential(q[:3], q[3], q[4], G, P)
    return v


def exact_gz(prob, P):
    G = float(prob.G)
    v = 0.0
    for q in np.asarray(getattr(prob, "prisms", np.zeros((0, 7)))).reshape(-1, 7):
        v += prism_gz(q[:3], q[3:6], q[6], G, P)
    for q in np.asarray(getattr(prob, "spheres", np.zeros((0, 5)))).reshape(-1, 5):
        v += sphere_gz(q[:3], q[3], q[4], G, P)
    return v


def run_paths(prob, kind, items, stream=None, threads=0, want_aux=False, want_exit=False, **overrides):
    """Runs the (station, local path) pairs in ``items``.  kind 0 = potential
    samples u_p; kind 1 = g_z samples (u+ - u-)/(2h).  Returns (u, steps) or
    (u, steps, aux, xe) with aux the (u+, u-) pairs of kind 1."""
    M = _Marshalled(prob, stream=stream, **overrides)
    items = np.ascontiguousarray(np.asarray(items, dtype=np.int64).reshape(-1, 2))
    n = len(items)
    u = np.zeros(n, dtype=np.float64)
    st = np.zeros(n, dtype=np.uint32)
    aux = np.zeros((n, 2), dtype=np.float64) if want_aux else None
    xe = np.zeros((n, 3), dtype=np.float64) if want_exit else None
    rc = lib().fko_run_paths(int(kind), _ptr(M.stations), len(M.stations), C.byref(M.box),
                             C.byref(M.src), C.byref(M.bc), C.byref(M.prm), _ptr(items), n,
                             _ptr(u), _ptr(st), _ptr(aux), _ptr(xe), int(threads))
    if rc != 0:
        raise ValueError("oracle: bad item list")
    if want_aux or want_exit:
        return u, st, aux, xe
    return u, st


def station_stats(u, steps):
    """Plain two-pass statistics of one station's samples in path order."""
    u = _f64(u)
    steps = np.ascontiguousarray(np.asarray(steps, dtype=np.uint32))
    s = Stat()
    lib().fko_station_stats(_ptr(u), _ptr(steps), len(u), C.byref(s))
    return {k: getattr(s, k) for k, _ in Stat._fields_}


def solve(prob, kind=0, n_paths=None, i_begin=0, stream=None, threads=0, **overrides):
    """All stations, local paths [i_begin, i_begin + n_paths).  Returns
    (stats list, u[S, n], steps[S, n])."""
    N = int(n_paths if n_paths is not None else prob.paths_per_station)
    S = len(np.asarray(prob.stations).reshape(-1, 3))
    ii = np.arange(i_begin, i_begin + N, dtype=np.int64)
    items = np.stack([np.repeat(np.arange(S, dtype=np.int64), N), np.tile(ii, S)], axis=1)
    u, st = run_paths(prob, kind, items, stream=stream, threads=threads, **overrides)
    u = u.reshape(S, N)
    st = st.reshape(S, N)
    stats = [station_stats(u[s], st[s]) for s in range(S)]
    return stats, u, st


def occupation(prob, kind, i_begin, i_end, stream=None, threads=0, **overrides):
    """Per-station voxel occupation counts (trapezoid weights) of the local
    paths [i_begin, i_end).  Returns (c_plus[S, nvox], c_minus or None)."""
    M = _Marshalled(prob, stream=stream, **overrides)
    S = len(M.stations)
    nvox = int(M.src.n[0]) * int(M.src.n[1]) * int(M.src.n[2])
    cp = np.zeros((S, nvox), dtype=np.uint64)
    cm = np.zeros((S, nvox), dtype=np.uint64) if kind == 1 else None
    rc = lib().fko_occupation(int(kind), _ptr(M.stations), S, C.byref(M.box), C.byref(M.src),
                              C.byref(M.bc), C.byref(M.prm), int(i_begin), int(i_end),
                              _ptr(cp), _ptr(cm), int(threads))
    if rc != 0:
        raise ValueError("oracle: occupation needs a voxel grid")
    return cp, cm


def moving_average(values, se=None, span=5):
    v = _f64(values).ravel()
    e = None if se is None else _f64(se).ravel()
    out = np.empty_like(v)
    oe = None if e is None else np.empty_like(e)
    if lib().fko_moving_average(_ptr(v), _ptr(e), len(v), int(span), _ptr(out), _ptr(oe)) != 0:
        raise ValueError("span must be a positive odd number")
    return out, oe


def max_threads():
    return lib().fko_max_threads()
