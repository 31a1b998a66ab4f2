"""The C interface without a GPU: the library loads, exports every function
include/fkgrav.h declares, its struct layouts match the binding's, and every
argument check rejects bad input on the host before anything is launched."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1709_07469_amd import fkgrav as F
from paper_1709_07469_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


# The argument-check tests hand the library stand-in device addresses that
# every check must reject before a launch; they run only where no GPU could
# ever receive such a launch.
host_only = pytest.mark.skipif(_gpu_present(), reason="passes stand-in device pointers; host-only")
HEADER = os.path.join(ROOT, "include", "fkgrav.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fk_[a-z0-9_]+)\s*\(", text)))


def test_header_functions_are_exported():
    L = F.lib()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


def test_enum_values_match_the_binding():
    # every enumerator of the header has the binding's value (and the
    # workload module's, where it names one)
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    found = dict((k, int(v)) for k, v in re.findall(r"\b(FK_[A-Z0-9_]+)\s*=\s*(-?\d+)", text))
    assert len(found) >= 25
    for name, value in found.items():
        assert getattr(F, name) == value, name
    assert (W.EXIT_OVERSHOOT, W.EXIT_INTERSECT, W.EXIT_BRIDGE) == (F.FK_EXIT_OVERSHOOT, F.FK_EXIT_INTERSECT,
                                                                   F.FK_EXIT_BRIDGE)
    assert (W.DOMAIN_BOX, W.DOMAIN_BALL) == (F.FK_DOMAIN_BOX, F.FK_DOMAIN_BALL)
    assert (W.BC_ZERO, W.BC_FACE_GRID, W.PREC_MIXED_KAHAN, W.PAIR_INDEPENDENT) == (
        F.FK_BC_ZERO, F.FK_BC_FACE_GRID, F.FK_MIXED_KAHAN, F.FK_PAIR_INDEPENDENT)


def test_struct_layouts_match_the_c_compiler(tmp_path):
    # every field offset and struct size of the binding against gcc's view of
    # the header
    structs = {"fk_box": F.fk_box, "fk_source": F.fk_source, "fk_boundary": F.fk_boundary,
               "fk_params": F.fk_params, "fk_stat": F.fk_stat, "fk_launch": F.fk_launch,
               "fk_problem": F.fk_problem}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fkgrav.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        name, field, val = line.split()
        cls = structs[name]
        got = C.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(val), (name, field, got, val)
        seen += 1
    assert seen == sum(len(c._fields_) + 1 for c in structs.values())


def _host_problem(**over):
    pr = W.cfg1(100)
    box = F.fk_box((C.c_double * 3)(*pr.box_lo), (C.c_double * 3)(*pr.box_hi))
    sp = np.ascontiguousarray(pr.spheres, dtype=np.float64)
    src = F.fk_source()
    src.spheres = sp.ctypes.data
    src.n_spheres = 1
    bcd = np.ascontiguousarray(pr.bc_data, dtype=np.float64)
    bc = F.fk_boundary()
    bc.kind = F.FK_BC_POINT_MASSES
    bc.data = bcd.ctypes.data
    bc.n_items = 1
    prm = F.make_params(pr, **over)
    return pr, box, src, bc, prm, (sp, bcd)


def _call(box, src, bc, prm, n_stations=8, ws_bytes=None, stations=1, out=1, ws=256):
    L = F.lib()
    if ws_bytes is None:
        ws_bytes = L.fk_workspace_bytes(0, n_stations, C.byref(prm)) or 1 << 20
    return L.fk_solve_potential(C.c_void_p(stations), n_stations, C.byref(box), C.byref(src), C.byref(bc),
                                C.byref(prm), C.c_void_p(out), C.c_void_p(ws), ws_bytes, None)


@host_only
@pytest.mark.parametrize("field,value,status", [
    ("dt", 0.0, F.FK_EINVAL), ("dt", float("nan"), F.FK_EINVAL), ("paths_per_station", 1, F.FK_EINVAL),
    ("precision", 3, F.FK_EINVAL), ("exit_rule", 3, F.FK_EINVAL), ("pairing", 5, F.FK_EINVAL),
    ("domain", 2, F.FK_EINVAL),
    ("max_steps", 0, F.FK_EINVAL), ("G", float("inf"), F.FK_EINVAL), ("h", -1.0, F.FK_EINVAL),
    ("path_offset", (1 << 32) - 50, F.FK_EUNSUPPORTED),
])
def test_bad_params_rejected(field, value, status):
    pr, box, src, bc, prm, keep = _host_problem()
    setattr(prm, field, value)
    assert _call(box, src, bc, prm, ws_bytes=1 << 30) == status
    assert F.lib().fk_last_error().decode() != ""


@host_only
def test_ball_and_bridge_arguments_rejected():
    pr, box, src, bc, prm, keep = _host_problem()
    prm.domain = 1                      # a ball needs a cubic box
    box.hi[0] = box.hi[0] + 0.5
    assert _call(box, src, bc, prm) == F.FK_EINVAL
    box.hi[0] = box.hi[0] - 0.5
    prm.domain = 0
    prm.exit_rule = 2                   # bridge: max_steps <= 2^30
    prm.max_steps = (1 << 30) + 1
    assert _call(box, src, bc, prm) == F.FK_EUNSUPPORTED


@host_only
def test_bad_box_source_boundary_workspace_rejected():
    pr, box, src, bc, prm, keep = _host_problem()
    L = F.lib()
    box.lo[1] = 2.0
    assert _call(box, src, bc, prm) == F.FK_EINVAL
    box.lo[1] = -1.0
    src.n_spheres = F.FK_MAX_SPHERES + 1
    assert _call(box, src, bc, prm) == F.FK_EUNSUPPORTED
    src.n_spheres = 1
    src.rho = 1024
    src.n = (C.c_int32 * 3)(4, 0, 4)
    assert _call(box, src, bc, prm) == F.FK_EINVAL
    src.n = (C.c_int32 * 3)(4, 4, 4)
    src.spacing = (C.c_double * 3)(0.1, -0.1, 0.1)
    assert _call(box, src, bc, prm) == F.FK_EINVAL
    src.spacing = (C.c_double * 3)(0.1, 0.1, 0.1)
    src.n = (C.c_int32 * 3)(1, 1 << 24, 1)  # an axis of 2^24 voxels (the row offset is a 24-bit product)
    assert _call(box, src, bc, prm) == F.FK_EUNSUPPORTED
    assert "2^24" in L.fk_last_error().decode()
    src.n = (C.c_int32 * 3)((1 << 24) - 1, 1 << 7, 2)   # 2^32 - 2^8 voxels
    assert _call(box, src, bc, prm) == F.FK_EUNSUPPORTED
    assert "2^31-1 voxels" in L.fk_last_error().decode()
    src.n = (C.c_int32 * 3)(4, 4, 4)
    src.rho_index = 2048                # the grid both as densities and by levels
    src.rho_levels = 4096
    assert _call(box, src, bc, prm) == F.FK_EINVAL
    assert "not both" in L.fk_last_error().decode()
    src.rho = None
    src.rho_levels = None               # an index grid without its levels
    assert _call(box, src, bc, prm) == F.FK_EINVAL
    assert "rho_levels" in L.fk_last_error().decode()
    src.rho_index = None
    src.rho = None
    bc.kind = 9
    assert _call(box, src, bc, prm) == F.FK_EINVAL
    bc.kind = F.FK_BC_PRISMS
    bc.n_items = 0
    assert _call(box, src, bc, prm) == F.FK_EUNSUPPORTED
    bc.kind = F.FK_BC_FACE_GRID
    bc.n_items = 0
    assert _call(box, src, bc, prm) == F.FK_EINVAL           # face_n all zero
    bc.kind = F.FK_BC_POINT_MASSES
    bc.n_items = 1
    need = L.fk_workspace_bytes(0, 8, C.byref(prm))
    assert _call(box, src, bc, prm, ws_bytes=need - 1) == F.FK_EWORKSPACE
    assert _call(box, src, bc, prm, ws=256 + 8) == F.FK_EWORKSPACE   # misaligned
    assert _call(box, src, bc, prm, out=0) == F.FK_EINVAL
    assert _call(box, src, bc, prm, stations=0) == F.FK_EINVAL
    # no stations: nothing to do, nothing launched, no device needed
    assert _call(box, src, bc, prm, n_stations=0, stations=0, out=0, ws=0) == F.FK_OK


def test_station_domain_check():
    pr, box, src, bc, prm, keep = _host_problem()
    st = np.array([[0.0, 0.0, 0.5], [0.0, 0.0, 0.99]])
    F.fk_check_stations(st, box, 0, prm)
    with pytest.raises(F.FkError) as e:
        F.fk_check_stations(st, box, 1, prm)           # 0.99 + sqrt(1e-3) leaves the box
    assert e.value.status == F.FK_EDOMAIN
    with pytest.raises(F.FkError) as e:
        F.fk_check_stations(np.array([[0.0, 0.0, 1.0]]), box, 0, prm)
    assert e.value.status == F.FK_EDOMAIN


def test_workspace_layout_and_launch_settings():
    pr = W.cfg2()
    prm = F.make_params(pr)
    v, s, t = F.fk_workspace_layout(0, 64, prm)
    T = 64 * pr.paths_per_station
    # the status block, then the per-walk values, step counts and exit records
    assert v == 256 and s >= v + 8 * T and s % 256 == 0 and t >= s + 4 * T + 32 * T
    v1, s1, t1 = F.fk_workspace_layout(1, 64, prm)
    assert s1 >= 16 * T and t1 > t
    assert F.fk_workspace_bytes(0, 64, prm) == t
    old = F.fk_get_launch(0)
    F.fk_set_launch(0, 128, 2, 16)
    assert F.fk_get_launch(0) == {"block": 128, "blocks_per_cu": 2, "grab": 16, "adjoint_table": 0, "stripes": 0,
                                  "refill_cost": 0}
    F.fk_set_launch(0, 128, 2, 16, adjoint_table=1, stripes=16, refill_cost=32)
    got = F.fk_get_launch(0)
    assert (got["adjoint_table"], got["stripes"], got["refill_cost"]) == (1, 16, 32)
    for bad in ({"adjoint_table": 2}, {"stripes": 33}, {"stripes": -1}, {"refill_cost": 9000}):
        with pytest.raises(F.FkError):
            F.fk_set_launch(0, 128, 2, 16, **bad)
    with pytest.raises(F.FkError):
        F.fk_set_launch(0, 96)
    with pytest.raises(F.FkError):
        F.fk_set_launch(0, 512)
    F.fk_set_launch_dict(0, old)
    assert F.fk_status_string(F.FK_EDOMAIN).startswith("station")
    assert F.fk_version() >= 100


def test_timing_read_without_solves():
    F.fk_timing_enable(True)
    assert F.fk_timing_read() == []
    F.fk_timing_enable(False)


def test_product_path_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        F.solve(W.cfg1(10), 0)


def test_bounded_workspace_sizes():
    # slice_walks > 0: the workspace holds one slice's records (36 B per walk)
    # and 48 B per (station, chunk) pair, whatever the walk count
    pr = W.cfg2()
    rec = F.make_params(pr)
    full = F.fk_workspace_bytes(1, 64, rec)
    sl = F.make_params(pr, slice_walks=1 << 20)
    small = F.fk_workspace_bytes(1, 64, sl)
    pairs = 64 * ((pr.paths_per_station + 8191) // 8192)
    assert 0 < small < full
    assert small >= 36 * (1 << 20) + 48 * pairs
    assert small <= 36 * (1 << 20) + 48 * pairs + 5 * 256
    big = F.make_params(pr.replace(paths_per_station=1 << 31), slice_walks=1 << 20)
    assert F.fk_workspace_bytes(1, 64, big) < 36 * (1 << 20) + 48 * 64 * (1 << 18) + 5 * 256
    # per-walk records exist in record mode only
    with pytest.raises(F.FkError) as e:
        F.fk_workspace_layout(1, 64, sl)
    assert e.value.status == F.FK_EINVAL
    # a slice holds at least one chunk of 8192 paths per walk of a pair
    for kind, bad in ((0, 8191), (1, 16383), (0, -1)):
        assert F.fk_workspace_bytes(kind, 64, F.make_params(pr, slice_walks=bad)) == 0
    assert F.fk_workspace_bytes(0, 64, F.make_params(pr, slice_walks=8192)) > 0


def test_batch_slice_walks_must_agree():
    from paper_1709_07469_amd import workloads as Wl
    a = Wl.cfg1(100)
    b = Wl.cfg1(100).replace(slice_walks=1 << 16)
    arr = (F.fk_problem * 2)()
    keep = []
    for m, pr in enumerate((a, b)):
        _, box, src, bc, prm, k = _host_problem(slice_walks=pr.slice_walks)
        keep.append(k)
        arr[m].kind = 0
        arr[m].stations = 4096
        arr[m].n_stations = 8
        arr[m].box = box
        arr[m].source = src
        arr[m].bc = bc
        arr[m].params = prm
        arr[m].out_offset = 8 * m
    assert F.lib().fk_batch_workspace_bytes(arr, 2) == 0
    assert "slice_walks" in F.lib().fk_last_error().decode()


def test_workspace_status_rejects_null():
    st = F.lib().fk_workspace_status(None, None, None)
    assert st == F.FK_EINVAL
    assert F.fk_status_string(F.FK_ENONFINITE) != "unknown status"
    assert F.fk_status_string(F.FK_ETRUNC) != "unknown status"


def test_batch_grids_of_one_kind():
    """A batch's grids are all FP32 densities or all given by levels: one
    kernel instance looks them up."""
    arr = (F.fk_problem * 2)()
    keep = []
    for m in range(2):
        _, box, src, bc, prm, k = _host_problem()
        keep.append(k)
        src.n = (C.c_int32 * 3)(4, 4, 4)
        src.spacing = (C.c_double * 3)(0.5, 0.5, 0.5)
        if m == 0:
            src.rho = 1024
        else:
            src.rho_index = 2048
            src.rho_levels = 4096
        arr[m].kind = 0
        arr[m].stations = 4096
        arr[m].n_stations = 8
        arr[m].box = box
        arr[m].source = src
        arr[m].bc = bc
        arr[m].params = prm
        arr[m].out_offset = 8 * m
    assert F.lib().fk_batch_workspace_bytes(arr, 2) == 0
    assert "levels" in F.lib().fk_last_error().decode()
    arr[1].source.rho_index = None
    arr[1].source.rho_levels = None
    arr[1].source.rho = 1024
    assert F.lib().fk_batch_workspace_bytes(arr, 2) > 0


def test_grid_levels_round_trip():
    rng = np.random.Generator(np.random.PCG64(7))
    vals = np.array([0.0, -0.0, 1.5, 2.0e3, np.float32(1) / 3, -7.25], dtype=np.float32)
    rho = vals[rng.integers(0, len(vals), size=(5, 6, 7))]
    index, levels = F.grid_levels(rho)
    assert index.dtype == np.uint8 and index.shape == rho.shape and levels.shape == (256,)
    back = levels[index]
    assert back.view(np.uint32).tolist() == rho.view(np.uint32).tolist()    # bit for bit, -0 kept
    assert np.isnan(levels[len(vals):]).all()
    with pytest.raises(ValueError):
        F.grid_levels(np.arange(257, dtype=np.float32).reshape(1, 1, 257))
