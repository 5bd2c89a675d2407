"""The C ABI without a GPU: the library loads, exports every declared entry
point, validates descriptors on the host and maps statistics to statuses."""
import ctypes as C
import os
import re

import pytest

from paper_1810_01780_amd import binding as B
from paper_1810_01780_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = declared_functions()
    assert set(names) >= {"rt_abi_version", "rt_validate", "rt_workspace_bytes",
                          "raytrace_launch", "rt_collect", "rt_last_error"}
    for n in names:
        assert hasattr(lib, n), n
    assert B.rt_abi_version() == B.ABI_VERSION == 8
    assert C.sizeof(B.rt_tuning) == 48 and B.rt_tuning.solve_fused.offset == 40


def test_struct_layouts_match_header():
    # sizes follow from the header's field lists on x86-64
    assert C.sizeof(B.rt_region) == 80
    assert C.sizeof(B.rt_anomaly) == 48
    assert C.sizeof(B.rt_field) == 104 and B.rt_field.n_anomalies.offset == 88
    assert C.sizeof(B.rt_plane) == 72
    assert C.sizeof(B.rt_step_limits) == 80
    assert C.sizeof(B.rt_stats) == 8 * len(B.STAT_FIELDS)
    assert C.sizeof(B.rt_outputs) == 8 * (len(B.RECORD_FIELDS) + 4)
    assert C.sizeof(B.rt_event) == 216 == B.EVENT_DTYPE.itemsize
    assert B.rt_event.pos.offset == 32 and B.rt_event.coef.offset == 152
    for f in B.EVENT_DTYPE.names:
        assert B.EVENT_DTYPE.fields[f][1] == getattr(B.rt_event, f).offset, f


def _descs(scene=None, **lim):
    scene = scene or W.point_source_fan(n_rays=8)
    d = B.HostDescriptors(scene)
    # fake (never dereferenced) device pointers: validation is host-only
    d.sources.xyz = 0x1000
    d.dirs.xyz = 0x2000
    d.dirs.src = 0x3000
    for k, v in lim.items():
        setattr(d.limits, k, v)
    return d


def _validate(d, tol=None):
    return B.rt_validate(d.field, d.bnd, d.sources, d.dirs, d.tol if tol is None else tol,
                         d.limits)


def test_validate_accepts_workloads():
    for sc in (W.point_source_fan(n_rays=8), W.two_layer(rays_per_source=1)):
        assert _validate(_descs(sc)) == B.RT_OK


@pytest.mark.parametrize("change,code", [
    (dict(h_min=0.0), B.RT_ERR_INVALID_ARG),
    (dict(h_min=20.0), B.RT_ERR_INVALID_ARG),          # h_min > h_max
    (dict(s_max=0.0), B.RT_ERR_INVALID_ARG),
    (dict(t_max=-1.0), B.RT_ERR_INVALID_ARG),
    (dict(amp_min=-0.1), B.RT_ERR_INVALID_ARG),
    (dict(max_generations=0), B.RT_ERR_INVALID_ARG),
    (dict(max_generations=5), B.RT_ERR_UNSUPPORTED),
    (dict(model=7), B.RT_ERR_INVALID_ARG),
    (dict(max_steps_per_ray=0), B.RT_ERR_INVALID_ARG),
])
def test_validate_rejects_bad_limits(change, code):
    d = _descs(**change)
    assert _validate(d) == code
    assert B.rt_last_error()


def test_validate_rejects_bad_descriptors():
    d = _descs()
    assert _validate(d, tol=0.0) == B.RT_ERR_INVALID_ARG
    assert _validate(d, tol=float("nan")) == B.RT_ERR_INVALID_ARG
    d = _descs()
    d.bnd.planes[0].normal = (C.c_double * 3)(0.0, 0.0, 0.0)
    assert _validate(d) == B.RT_ERR_INVALID_ARG and "normal" in B.rt_last_error()
    d = _descs()
    d.bnd.planes[0].region_pos = 9
    assert _validate(d) == B.RT_ERR_INVALID_ARG
    d = _descs()
    d.bnd.planes[0].kind = 5
    assert _validate(d) == B.RT_ERR_INVALID_ARG
    d = _descs()
    d.bnd.n_planes = B.RT_MAX_PLANES + 1
    assert _validate(d) == B.RT_ERR_INVALID_ARG
    d = _descs()
    d.field.n_regions = 0
    assert _validate(d) == B.RT_ERR_INVALID_ARG
    d = _descs()
    d.bnd.box_lo = (C.c_double * 3)(0.0, 0.0, 5.0)
    d.bnd.box_hi = (C.c_double * 3)(1.0, 1.0, 5.0)
    assert _validate(d) == B.RT_ERR_INVALID_ARG
    d = _descs()
    d.dirs.xyz = None
    assert _validate(d) == B.RT_ERR_INVALID_ARG
    d = _descs()
    d.dirs.n = 0          # an empty launch is valid
    assert _validate(d) == B.RT_OK


def test_validate_grid_descriptor():
    sc = W.gridded(rays_per_source=1, n_sources=2, nx=4, ny=4, nz=4)
    d = _descs(sc)
    assert _validate(d) == B.RT_ERR_INVALID_ARG  # grid data pointer still NULL
    d.field.grid.n = 0x4000
    assert _validate(d) == B.RT_OK
    d.field.grid.nz = 1
    assert _validate(d) == B.RT_ERR_INVALID_ARG
    d.field.grid.nz = 4
    d.field.grid.spacing = (C.c_double * 3)(10.0, 0.0, 10.0)
    assert _validate(d) == B.RT_ERR_INVALID_ARG
    # the prepared nodes are addressed with 32-bit byte offsets: 512 x 512 x
    # 128 = 2^25 bricks of 128 bytes are one byte too many (nz = 255 still
    # needs 128 brick layers), 127 layers are accepted
    d.field.grid.spacing = (C.c_double * 3)(10.0, 10.0, 10.0)
    d.field.grid.nx, d.field.grid.ny = 1024, 1024
    for nz, want in ((256, B.RT_ERR_UNSUPPORTED), (255, B.RT_ERR_UNSUPPORTED), (254, B.RT_OK)):
        d.field.grid.nz = nz
        assert _validate(d) == want, nz


def test_workspace_bytes():
    d = _descs()
    # counters, then the overflow queue, the hand-out order and its per-chunk
    # sorted form (4 B per record each, padded to 4 KiB), the chunk keys
    # (8 B per 16,384 records, one more, padded), then the grid nodes in
    # bricks of 2 x 2 x 2 float4
    assert B.rt_workspace_bytes(d.field, 0) == 4096 + 4096
    assert B.rt_workspace_bytes(d.field, 1) == 4096 + 3 * 4096 + 4096
    assert B.rt_workspace_bytes(d.field, 2048) == 4096 + 3 * 8192 + 4096
    assert B.rt_workspace_bytes(d.field, 1 << 30) == 4096 + 3 * (4 << 30) + 528384
    sc = W.gridded(rays_per_source=1, n_sources=2, nx=4, ny=5, nz=6)
    d = _descs(sc)
    assert B.rt_workspace_bytes(d.field, 1024) == 4096 + 3 * 4096 + 4096 + 2 * 3 * 3 * 128


def test_collect_maps_statistics():
    s = B.rt_stats()
    s.needed = 10
    assert B.rt_collect(s, 10) == B.RT_OK
    assert B.rt_collect(s, 9) == B.RT_ERR_CAPACITY
    s.invalid = 1
    assert B.rt_collect(s, 10) == B.RT_ERR_INVALID_ARG
    s.sched_errors = 1
    assert B.rt_collect(s, 10) == B.RT_ERR_DEVICE
    s2 = B.rt_stats()
    s2.nonfinite = 3          # per-ray status, not a launch failure
    assert B.rt_collect(s2, 0) == B.RT_OK
    s3 = B.rt_stats()
    s3.events, s3.events_lost = 12, 2
    assert B.rt_collect(s3, 0) == B.RT_ERR_CAPACITY and "ev_capacity >= 12" in B.rt_last_error()


def test_launch_validates_before_touching_the_device():
    d = _descs(h_min=-1.0)
    out = B.rt_outputs()
    st = B.raytrace_launch(d.field, d.bnd, d.sources, d.dirs, d.tol, d.limits, out, 0, 0, 0)
    assert st == B.RT_ERR_INVALID_ARG
    d = _descs()
    st = B.raytrace_launch(d.field, d.bnd, d.sources, d.dirs, d.tol, d.limits, out, 0, 0, 0)
    assert st == B.RT_ERR_INVALID_ARG and "null" in B.rt_last_error()
    # fake (never dereferenced) output arrays: the event arguments are checked
    # on the host before anything is enqueued
    out = B.rt_outputs(*([0x10000 * (i + 1) for i in range(len(B.RECORD_FIELDS))]
                         + [d.dirs.n, 0x900000, None, -1]))
    ws = 0xA00000
    st = B.raytrace_launch(d.field, d.bnd, d.sources, d.dirs, d.tol, d.limits, out, ws, 0, 0)
    assert st == B.RT_ERR_INVALID_ARG and "ev_capacity" in B.rt_last_error()
    out.ev_capacity = 16
    st = B.raytrace_launch(d.field, d.bnd, d.sources, d.dirs, d.tol, d.limits, out, ws, 0, 0)
    assert st == B.RT_ERR_INVALID_ARG and "ev_capacity" in B.rt_last_error()
    out.ev_capacity = 0   # then the workspace size is the next check
    st = B.raytrace_launch(d.field, d.bnd, d.sources, d.dirs, d.tol, d.limits, out, ws, 0, 0)
    assert st == B.RT_ERR_INVALID_ARG and "workspace" in B.rt_last_error()


# --- emitter -> receiver solves ---------------------------------------------
def _solve_descs(**lim):
    d = B.HostDescriptors(W.solve_pairs(8).scene)
    for k, v in lim.items():
        setattr(d.limits, k, v)
    return d


def test_solve_validate():
    d = _solve_descs()
    p = B.solve_params()
    assert B.rt_solve_validate(d.field, d.bnd, d.tol, d.limits, p) == B.RT_OK
    assert B.rt_solve_validate(d.field, d.bnd, d.tol, d.limits, None) == B.RT_OK
    # unused by shots: s_max, amp_min, max_generations
    d2 = _solve_descs(s_max=0.0, amp_min=-1.0, max_generations=9)
    assert B.rt_solve_validate(d2.field, d2.bnd, d2.tol, d2.limits, p) == B.RT_OK
    d3 = _solve_descs(t_max=1e-6)
    assert B.rt_solve_validate(d3.field, d3.bnd, d3.tol, d3.limits, p) == B.RT_ERR_INVALID_ARG
    assert B.rt_solve_validate(d.field, d.bnd, 0.0, d.limits, p) == B.RT_ERR_INVALID_ARG
    for bad in (dict(n_scan=1), dict(n_scan=5000), dict(max_iter=0), dict(max_brackets=17),
                dict(miss_tol=0.0), dict(miss_tol=1e-3, accept_tol=1e-4),
                dict(slope_max=-1.0), dict(slope_max=float("inf"))):
        q = B.solve_params(**bad)
        assert B.rt_solve_validate(d.field, d.bnd, d.tol, d.limits, q) == B.RT_ERR_INVALID_ARG
        assert B.rt_last_error()


def test_solve_validate_boundaries():
    p = B.solve_params()
    d = _solve_descs()
    d.bnd.has_box = 1
    d.bnd.box_lo = (C.c_double * 3)(-1.0, -1.0, -1.0)
    d.bnd.box_hi = (C.c_double * 3)(1.0, 1.0, 1.0)
    assert B.rt_solve_validate(d.field, d.bnd, d.tol, d.limits, p) == B.RT_ERR_INVALID_ARG
    d = _solve_descs()
    d.bnd.planes[0].kind = 1     # RT_PLANE_ABSORB: not a reflecting surface
    assert B.rt_solve_validate(d.field, d.bnd, d.tol, d.limits, p) == B.RT_ERR_INVALID_ARG
    d = _solve_descs()
    d.bnd.n_planes = 0
    assert B.rt_solve_validate(d.field, d.bnd, d.tol, d.limits, p) == B.RT_ERR_INVALID_ARG
    g = B.HostDescriptors(W.gridded(rays_per_source=1, n_sources=2, nx=4, ny=4, nz=4))
    g.field.grid.n = 0x4000
    g.bnd.has_box = 0
    g.limits.t_max = 0.0
    assert B.rt_solve_validate(g.field, g.bnd, g.tol, g.limits, p) == B.RT_ERR_UNSUPPORTED


def test_solve_workspace_bytes():
    d = _solve_descs()
    p = B.solve_params(n_scan=64, max_brackets=4)
    assert B.rt_solve_workspace_bytes(d.field, 0) == 4096
    # 20 (pair, family) entries: 64 misses x 8 B = 10240 -> 12288; 4 brackets x 80 B = 6400 -> 8192
    assert B.rt_solve_workspace_bytes(d.field, 10, p) == 4096 + 12288 + 8192
    with pytest.raises(B.RTError):
        B.rt_solve_workspace_bytes(d.field, 10, None)


def test_solve_and_shoot_validate_before_touching_the_device():
    d = _solve_descs()
    p = B.solve_params()
    pairs = B.rt_pairs(0x1000, 0x2000, 0x3000, 4)
    out = B.rt_solve_outputs()
    st = B.raytrace_solve(d.field, d.bnd, d.tol, d.limits, pairs, p, out, 0, 0, 0)
    assert st == B.RT_ERR_INVALID_ARG and "null" in B.rt_last_error()
    shots = B.rt_shots(0x1000, 0x2000, 0x3000, 0x4000, 0x5000, 4)
    sout = B.rt_shot_outputs()
    st = B.raytrace_shoot(d.field, d.bnd, d.tol, d.limits, shots, sout, 0, 0, 0)
    assert st == B.RT_ERR_INVALID_ARG and "null" in B.rt_last_error()
    bad = B.solve_params(max_iter=0)
    st = B.raytrace_solve(d.field, d.bnd, d.tol, d.limits, pairs, bad, out, 0, 0, 0)
    assert st == B.RT_ERR_INVALID_ARG


def test_validate_curved_boundaries():
    d = _descs(W.curved(n_sources=1, rays_per_source=4))
    assert _validate(d) == B.RT_OK
    d.bnd.planes[1].param = 0.0           # sphere of radius 0
    assert _validate(d) == B.RT_ERR_INVALID_ARG and "radius" in B.rt_last_error()
    d = _descs(W.curved(n_sources=1, rays_per_source=4))
    d.bnd.planes[2].param = float("inf")  # paraboloid curvature
    assert _validate(d) == B.RT_ERR_INVALID_ARG
    d = _descs(W.curved(n_sources=1, rays_per_source=4))
    d.bnd.planes[1].shape = 7
    assert _validate(d) == B.RT_ERR_INVALID_ARG and "shape" in B.rt_last_error()
    # solves follow planes only
    s = _solve_descs()
    s.bnd.planes[1].shape = B.RT_SHAPE_SPHERE if hasattr(B, "RT_SHAPE_SPHERE") else 1
    s.bnd.planes[1].param = 10.0
    assert B.rt_solve_validate(s.field, s.bnd, s.tol, s.limits, B.solve_params()) == \
        B.RT_ERR_UNSUPPORTED


def test_validate_non_stratified_fields():
    d = _descs(W.field3d(n_sources=1, rays_per_source=4))
    assert _validate(d) == B.RT_OK
    d.field.anomalies[0].sigma = 0.0
    assert _validate(d) == B.RT_ERR_INVALID_ARG and "sigma" in B.rt_last_error()
    d = _descs(W.field3d(n_sources=1, rays_per_source=4))
    d.field.anomalies[1].region = 5
    assert _validate(d) == B.RT_ERR_INVALID_ARG and "region" in B.rt_last_error()
    d = _descs(W.field3d(n_sources=1, rays_per_source=4))
    d.field.n_anomalies = B.RT_MAX_ANOMALIES + 1
    assert _validate(d) == B.RT_ERR_INVALID_ARG
    d = _descs(W.field3d(n_sources=1, rays_per_source=4))
    d.field.regions[1].axis[0] = float("nan")
    assert _validate(d) == B.RT_ERR_INVALID_ARG and "axis" in B.rt_last_error()
    # solves take depth-stratified fields only: an axis along +z of any length
    # is depth, any other axis or an anomaly is not
    s = _solve_descs()
    p = B.solve_params()
    s.field.regions[1].axis[2] = 3.0
    assert B.rt_solve_validate(s.field, s.bnd, s.tol, s.limits, p) == B.RT_OK
    s.field.regions[1].axis[0] = 0.1
    assert B.rt_solve_validate(s.field, s.bnd, s.tol, s.limits, p) == B.RT_ERR_UNSUPPORTED
    s = _solve_descs()
    s.field.regions[1].axis[2] = -1.0
    assert B.rt_solve_validate(s.field, s.bnd, s.tol, s.limits, p) == B.RT_ERR_UNSUPPORTED
    s = _solve_descs()
    an = (B.rt_anomaly * 1)(B.rt_anomaly((C.c_double * 3)(0.0, 0.0, 100.0), 0.01, 5.0, 1))
    s.field.n_anomalies, s.field.anomalies = 1, C.cast(an, C.POINTER(B.rt_anomaly))
    assert B.rt_solve_validate(s.field, s.bnd, s.tol, s.limits, p) == B.RT_ERR_UNSUPPORTED


def test_validate_step_budget_and_resume():
    d = _descs()
    d.limits.max_steps_per_launch = 1000
    d.limits.resume = 1
    assert _validate(d) == B.RT_OK
    d.limits.max_steps_per_launch = -1
    assert _validate(d) == B.RT_ERR_INVALID_ARG and "max_steps_per_launch" in B.rt_last_error()
    d = _descs()
    d.limits.resume = 2
    assert _validate(d) == B.RT_ERR_INVALID_ARG and "resume" in B.rt_last_error()
    # solves take neither
    s = _solve_descs()
    s.limits.max_steps_per_launch = 10
    assert B.rt_solve_validate(s.field, s.bnd, s.tol, s.limits, B.solve_params()) == \
        B.RT_ERR_INVALID_ARG


def test_collect_reports_interruption():
    s = B.rt_stats()
    s.interrupted = 1
    assert B.rt_collect(s, 10) == B.RT_INTERRUPTED and "resume" in B.rt_last_error()
    s.needed = 11   # slots short takes precedence: resuming cannot fix it
    assert B.rt_collect(s, 10) == B.RT_ERR_CAPACITY
