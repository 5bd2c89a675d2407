"""Thin ctypes binding of the radiotrace C ABI (include/radiotrace.h and
include/radiotrace_solve.h).

The functions carry the C names (rt_abi_version, rt_validate,
rt_workspace_bytes, raytrace_launch, rt_collect, rt_last_error,
rt_solve_validate, rt_solve_workspace_bytes, raytrace_solve, raytrace_shoot,
rt_solve_autotune)
and only marshal arguments; every step of the tracing and solving runs in the
HIP kernels.  PyTorch
supplies device memory and the stream.  The library must have been built
(``paper_1810_01780_amd.build.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

from . import workloads as W

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libradiotrace.so")

RT_OK, RT_ERR_INVALID_ARG, RT_ERR_CAPACITY, RT_ERR_DEVICE, RT_ERR_UNSUPPORTED, \
    RT_INTERRUPTED = range(6)
RT_ST_PARKED, RT_ST_QUEUED, RT_ST_EMPTY = -2, -1, 0
(RT_ST_PATH, RT_ST_BOX, RT_ST_TIME, RT_ST_AMP, RT_ST_ABSORB, RT_ST_STEPCAP,
 RT_ST_NONFINITE, RT_ST_INVALID) = range(1, 9)
RT_MAX_REGIONS, RT_MAX_PLANES, RT_MAX_GENERATIONS, RT_MAX_ANOMALIES = 8, 16, 4, 8
RT_SHAPE_PLANE, RT_SHAPE_SPHERE, RT_SHAPE_PARABOLOID = 0, 1, 2


class rt_region(C.Structure):
    _fields_ = [("a", C.c_double), ("b", C.c_double), ("dn", C.c_double), ("z0", C.c_double),
                ("z_top", C.c_double), ("z_bot", C.c_double), ("use_grid", C.c_int32),
                ("axis", C.c_double * 3)]


class rt_anomaly(C.Structure):
    _fields_ = [("centre", C.c_double * 3), ("amplitude", C.c_double), ("sigma", C.c_double),
                ("region", C.c_int32)]


class rt_grid(C.Structure):
    _fields_ = [("n", C.c_void_p), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("origin", C.c_double * 3), ("spacing", C.c_double * 3)]


class rt_field(C.Structure):
    _fields_ = [("n_regions", C.c_int32), ("regions", C.POINTER(rt_region)), ("grid", rt_grid),
                ("n_anomalies", C.c_int32), ("anomalies", C.POINTER(rt_anomaly))]


class rt_plane(C.Structure):
    _fields_ = [("point", C.c_double * 3), ("normal", C.c_double * 3),
                ("region_pos", C.c_int32), ("region_neg", C.c_int32), ("kind", C.c_int32),
                ("shape", C.c_int32), ("param", C.c_double)]


class rt_boundaries(C.Structure):
    _fields_ = [("n_planes", C.c_int32), ("planes", C.POINTER(rt_plane)),
                ("has_box", C.c_int32), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3)]


class rt_sources(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("n", C.c_int32)]


class rt_directions(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("src", C.c_void_p), ("n", C.c_int64)]


class rt_step_limits(C.Structure):
    _fields_ = [("h_min", C.c_double), ("h_max", C.c_double), ("h_init", C.c_double),
                ("s_max", C.c_double), ("t_max", C.c_double), ("amp_min", C.c_double),
                ("max_generations", C.c_int32), ("model", C.c_int32),
                ("max_steps_per_ray", C.c_int64), ("max_steps_per_launch", C.c_int64),
                ("resume", C.c_int32)]


STAT_FIELDS = ["accepted", "rejected", "relocation", "forced", "events", "spawned",
               "suppressed_gen", "suppressed_amp", "records", "needed", "nonfinite",
               "max_gen", "invalid", "refills", "sched_errors", "spilled", "interrupted",
               "events_lost", "max_queue"]


class rt_stats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in STAT_FIELDS]


F64_FIELDS = ["x", "y", "z", "ux", "uy", "uz", "s", "t", "as_re", "as_im", "ap_re", "ap_im", "h"]
U64_FIELDS = ["key", "parent"]
I32_FIELDS = ["gen", "status", "n_acc", "n_rej", "n_ev", "region"]
U32_FIELDS = ["side"]
RECORD_FIELDS = F64_FIELDS + U64_FIELDS + I32_FIELDS + U32_FIELDS


class rt_outputs(C.Structure):
    _fields_ = ([(f, C.c_void_p) for f in RECORD_FIELDS]
                + [("capacity", C.c_int64), ("stats", C.c_void_p), ("events", C.c_void_p),
                   ("ev_capacity", C.c_int64)])


RT_EV_SPAWNED, RT_EV_TIR, RT_EV_GEN, RT_EV_AMP = range(4)


class rt_event(C.Structure):
    _fields_ = [("key", C.c_uint64), ("ordinal", C.c_int32), ("boundary", C.c_int32),
                ("outcome", C.c_int32), ("gen", C.c_int32), ("region_in", C.c_int32),
                ("region_out", C.c_int32), ("pos", C.c_double * 3), ("dir", C.c_double * 3),
                ("s", C.c_double), ("t", C.c_double), ("cos_i", C.c_double),
                ("n1", C.c_double), ("n2", C.c_double), ("amp", C.c_double * 4),
                ("coef", C.c_double * 8)]


# the same layout as a numpy record type (for event arrays copied from the device)
EVENT_DTYPE = np.dtype([("key", np.uint64), ("ordinal", np.int32), ("boundary", np.int32),
                        ("outcome", np.int32), ("gen", np.int32), ("region_in", np.int32),
                        ("region_out", np.int32), ("pos", np.float64, 3),
                        ("dir", np.float64, 3), ("s", np.float64), ("t", np.float64),
                        ("cos_i", np.float64), ("n1", np.float64), ("n2", np.float64),
                        ("amp", np.float64, 4), ("coef", np.float64, 8)])


class rt_tuning(C.Structure):
    _fields_ = [("block_size", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("refill_threshold", C.c_int32), ("ev_trace_begin", C.c_void_p),
                ("ev_trace_end", C.c_void_p), ("local_queue", C.c_int32),
                ("scan_chunk", C.c_int32), ("solve_fused", C.c_int32)]


# --- emitter -> receiver solves (include/radiotrace_solve.h) -----------------
RT_FAMILY_DIRECT, RT_FAMILY_REFLECTED = 0, 1
RT_SHOT_RECEIVER, RT_SHOT_SURFACE, RT_SHOT_LOST, RT_SHOT_INVALID = range(4)


class rt_pairs(C.Structure):
    _fields_ = [("zs", C.c_void_p), ("zr", C.c_void_p), ("dist", C.c_void_p), ("n", C.c_int64)]


class rt_solve_params(C.Structure):
    _fields_ = [("n_scan", C.c_int32), ("max_iter", C.c_int32), ("max_brackets", C.c_int32),
                ("miss_tol", C.c_double), ("accept_tol", C.c_double),
                ("slope_max", C.c_double)]


SOLVE_STAT_FIELDS = ["shots", "accepted", "rejected", "relocation", "forced", "events",
                     "brackets", "found", "invalid"]


class rt_solve_stats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in SOLVE_STAT_FIELDS]


SOLVE_I32 = ["found", "shots", "roots"]
SOLVE_F64 = ["theta", "miss", "t", "s", "as_re", "as_im", "ap_re", "ap_im"]


class rt_solve_outputs(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in SOLVE_I32 + SOLVE_F64] + [("stats", C.c_void_p)]


class rt_shots(C.Structure):
    _fields_ = [("zs", C.c_void_p), ("zr", C.c_void_p), ("dist", C.c_void_p),
                ("theta", C.c_void_p), ("family", C.c_void_p), ("n", C.c_int64)]


SHOT_I32 = ["status", "n_acc", "n_rej"]
SHOT_F64 = ["miss", "t", "s", "as_re", "as_im", "ap_re", "ap_im"]


class rt_shot_outputs(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in SHOT_I32 + SHOT_F64] + [("stats", C.c_void_p)]


# --- surrogate network (include/radiotrace_mlp.h) ---------------------------
RT_MLP_IN, RT_MLP_WIDTH, RT_MLP_HIDDEN, RT_MLP_OUT, RT_MLP_TARGETS = 5, 256, 4, 10, 8


class rt_adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


RT_PATH_SURROGATE, RT_PATH_TRACER = 0, 1


class rt_surrogate_params(C.Structure):
    _fields_ = [("z0", C.c_double), ("dn", C.c_double), ("verify_tol", C.c_double),
                ("dseed", C.c_double), ("max_shots", C.c_int32), ("absent_logit", C.c_float),
                ("multi_logit", C.c_float)]


_lib = None
# RT_ABI_VERSION of the header the structures above follow
ABI_VERSION = 8


def lib() -> C.CDLL:
    """Load libradiotrace.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                               "paper_1810_01780_amd.build.build() (no fallback path exists)")
        # PyTorch ships its own HIP runtime under the same soname; loading torch
        # first makes this library bind to that one runtime instead of a second
        # copy (device pointers and streams must come from one runtime).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(_LIB_PATH)
        L.rt_abi_version.restype = C.c_int32
        L.rt_abi_version.argtypes = []
        if L.rt_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{_LIB_PATH} has ABI version {L.rt_abi_version()}, the binding "
                               f"expects {ABI_VERSION}: rebuild it")
        L.rt_validate.restype = C.c_int
        L.rt_validate.argtypes = [C.POINTER(rt_field), C.POINTER(rt_boundaries),
                                  C.POINTER(rt_sources), C.POINTER(rt_directions), C.c_double,
                                  C.POINTER(rt_step_limits)]
        L.rt_workspace_bytes.restype = C.c_int
        L.rt_workspace_bytes.argtypes = [C.POINTER(rt_field), C.c_int64, C.POINTER(C.c_size_t)]
        L.raytrace_launch.restype = C.c_int
        L.raytrace_launch.argtypes = [C.POINTER(rt_field), C.POINTER(rt_boundaries),
                                      C.POINTER(rt_sources), C.POINTER(rt_directions), C.c_double,
                                      C.POINTER(rt_step_limits), C.POINTER(rt_outputs),
                                      C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(rt_tuning)]
        L.raytrace_launch_static.restype = C.c_int
        L.raytrace_launch_static.argtypes = [C.POINTER(rt_field), C.POINTER(rt_boundaries),
                                             C.POINTER(rt_sources), C.POINTER(rt_directions),
                                             C.c_double, C.POINTER(rt_step_limits),
                                             C.POINTER(rt_outputs), C.c_void_p,
                                             C.POINTER(rt_tuning)]
        L.rt_probe_read_bandwidth.restype = C.c_int
        L.rt_probe_read_bandwidth.argtypes = [C.c_void_p, C.c_size_t, C.c_int32, C.c_int32,
                                              C.c_void_p, C.POINTER(C.c_double)]
        L.rt_collect.restype = C.c_int
        L.rt_collect.argtypes = [C.POINTER(rt_stats), C.c_int64]
        L.rt_last_error.restype = C.c_char_p
        L.rt_last_error.argtypes = []
        L.rt_solve_validate.restype = C.c_int
        L.rt_solve_validate.argtypes = [C.POINTER(rt_field), C.POINTER(rt_boundaries),
                                        C.c_double, C.POINTER(rt_step_limits),
                                        C.POINTER(rt_solve_params)]
        L.rt_solve_workspace_bytes.restype = C.c_int
        L.rt_solve_workspace_bytes.argtypes = [C.POINTER(rt_field), C.c_int64,
                                               C.POINTER(rt_solve_params),
                                               C.POINTER(C.c_size_t)]
        L.raytrace_solve.restype = C.c_int
        L.raytrace_solve.argtypes = [C.POINTER(rt_field), C.POINTER(rt_boundaries), C.c_double,
                                     C.POINTER(rt_step_limits), C.POINTER(rt_pairs),
                                     C.POINTER(rt_solve_params), C.POINTER(rt_solve_outputs),
                                     C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(rt_tuning)]
        L.raytrace_shoot.restype = C.c_int
        L.raytrace_shoot.argtypes = [C.POINTER(rt_field), C.POINTER(rt_boundaries), C.c_double,
                                     C.POINTER(rt_step_limits), C.POINTER(rt_shots),
                                     C.POINTER(rt_shot_outputs), C.c_void_p, C.c_size_t,
                                     C.c_void_p, C.POINTER(rt_tuning)]
        L.rt_solve_autotune.restype = C.c_int
        L.rt_solve_autotune.argtypes = [C.POINTER(rt_field), C.POINTER(rt_boundaries),
                                        C.c_double, C.POINTER(rt_step_limits),
                                        C.POINTER(rt_pairs), C.POINTER(rt_solve_params),
                                        C.POINTER(rt_solve_outputs), C.c_void_p, C.c_size_t,
                                        C.c_void_p, C.POINTER(rt_tuning),
                                        C.POINTER(C.c_float)]
        L.rt_mlp_param_count.restype = C.c_int64
        L.rt_mlp_param_count.argtypes = []
        L.rt_mlp_workspace_bytes.restype = C.c_int
        L.rt_mlp_workspace_bytes.argtypes = [C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]
        L.rt_mlp_pack.restype = C.c_int
        L.rt_mlp_pack.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.rt_mlp_forward.restype = C.c_int
        L.rt_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_size_t, C.c_void_p]
        L.rt_mlp_forward_layers.restype = C.c_int
        L.rt_mlp_forward_layers.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                            C.c_void_p, C.c_size_t, C.c_void_p]
        L.rt_mlp_gradients.restype = C.c_int
        L.rt_mlp_gradients.argtypes = [C.c_void_p] * 4 + [C.c_int64, C.c_void_p, C.c_void_p,
                                                         C.c_void_p, C.c_size_t, C.c_void_p]
        L.rt_mlp_adam.restype = C.c_int
        L.rt_mlp_adam.argtypes = [C.c_void_p] * 4 + [C.c_int64, C.POINTER(rt_adam), C.c_void_p,
                                                    C.c_size_t, C.c_void_p]
        L.raytrace_solve_seeded.restype = C.c_int
        L.raytrace_solve_seeded.argtypes = [
            C.POINTER(rt_field), C.POINTER(rt_boundaries), C.c_double, C.POINTER(rt_step_limits),
            C.POINTER(rt_pairs), C.c_void_p, C.c_void_p, C.POINTER(rt_surrogate_params),
            C.POINTER(rt_solve_outputs), C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
            C.POINTER(rt_tuning)]
        L.rt_surrogate_features.restype = C.c_int
        L.rt_surrogate_features.argtypes = [C.POINTER(rt_pairs), C.c_double, C.c_double,
                                            C.c_void_p, C.c_void_p]
        L.rt_surrogate_targets.restype = C.c_int
        L.rt_surrogate_targets.argtypes = [C.POINTER(rt_solve_outputs), C.c_int64, C.c_void_p,
                                           C.c_void_p, C.c_void_p]
        L.rt_surrogate_workspace_bytes.restype = C.c_int
        L.rt_surrogate_workspace_bytes.argtypes = [C.POINTER(rt_field), C.c_int64,
                                                   C.POINTER(rt_solve_params),
                                                   C.POINTER(C.c_size_t)]
        L.raytrace_solve_surrogate.restype = C.c_int
        L.raytrace_solve_surrogate.argtypes = [
            C.POINTER(rt_field), C.POINTER(rt_boundaries), C.c_double, C.POINTER(rt_step_limits),
            C.POINTER(rt_pairs), C.POINTER(rt_solve_params), C.POINTER(rt_surrogate_params),
            C.c_void_p, C.POINTER(rt_solve_outputs), C.c_void_p, C.c_void_p, C.c_void_p,
            C.c_size_t, C.c_void_p, C.POINTER(rt_tuning)]
        _lib = L
    return _lib


# --- the C entry points, same names ------------------------------------------
def rt_abi_version() -> int:
    return int(lib().rt_abi_version())


def rt_validate(field, boundaries, sources, directions, tol, limits) -> int:
    return int(lib().rt_validate(C.byref(field), C.byref(boundaries), C.byref(sources),
                                 C.byref(directions), float(tol), C.byref(limits)))


def rt_workspace_bytes(field, capacity: int) -> int:
    n = C.c_size_t(0)
    st = lib().rt_workspace_bytes(C.byref(field), C.c_int64(capacity), C.byref(n))
    if st != RT_OK:
        raise RTError(st, rt_last_error())
    return int(n.value)


def raytrace_launch(field, boundaries, sources, directions, tol, limits, outputs, workspace,
                    workspace_bytes, stream, tuning=None) -> int:
    return int(lib().raytrace_launch(
        C.byref(field), C.byref(boundaries), C.byref(sources), C.byref(directions), float(tol),
        C.byref(limits), C.byref(outputs), C.c_void_p(workspace), C.c_size_t(workspace_bytes),
        C.c_void_p(stream), C.byref(tuning) if tuning is not None else None))


def raytrace_launch_static(field, boundaries, sources, directions, tol, limits, outputs,
                           stream, tuning=None) -> int:
    return int(lib().raytrace_launch_static(C.byref(field), C.byref(boundaries),
                                            C.byref(sources), C.byref(directions), tol,
                                            C.byref(limits), C.byref(outputs), stream,
                                            C.byref(tuning) if tuning is not None else None))


RT_STATIC_SCRATCH_BYTES = 64 << 20
RT_PROBE_STREAM, RT_PROBE_GATHER = 0, 1


def rt_probe_read_bandwidth(buffer, nbytes: int, pattern: int, passes: int, stream) -> float:
    """GB/s of float4 reads served from a device buffer (see radiotrace_probe.h)."""
    out = C.c_double()
    st = lib().rt_probe_read_bandwidth(buffer, nbytes, pattern, passes, stream, C.byref(out))
    if st != RT_OK:
        raise RTError(st, rt_last_error())
    return float(out.value)


def rt_collect(stats, capacity: int) -> int:
    return int(lib().rt_collect(C.byref(stats), C.c_int64(capacity)))


def rt_last_error() -> str:
    return lib().rt_last_error().decode()


class RTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"radiotrace status {status}: {msg}")
        self.status = status


# --- descriptor marshalling for workload scenes ------------------------------
class HostDescriptors:
    """ctypes descriptors of a Scene's host-side parts (regions, planes, box,
    limits); device pointers are filled in by DeviceScene."""

    def __init__(self, scene: W.Scene):
        self.scene = scene
        regs = (rt_region * max(1, len(scene.regions)))()
        for i, r in enumerate(scene.regions):
            regs[i] = rt_region(r.a, r.b, r.dn, r.z0, r.z_top, r.z_bot, int(r.use_grid),
                                (C.c_double * 3)(*r.axis))
        anoms = (rt_anomaly * max(1, len(scene.anomalies)))()
        for i, q in enumerate(scene.anomalies):
            anoms[i] = rt_anomaly((C.c_double * 3)(*q.centre), q.amplitude, q.sigma, q.region)
        pls = (rt_plane * max(1, len(scene.planes)))()
        for i, p in enumerate(scene.planes):
            pls[i] = rt_plane((C.c_double * 3)(*p.point), (C.c_double * 3)(*p.normal),
                              p.region_pos, p.region_neg, p.kind, p.shape, p.param)
        self._keep = [regs, pls, anoms]
        self.field = rt_field(len(scene.regions), C.cast(regs, C.POINTER(rt_region)), rt_grid(),
                              len(scene.anomalies), C.cast(anoms, C.POINTER(rt_anomaly)))
        if scene.grid is not None:
            nz, ny, nx = scene.grid.n.shape
            self.field.grid.nx, self.field.grid.ny, self.field.grid.nz = nx, ny, nz
            self.field.grid.origin = (C.c_double * 3)(*scene.grid.origin)
            self.field.grid.spacing = (C.c_double * 3)(*scene.grid.spacing)
        self.bnd = rt_boundaries(len(scene.planes), C.cast(pls, C.POINTER(rt_plane)), 0)
        if scene.box_lo is not None:
            self.bnd.has_box = 1
            self.bnd.box_lo = (C.c_double * 3)(*scene.box_lo)
            self.bnd.box_hi = (C.c_double * 3)(*scene.box_hi)
        lim = scene.limits
        self.limits = rt_step_limits(lim.h_min, lim.h_max, lim.h_init, lim.s_max, lim.t_max,
                                     lim.amp_min, lim.max_generations, lim.model,
                                     lim.max_steps_per_ray, lim.max_steps_per_launch, 0)
        self.tol = lim.tol
        self.sources = rt_sources(None, int(scene.sources.shape[0]))
        self.dirs = rt_directions(None, None, int(scene.n_rays))


class DeviceScene:
    """Device-resident inputs, outputs and workspace for one Scene (torch
    tensors on cuda:0 by default), reusable across launches."""

    def __init__(self, scene: W.Scene, capacity: Optional[int] = None, device="cuda",
                 ev_capacity: int = 0, static_scratch: bool = False):
        import torch
        self.torch = torch
        self.scene = scene
        self.desc = HostDescriptors(scene)
        dev = torch.device(device)
        self.device = dev
        self.src = torch.as_tensor(np.ascontiguousarray(scene.sources, np.float64), device=dev)
        self.dirs = torch.as_tensor(np.ascontiguousarray(scene.dirs, np.float64), device=dev)
        self.ray_src = torch.as_tensor(np.ascontiguousarray(scene.ray_src, np.int32), device=dev)
        self.desc.sources.xyz = self.src.data_ptr()
        self.desc.dirs.xyz = self.dirs.data_ptr()
        self.desc.dirs.src = self.ray_src.data_ptr()
        if scene.grid is not None:
            self.grid = torch.as_tensor(np.ascontiguousarray(scene.grid.n, np.float32), device=dev)
            self.desc.field.grid.n = self.grid.data_ptr()
        self.capacity = int(capacity if capacity is not None else scene.capacity_hint())
        self.capacity = max(self.capacity, scene.n_rays)
        cap = max(1, self.capacity)
        self.rec: Dict[str, "torch.Tensor"] = {}
        for f in F64_FIELDS:
            self.rec[f] = torch.empty(cap, dtype=torch.float64, device=dev)
        for f in U64_FIELDS:
            self.rec[f] = torch.empty(cap, dtype=torch.int64, device=dev)
        for f in I32_FIELDS + U32_FIELDS:
            self.rec[f] = torch.empty(cap, dtype=torch.int32, device=dev)
        self.stats_dev = torch.zeros(len(STAT_FIELDS), dtype=torch.int64, device=dev)
        self.ev_capacity = int(ev_capacity)
        self.events_dev = None
        if self.ev_capacity > 0:
            self.events_dev = torch.empty(self.ev_capacity * EVENT_DTYPE.itemsize,
                                          dtype=torch.uint8, device=dev)
        self.out = rt_outputs(*([self.rec[f].data_ptr() for f in RECORD_FIELDS]
                                + [self.capacity, self.stats_dev.data_ptr(),
                                   self.events_dev.data_ptr() if self.ev_capacity else None,
                                   self.ev_capacity]))
        self.ws_bytes = rt_workspace_bytes(self.desc.field, self.capacity)
        # static_scratch: launches use raytrace_launch_static, whose scratch
        # is the library's own device array (no workspace is allocated)
        self.static_scratch = static_scratch
        self.workspace = None
        if not static_scratch:
            self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)

    def launch(self, stream=None, tuning: Optional[rt_tuning] = None, resume: bool = False) -> None:
        """Enqueue one trace on the stream (torch's current stream by default);
        resume=True continues a launch that stopped at its step budget."""
        torch = self.torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.desc.limits.resume = 1 if resume else 0
        try:
            if self.static_scratch:
                st = raytrace_launch_static(self.desc.field, self.desc.bnd, self.desc.sources,
                                            self.desc.dirs, self.desc.tol, self.desc.limits,
                                            self.out, stream.cuda_stream, tuning)
            else:
                st = raytrace_launch(self.desc.field, self.desc.bnd, self.desc.sources,
                                     self.desc.dirs, self.desc.tol, self.desc.limits, self.out,
                                     self.workspace.data_ptr(), self.ws_bytes,
                                     stream.cuda_stream, tuning)
        finally:
            self.desc.limits.resume = 0
        if st != RT_OK:
            raise RTError(st, rt_last_error())

    def stats(self) -> Dict[str, int]:
        v = self.stats_dev.cpu().numpy()
        return {f: int(v[i]) for i, f in enumerate(STAT_FIELDS)}

    def collect(self, check: bool = True):
        """Synchronise, then return (records as numpy arrays in slot order,
        stats); raises RTError on a failing status when check is set."""
        self.torch.cuda.synchronize(self.device)
        stats = self.stats()
        host = rt_stats(*[stats[f] for f in STAT_FIELDS])
        st = rt_collect(host, self.capacity)
        if check and st != RT_OK:
            raise RTError(st, rt_last_error())
        n = min(stats["records"] + stats["invalid"], self.capacity)
        out = {}
        for f in RECORD_FIELDS:
            a = self.rec[f][:n].cpu().numpy()
            if f in U64_FIELDS:
                a = a.view(np.uint64)
            elif f in U32_FIELDS:
                a = a.view(np.uint32)
            out[f] = a
        return out, stats

    def events(self):
        """Event records written by the last launch (after collect), as a
        dict of numpy arrays sorted by (key, ordinal)."""
        if self.events_dev is None:
            return None
        m = min(self.stats()["events"], self.ev_capacity)
        raw = self.events_dev[:m * EVENT_DTYPE.itemsize].cpu().numpy()
        ev = raw.view(EVENT_DTYPE)
        order = np.lexsort((ev["ordinal"], ev["key"]))
        return {f: np.ascontiguousarray(ev[f][order]) for f in EVENT_DTYPE.names}


def trace(scene: W.Scene, capacity: Optional[int] = None, tuning: Optional[rt_tuning] = None,
          check: bool = True, ev_capacity: Optional[int] = None):
    """Trace a scene on the GPU; returns (records in slot order, stats), and
    with ev_capacity also the event records: (records, stats, events)."""
    ds = DeviceScene(scene, capacity=capacity, ev_capacity=ev_capacity or 0)
    ds.launch(tuning=tuning)
    out, stats = ds.collect(check=check)
    if ev_capacity:
        return out, stats, ds.events()
    return out, stats


# --- emitter -> receiver solves: C entry points and device-side helpers -------
def rt_solve_validate(field, boundaries, tol, limits, params=None) -> int:
    return int(lib().rt_solve_validate(C.byref(field), C.byref(boundaries), float(tol),
                                       C.byref(limits),
                                       C.byref(params) if params is not None else None))


def rt_solve_workspace_bytes(field, n_pairs: int, params=None) -> int:
    n = C.c_size_t(0)
    st = lib().rt_solve_workspace_bytes(C.byref(field), C.c_int64(n_pairs),
                                        C.byref(params) if params is not None else None,
                                        C.byref(n))
    if st != RT_OK:
        raise RTError(st, rt_last_error())
    return int(n.value)


def raytrace_solve(field, boundaries, tol, limits, pairs, params, outputs, workspace,
                   workspace_bytes, stream, tuning=None) -> int:
    return int(lib().raytrace_solve(
        C.byref(field), C.byref(boundaries), float(tol), C.byref(limits), C.byref(pairs),
        C.byref(params), C.byref(outputs), C.c_void_p(workspace), C.c_size_t(workspace_bytes),
        C.c_void_p(stream), C.byref(tuning) if tuning is not None else None))


def raytrace_shoot(field, boundaries, tol, limits, shots, outputs, workspace, workspace_bytes,
                   stream, tuning=None) -> int:
    return int(lib().raytrace_shoot(
        C.byref(field), C.byref(boundaries), float(tol), C.byref(limits), C.byref(shots),
        C.byref(outputs), C.c_void_p(workspace), C.c_size_t(workspace_bytes),
        C.c_void_p(stream), C.byref(tuning) if tuning is not None else None))


def rt_solve_autotune(field, boundaries, tol, limits, pairs, params, outputs, workspace,
                      workspace_bytes, stream):
    """Returns (status, best rt_tuning, its time in ms)."""
    best = rt_tuning()
    ms = C.c_float(0.0)
    st = lib().rt_solve_autotune(
        C.byref(field), C.byref(boundaries), float(tol), C.byref(limits), C.byref(pairs),
        C.byref(params), C.byref(outputs), C.c_void_p(workspace), C.c_size_t(workspace_bytes),
        C.c_void_p(stream), C.byref(best), C.byref(ms))
    return int(st), best, float(ms.value)


def solve_params(n_scan=64, max_iter=60, max_brackets=4, miss_tol=1e-4, accept_tol=1e-3,
                 slope_max=1e7):
    return rt_solve_params(n_scan, max_iter, max_brackets, miss_tol, accept_tol, slope_max)


class DeviceSolve:
    """Device-resident pairs, outputs and workspace for solving source /
    receiver pairs in a scene's medium (planes[0] = surface), reusable across
    launches and capturable into a graph."""

    def __init__(self, scene: W.Scene, zs, zr, dist, params: Optional[rt_solve_params] = None,
                 device="cuda"):
        import torch
        self.torch = torch
        self.desc = HostDescriptors(scene)
        dev = torch.device(device)
        self.device = dev
        self.params = params if params is not None else solve_params()
        f64 = dict(dtype=torch.float64, device=dev)
        self.zs = torch.as_tensor(np.ascontiguousarray(zs, np.float64), device=dev)
        self.zr = torch.as_tensor(np.ascontiguousarray(zr, np.float64), device=dev)
        self.dist = torch.as_tensor(np.ascontiguousarray(dist, np.float64), device=dev)
        n = int(self.zs.shape[0])
        self.n = n
        self.pairs = rt_pairs(self.zs.data_ptr(), self.zr.data_ptr(), self.dist.data_ptr(), n)
        m = max(1, 2 * n)
        self.res = {f: torch.zeros(m, dtype=torch.int32, device=dev) for f in SOLVE_I32}
        self.res.update({f: torch.zeros(m, **f64) for f in SOLVE_F64})
        self.stats_dev = torch.zeros(len(SOLVE_STAT_FIELDS), dtype=torch.int64, device=dev)
        self.out = rt_solve_outputs(*([self.res[f].data_ptr() for f in SOLVE_I32 + SOLVE_F64]
                                      + [self.stats_dev.data_ptr()]))
        self.ws_bytes = rt_solve_workspace_bytes(self.desc.field, n, self.params)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)

    def launch(self, stream=None, tuning: Optional[rt_tuning] = None) -> None:
        torch = self.torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        st = raytrace_solve(self.desc.field, self.desc.bnd, self.desc.tol, self.desc.limits,
                            self.pairs, self.params, self.out, self.workspace.data_ptr(),
                            self.ws_bytes, stream.cuda_stream, tuning)
        if st != RT_OK:
            raise RTError(st, rt_last_error())

    def autotune(self, stream=None):
        """Measure the launch tunings on these pairs; returns (rt_tuning, ms)."""
        torch = self.torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        st, best, ms = rt_solve_autotune(self.desc.field, self.desc.bnd, self.desc.tol,
                                         self.desc.limits, self.pairs, self.params, self.out,
                                         self.workspace.data_ptr(), self.ws_bytes,
                                         stream.cuda_stream)
        if st != RT_OK:
            raise RTError(st, rt_last_error())
        return best, ms

    def stats(self) -> Dict[str, int]:
        v = self.stats_dev.cpu().numpy()
        return {f: int(v[i]) for i, f in enumerate(SOLVE_STAT_FIELDS)}

    def collect(self):
        """Synchronise; results as numpy arrays shaped (n, 2) [pair, family]."""
        self.torch.cuda.synchronize(self.device)
        out = {f: t[:2 * self.n].cpu().numpy().reshape(self.n, 2) for f, t in self.res.items()}
        return out, self.stats()


def solve(scene: W.Scene, zs, zr, dist, params: Optional[rt_solve_params] = None,
          tuning: Optional[rt_tuning] = None):
    """Solve source/receiver pairs on the GPU; returns (results shaped
    (n, 2), stats)."""
    ds = DeviceSolve(scene, zs, zr, dist, params)
    ds.launch(tuning=tuning)
    return ds.collect()


def shoot(scene: W.Scene, zs, zr, dist, theta, family, tuning: Optional[rt_tuning] = None):
    """Single shots on the GPU; returns (per-shot results, stats)."""
    import torch
    desc = HostDescriptors(scene)
    dev = torch.device("cuda")
    cols = [torch.as_tensor(np.ascontiguousarray(a, np.float64), device=dev)
            for a in (zs, zr, dist, theta)]
    fam = torch.as_tensor(np.ascontiguousarray(family, np.int32), device=dev)
    n = int(cols[0].shape[0])
    shots = rt_shots(*[c.data_ptr() for c in cols], fam.data_ptr(), n)
    m = max(1, n)
    res = {f: torch.zeros(m, dtype=torch.int32, device=dev) for f in SHOT_I32}
    res.update({f: torch.zeros(m, dtype=torch.float64, device=dev) for f in SHOT_F64})
    stats_dev = torch.zeros(len(SOLVE_STAT_FIELDS), dtype=torch.int64, device=dev)
    out = rt_shot_outputs(*([res[f].data_ptr() for f in SHOT_I32 + SHOT_F64]
                            + [stats_dev.data_ptr()]))
    ws_bytes = rt_solve_workspace_bytes(desc.field, 0)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    st = raytrace_shoot(desc.field, desc.bnd, desc.tol, desc.limits, shots, out, ws.data_ptr(),
                        ws_bytes, torch.cuda.current_stream().cuda_stream, tuning)
    if st != RT_OK:
        raise RTError(st, rt_last_error())
    torch.cuda.synchronize()
    v = stats_dev.cpu().numpy()
    return ({f: t[:n].cpu().numpy() for f, t in res.items()},
            {f: int(v[i]) for i, f in enumerate(SOLVE_STAT_FIELDS)})


# --- surrogate network: C entry points and a device-side holder ---------------
def rt_mlp_param_count() -> int:
    return int(lib().rt_mlp_param_count())


def rt_mlp_workspace_bytes(batch: int, training: bool) -> int:
    n = C.c_size_t(0)
    st = lib().rt_mlp_workspace_bytes(C.c_int64(batch), C.c_int32(1 if training else 0),
                                      C.byref(n))
    if st != RT_OK:
        raise RTError(st, rt_last_error())
    return int(n.value)


def rt_mlp_pack(params, workspace, workspace_bytes, stream) -> int:
    return int(lib().rt_mlp_pack(C.c_void_p(params), C.c_void_p(workspace),
                                 C.c_size_t(workspace_bytes), C.c_void_p(stream)))


def rt_mlp_forward(params, x, batch, y, workspace, workspace_bytes, stream) -> int:
    return int(lib().rt_mlp_forward(C.c_void_p(params), C.c_void_p(x), C.c_int64(batch),
                                    C.c_void_p(y), C.c_void_p(workspace),
                                    C.c_size_t(workspace_bytes), C.c_void_p(stream)))


def rt_mlp_forward_layers(params, x, batch, y, workspace, workspace_bytes, stream) -> int:
    return int(lib().rt_mlp_forward_layers(C.c_void_p(params), C.c_void_p(x),
                                           C.c_int64(batch), C.c_void_p(y),
                                           C.c_void_p(workspace), C.c_size_t(workspace_bytes),
                                           C.c_void_p(stream)))


def rt_mlp_gradients(params, x, targets, mask, batch, grad, loss, workspace, workspace_bytes,
                     stream) -> int:
    return int(lib().rt_mlp_gradients(
        C.c_void_p(params), C.c_void_p(x), C.c_void_p(targets), C.c_void_p(mask),
        C.c_int64(batch), C.c_void_p(grad), C.c_void_p(loss), C.c_void_p(workspace),
        C.c_size_t(workspace_bytes), C.c_void_p(stream)))


def rt_mlp_adam(params, m, v, grad, step, hp, workspace, workspace_bytes, stream) -> int:
    return int(lib().rt_mlp_adam(C.c_void_p(params), C.c_void_p(m), C.c_void_p(v),
                                 C.c_void_p(grad), C.c_int64(step), C.byref(hp),
                                 C.c_void_p(workspace), C.c_size_t(workspace_bytes),
                                 C.c_void_p(stream)))


class DeviceMLP:
    """FP32 parameters, Adam moments, gradient and workspace of the surrogate
    network on the GPU (torch tensors), for batches of up to max_batch rows."""

    def __init__(self, params, max_batch: int, training: bool = True, device="cuda"):
        import torch
        self.torch = torch
        dev = torch.device(device)
        self.device = dev
        n = rt_mlp_param_count()
        p = np.ascontiguousarray(params, np.float32)
        assert p.shape == (n,), f"expected {n} parameters"
        self.params = torch.as_tensor(p.copy(), device=dev)
        self.training = training
        self.max_batch = int(max_batch)
        self.ws_bytes = rt_mlp_workspace_bytes(self.max_batch, training)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        if training:
            self.m = torch.zeros(n, dtype=torch.float32, device=dev)
            self.v = torch.zeros(n, dtype=torch.float32, device=dev)
            self.grad = torch.zeros(n, dtype=torch.float32, device=dev)
            self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
            self.step = 0
        self.pack()

    def _stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def _check(self, st):
        if st != RT_OK:
            raise RTError(st, rt_last_error())

    def pack(self):
        self._check(rt_mlp_pack(self.params.data_ptr(), self.workspace.data_ptr(),
                                self.ws_bytes, self._stream()))

    def forward(self, x, y, layers: bool = False):
        """x: device FP32 [B][5] tensor; y: device FP32 [B][12] tensor
        (written); layers=True: one launch per layer (rt_mlp_forward_layers)."""
        B = int(x.shape[0])
        fn = rt_mlp_forward_layers if layers else rt_mlp_forward
        self._check(fn(self.params.data_ptr(), x.data_ptr(), B, y.data_ptr(),
                       self.workspace.data_ptr(), self.ws_bytes, self._stream()))

    def gradients(self, x, t, m):
        """Fills self.grad and self.loss for a batch of device tensors."""
        B = int(x.shape[0])
        self._check(rt_mlp_gradients(self.params.data_ptr(), x.data_ptr(), t.data_ptr(),
                                     m.data_ptr(), B, self.grad.data_ptr(), self.loss.data_ptr(),
                                     self.workspace.data_ptr(), self.ws_bytes, self._stream()))

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        hp = rt_adam(lr, beta1, beta2, eps)
        self._check(rt_mlp_adam(self.params.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                self.grad.data_ptr(), self.step, hp, self.workspace.data_ptr(),
                                self.ws_bytes, self._stream()))

    def train_step(self, x, t, m, lr):
        self.gradients(x, t, m)
        self.adam(lr)


# --- surrogate-seeded solves ----------------------------------------------------
def surrogate_params(z0=75.0, dn=0.43, verify_tol=0.01, dseed=1e-4, max_shots=8,
                     absent_logit=-2.0, multi_logit=-10.0):
    return rt_surrogate_params(z0, dn, verify_tol, dseed, max_shots, absent_logit, multi_logit)


def raytrace_solve_seeded(field, boundaries, tol, limits, pairs, seed, seed_try, sp, outputs,
                          verify, workspace, workspace_bytes, stream, tuning=None) -> int:
    return int(lib().raytrace_solve_seeded(
        C.byref(field), C.byref(boundaries), float(tol), C.byref(limits), C.byref(pairs),
        C.c_void_p(seed), C.c_void_p(seed_try), C.byref(sp), C.byref(outputs),
        C.c_void_p(verify), C.c_void_p(workspace), C.c_size_t(workspace_bytes),
        C.c_void_p(stream), C.byref(tuning) if tuning is not None else None))


def rt_surrogate_features(pairs, z0, dn, x, stream) -> int:
    return int(lib().rt_surrogate_features(C.byref(pairs), float(z0), float(dn), C.c_void_p(x),
                                           C.c_void_p(stream)))


def rt_surrogate_targets(solved, n, targets, mask, stream) -> int:
    return int(lib().rt_surrogate_targets(C.byref(solved), C.c_int64(n), C.c_void_p(targets),
                                          C.c_void_p(mask), C.c_void_p(stream)))


def rt_surrogate_workspace_bytes(field, n_pairs, fallback) -> int:
    n = C.c_size_t(0)
    st = lib().rt_surrogate_workspace_bytes(C.byref(field), C.c_int64(n_pairs), C.byref(fallback),
                                            C.byref(n))
    if st != RT_OK:
        raise RTError(st, rt_last_error())
    return int(n.value)


def raytrace_solve_surrogate(field, boundaries, tol, limits, pairs, fallback, sp, mlp_params,
                             outputs, path, fallback_pairs, workspace, workspace_bytes, stream,
                             tuning=None) -> int:
    return int(lib().raytrace_solve_surrogate(
        C.byref(field), C.byref(boundaries), float(tol), C.byref(limits), C.byref(pairs),
        C.byref(fallback), C.byref(sp), C.c_void_p(mlp_params), C.byref(outputs),
        C.c_void_p(path), C.c_void_p(fallback_pairs), C.c_void_p(workspace),
        C.c_size_t(workspace_bytes), C.c_void_p(stream),
        C.byref(tuning) if tuning is not None else None))


def solve_seeded(scene: W.Scene, zs, zr, dist, seed, seed_try, sp=None, tuning=None):
    """Seeded secant on the GPU (seed, seed_try shaped [n, 2]); returns
    (results shaped (n, 2) incl. 'verify', stats)."""
    import torch
    ds = DeviceSolve(scene, zs, zr, dist)
    n = ds.n
    sd = torch.as_tensor(np.ascontiguousarray(np.asarray(seed, np.float64).reshape(2 * n)),
                         device=ds.device)
    tr = torch.as_tensor(np.ascontiguousarray(np.asarray(seed_try, np.int32).reshape(2 * n)),
                         device=ds.device)
    verify = torch.full((max(1, 2 * n),), -1, dtype=torch.int32, device=ds.device)
    ws = torch.empty(4096, dtype=torch.uint8, device=ds.device)
    sp = sp if sp is not None else surrogate_params()
    st = raytrace_solve_seeded(ds.desc.field, ds.desc.bnd, ds.desc.tol, ds.desc.limits, ds.pairs,
                               sd.data_ptr(), tr.data_ptr(), sp, ds.out, verify.data_ptr(),
                               ws.data_ptr(), 4096, torch.cuda.current_stream().cuda_stream,
                               tuning)
    if st != RT_OK:
        raise RTError(st, rt_last_error())
    res, stats = ds.collect()
    res["verify"] = verify[:2 * n].cpu().numpy().reshape(n, 2)
    return res, stats


class DeviceSurrogateSolve:
    """Device-resident pairs, outputs and workspace for raytrace_solve_surrogate."""

    def __init__(self, scene: W.Scene, zs, zr, dist, sp, fallback=None, device="cuda"):
        import torch
        self.torch = torch
        self.base = DeviceSolve(scene, zs, zr, dist, fallback, device=device)
        self.sp = sp
        dev = self.base.device
        n = self.base.n
        self.path = torch.zeros(max(1, 2 * n), dtype=torch.int32, device=dev)
        self.fallback_pairs = torch.zeros(1, dtype=torch.int64, device=dev)
        self.ws_bytes = rt_surrogate_workspace_bytes(self.base.desc.field, n, self.base.params)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)

    def launch(self, mlp_params, stream=None, tuning=None):
        b = self.base
        if stream is None:
            stream = self.torch.cuda.current_stream(b.device)
        st = raytrace_solve_surrogate(b.desc.field, b.desc.bnd, b.desc.tol, b.desc.limits,
                                      b.pairs, b.params, self.sp, mlp_params.data_ptr(), b.out,
                                      self.path.data_ptr(), self.fallback_pairs.data_ptr(),
                                      self.workspace.data_ptr(), self.ws_bytes,
                                      stream.cuda_stream, tuning)
        if st != RT_OK:
            raise RTError(st, rt_last_error())

    def collect(self):
        res, stats = self.base.collect()
        n = self.base.n
        res["path"] = self.path[:2 * n].cpu().numpy().reshape(n, 2)
        stats["fallback_pairs"] = int(self.fallback_pairs.cpu().numpy()[0])
        return res, stats
