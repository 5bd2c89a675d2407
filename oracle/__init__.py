"""CPU oracle for the ray tracer -- TEST INFRASTRUCTURE ONLY.

A plain scalar FP64 C implementation of RadioPropa's method (paper §2:
eq. 1/eq. 2 integrated with Cash-Karp, planar boundaries with reflection, a
refracted secondary and Fresnel amplitudes).  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import this package; the
GPU library never does, and the two share no code.

``trace(scene)`` returns the records as numpy arrays sorted by ray key, plus
the run statistics.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "raytrace_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODEL_PAPER, MODEL_EXACT = 0, 1
ST_PATH, ST_BOX, ST_TIME, ST_AMP, ST_ABSORB, ST_STEPCAP, ST_NONFINITE = range(1, 8)


def build(force: bool = True) -> str:
    """Compile the oracle with plain IEEE semantics (no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Region(C.Structure):
    _fields_ = [("a", C.c_double), ("b", C.c_double), ("dn", C.c_double),
                ("z0", C.c_double), ("z_top", C.c_double), ("z_bot", C.c_double),
                ("use_grid", C.c_int32), ("axis", C.c_double * 3)]


class Anomaly(C.Structure):
    _fields_ = [("centre", C.c_double * 3), ("amplitude", C.c_double),
                ("sigma", C.c_double), ("region", C.c_int32)]


class Plane(C.Structure):
    _fields_ = [("point", C.c_double * 3), ("normal", C.c_double * 3),
                ("region_pos", C.c_int32), ("region_neg", C.c_int32),
                ("kind", C.c_int32), ("shape", C.c_int32), ("param", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("n_regions", C.c_int32), ("regions", C.POINTER(Region)),
                ("n_planes", C.c_int32), ("planes", C.POINTER(Plane)),
                ("has_box", C.c_int32), ("box_lo", C.c_double * 3),
                ("box_hi", C.c_double * 3),
                ("grid", C.POINTER(C.c_float)), ("nx", C.c_int32),
                ("ny", C.c_int32), ("nz", C.c_int32),
                ("origin", C.c_double * 3), ("spacing", C.c_double * 3),
                ("n_sources", C.c_int32), ("src_xyz", C.POINTER(C.c_double)),
                ("n_rays", C.c_int64), ("dir_xyz", C.POINTER(C.c_double)),
                ("ray_src", C.POINTER(C.c_int32)),
                ("tol", C.c_double), ("h_min", C.c_double), ("h_max", C.c_double),
                ("h_init", C.c_double), ("s_max", C.c_double), ("t_max", C.c_double),
                ("amp_min", C.c_double), ("max_gen", C.c_int32),
                ("model", C.c_int32), ("max_steps", C.c_int64),
                ("n_anomalies", C.c_int32), ("anomalies", C.POINTER(Anomaly))]


F64_FIELDS = ["x", "y", "z", "ux", "uy", "uz", "s", "t",
              "as_re", "as_im", "ap_re", "ap_im", "h"]
U64_FIELDS = ["key", "parent"]
I32_FIELDS = ["gen", "status", "n_acc", "n_rej", "n_ev", "region"]


class Records(C.Structure):
    _fields_ = ([(f, C.POINTER(C.c_double)) for f in F64_FIELDS]
                + [(f, C.POINTER(C.c_uint64)) for f in U64_FIELDS]
                + [(f, C.POINTER(C.c_int32)) for f in I32_FIELDS]
                + [("capacity", C.c_int64)])


STAT_FIELDS = ["accepted", "rejected", "relocation", "forced", "events", "spawned",
               "suppressed_gen", "suppressed_amp", "records", "needed",
               "nonfinite", "max_gen"]


class Stats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in STAT_FIELDS]


EV_SPAWNED, EV_TIR, EV_GEN, EV_AMP = range(4)
# event record fields: name -> (ctype, numpy dtype, values per event)
EVENT_FIELDS = {"key": (C.c_uint64, np.uint64, 1), "ordinal": (C.c_int32, np.int32, 1),
                "boundary": (C.c_int32, np.int32, 1), "outcome": (C.c_int32, np.int32, 1),
                "gen": (C.c_int32, np.int32, 1), "region_in": (C.c_int32, np.int32, 1),
                "region_out": (C.c_int32, np.int32, 1), "pos": (C.c_double, np.float64, 3),
                "dir": (C.c_double, np.float64, 3), "s": (C.c_double, np.float64, 1),
                "t": (C.c_double, np.float64, 1), "cos_i": (C.c_double, np.float64, 1),
                "n1": (C.c_double, np.float64, 1), "n2": (C.c_double, np.float64, 1),
                "amp": (C.c_double, np.float64, 4), "coef": (C.c_double, np.float64, 8)}


class Events(C.Structure):
    _fields_ = ([(f, C.POINTER(ct)) for f, (ct, _, _) in EVENT_FIELDS.items()]
                + [("capacity", C.c_int64)])


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        L.orc_trace.restype = C.c_int
        L.orc_trace.argtypes = [C.POINTER(Problem), C.POINTER(C.c_int64), C.c_int64,
                                C.POINTER(Records), C.POINTER(Stats), C.c_int]
        L.orc_trace_events.restype = C.c_int
        L.orc_trace_events.argtypes = [C.POINTER(Problem), C.POINTER(C.c_int64), C.c_int64,
                                       C.POINTER(Records), C.POINTER(Stats),
                                       C.POINTER(Events), C.POINTER(C.c_int64), C.c_int]
        L.orc_ck_trial.restype = None
        L.orc_ck_trial.argtypes = [C.POINTER(Problem), C.c_int32,
                                   C.POINTER(C.c_double), C.c_double,
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_field.restype = None
        L.orc_field.argtypes = [C.POINTER(Problem), C.c_int32, C.POINTER(C.c_double),
                                C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_fresnel.restype = C.c_int
        L.orc_fresnel.argtypes = [C.c_double, C.c_double, C.c_double,
                                  C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class _Prepared:
    """Holds the ctypes problem and keeps its arrays alive."""

    def __init__(self, scene):
        lim = scene.limits
        self.keep = []
        regs = (Region * max(1, len(scene.regions)))()
        for i, r in enumerate(scene.regions):
            regs[i] = Region(r.a, r.b, r.dn, r.z0, r.z_top, r.z_bot, int(r.use_grid),
                             (C.c_double * 3)(*r.axis))
        anoms = (Anomaly * max(1, len(scene.anomalies)))()
        for i, q in enumerate(scene.anomalies):
            anoms[i] = Anomaly((C.c_double * 3)(*q.centre), q.amplitude, q.sigma, q.region)
        pls = (Plane * max(1, len(scene.planes)))()
        for i, p in enumerate(scene.planes):
            pls[i] = Plane((C.c_double * 3)(*p.point), (C.c_double * 3)(*p.normal),
                           p.region_pos, p.region_neg, p.kind, p.shape, p.param)
        src = np.ascontiguousarray(scene.sources, dtype=np.float64)
        dirs = np.ascontiguousarray(scene.dirs, dtype=np.float64)
        rsrc = np.ascontiguousarray(scene.ray_src, dtype=np.int32)
        self.keep += [regs, pls, anoms, src, dirs, rsrc]
        P = Problem()
        P.n_regions = len(scene.regions)
        P.regions = C.cast(regs, C.POINTER(Region))
        P.n_anomalies = len(scene.anomalies)
        P.anomalies = C.cast(anoms, C.POINTER(Anomaly))
        P.n_planes = len(scene.planes)
        P.planes = C.cast(pls, C.POINTER(Plane))
        if scene.box_lo is not None:
            P.has_box = 1
            P.box_lo = (C.c_double * 3)(*scene.box_lo)
            P.box_hi = (C.c_double * 3)(*scene.box_hi)
        if scene.grid is not None:
            g = np.ascontiguousarray(scene.grid.n, dtype=np.float32)
            self.keep.append(g)
            P.grid = _ptr(g, C.c_float)
            P.nz, P.ny, P.nx = g.shape
            P.origin = (C.c_double * 3)(*scene.grid.origin)
            P.spacing = (C.c_double * 3)(*scene.grid.spacing)
        P.n_sources = src.shape[0]
        P.src_xyz = _ptr(src, C.c_double)
        P.n_rays = dirs.shape[0]
        P.dir_xyz = _ptr(dirs, C.c_double)
        P.ray_src = _ptr(rsrc, C.c_int32)
        P.tol, P.h_min, P.h_max = lim.tol, lim.h_min, lim.h_max
        P.h_init, P.s_max, P.t_max, P.amp_min = lim.h_init, lim.s_max, lim.t_max, lim.amp_min
        P.max_gen, P.model, P.max_steps = lim.max_generations, lim.model, lim.max_steps_per_ray
        self.P = P


def trace(scene, roots=None, threads: int | None = None, capacity: int | None = None,
          events: bool = False):
    """Trace (a subset of the root rays of) ``scene``; records sorted by key.
    With events=True also returns the Fresnel event records sorted by
    (key, ordinal): (records, stats, events)."""
    if events:
        return _trace_events(scene, roots, threads, capacity)
    L = lib()
    prep = _Prepared(scene)
    n_roots = scene.n_rays if roots is None else len(roots)
    if capacity is None:
        capacity = max(16, 8 * n_roots + 64)
    if threads is None:
        threads = max(1, min(os.cpu_count() or 1, 16))
    arrs = {}
    for f in F64_FIELDS:
        arrs[f] = np.zeros(capacity, np.float64)
    for f in U64_FIELDS:
        arrs[f] = np.zeros(capacity, np.uint64)
    for f in I32_FIELDS:
        arrs[f] = np.zeros(capacity, np.int32)
    rec = Records(*([_ptr(arrs[f], C.c_double) for f in F64_FIELDS]
                    + [_ptr(arrs[f], C.c_uint64) for f in U64_FIELDS]
                    + [_ptr(arrs[f], C.c_int32) for f in I32_FIELDS]
                    + [capacity]))
    st = Stats()
    rptr = None
    if roots is not None:
        ra = np.ascontiguousarray(roots, dtype=np.int64)
        prep.keep.append(ra)
        rptr = _ptr(ra, C.c_int64)
    rc = L.orc_trace(C.byref(prep.P), rptr, n_roots, C.byref(rec), C.byref(st), threads)
    stats = {f: int(getattr(st, f)) for f in STAT_FIELDS}
    if rc == -2:
        raise ValueError("oracle: unsupported problem (generations must be 1..4, planes <= 16)")
    if rc != 0:
        raise RuntimeError(f"oracle: record capacity {capacity} < needed {stats['needed']}")
    n = stats["records"]
    order = np.argsort(arrs["key"][:n], kind="stable")
    out = {f: a[:n][order] for f, a in arrs.items()}
    return out, stats


class TrialLog(C.Structure):
    _fields_ = [("h", C.POINTER(C.c_double)), ("err", C.POINTER(C.c_double)),
                ("outcome", C.POINTER(C.c_int32)), ("cap", C.c_int64), ("n", C.c_int64)]


def trace_log(scene, roots, cap: int = 1 << 20):
    """The step controller's trials of the listed roots' trees, in order, on
    one thread: (h, err / tol, outcome: 0 rejected, 1 accepted, 2 forced)."""
    L = lib()
    L.orc_trace_log.restype = C.c_int
    L.orc_trace_log.argtypes = [C.POINTER(Problem), C.POINTER(C.c_int64), C.c_int64,
                                C.POINTER(Records), C.POINTER(Stats), C.POINTER(TrialLog)]
    prep = _Prepared(scene)
    ra = np.ascontiguousarray(roots, dtype=np.int64)
    capacity = max(16, 8 * len(ra) + 64)
    arrs = {f: np.zeros(capacity, np.float64) for f in F64_FIELDS}
    arrs.update({f: np.zeros(capacity, np.uint64) for f in U64_FIELDS})
    arrs.update({f: np.zeros(capacity, np.int32) for f in I32_FIELDS})
    rec = Records(*([_ptr(arrs[f], C.c_double) for f in F64_FIELDS]
                    + [_ptr(arrs[f], C.c_uint64) for f in U64_FIELDS]
                    + [_ptr(arrs[f], C.c_int32) for f in I32_FIELDS]
                    + [capacity]))
    h, err = np.zeros(cap, np.float64), np.zeros(cap, np.float64)
    outcome = np.zeros(cap, np.int32)
    log = TrialLog(_ptr(h, C.c_double), _ptr(err, C.c_double), _ptr(outcome, C.c_int32), cap, 0)
    st = Stats()
    rc = L.orc_trace_log(C.byref(prep.P), _ptr(ra, C.c_int64), len(ra), C.byref(rec),
                         C.byref(st), C.byref(log))
    if rc != 0:
        raise RuntimeError(f"oracle: trace_log returned {rc}")
    n = log.n
    return h[:n].copy(), err[:n].copy(), outcome[:n].copy()


def _trace_events(scene, roots, threads, capacity, ev_capacity=None):
    L = lib()
    prep = _Prepared(scene)
    n_roots = scene.n_rays if roots is None else len(roots)
    if capacity is None:
        capacity = max(16, 8 * n_roots + 64)
    if threads is None:
        threads = max(1, min(os.cpu_count() or 1, 16))
    if ev_capacity is None:
        ev_capacity = max(16, 4 * n_roots + 64)
    arrs = {}
    for f in F64_FIELDS:
        arrs[f] = np.zeros(capacity, np.float64)
    for f in U64_FIELDS:
        arrs[f] = np.zeros(capacity, np.uint64)
    for f in I32_FIELDS:
        arrs[f] = np.zeros(capacity, np.int32)
    rec = Records(*([_ptr(arrs[f], C.c_double) for f in F64_FIELDS]
                    + [_ptr(arrs[f], C.c_uint64) for f in U64_FIELDS]
                    + [_ptr(arrs[f], C.c_int32) for f in I32_FIELDS]
                    + [capacity]))
    ev = {f: np.zeros((ev_capacity, k) if k > 1 else ev_capacity, dt)
          for f, (_, dt, k) in EVENT_FIELDS.items()}
    evs = Events(*([_ptr(ev[f], ct) for f, (ct, _, _) in EVENT_FIELDS.items()]
                   + [ev_capacity]))
    st = Stats()
    n_ev = C.c_int64(0)
    rptr = None
    if roots is not None:
        ra = np.ascontiguousarray(roots, dtype=np.int64)
        prep.keep.append(ra)
        rptr = _ptr(ra, C.c_int64)
    rc = L.orc_trace_events(C.byref(prep.P), rptr, n_roots, C.byref(rec), C.byref(st),
                            C.byref(evs), C.byref(n_ev), threads)
    stats = {f: int(getattr(st, f)) for f in STAT_FIELDS}
    if rc == -2:
        raise ValueError("oracle: unsupported problem (generations must be 1..4, planes <= 16)")
    if rc == -1:
        raise RuntimeError(f"oracle: record capacity {capacity} < needed {stats['needed']}")
    if rc == -3:  # more events than room: trace again with room for all of them
        return _trace_events(scene, roots, threads, capacity, int(n_ev.value))
    n = stats["records"]
    order = np.argsort(arrs["key"][:n], kind="stable")
    out = {f: a[:n][order] for f, a in arrs.items()}
    m = int(n_ev.value)
    order = np.lexsort((ev["ordinal"][:m], ev["key"][:m]))
    evout = {f: a[:m][order] for f, a in ev.items()}
    return out, stats, evout


def ck_trial(scene, region: int, y0, h: float):
    L = lib()
    prep = _Prepared(scene)
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    y5 = np.zeros(7)
    dl = np.zeros(7)
    L.orc_ck_trial(C.byref(prep.P), region, _ptr(y0, C.c_double), h,
                   _ptr(y5, C.c_double), _ptr(dl, C.c_double))
    return y5, dl


def field(scene, region: int, r):
    L = lib()
    prep = _Prepared(scene)
    r = np.ascontiguousarray(r, dtype=np.float64)
    n = np.zeros(1)
    g = np.zeros(3)
    L.orc_field(C.byref(prep.P), region, _ptr(r, C.c_double), _ptr(n, C.c_double),
                _ptr(g, C.c_double))
    return float(n[0]), g


def fresnel(n1: float, n2: float, ci: float):
    """(rs, rp, ts, tp) as complex numbers, cos_t, tir flag."""
    out = np.zeros(9)
    tir = lib().orc_fresnel(n1, n2, ci, _ptr(out, C.c_double))
    rs, rp = complex(out[0], out[1]), complex(out[2], out[3])
    ts, tp = complex(out[4], out[5]), complex(out[6], out[7])
    return rs, rp, ts, tp, float(out[8]), bool(tir)


# --- emitter -> receiver solves ---------------------------------------------
class SolveSpec(C.Structure):
    _fields_ = [("zs", C.POINTER(C.c_double)), ("zr", C.POINTER(C.c_double)),
                ("dist", C.POINTER(C.c_double)), ("n_scan", C.c_int32),
                ("max_iter", C.c_int32), ("max_brackets", C.c_int32),
                ("miss_tol", C.c_double), ("accept_tol", C.c_double),
                ("slope_max", C.c_double)]


SOLVE_I32 = ["found", "shots", "roots"]
SOLVE_F64 = ["theta", "miss", "t", "s", "as_re", "as_im", "ap_re", "ap_im"]


class SolveOut(C.Structure):
    _fields_ = ([(f, C.POINTER(C.c_int32)) for f in SOLVE_I32]
                + [(f, C.POINTER(C.c_double)) for f in SOLVE_F64])


def solve(scene, zs, zr, dist, pairs=None, n_scan=64, max_iter=60, max_brackets=4,
          miss_tol=1e-4, accept_tol=1e-3, slope_max=1e7, threads=None):
    """Shooting solves for source/receiver pairs; arrays indexed [pair, family]
    with family 0 = direct, 1 = reflected once at the surface."""
    L = lib()
    L.orc_solve.restype = C.c_int
    L.orc_solve.argtypes = [C.POINTER(Problem), C.POINTER(SolveSpec), C.POINTER(C.c_int64),
                            C.c_int64, C.POINTER(SolveOut), C.c_int]
    prep = _Prepared(scene)
    zs = np.ascontiguousarray(zs, np.float64)
    zr = np.ascontiguousarray(zr, np.float64)
    dist = np.ascontiguousarray(dist, np.float64)
    prep.keep += [zs, zr, dist]
    spec = SolveSpec(_ptr(zs, C.c_double), _ptr(zr, C.c_double), _ptr(dist, C.c_double),
                     n_scan, max_iter, max_brackets, miss_tol, accept_tol, slope_max)
    n = len(zs)
    arrs = {f: np.zeros(2 * n, np.int32) for f in SOLVE_I32}
    arrs.update({f: np.zeros(2 * n, np.float64) for f in SOLVE_F64})
    out = SolveOut(*([_ptr(arrs[f], C.c_int32) for f in SOLVE_I32]
                     + [_ptr(arrs[f], C.c_double) for f in SOLVE_F64]))
    rptr, n_pairs = None, n
    if pairs is not None:
        pa = np.ascontiguousarray(pairs, np.int64)
        prep.keep.append(pa)
        rptr, n_pairs = _ptr(pa, C.c_int64), len(pa)
    if threads is None:
        threads = max(1, min(os.cpu_count() or 1, 16))
    rc = L.orc_solve(C.byref(prep.P), C.byref(spec), rptr, n_pairs, C.byref(out), threads)
    if rc != 0:
        raise ValueError("oracle: unsupported solve problem (planes[0] must be the surface; "
                         "no box or time limit)")
    return {f: a.reshape(n, 2) for f, a in arrs.items()}


SHOT_I32 = ["status", "n_acc", "n_rej"]
SHOT_F64 = ["miss", "t", "s", "as_re", "as_im", "ap_re", "ap_im"]


class ShotOut(C.Structure):
    _fields_ = ([(f, C.POINTER(C.c_int32)) for f in SHOT_I32]
                + [(f, C.POINTER(C.c_double)) for f in SHOT_F64])


def shoot(scene, zs, zr, dist, theta, family, threads=None):
    """Single shots (the building block of solve): status 0 receiver plane,
    1 surface touched where the family forbids it, 2 lost, 3 invalid."""
    L = lib()
    L.orc_shoot.restype = C.c_int
    L.orc_shoot.argtypes = [C.POINTER(Problem)] + [C.POINTER(C.c_double)] * 4 + [
        C.POINTER(C.c_int32), C.c_int64, C.POINTER(ShotOut), C.c_int]
    prep = _Prepared(scene)
    cols = [np.ascontiguousarray(a, np.float64) for a in (zs, zr, dist, theta)]
    fam = np.ascontiguousarray(family, np.int32)
    n = len(cols[0])
    assert all(len(c) == n for c in cols) and len(fam) == n
    prep.keep += cols + [fam]
    arrs = {f: np.zeros(n, np.int32) for f in SHOT_I32}
    arrs.update({f: np.zeros(n, np.float64) for f in SHOT_F64})
    out = ShotOut(*([_ptr(arrs[f], C.c_int32) for f in SHOT_I32]
                    + [_ptr(arrs[f], C.c_double) for f in SHOT_F64]))
    if threads is None:
        threads = max(1, min(os.cpu_count() or 1, 16))
    rc = L.orc_shoot(C.byref(prep.P), *[_ptr(c, C.c_double) for c in cols],
                     _ptr(fam, C.c_int32), n, C.byref(out), threads)
    if rc != 0:
        raise ValueError("oracle: unsupported shoot problem (planes[0] must be the surface; "
                         "no box or time limit)")
    return arrs


class SeedSpec(C.Structure):
    _fields_ = [("verify_tol", C.c_double), ("dseed", C.c_double), ("max_shots", C.c_int32)]


def solve_seeded(scene, zs, zr, dist, seed, try_, verify_tol=0.01, dseed=1e-4, max_shots=6,
                 threads=None):
    """Seeded secant per entry (seed and try_ shaped [n, 2]); results shaped
    [n, 2] plus 'verify' (1 verified, 0 not, -1 not tried)."""
    L = lib()
    L.orc_solve_seeded.restype = C.c_int
    L.orc_solve_seeded.argtypes = [C.POINTER(Problem)] + [C.POINTER(C.c_double)] * 3 + [
        C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(SeedSpec),
        C.POINTER(SolveOut), C.POINTER(C.c_int32), C.c_int]
    prep = _Prepared(scene)
    cols = [np.ascontiguousarray(a, np.float64) for a in (zs, zr, dist)]
    n = len(cols[0])
    sd = np.ascontiguousarray(np.asarray(seed, np.float64).reshape(2 * n))
    tr = np.ascontiguousarray(np.asarray(try_, np.int32).reshape(2 * n))
    prep.keep += cols + [sd, tr]
    arrs = {f: np.zeros(2 * n, np.int32) for f in SOLVE_I32}
    arrs.update({f: np.zeros(2 * n, np.float64) for f in SOLVE_F64})
    verify = np.full(2 * n, -1, np.int32)
    out = SolveOut(*([_ptr(arrs[f], C.c_int32) for f in SOLVE_I32]
                     + [_ptr(arrs[f], C.c_double) for f in SOLVE_F64]))
    spec = SeedSpec(verify_tol, dseed, max_shots)
    if threads is None:
        threads = max(1, min(os.cpu_count() or 1, 16))
    rc = L.orc_solve_seeded(C.byref(prep.P), *[_ptr(c, C.c_double) for c in cols], n,
                            _ptr(sd, C.c_double), _ptr(tr, C.c_int32), C.byref(spec),
                            C.byref(out), _ptr(verify, C.c_int32), threads)
    if rc != 0:
        raise ValueError("oracle: unsupported solve problem")
    res = {f: a.reshape(n, 2) for f, a in arrs.items()}
    res["verify"] = verify.reshape(n, 2)
    return res
