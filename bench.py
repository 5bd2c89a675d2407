#!/usr/bin/env python
"""Throughput benchmark of the FP64 ray tracer on one MI355X.

Default workload: the two-layer firn model -- 1,048,576 rays launched
isotropically from 64 seeded sources (depths 10-1500 m), n = 1.78 -
0.43 exp(-z/75 m) with +0.01 below the layer plane at 150 m, Fresnel surface
and layer plane spawning secondaries up to four generations, 5 km path limit,
Cash-Karp tolerance 1e-6, steps 1 mm - 10 m, paper model (eq. 2).

A step is one raytrace_launch (initialisation and the whole ray tree) over
the full batch, with inputs already resident in device memory.  The headline
value is accepted Runge-Kutta steps per second over primaries and
secondaries.  The trace kernel's own duration is measured with HIP events
recorded on the launch stream, and the CPU oracle is timed on a bounded
sample of the same workload.  The default line also carries the metric's
second part under "solves": emitter -> receiver solves/s of the
surrogate-seeded path and of the tracer alone on one batch of 1,048,576
pairs (network trained first, not timed; see surrogate_run).  Prints one
JSON line.
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 work of one Cash-Karp trial step (FMA = 2 FLOP): the
# generic 3-D count of the method's step, paper model, analytic layered field
# with planes -- 15 h a_kj products, 105 stage-combination FMAs, outputs 60,
# error vector 66, error norm 20, controller with pow 65, renormalisation 18,
# six right-hand sides of ~48 (exp ~30 by range reduction + polynomial,
# reciprocal ~8), plane tests + s += h ~15: ~750 FLOP (exact model ~830).
# The stratified kernel skips the horizontal components and uses the Nystrom
# form of the step, so it executes fewer operations per trial (~458); the
# roofline counts the method's work, not the kernel's.
FLOP_PER_TRIAL = {0: 750, 1: 830}      # by model (paper, exact)
FLOP_PLANES_IN_BASE = 15               # the plane tests included above
# Boundary tests per trial by surface: plane 3 FMA; sphere 3 sub + 2 FMA +
# mul + sqrt + sub; paraboloid 4 sub + FMA + 2 mul; box face as a plane;
# travel-time limit 2.
SURFACE_FLOP = {0: 6, 1: 17, 2: 8}
# Non-stratified analytic media add to each of the six field evaluations the
# projection on the stratification axis (5) and 49 per Gaussian anomaly of the
# ray's region.
FLOP_AXIS = 6 * 5
FLOP_PER_ANOMALY = 6 * 49
# Gridded media, paper model: per stage 8 float4 node loads (128 B) -> 768 B
# of node data per trial step.
BYTES_PER_TRIAL_GRID = 768

# HBM bytes per launch of the dominant kernel, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, per dispatch), each divided by what the same
# counter reads per byte of a plain 1 GiB device copy (--workload copy).
# Valid only for the kernel sources with the listed SHA-256 digest (of their
# code: comments and whitespace removed); after a change to the code the
# traffic is reported as null until measured again.
TRAFFIC = {  # workload -> (fetch bytes, write bytes, digest)
    "twolayer": (2.9294e+09, 4.1181e+09,
                 "89e253342b7b13119e670cac1e30a8686dabadd1e05632db276fd97c85f56764"),
    "grid256": (1.0167e+11, 2.5759e+09,
                "89e253342b7b13119e670cac1e30a8686dabadd1e05632db276fd97c85f56764"),
}
TRACE_SOURCES = ("rt_kernels.hip", "rt_strat.hip", "rt_trace.hpp", "rt_device.hpp",
                 "rt_params.hpp")


def code_of(text):
    """C/C++ source without comments and whitespace."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return "".join(text.split())


def kernel_digest(sources=None):
    import hashlib
    h = hashlib.sha256()
    for f in TRACE_SOURCES:
        if sources is None:
            with open(os.path.join(ROOT, "paper_1810_01780_amd", "csrc", f)) as fh:
                text = fh.read()
        else:
            text = sources[f]
        h.update(code_of(text).encode())
    return h.hexdigest()


# L2 hit fraction of the trace kernel's requests (rocprofv3 TCC_HIT_sum,
# TCC_MISS_sum of one launch), valid for the listed code digest like TRAFFIC.
L2_HIT = {  # workload -> (hits, misses, digest)
    "grid256": (3.9961e+09, 8.7349e+08,
                "89e253342b7b13119e670cac1e30a8686dabadd1e05632db276fd97c85f56764"),
}

# FP64 instructions the trace kernel issues per launch (rocprofv3
# SQ_INSTS_VALU_FMA_F64, _MUL_F64, _ADD_F64, _TRANS_F64: wave instructions,
# masked lanes included) and the trial steps of that launch, valid for the
# listed code digest like TRAFFIC.  The headline FLOP/s counts the method's
# work per trial (FLOP_PER_TRIAL); this is what the kernel executes for it.
EXEC_FP64 = {  # workload -> (fma, mul, add, trans, trial steps, digest)
    "twolayer": (4.49195e9, 1.33698e9, 2.18356e8, 2.21103e8, 1621800464,
                 "89e253342b7b13119e670cac1e30a8686dabadd1e05632db276fd97c85f56764"),
}


def executed_fp64(workload, kern_s):
    t = EXEC_FP64.get(workload)
    if t is None or t[5] != kernel_digest():
        return None
    flop = 64.0 * (2.0 * t[0] + t[1] + t[2] + t[3])
    return {"flop_per_trial": flop / t[4], "tflops": flop / kern_s / 1e12,
            "frac": flop / kern_s / 1e12 / PEAK_FP64_VECTOR_TFLOPS,
            "source": "SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F64 x 64 lanes, FMA as 2"}


def measured_l2_hit(workload):
    t = L2_HIT.get(workload)
    if t is None or t[2] != kernel_digest():
        return None
    return t[0] / (t[0] + t[1])


def measured_traffic(workload):
    t = TRAFFIC.get(workload)
    if t is None or t[2] != kernel_digest():
        return None
    return t[0] + t[1]


PEAK_FP64_VECTOR_TFLOPS = 78.6   # MI355X: 256 CU x 128 FLOP/clk x 2.4 GHz
PEAK_HBM_GBS = 8000.0            # MI355X HBM3E
PEAK_BF16_TFLOPS = 2500.0        # MI355X dense BF16 matrix cores


def _hip():
    # the HIP runtime torch already loaded (same soname as the library's)
    lib = ctypes.CDLL("libamdhip64.so.7")
    lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                        ctypes.c_void_p]
    lib.hipEventSynchronize.argtypes = [ctypes.c_void_p]
    lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
    return lib


def device_info():
    """The GPU the run used: name, compute units, peak engine clock."""
    import torch
    hip = _hip()
    v = ctypes.c_int()
    dev = torch.cuda.current_device()
    info = {"name": torch.cuda.get_device_name(dev)}
    for key, attr in (("compute_units", 63), ("clock_mhz", 5)):
        # hipDeviceAttributeMultiprocessorCount, hipDeviceAttributeClockRate (kHz)
        if hip.hipDeviceGetAttribute(ctypes.byref(v), attr, dev) == 0:
            info[key] = v.value // 1000 if key == "clock_mhz" else v.value
    return info


def make_scene(name):
    from paper_1810_01780_amd import workloads as W
    if name == "twolayer":
        return W.two_layer(), dict(workload="twolayer", rays=1048576, sources=64,
                                   generations=4, tol=1e-6, s_max_m=5000, model="paper")
    if name == "grid256":
        return W.gridded(), dict(workload="grid256", rays=4194304, sources=256,
                                 grid=[256, 256, 128], spacing_m=10, tol=1e-7, s_max_m=3000,
                                 model="paper")
    if name == "curved":
        return W.curved(rays_per_source=262144), dict(
            workload="curved", rays=1048576, sources=4, generations=3, tol=1e-6, s_max_m=1500,
            model="paper", surfaces="plane, sphere R 25 m, paraboloid bed")
    if name == "field3d":
        return W.field3d(rays_per_source=262144), dict(
            workload="field3d", rays=1048576, sources=4, generations=2, tol=1e-6, s_max_m=1500,
            model="paper", field="firn along an axis tilted 8 deg, 2 Gaussian anomalies")
    if name == "fan1024":
        return W.point_source_fan(), dict(workload="fan1024", rays=1024, sources=1,
                                          generations=2, tol=1e-6, s_max_m=2000, model="paper")
    raise SystemExit(f"unknown workload {name}")


def is_general(scene):
    """True when the scene runs on the general 3-D kernel."""
    return bool(scene.anomalies) or any(
        r.use_grid or r.axis[0] != 0.0 or r.axis[1] != 0.0 or r.axis[2] < 0.0
        for r in scene.regions)


def trace_kernel_name(scene):
    """The trace kernel a launch on this scene runs: gridded and general
    fields take the general 3-D kernel, depth-stratified ones the
    stratified kernel (the same test as the C launcher's)."""
    return "trace_general_kernel" if is_general(scene) else "trace_strat_kernel"


def flop_per_trial(scene, region):
    """Algorithmic FP64 work of one trial step of a ray in region (analytic
    media): the method's per-step count for the model, with the boundary
    tests of this scene's surfaces and the non-stratified field terms."""
    bnd = sum(SURFACE_FLOP[p.shape] for p in scene.planes) + 1
    bnd += 36 if scene.box_lo is not None else 0
    bnd += 2 if scene.limits.t_max > 0 else 0
    f = FLOP_PER_TRIAL[scene.limits.model] - FLOP_PLANES_IN_BASE + bnd
    if is_general(scene):
        n_an = sum(1 for q in scene.anomalies if q.region == region)
        f += FLOP_AXIS + FLOP_PER_ANOMALY * n_an
    return f


def trial_flops(scene, rec, trials):
    """FLOP of a launch: each record's trials at its region's rate (a record
    stays in one region: the parent reflects, the secondary carries the
    refraction), event-search trials at the mean rate."""
    import numpy as np
    per = np.array([flop_per_trial(scene, r) for r in range(len(scene.regions))], float)
    n = rec["n_acc"].astype(np.float64) + rec["n_rej"]
    w = float((n * per[rec["region"]]).sum())
    return w * trials / max(1.0, float(n.sum()))


def host_cpu():
    """(logical CPUs this process may use, all logical CPUs, CPU model)."""
    allowed = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return allowed or os.cpu_count() or 1, os.cpu_count() or 1, model


def _oracle_rate(scene, threads, target_s, log):
    """Accepted steps/s of the oracle on an evenly strided sample of root rays
    sized for about target_s seconds: (rate, description of the sample)."""
    import numpy as np
    import oracle
    n = scene.n_rays
    probe = np.arange(0, n, max(1, n // 512), dtype=np.int64)
    t0 = time.perf_counter()
    _, st = oracle.trace(scene, roots=probe, threads=threads)
    per_root = (time.perf_counter() - t0) / len(probe)
    for attempt in range(2):
        # the probe is short and its time noisy: a sample that ran for less
        # than half the target is sized again from its own rate, once
        stride = max(1, int(np.ceil(n * per_root / target_s)))
        roots = np.arange(0, n, stride, dtype=np.int64)
        log(f"cpu baseline: {len(roots)} of {n} roots (one in {stride}), {threads} threads")
        t0 = time.perf_counter()
        _, st = oracle.trace(scene, roots=roots, threads=threads)
        dt = time.perf_counter() - t0
        if dt >= 0.5 * target_s or stride == 1:
            break
        per_root = dt / len(roots)
    return st["accepted"] / dt, (f"one root ray in {stride} ({len(roots)} of {n}) with its "
                                 f"full secondary tree: {st['accepted']} accepted steps in "
                                 f"{dt:.1f} s")


def cpu_baseline(scene, target_s, max_threads, log):
    """The CPU oracle on the host: one thread, then every core this process
    may use (at most max_threads), each on its own strided sample of root
    rays sized for about target_s / 2 seconds."""
    allowed, nproc, model = host_cpu()
    threads = max(1, min(allowed, max_threads))
    one, one_sample = _oracle_rate(scene, 1, 0.4 * target_s, log)
    rate, sample = _oracle_rate(scene, threads, 0.6 * target_s, log)
    return {"value": rate, "unit": "ray-steps/s", "cores": threads, "kind": "oracle",
            "sample": sample, "one_thread": {"value": one, "sample": one_sample},
            "host": {"cpus_allowed": allowed, "nproc": nproc, "model": model}}


def cpu_solve_baseline(sp, target_s, threads, log):
    """Time the CPU oracle's solves on an evenly strided sample of the pairs."""
    import numpy as np
    import oracle
    n = sp.n
    probe = np.arange(0, n, max(1, n // 256), dtype=np.int64)
    t0 = time.perf_counter()
    oracle.solve(sp.scene, sp.zs, sp.zr, sp.dist, pairs=probe, threads=threads)
    per_pair = (time.perf_counter() - t0) / len(probe)
    for attempt in range(2):
        stride = max(1, int(np.ceil(n * per_pair / target_s)))
        pick = np.arange(0, n, stride, dtype=np.int64)
        log(f"cpu baseline: {len(pick)} of {n} pairs (one in {stride}), {threads} threads")
        t0 = time.perf_counter()
        oracle.solve(sp.scene, sp.zs, sp.zr, sp.dist, pairs=pick, threads=threads)
        dt = time.perf_counter() - t0
        if dt >= 0.5 * target_s or stride == 1:
            break
        per_pair = dt / len(pick)
    return {"value": len(pick) / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"one pair in {stride} ({len(pick)} of {n}), both families, "
                      f"in {dt:.1f} s"}


def bench_solve(args, log):
    """Batched emitter -> receiver solves: 65,536 seeded pairs (source depth
    50-2000 m, receiver depth 0-200 m, distance 10 m - 3 km) in the two-layer
    firn model, direct and surface-reflected solution of each.  A step is one
    raytrace_solve of the whole batch replayed from a captured graph, with the
    launch tuning chosen by rt_solve_autotune on the whole batch."""
    import torch
    from paper_1810_01780_amd import binding
    from paper_1810_01780_amd import workloads as W
    sp = W.solve_pairs()
    prm = binding.solve_params()
    cfg = dict(workload="solve65536", pairs=sp.n, n_scan=prm.n_scan, max_iter=prm.max_iter,
               max_brackets=prm.max_brackets, miss_tol_m=prm.miss_tol,
               accept_tol_m=prm.accept_tol, slope_max_m_per_rad=prm.slope_max,
               tol=sp.scene.limits.tol, model="paper")
    log(f"workload solve65536: {sp.n} pairs")
    if args.block or args.refill or args.scan_chunk or args.fused is not None:
        tun = binding.rt_tuning(block_size=args.block, refill_threshold=args.refill,
                                scan_chunk=args.scan_chunk, solve_fused=args.fused or 0)
        cfg["tuning"] = "fixed"
    else:
        # the whole batch: a 16,384-pair sample picked tunings 6 % apart from
        # run to run on the full solve
        m = sp.n
        sample = binding.DeviceSolve(sp.scene, sp.zs[:m], sp.zr[:m], sp.dist[:m], prm)
        tun, ms = sample.autotune()
        log(f"autotune on {m} pairs: block {tun.block_size} refill {tun.refill_threshold} "
            f"scan chunk {tun.scan_chunk} fused {tun.solve_fused} ({ms:.2f} ms)")
        cfg["tuning"] = "autotuned"
        del sample
    fused = tun.solve_fused == 1 and prm.n_scan <= 64 and prm.max_brackets <= 4
    cfg.update(block=tun.block_size, refill=tun.refill_threshold, scan_chunk=tun.scan_chunk,
               launches="fused" if fused else "scan+refine+select")
    ds = binding.DeviceSolve(sp.scene, sp.zs, sp.zr, sp.dist, prm)
    hip = _hip()

    def event():
        e = ctypes.c_void_p()
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
        return e

    def elapsed(b, e):
        ms = ctypes.c_float()
        hip.hipEventElapsedTime(ctypes.byref(ms), b, e)
        return ms.value

    # shot-kernel time (the fused launch, or scan + refinement) from eager
    # launches, events on the stream
    kern = []
    for i in range(args.warmup + 1):
        b, e = event(), event()
        ds.launch(tuning=binding.rt_tuning(
            block_size=tun.block_size, refill_threshold=tun.refill_threshold, ev_trace_begin=b,
            ev_trace_end=e, scan_chunk=tun.scan_chunk, solve_fused=tun.solve_fused))
        res, st = ds.collect()
        if i >= args.warmup:
            kern.append(elapsed(b, e))
        log(f"eager {i}: found {st['found']} of {2 * sp.n}, {st['shots']} shots, "
            f"{elapsed(b, e):.2f} ms shot kernels")
    # capture the whole solve and time graph replays
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ds.launch(stream=s, tuning=tun)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        ds.launch(tuning=tun)
    g.replay()
    torch.cuda.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    res2, st2 = ds.collect()
    assert st2 == st, "graph replay differs from the eager solve"
    kern_s = sum(kern) / len(kern) / 1e3
    trials = st["accepted"] + st["rejected"] + st["relocation"]
    achieved = trials * FLOP_PER_TRIAL[0] / kern_s / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS, "traffic": None,
            "kernel": "shot_kernel (fused scan, refine and select)" if fused
            else "shot_kernel (scan + refine)", "kernel_ms": kern_s * 1e3}
    cfg.update(shots=st["shots"], trial_steps=trials, accepted_steps=st["accepted"],
               found=st["found"], brackets=st["brackets"])
    log(f"timed {args.steps} graph replays: {wall:.3f} s; shot kernels {kern_s * 1e3:.2f} ms")
    out = {"metric": "emitter->receiver solves/s (FP64 tracer)",
           "value": sp.n * args.steps / wall, "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": cfg, "roofline": roof}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_solve_baseline(sp, args.cpu_seconds,
                                                 min(args.cpu_threads, host_cpu()[0]), log)
    print(json.dumps(out), flush=True)


def surrogate_run(n_pairs, steps, warmup, log, net=None, multi_logit=-10.0):
    """Surrogate-seeded solves against the tracer alone on the same GPU.

    The network is trained first (the default recipe: tracer solves of
    2,048 seeded profiles x 8,192 pairs, 8,000 Adam steps of 16,384 rows; not
    timed) unless given.  Then n_pairs seeded pairs of the two-layer workload
    are solved as one batch, by the captured raytrace_solve_surrogate graph
    (network inference on the whole batch, seeded secant with shot
    verification, tracer for every other entry) and by the tracer's captured
    raytrace_solve graph, both with the tracer launch tuning that
    rt_solve_autotune picks on the batch's first 65,536 pairs; each is
    replayed warmup + steps times, the steps timed.  Returns the measured figures and the entry classification."""
    import numpy as np
    import torch
    from paper_1810_01780_amd import binding
    from paper_1810_01780_amd import surrogate
    from paper_1810_01780_amd import workloads as W
    out = {}
    if net is None:
        t0 = time.perf_counter()
        net, losses = surrogate.default_model(seed=0, log=log)
        out.update(training_pairs=2048 * 8192, training_steps=8000, training_batch=16384,
                   training_s=round(time.perf_counter() - t0, 1), final_loss=losses[-1][1])
    sp = W.solve_pairs(n_pairs)
    prm = binding.solve_params()
    spar = binding.surrogate_params(z0=75.0, dn=0.43, multi_logit=multi_logit)
    # one launch tuning for the tracer's solve in both graphs (the surrogate's
    # tracer entries and the tracer alone), picked by rt_solve_autotune on the
    # batch's first 65,536 pairs
    m = min(sp.n, 1 << 16)
    sample = binding.DeviceSolve(sp.scene, sp.zs[:m], sp.zr[:m], sp.dist[:m], prm)
    tun, _ = sample.autotune()
    del sample
    out.update(tuning=dict(block=tun.block_size, refill=tun.refill_threshold,
                           scan_chunk=tun.scan_chunk, fused=tun.solve_fused,
                           picked_on_pairs=m))
    log(f"tracer tuning (autotuned on {m} pairs): block {tun.block_size} refill "
        f"{tun.refill_threshold} scan chunk {tun.scan_chunk} fused {tun.solve_fused}")
    ds = binding.DeviceSurrogateSolve(sp.scene, sp.zs, sp.zr, sp.dist, spar, prm)
    tr = binding.DeviceSolve(sp.scene, sp.zs, sp.zr, sp.dist, prm)

    def graph_of(fn):
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn(s)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            fn(None)
        return g

    g_su = graph_of(lambda s: ds.launch(net.params, stream=s, tuning=tun))
    g_tr = graph_of(lambda s: tr.launch(stream=s, tuning=tun))

    def timed(g):
        for _ in range(warmup):
            g.replay()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps
    t_su = timed(g_su)
    t_tr = timed(g_tr)
    res, st = ds.collect()
    rres, rst = tr.collect()
    path = res["path"]
    sur = path == binding.RT_PATH_SURROGATE
    both = sur & (rres["found"] == 1)
    dt = res["t"][both] - rres["t"][both]
    # network forward alone on the whole batch (events on the stream)
    hip = _hip()
    e0, e1 = ctypes.c_void_p(), ctypes.c_void_p()
    hip.hipEventCreate(ctypes.byref(e0))
    hip.hipEventCreate(ctypes.byref(e1))
    inf = binding.DeviceMLP(net.params.cpu().numpy(), max_batch=sp.n, training=False)
    x = torch.randn((sp.n, 5), device="cuda")
    y = torch.empty((sp.n, 12), device="cuda")
    inf.forward(x, y)
    stream = torch.cuda.current_stream().cuda_stream
    hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    hip.hipEventRecord(e0, ctypes.c_void_p(stream))
    for _ in range(10):
        inf.forward(x, y)
    hip.hipEventRecord(e1, ctypes.c_void_p(stream))
    hip.hipEventSynchronize(e1)
    ms = ctypes.c_float()
    hip.hipEventElapsedTime(ctypes.byref(ms), e0, e1)
    mlp_s = ms.value / 10 / 1e3
    mlp_flop = 2.0 * sp.n * (5 * 256 + 3 * 256 * 256 + 256 * 12)
    out.update(pairs=sp.n, network="5-256x4-12 SiLU, BF16 MFMA", verify_tol_m=spar.verify_tol,
               max_shots=spar.max_shots, absent_logit=spar.absent_logit,
               multi_logit=spar.multi_logit, surrogate_solves_per_s=sp.n / t_su,
               tracer_solves_per_s=sp.n / t_tr, gain_vs_tracer=t_tr / t_su,
               surrogate_ms=t_su * 1e3, tracer_ms=t_tr * 1e3,
               surrogate_entries=int(sur.sum()), tracer_entries=int((~sur).sum()),
               fallback_pairs=st["fallback_pairs"], found=int(res["found"].sum()),
               tracer_found=int(rres["found"].sum()),
               tracer_found_missed=int(((rres["found"] == 1) & (res["found"] == 0)).sum()),
               later_than_tracer=int((dt > 1e-10).sum()),
               earlier_than_tracer=int((dt < -1e-10).sum()),
               shots=st["shots"], tracer_shots=rst["shots"],
               trial_steps=st["accepted"] + st["rejected"] + st["relocation"],
               mlp_forward_ms=mlp_s * 1e3, mlp_tflops=mlp_flop / mlp_s / 1e12,
               mlp_bf16_frac=mlp_flop / mlp_s / 1e12 / PEAK_BF16_TFLOPS)
    log(f"surrogate {t_su * 1e3:.2f} ms vs tracer {t_tr * 1e3:.2f} ms per {sp.n} pairs; "
        f"{st['fallback_pairs']} pairs with tracer entries")
    return out, net, sp


def bench_surrogate(args, log):
    """Surrogate-seeded solves of a 1,048,576-pair batch (surrogate_run); the
    JSON line carries the tracer's rate on the same pairs and GPU."""
    r, _, sp = surrogate_run(1 << 20, args.steps, args.warmup, log,
                             multi_logit=args.multi_logit)
    t_su = r["surrogate_ms"] / 1e3
    achieved = r["trial_steps"] * FLOP_PER_TRIAL[0] / t_su / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS, "traffic": None,
            "kernel": "shot_kernel (seeded + tracer entries), whole-launch time",
            "kernel_ms": t_su * 1e3}
    out = {"metric": "emitter->receiver solves/s (surrogate-seeded, shot-verified)",
           "value": r["surrogate_solves_per_s"], "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_su * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64+bf16", "data": "synthetic",
           "config": dict(workload="solve1M-surrogate", **r), "roofline": roof}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_solve_baseline(sp, args.cpu_seconds,
                                                 min(args.cpu_threads, host_cpu()[0]), log)
    print(json.dumps(out), flush=True)


def bench_copy(args, log):
    """A plain device-to-device copy of 1 GiB per step: the calibration of the
    HBM byte counters (reads 2^30 bytes, writes 2^30 bytes)."""
    import torch
    n = 1 << 27
    x = torch.rand(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    log(f"copy: {dt * 1e3:.3f} ms per GiB copied")
    out = {"metric": "device copy bandwidth (read + write)", "value": 2 * n * 8 / dt / 1e9,
           "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "copy", "bytes_read": n * 8, "bytes_written": n * 8}}
    print(json.dumps(out), flush=True)


def probe_levels(log, passes=20):
    """Read bandwidth (GB/s) of float4 streams and gathers from buffers sized
    for each XCD's L2 (2 MiB), the MALL (128 MiB, the size of the gridded
    workload's node array) and HBM (4 GiB)."""
    import torch
    from paper_1810_01780_amd import binding
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    for name, nbytes in (("l2", 2 << 20), ("mall", 128 << 20), ("hbm", 4 << 30)):
        buf = torch.rand(nbytes // 4, dtype=torch.float32, device="cuda")
        for pat, pname in ((binding.RT_PROBE_STREAM, "stream"), (binding.RT_PROBE_GATHER, "gather")):
            gbs = binding.rt_probe_read_bandwidth(buf.data_ptr(), nbytes, pat, passes, stream)
            out[f"{pname}_{name}"] = gbs
            log(f"probe {pname} {name} ({nbytes >> 20} MiB): {gbs:.0f} GB/s")
        del buf
    return out


def bench_probe(args, log):
    """The read-bandwidth probe alone: one JSON line of GB/s per level and
    pattern (value: the L2 gather rate)."""
    t0 = time.perf_counter()
    lv = probe_levels(log)
    dt = time.perf_counter() - t0
    out = {"metric": "float4 read bandwidth by serving level", "value": lv["gather_l2"],
           "unit": "GB/s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": dt * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": {"workload": "probe", **lv}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="twolayer",
                    choices=["twolayer", "grid256", "curved", "field3d", "fan1024", "solve",
                             "surrogate", "copy", "probe"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--refill", type=int, default=0)
    ap.add_argument("--scan-chunk", type=int, default=0,
                    help="solve: entries whose angle scans interleave (0 = autotune)")
    ap.add_argument("--fused", type=int, default=None, choices=[0, 1],
                    help="solve: 1 = one fused launch, 0 = scan, refine and select launches "
                         "(default: autotune)")
    ap.add_argument("--multi-logit", type=float, default=-10.0,
                    help="surrogate: several-roots logit above which the tracer solves an entry")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="at most this many oracle threads (one GPU's share of a box's CPUs)")
    ap.add_argument("--ev-capacity", type=int, default=0,
                    help="record Fresnel events too (rt_event array of this many entries)")
    ap.add_argument("--no-solves", action="store_true",
                    help="twolayer: leave out the solves figures (surrogate vs tracer)")
    args = ap.parse_args()
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: one GPU per process; rays shard across GPUs by root index, which "
              "is left to the caller, so only --gpus 1 is measured", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1810_01780_amd import binding

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    if args.workload == "copy":
        return bench_copy(args, log)
    if args.workload == "probe":
        return bench_probe(args, log)
    if args.workload == "solve":
        return bench_solve(args, log)
    if args.workload == "surrogate":
        return bench_surrogate(args, log)
    scene, cfg = make_scene(args.workload)
    log(f"workload {cfg['workload']}: {scene.n_rays} rays")
    ds = binding.DeviceScene(scene, ev_capacity=args.ev_capacity)
    hip = _hip()

    def event():
        e = ctypes.c_void_p()
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
        return e

    def tuning(b=None, e=None):
        return binding.rt_tuning(args.block, 0, args.refill, b, e)

    for i in range(args.warmup):
        ds.launch(tuning=tuning())
        rec, st = ds.collect()
        log(f"warmup {i}: {st['records']} records, {st['accepted']} accepted steps")
    pairs = [(event(), event()) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, e in pairs:
        ds.launch(tuning=tuning(b, e))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rec, st = ds.collect()
    kern_ms = []
    for b, e in pairs:
        ms = ctypes.c_float()
        hip.hipEventElapsedTime(ctypes.byref(ms), b, e)
        kern_ms.append(ms.value)
        hip.hipEventDestroy(b)
        hip.hipEventDestroy(e)
    kern_s = sum(kern_ms) / len(kern_ms) / 1e3
    log(f"timed {args.steps} launches: {wall:.3f} s wall, trace kernel {kern_s * 1e3:.3f} ms avg; "
        f"stats {st}")

    trials = st["accepted"] + st["rejected"] + st["relocation"]
    if args.workload == "grid256":
        # HBM: the measured traffic of the trace kernel (counter runs) over
        # its time; the node data the trials request is mostly served by the
        # L2 and the MALL, so it is set against those levels' measured peaks,
        # mixed by the L2 hit fraction of the same kernel's requests
        traffic = measured_traffic(args.workload)
        hbm = traffic / kern_s / 1e9 if traffic else None
        roof = {"bound": "hbm", "achieved": hbm, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": hbm / PEAK_HBM_GBS if hbm else None, "traffic": traffic}
        req = trials * BYTES_PER_TRIAL_GRID / kern_s / 1e9
        lv = probe_levels(log)
        hit = measured_l2_hit(args.workload)
        serving = {"requested_GBps": req, "bytes_per_trial": BYTES_PER_TRIAL_GRID,
                   "peak_stream_l2": lv["stream_l2"], "peak_stream_mall": lv["stream_mall"],
                   "peak_gather_l2": lv["gather_l2"], "peak_gather_mall": lv["gather_mall"],
                   "l2_hit": hit}
        if hit is not None:
            mix = 1.0 / (hit / lv["stream_l2"] + (1.0 - hit) / lv["stream_mall"])
            serving.update(peak_mix=mix, frac=req / mix)
        roof["serving"] = serving
    else:
        method = trial_flops(scene, rec, trials)
        achieved = method / kern_s / 1e12
        # achieved counts the method's work per trial step; executed_fp64
        # what the kernel's FP64 instructions amount to (counter runs)
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
                "traffic": measured_traffic(args.workload),
                "method_flop_per_trial": method / trials if trials else None,
                "executed_fp64": executed_fp64(args.workload, kern_s)}
    roof["kernel"] = trace_kernel_name(scene)
    roof["kernel_ms"] = kern_s * 1e3

    if args.ev_capacity:
        cfg.update(event_records=st["events"])
    cfg.update(trial_steps=trials, accepted_steps=st["accepted"], records=st["records"],
               spawned=st["spawned"])
    value = st["accepted"] * args.steps / wall
    out = {"metric": "accepted RK45 ray-steps/s (FP64)", "value": value, "unit": "ray-steps/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": cfg,
           "roofline": roof, "device": device_info()}
    if args.workload == "twolayer" and not args.no_solves:
        # the metric's second part: emitter -> receiver solves/s of the
        # surrogate path and of the tracer alone, on a 1,048,576-pair batch
        del ds
        torch.cuda.empty_cache()
        try:
            r, _, _ = surrogate_run(1 << 20, 3, 1, log)
            out["solves"] = dict(workload="solve1M two-layer", **r)
        except Exception as e:  # the trace figures stand on their own
            out["solves"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, args.cpu_seconds, args.cpu_threads, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
