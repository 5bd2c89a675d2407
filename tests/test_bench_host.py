"""Host-side logic of bench.py (no GPU): the FLOP model per trial step, the
traffic figure's validity rule, and the one-GPU contract."""
import os
import subprocess
import sys

import pytest

import bench
from paper_1810_01780_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_flop_model_per_trial():
    # the method's step: ~750 FLOP (paper model) including ~15 of plane
    # tests, here replaced by this scene's two planes (6 each) and s += h
    sc = W.two_layer(rays_per_source=1)
    assert not bench.is_general(sc)
    assert [bench.flop_per_trial(sc, r) for r in range(3)] == [748, 748, 748]
    # a sphere and a paraboloid next to the surface plane
    cv = W.curved(rays_per_source=1)
    assert bench.flop_per_trial(cv, 1) == 750 - 15 + 6 + 17 + 8 + 1
    # non-stratified media: axis projection and 294 per anomaly of the region
    f3 = W.field3d(rays_per_source=1)
    assert bench.is_general(f3)
    assert bench.flop_per_trial(f3, 0) == 750 - 15 + 7 + 30
    assert bench.flop_per_trial(f3, 1) == 750 - 15 + 7 + 30 + 2 * 294
    # exact model: ~830
    ex = W.two_layer(rays_per_source=1, model=W.MODEL_EXACT)
    assert bench.flop_per_trial(ex, 1) == 830 - 15 + 13


def test_trial_flops_weights_records_by_region():
    import numpy as np
    sc = W.field3d(rays_per_source=1)
    rec = {"n_acc": np.array([10, 20]), "n_rej": np.array([0, 5]), "region": np.array([0, 1])}
    want = 10 * bench.flop_per_trial(sc, 0) + 25 * bench.flop_per_trial(sc, 1)
    assert bench.trial_flops(sc, rec, 35) == pytest.approx(want)
    # event-search trials (beyond the records' own counts) at the mean rate
    assert bench.trial_flops(sc, rec, 70) == pytest.approx(2 * want)


def test_traffic_only_for_the_measured_sources(monkeypatch):
    d = bench.kernel_digest()
    monkeypatch.setattr(bench, "TRAFFIC", {"twolayer": (100.0, 50.0, d),
                                           "grid256": (1.0, 2.0, "0" * 64)})
    assert bench.measured_traffic("twolayer") == 150.0
    assert bench.measured_traffic("grid256") is None   # sources changed since
    assert bench.measured_traffic("curved") is None    # never measured


def test_executed_fp64_from_counters(monkeypatch):
    """Executed FP64 counts every lane of each FP64 instruction, FMA as two
    operations, and is reported only for the measured sources."""
    d = bench.kernel_digest()
    monkeypatch.setattr(bench, "EXEC_FP64", {"twolayer": (10.0, 4.0, 2.0, 1.0, 64, d),
                                             "grid256": (1.0, 1.0, 1.0, 1.0, 1, "f" * 64)})
    e = bench.executed_fp64("twolayer", 2.0)
    assert e["flop_per_trial"] == pytest.approx(64 * (20 + 4 + 2 + 1) / 64)
    assert e["tflops"] == pytest.approx(64 * 27 / 2.0 / 1e12)
    assert e["frac"] == pytest.approx(e["tflops"] / bench.PEAK_FP64_VECTOR_TFLOPS)
    assert bench.executed_fp64("grid256", 1.0) is None
    assert bench.executed_fp64("curved", 1.0) is None


def test_counter_constants_belong_to_the_committed_sources():
    """The traffic, L2 and FP64 counts in bench.py were measured on the trace
    sources as committed (a kernel change must re-measure them)."""
    d = bench.kernel_digest()
    for table, at in ((bench.TRAFFIC, 2), (bench.L2_HIT, 2), (bench.EXEC_FP64, 5)):
        for w, t in table.items():
            assert t[at] == d, w


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_digest_follows_code_not_comments():
    src = {f: open(os.path.join(ROOT, "paper_1810_01780_amd", "csrc", f)).read()
           for f in bench.TRACE_SOURCES}
    d = bench.kernel_digest(src)
    assert d == bench.kernel_digest()
    f0 = bench.TRACE_SOURCES[0]
    commented = dict(src, **{f0: "// a note\n" + src[f0].replace("\n", "\n  ", 3) + "/* end */\n"})
    assert bench.kernel_digest(commented) == d
    changed = dict(src, **{f0: src[f0] + "\nint x_ = 1;\n"})
    assert bench.kernel_digest(changed) != d


def test_kernel_named_after_the_scene():
    # the roofline names the kernel that rocprofv3 lists for the workload
    names = {w: bench.trace_kernel_name(bench.make_scene(w)[0])
             for w in ("twolayer", "grid256", "curved", "field3d", "fan1024")}
    assert names == {"twolayer": "trace_strat_kernel", "grid256": "trace_general_kernel",
                     "curved": "trace_strat_kernel", "field3d": "trace_general_kernel",
                     "fan1024": "trace_strat_kernel"}
