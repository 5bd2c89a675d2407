"""GPU event records (one per Fresnel boundary event, rt_event) through the
C ABI: element by element against the oracle's event records, and held to
the geometric, energy and ray-tree checks of tests/event_checks.py."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_1810_01780_amd import workloads as W

from .event_checks import check_geometry, check_tree
from .parity import AMP_DIR_SENS_GRID, compare, compare_events, event_pairs, sort_by_key
from .scenes import maximal, void_chord

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_01780_amd import binding
    binding.lib()
    return binding


def _announce(name, scene):
    print(f"\n[gpu-case] {name}: {scene.n_rays} rays, model {scene.limits.model}", flush=True)
    sys.stdout.flush()


CASES = {
    "fan-exact": lambda: W.point_source_fan(model=W.MODEL_EXACT),
    "twolayer-paper": lambda: W.two_layer(rays_per_source=16),
    "twolayer-exact": lambda: W.two_layer(rays_per_source=16, model=W.MODEL_EXACT),
    "curved-fresnel-bed": lambda: W.curved(rays_per_source=128, bed_kind=W.PLANE_FRESNEL),
    "paper-example-cuts": lambda: W.paper_example(n_rays=256),
    "field3d": lambda: W.field3d(rays_per_source=128),
    "void-chord-paper": lambda: void_chord(W.MODEL_PAPER),
    "void-chord-exact": lambda: void_chord(W.MODEL_EXACT),
    # every descriptor slot in use: 8 media, 16 boundaries + box + time limit
    "maximal-tables": lambda: maximal(),
    "maximal-tables-anomalies-exact": lambda: maximal(anomalies=True, model=W.MODEL_EXACT),
}


@pytest.mark.parametrize("name", list(CASES))
def test_events_match_oracle(gpu, oracle_lib, name):
    sc = CASES[name]()
    _announce("events-" + name, sc)
    ref, rst, rev = oracle_lib.trace(sc, events=True)
    got, gst, gev = gpu.trace(sc, ev_capacity=2 * len(rev["key"]) + 64)
    assert gst["events_lost"] == 0
    compare(got, ref, sc.limits.tol, label=name)
    summ = compare_events(gev, rev, got, ref, label=name)
    print(f"[gpu-case] events-{name}: {summ}", flush=True)
    stratified = not sc.anomalies and all(not any(r.axis) for r in sc.regions)
    check_geometry(sc, gev, media=stratified)
    check_tree(sc, sort_by_key(got), gst, gev, amp_tol=1e-14)


def test_events_leave_records_unchanged(gpu):
    """The instances that write events trace the same rays bit for bit."""
    sc = W.two_layer(rays_per_source=16)
    _announce("events-records-unchanged", sc)
    a, sa = gpu.trace(sc)
    b, sb, ev = gpu.trace(sc, ev_capacity=1 << 16)
    assert len(ev["key"]) == sb["events"] > 0
    a, b = sort_by_key(a), sort_by_key(b)
    for f in a:
        assert np.array_equal(a[f], b[f]), f
    for f in ("accepted", "rejected", "relocation", "events", "spawned", "records"):
        assert sa[f] == sb[f], f


def test_events_gridded(gpu, oracle_lib):
    """The gridded instance (256 x 256 x 128 nodes, tolerance 1e-6, where
    every ray is well conditioned): surface reflections with the refracted
    branch beyond the generation limit."""
    sc = W.gridded(rays_per_source=4, tol=1e-6)
    _announce("events-gridded", sc)
    ref, rst, rev = oracle_lib.trace(sc, events=True)
    got, gst, gev = gpu.trace(sc, ev_capacity=1 << 14)
    assert gst["events"] > 0 and gst["events_lost"] == 0
    compare(got, ref, sc.limits.tol, label="grid-events", amp_dir_sens=AMP_DIR_SENS_GRID)
    summ = compare_events(gev, rev, got, ref, label="grid-events",
                          amp_dir_sens=AMP_DIR_SENS_GRID)
    print(f"[gpu-case] events-gridded: {summ}", flush=True)
    check_geometry(sc, gev, media=False)
    check_tree(sc, sort_by_key(got), gst, gev, amp_tol=1e-14)


def test_event_capacity_overflow(gpu):
    """Too small an ev_capacity: RT_ERR_CAPACITY with the lost count; the
    records written are events of the full run, bit for bit."""
    sc = W.two_layer(rays_per_source=16)
    _announce("events-overflow", sc)
    full, fst, fev = gpu.trace(sc, ev_capacity=1 << 16)
    ds = gpu.DeviceScene(sc, ev_capacity=100)
    ds.launch()
    rec, st = ds.collect(check=False)
    assert st["events"] == fst["events"] > 100
    assert st["events_lost"] == st["events"] - 100
    host = gpu.rt_stats(*[st[f] for f in gpu.STAT_FIELDS])
    assert gpu.rt_collect(host, ds.capacity) == gpu.RT_ERR_CAPACITY
    assert "ev_capacity" in gpu.rt_last_error()
    ev = ds.events()
    assert len(ev["key"]) == 100
    idx = np.searchsorted(event_pairs(fev), event_pairs(ev))
    assert np.array_equal(event_pairs(fev)[idx], event_pairs(ev))
    for f in ev:
        assert np.array_equal(ev[f], fev[f][idx]), f


def test_events_across_interrupt_and_resume(gpu):
    """Events accumulate over interrupted and resumed launches and equal
    those of one uninterrupted launch bit for bit."""
    sc = W.two_layer(rays_per_source=16)
    _announce("events-resume", sc)
    base, bst, bev = gpu.trace(sc, ev_capacity=1 << 16)
    total = bst["accepted"] + bst["rejected"] + bst["relocation"]
    lim = dataclasses.replace(sc.limits, max_steps_per_launch=total // 5)
    ds = gpu.DeviceScene(dataclasses.replace(sc, limits=lim), ev_capacity=1 << 16)
    ds.launch()
    rec, st = ds.collect(check=False)
    n_int = 0
    while st["interrupted"]:
        n_int += 1
        assert n_int < 50 and st["sched_errors"] == 0
        ds.launch(resume=True)
        rec, st = ds.collect(check=False)
    assert n_int >= 2
    ev = ds.events()
    assert st["events"] == bst["events"] and st["events_lost"] == 0
    for f in ev:
        assert np.array_equal(ev[f], bev[f]), f


def test_events_full_size_sampled(gpu, oracle_lib):
    """The benchmark workload at full size (1,048,576 primaries, four
    generations, 5.8e6 events) with event records on: the records and events
    of 512 evenly spaced primaries' trees against the oracle's."""
    sc = W.two_layer()
    _announce("events-twolayer-full", sc)
    got, gst, gev = gpu.trace(sc, ev_capacity=8 << 20)
    assert gst["events_lost"] == 0 and len(gev["key"]) == gst["events"]
    roots = np.arange(0, sc.n_rays, sc.n_rays // 512, dtype=np.int64)
    ref, rst, rev = oracle_lib.trace(sc, roots=roots, events=True)
    sel = np.isin((got["key"] >> np.uint64(24)).astype(np.int64), roots)
    sub = {f: a[sel] for f, a in got.items()}
    esel = np.isin((gev["key"] >> np.uint64(24)).astype(np.int64), roots)
    esub = {f: a[esel] for f, a in gev.items()}
    compare(sub, ref, sc.limits.tol, label="events-twolayer-full")
    summ = compare_events(esub, rev, sub, ref, label="events-twolayer-full")
    print(f"[gpu-case] events-twolayer-full: {summ}", flush=True)
    assert summ["events"] == len(rev["key"]) > 1000
