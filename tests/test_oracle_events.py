"""Pins of the oracle's Fresnel event records (section 2, boundary
paragraph: a ray passing a boundary is reflected and casts a refracted
secondary from the intersection point, amplitudes by Fresnel's equations).

The fan of 1,024 rays from 200 m under a flat surface fixes every event by
Snell's law in the stratified medium: the invariant I = n(z_s) sin(theta_0)
of a ray decides whether it refracts out (I < n_air = 1), is totally
reflected (1 <= I < n(0) = 1.35) or turns before the surface (I >= 1.35),
and the angle of incidence at the surface follows from n(0) sin(theta_i) = I.
The other scenes are held to the geometric, energy and bookkeeping
invariants of tests/event_checks.py."""
import numpy as np
import pytest

from paper_1810_01780_amd import workloads as W

from .event_checks import GEN, SPAWNED, TIR, check_geometry, check_tree
from .scenes import void_chord

N_SURF = 1.78 - 0.43
W_C0 = 299792458.0


def _fan(model):
    return W.point_source_fan(model=model)


@pytest.mark.parametrize("model", [W.MODEL_EXACT, W.MODEL_PAPER])
def test_fan_events_follow_snell(oracle_lib, model):
    sc = _fan(model)
    rec, st, ev = oracle_lib.trace(sc, events=True)
    th = (np.arange(1024) + 0.5) * np.pi / 1024
    inv = (1.78 - 0.43 * np.exp(-200.0 / 75.0)) * np.sin(th)
    up = th < np.pi / 2  # rays launched downward bend further down
    want_out = np.nonzero(up & (inv < 1.0))[0]
    want_tir = np.nonzero(up & (inv >= 1.0) & (inv < N_SURF))[0]
    assert len(want_out) == 198 and len(want_tir) == 89
    roots = (ev["key"] >> np.uint64(24)).astype(np.int64)
    assert np.all(ev["ordinal"] == 1) and np.all(ev["gen"] == 0) and np.all(ev["boundary"] == 0)
    # eq. 1 keeps the invariant to the tolerance; eq. 2 drifts by up to a few
    # 1e-3 at h_max = 10 m (first order in the step), so there only rays
    # farther than that from a threshold are held to their class
    margin = 1e-9 if model == W.MODEL_EXACT else 1e-2
    sure = (np.abs(inv - 1.0) > margin) & (np.abs(inv - N_SURF) > margin)
    got_out = set(roots[ev["outcome"] == SPAWNED].tolist())
    got_tir = set(roots[ev["outcome"] == TIR].tolist())
    for name, got, want in (("out", got_out, want_out), ("tir", got_tir, want_tir)):
        assert {i for i in got if sure[i]} == {i for i in want.tolist() if sure[i]}, name
    assert all(i in got_out | got_tir for i in range(1024) if up[i] and inv[i] < N_SURF - margin)
    if model == W.MODEL_EXACT:
        assert got_out == set(want_out.tolist()) and got_tir == set(want_tir.tolist())
        assert len(ev["key"]) == st["events"] == 287
    # on the surface, arriving from the firn, incident amplitudes of a primary
    assert np.max(np.abs(ev["pos"][:, 2])) <= 1e-10
    assert np.allclose(ev["pos"][:, 1], 0.0, atol=1e-12)
    assert np.max(np.abs(ev["n1"] - N_SURF)) <= 1e-15 and np.all(ev["n2"] == 1.0)
    assert np.all(ev["amp"] == np.array([1.0, 0.0, 1.0, 0.0]))
    # Snell's invariant at the surface: exact to the integration tolerance
    # for eq. 1; eq. 2 drifts with the step length (first order in h)
    sin_i = np.sqrt(1.0 - ev["cos_i"] ** 2)
    drift = np.abs(N_SURF * sin_i - inv[roots])
    assert drift.max() <= (1e-9 if model == W.MODEL_EXACT else 1e-2)
    # the path reaches the surface no sooner than the straight chord
    chord = np.hypot(ev["pos"][:, 0], 200.0)
    assert np.all(ev["s"] >= chord - 1e-9)
    assert np.all(ev["t"] * W_C0 > ev["s"] * N_SURF) and np.all(ev["t"] * W_C0 < ev["s"] * 1.78)
    check_geometry(sc, ev)
    check_tree(sc, rec, st, ev)


@pytest.mark.parametrize("model", [W.MODEL_PAPER, W.MODEL_EXACT])
def test_two_layer_events(oracle_lib, model):
    sc = W.two_layer(rays_per_source=8, model=model)
    rec, st, ev = oracle_lib.trace(sc, events=True)
    assert st["spawned"] > 0 and st["max_gen"] >= 2
    assert set(np.unique(ev["boundary"])) == {0, 1}
    check_geometry(sc, ev)
    check_tree(sc, rec, st, ev)


@pytest.mark.parametrize("bed", [W.PLANE_ABSORB, W.PLANE_FRESNEL])
def test_curved_events(oracle_lib, bed):
    sc = W.curved(rays_per_source=64, bed_kind=bed)
    rec, st, ev = oracle_lib.trace(sc, events=True)
    assert st["suppressed_amp"] > 0 or st["spawned"] > 0
    hit = set(np.unique(ev["boundary"]))
    assert 1 in hit and (2 in hit) == (bed == W.PLANE_FRESNEL)
    check_geometry(sc, ev)
    check_tree(sc, rec, st, ev)


def test_events_leave_records_unchanged(oracle_lib):
    sc = W.two_layer(rays_per_source=4)
    a, sa = oracle_lib.trace(sc)
    b, sb, ev = oracle_lib.trace(sc, events=True)
    assert sa == sb
    for f in a:
        assert np.array_equal(a[f], b[f]), f


def test_small_event_capacity_is_retried(oracle_lib):
    sc = W.two_layer(rays_per_source=4)
    rec, st, ev = oracle_lib.trace(sc, events=True)
    rec2, st2, ev2 = oracle_lib._trace_events(sc, None, None, None, ev_capacity=3)
    assert len(ev2["key"]) == st["events"] > 3
    for f in ev:
        assert np.array_equal(ev[f], ev2[f]), f


def test_planted_mistake_is_caught(oracle_lib):
    """A dropped factor in the amplitude chain or an event off its boundary
    fails the checks."""
    sc = W.two_layer(rays_per_source=8)
    rec, st, ev = oracle_lib.trace(sc, events=True)
    bad = {f: a.copy() for f, a in ev.items()}
    j = int(np.nonzero(bad["ordinal"] == 2)[0][0])
    bad["amp"][j, 0] *= -1.0
    with pytest.raises(AssertionError):
        check_tree(sc, rec, st, bad)
    bad = {f: a.copy() for f, a in ev.items()}
    bad["pos"][0, 2] += 1e-6
    with pytest.raises(AssertionError):
        check_geometry(sc, bad)


@pytest.mark.parametrize("model", [W.MODEL_PAPER, W.MODEL_EXACT])
def test_short_chord_through_a_void(oracle_lib, model):
    """Closed form in constant media: the refracted secondary crosses the
    void along a chord of 2 R cos(theta_t) = 5.3 m, shorter than its step,
    and meets the wall again where the straight line leaves the sphere; it
    keeps bouncing inside along chords of the same length and incidence (it
    must not stall on the wall it was cast from)."""
    R, c = 10.0, np.array([0.0, 0.0, 100.0])
    sc = void_chord(model)
    rec, st, ev = oracle_lib.trace(sc, events=True)
    th = np.radians(40.0)
    p1 = np.array([R * np.sin(th), 0.0, 100.0 - R * np.cos(th)])
    prim = ev["gen"] == 0
    assert np.linalg.norm(ev["pos"][prim][0] - p1) <= 1e-9
    assert abs(ev["cos_i"][prim][0] - np.cos(th)) <= 1e-12
    assert ev["outcome"][prim][0] == SPAWNED
    # Snell's law in vector form at p1 (normal pointing back into the ice)
    u = np.array([0.0, 0.0, 1.0])
    nin = (p1 - c) / R
    ci = -u @ nin
    eta = 1.5 / 1.0
    ct = np.sqrt(1.0 - eta ** 2 * (1.0 - ci ** 2))
    ut = eta * u + (eta * ci - ct) * nin
    chord = 2.0 * R * ct
    assert 5.0 < chord < 6.0
    child = ev["gen"] == 1
    pos, s, t = ev["pos"][child], ev["s"][child], ev["t"][child]
    assert len(pos) >= 2
    assert np.linalg.norm(pos[0] - (p1 + chord * ut)) <= 1e-9
    # the search stops within 1e-10 m of the wall: the normal there turns by
    # up to 1e-11 per bounce
    assert np.all(np.abs(ev["cos_i"][child] - ct) <= 1e-10)
    assert np.all(np.abs(np.linalg.norm(np.diff(pos, axis=0), axis=1) - chord) <= 1e-9)
    assert abs(s[0] - ev["s"][prim][0] - chord) <= 1e-9
    assert np.all(np.abs(np.diff(s) - chord) <= 1e-9)
    assert np.all(np.abs(np.diff(t) - chord / W_C0) <= 1e-17)
    # inside the void the secondary is beyond the generation limit: no more rays
    assert np.all(ev["outcome"][child] == GEN) and st["records"] == 2
    assert np.all(rec["status"] == oracle_lib.ST_PATH)
    check_geometry(sc, ev)
    check_tree(sc, rec, st, ev)


@pytest.mark.parametrize("anomalies", [False, True])
def test_full_descriptor_tables(oracle_lib, anomalies):
    """8 media, 16 boundaries, a box, a travel-time and an amplitude limit
    (and 8 anomalies): every event valid and tied to the records, and every
    kind of end occurs."""
    from .scenes import maximal
    sc = maximal(anomalies=anomalies)
    rec, st, ev = oracle_lib.trace(sc, events=True)
    ends = set(np.unique(rec["status"]).tolist())
    assert {oracle_lib.ST_BOX, oracle_lib.ST_TIME, oracle_lib.ST_AMP, oracle_lib.ST_ABSORB} <= ends
    assert st["max_gen"] == 3 and st["suppressed_gen"] > 0
    check_geometry(sc, ev, media=not anomalies)
    check_tree(sc, rec, st, ev)
