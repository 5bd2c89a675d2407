"""Checks on Fresnel event records that hold by construction of the method
(section 2, boundary paragraph), written from the scene description alone:
where a boundary is, which media meet there, energy conservation of the
Fresnel coefficients, and the ray-tree and amplitude bookkeeping that ties
the events to the final records.  They apply to the oracle's events and to
the GPU's alike."""
import numpy as np

from paper_1810_01780_amd import workloads as W

C0 = 299792458.0
# event outcomes (RT_EV_* of the C ABI, EV_* of the oracle)
SPAWNED, TIR, GEN, AMP = 0, 1, 2, 3


def boundary_g(plane, p):
    """Signed distance-like function of a boundary (positive on region_pos)."""
    pt = np.asarray(plane.point, np.float64)
    if plane.shape == W.SHAPE_SPHERE:
        return np.linalg.norm(p - pt, axis=-1) - plane.param
    if plane.shape == W.SHAPE_PARABOLOID:
        rho2 = (p[..., 0] - pt[0]) ** 2 + (p[..., 1] - pt[1]) ** 2
        return p[..., 2] - pt[2] - plane.param * rho2
    nrm = np.asarray(plane.normal, np.float64)
    nrm = nrm / np.linalg.norm(nrm)
    return (p - pt) @ nrm


def boundary_normal(plane, p):
    """Unit normal (gradient direction of boundary_g) at p."""
    pt = np.asarray(plane.point, np.float64)
    if plane.shape == W.SHAPE_SPHERE:
        d = p - pt
    elif plane.shape == W.SHAPE_PARABOLOID:
        d = np.stack([-2 * plane.param * (p[..., 0] - pt[0]),
                      -2 * plane.param * (p[..., 1] - pt[1]), np.ones(p.shape[:-1])], axis=-1)
    else:
        d = np.broadcast_to(np.asarray(plane.normal, np.float64), p.shape)
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def region_n(region, p):
    """Index of an analytic region stratified in depth (no anomalies)."""
    z = p[..., 2]
    n = region.a + region.b * z
    if region.dn != 0.0:
        n = n - region.dn * np.exp(-z / region.z0)
    return n


def cmul(a_re, a_im, b_re, b_im):
    return a_re * b_re - a_im * b_im, a_re * b_im + a_im * b_re


def check_geometry(scene, ev, g_tol=1e-9, cos_tol=1e-12, n_tol=1e-12, media=True):
    """Each event lies on its boundary, cos_i is the incidence cosine of the
    recorded direction, n1 / n2 are the indices of the media on the incident
    and the far side (stratified scenes), and the Fresnel coefficients
    conserve energy: |r|^2 + (n2 cos_t)/(n1 cos_i) |t|^2 = 1 per polarisation,
    |r| = 1 and t = 0 under total internal reflection."""
    m = len(ev["key"])
    assert m > 0
    for j in range(m):
        pl = scene.planes[ev["boundary"][j]]
        p = ev["pos"][j]
        assert abs(boundary_g(pl, p[None])[0]) <= g_tol, (j, boundary_g(pl, p[None]))
        nb = boundary_normal(pl, p[None])[0]
        u = ev["dir"][j]
        assert abs(np.linalg.norm(u) - 1.0) <= 1e-14
        un = float(u @ nb)
        assert abs(ev["cos_i"][j] - abs(un)) <= cos_tol, (j, ev["cos_i"][j], un)
        # moving against the normal: the ray passes into region_neg
        r_out = pl.region_neg if un < 0 else pl.region_pos
        assert ev["region_out"][j] == r_out, j
        if media:
            n1 = region_n(scene.regions[ev["region_in"][j]], p)
            n2 = region_n(scene.regions[r_out], p)
            assert abs(ev["n1"][j] - n1) <= n_tol and abs(ev["n2"][j] - n2) <= n_tol, \
                (j, ev["n1"][j], n1, ev["n2"][j], n2)
    ci, n1, n2, c = ev["cos_i"], ev["n1"], ev["n2"], ev["coef"]
    st2 = (n1 / n2) ** 2 * (1.0 - ci ** 2)
    tir = st2 > 1.0
    assert np.array_equal(tir, ev["outcome"] == TIR), "TIR outcome and Snell disagree"
    r2s = c[:, 0] ** 2 + c[:, 1] ** 2
    r2p = c[:, 2] ** 2 + c[:, 3] ** 2
    t2s = c[:, 4] ** 2 + c[:, 5] ** 2
    t2p = c[:, 6] ** 2 + c[:, 7] ** 2
    ok = ~tir & (ci > 1e-6)
    ct = np.sqrt(np.maximum(0.0, 1.0 - st2[ok]))
    k = n2[ok] * ct / (n1[ok] * ci[ok])
    assert np.max(np.abs(r2s[ok] + k * t2s[ok] - 1.0), initial=0.0) <= 1e-12
    assert np.max(np.abs(r2p[ok] + k * t2p[ok] - 1.0), initial=0.0) <= 1e-12
    assert np.max(np.abs(r2s[tir] - 1.0), initial=0.0) <= 1e-12
    assert np.max(np.abs(r2p[tir] - 1.0), initial=0.0) <= 1e-12
    assert np.all(t2s[tir] == 0.0) and np.all(t2p[tir] == 0.0)


def check_tree(scene, rec, stats, ev, amp_tol=1e-15):
    """The events of a ray carry ordinals 1..n_ev of its final record, in
    increasing path length and travel time; a SPAWNED event has exactly one
    child record (its key extends the parent's by the ordinal); the
    incident amplitudes chain through the reflection coefficients from the
    launch amplitude (1, or the parent's incident amplitude times t) to the
    final record's amplitude; outcome counts equal the statistics."""
    keys = rec["key"]
    idx = {int(k): i for i, k in enumerate(keys)}
    assert len(idx) == len(keys)
    oc = ev["outcome"]
    assert len(ev["key"]) == stats["events"]
    assert int(np.sum(oc == SPAWNED)) == stats["spawned"]
    assert int(np.sum(oc == GEN)) == stats["suppressed_gen"]
    assert int(np.sum(oc == AMP)) == stats["suppressed_amp"]
    # events grouped per key, in ordinal order (the caller sorts by key, ordinal)
    start = {}
    for j, k in enumerate(ev["key"]):
        start.setdefault(int(k), []).append(j)
    for k, js in start.items():
        i = idx[k]
        assert [int(ev["ordinal"][j]) for j in js] == list(range(1, rec["n_ev"][i] + 1)), k
        assert np.all(ev["gen"][js] == rec["gen"][i])
        # the reflected ray stays in its medium: the last event's is the final one
        assert np.all(ev["region_in"][js] == rec["region"][i])
        assert np.all(np.diff(ev["s"][js]) >= 0) and np.all(np.diff(ev["t"][js]) >= 0)
        assert ev["s"][js[-1]] <= rec["s"][i] and ev["t"][js[-1]] <= rec["t"][i]
    assert all(rec["n_ev"][idx[k]] == 0 for k in idx if k not in start)
    # launch amplitude of every ray
    launch = {}
    children = set()
    for j in np.nonzero(oc == SPAWNED)[0]:
        g = int(ev["gen"][j])
        ck = int(ev["key"][j]) | (int(ev["ordinal"][j]) << (8 * (2 - g)))
        assert ck in idx, f"child {ck:#x} of an event has no record"
        i = idx[ck]
        assert int(rec["parent"][i]) == int(ev["key"][j]) and rec["gen"][i] == g + 1
        assert rec["region"][i] == ev["region_out"][j]
        a = ev["amp"][j]
        c = ev["coef"][j]
        launch[ck] = cmul(a[0], a[1], c[4], c[5]) + cmul(a[2], a[3], c[6], c[7])
        children.add(ck)
    assert children == {int(k) for k, g in zip(keys, rec["gen"]) if g > 0}
    for k, i in idx.items():
        a = launch.get(k, (1.0, 0.0, 1.0, 0.0))
        for j in start.get(k, []):
            assert np.max(np.abs(ev["amp"][j] - np.array(a))) <= amp_tol, (k, j)
            c = ev["coef"][j]
            a = cmul(a[0], a[1], c[0], c[1]) + cmul(a[2], a[3], c[2], c[3])
        fin = np.array([rec["as_re"][i], rec["as_im"][i], rec["ap_re"][i], rec["ap_im"][i]])
        assert np.max(np.abs(fin - np.array(a))) <= amp_tol, (k, fin, a)
