"""Element-by-element comparison of GPU records with the CPU oracle.

Bars (FP64 path): positions |dr| <= 1e-9 * max(s, 1 m); path length and
travel time 1e-9 relative; amplitudes 1e-12 absolute per component; the
discrete results -- ray tree (keys), generation, parent, final status and
medium, accepted/rejected step counts -- equal.

The adaptive controller turns a continuous error estimate into an accept or
reject decision.  The GPU evaluates exp, division and square root with
different (1-ulp) rounding and contracts products into FMAs, so a trial whose
error estimate lies within ~1e-12 of the threshold could be decided the other
way; such a "flipped" ray would follow a different but equally valid step
sequence.  Analytic media show none, so by default none is allowed; a caller
that expects them passes max_flips, and flipped rays are then held to
10 * tol.

A Fresnel factor is a function of the incidence at its event, which both
sides know to rounding times the event's conditioning; the amplitude of a
record is the product of the factors of every event on its path (its own
and its ancestors' up to its casting), so the amplitude bar is 1e-12 per
event on that path (1e-12 for a ray without events).

Gridded media (trilinear, C0 gradient) move the direction at the end of a
ray by more than rounding, and a Fresnel factor moves with the incidence:
their comparisons pass amp_dir_sens = 10, which adds 10 |du| to the
amplitude bar of each record (|du| the difference of the final unit
directions); the records above 1e-12 are counted and reported.  Analytic
media get no such allowance: the per-event bar alone.
"""
import numpy as np

POS_REL = 1e-9
AMP_ABS = 1e-12
# allowance per unit direction difference for gridded media (see above)
AMP_DIR_SENS_GRID = 10.0


def events_on_path(rec):
    """Fresnel events on the path of each record: its own plus, for a
    secondary, the event ordinals of its ancestors at which each generation
    was cast (the key's low three bytes)."""
    key = rec["key"].astype(np.uint64)
    n = rec["n_ev"].astype(np.int64)
    for shift in (16, 8, 0):
        n = n + ((key >> np.uint64(shift)) & np.uint64(0xFF)).astype(np.int64)
    return n


def sort_by_key(rec):
    order = np.argsort(rec["key"], kind="stable")
    return {f: a[order] for f, a in rec.items()}


def compare(got, ref, tol, label="", max_flips=0, amp_dir_sens=0.0):
    """Returns a summary dict; raises AssertionError when a bar is missed."""
    g = sort_by_key(got)
    r = ref  # the oracle returns key order
    gk, rk = g["key"], r["key"]
    common, gi, ri = np.intersect1d(gk, rk, assume_unique=True, return_indices=True)
    n_ref = len(rk)
    missing = n_ref - len(common)
    extra = len(gk) - len(common)
    for f in ("gen", "parent"):
        assert np.array_equal(g[f][gi], r[f][ri]), f"{label}: {f} differs"
    same_steps = (g["n_acc"][gi] == r["n_acc"][ri]) & (g["n_rej"][gi] == r["n_rej"][ri])
    flips = int(np.sum(~same_steps))
    n = len(common)
    if max_flips == 0:
        assert missing == 0 and extra == 0, \
            f"{label}: ray trees differ: {missing} missing, {extra} extra of {n_ref}"
    else:
        assert missing + extra <= 4 * max_flips, \
            f"{label}: ray trees differ: {missing} missing, {extra} extra of {n_ref}"
    assert flips <= max_flips, f"{label}: {flips} of {n} rays flipped (at most {max_flips})"

    s = np.maximum(r["s"][ri], 1.0)
    dpos = np.sqrt((g["x"][gi] - r["x"][ri]) ** 2 + (g["y"][gi] - r["y"][ri]) ** 2
                   + (g["z"][gi] - r["z"][ri]) ** 2) / s
    ds = np.abs(g["s"][gi] - r["s"][ri]) / s
    dt = np.abs(g["t"][gi] - r["t"][ri]) / np.maximum(np.abs(r["t"][ri]), 1e-300)
    damp = np.max(np.stack([np.abs(g[f][gi] - r[f][ri]) for f in
                            ("as_re", "as_im", "ap_re", "ap_im")]), axis=0)
    du = np.sqrt((g["ux"][gi] - r["ux"][ri]) ** 2 + (g["uy"][gi] - r["uy"][ri]) ** 2
                 + (g["uz"][gi] - r["uz"][ri]) ** 2)
    amp_bar = AMP_ABS * np.maximum(1, events_on_path(r)[ri])
    amp_excess = damp - (amp_bar + amp_dir_sens * du)
    ok = same_steps
    plain = ok & (du <= 1e-12) & (amp_dir_sens == 0.0)
    summary = dict(rays=n_ref, common=n, flips=flips, missing=missing, extra=extra,
                   pos=float(dpos[ok].max(initial=0.0)), s=float(ds[ok].max(initial=0.0)),
                   t=float(dt[ok].max(initial=0.0)), amp=float(damp[ok].max(initial=0.0)),
                   dir=float(du[ok].max(initial=0.0)),
                   amp_excess=float(amp_excess[ok].max(initial=-1.0)),
                   amp_over_1e12=int(np.sum(ok & (damp > AMP_ABS))),
                   amp_plain=float((damp - amp_bar)[plain].max(initial=-1.0)))
    if n:
        w = int(np.argmax(np.where(ok, dpos, -1.0)))
        summary["worst_pos"] = dict(key=int(r["key"][ri][w]), gen=int(r["gen"][ri][w]),
                                    status=int(r["status"][ri][w]), n_ev=int(r["n_ev"][ri][w]),
                                    n_acc=int(r["n_acc"][ri][w]), s=float(r["s"][ri][w]),
                                    z=float(r["z"][ri][w]), dpos=float(dpos[w]))
    assert np.array_equal(g["status"][gi][ok], r["status"][ri][ok]), f"{label}: status differs"
    assert np.array_equal(g["region"][gi][ok], r["region"][ri][ok]), f"{label}: region differs"
    assert summary["pos"] <= POS_REL, f"{label}: position {summary}"
    assert summary["s"] <= POS_REL, f"{label}: path length {summary}"
    assert summary["t"] <= POS_REL, f"{label}: travel time {summary}"
    assert summary["amp_excess"] <= 0.0, f"{label}: amplitude {summary}"
    assert summary["amp_plain"] <= 0.0, f"{label}: amplitude {summary}"
    if flips:
        bad = ~ok
        loose = 10 * tol
        assert np.all(dpos[bad] <= max(loose, POS_REL)), f"{label}: flipped rays {summary}"
    return summary


def perturbed(scene, eps=1e-15):
    """Copy of a scene with every launch direction scaled by (1 + O(eps)) per
    component: an input change at the rounding level."""
    import dataclasses
    pat = np.array([1.0, -1.0, 0.5])
    return dataclasses.replace(scene, dirs=scene.dirs * (1.0 + eps * pat))


def compare_conditioned(got, ref, ref_pert, tol, label="", ill_factor=10.0, ill_cap=1e-3,
                        amp_dir_sens=0.0, amp_cap=1e-2):
    """Parity where the method itself is ill-conditioned for some rays.

    The oracle run on the same rays with launch directions changed by 1e-15
    ('ref_pert') shows each record's own sensitivity.  Rays whose oracle
    result is stable under that perturbation -- same step counts, positions
    within 1e-12 relative, amplitudes within a tenth of their per-event bar
    -- must meet the standard bars (compare): the GPU's own rounding
    differences act like a perturbation some 100 times larger, which such a
    ray turns into at most ~1e-10.  For the others the GPU deviation
    from the oracle must be of the size of the oracle's own deviation under
    the perturbation: median within ill_factor times the median spread (or
    the standard bar, whichever is larger), and every ray within ill_cap
    relative in position and amp_cap in amplitude (the amplitude of such a
    ray follows its incidence at each event, which moves with the
    trajectory: the oracle's own spread reaches a few 1e-3).  This is how a
    trilinear
    (C0-gradient) field at tight tolerance, where the step controller
    amplifies rounding, and rays that graze a boundary many times, whose
    Fresnel factors are steep in the incidence, are judged.  The ray tree
    and final statuses must agree for every ray.
    """
    g = sort_by_key(got)
    r, p = ref, ref_pert
    assert np.array_equal(r["key"], p["key"]), f"{label}: perturbed oracle changed the tree"
    assert np.array_equal(g["key"], r["key"]), f"{label}: ray trees differ"
    assert np.array_equal(g["status"], r["status"]), f"{label}: statuses differ"
    s = np.maximum(r["s"], 1.0)

    def dpos(a, b):
        return np.maximum(np.sqrt((a["x"] - b["x"]) ** 2 + (a["y"] - b["y"]) ** 2
                                  + (a["z"] - b["z"]) ** 2) / s, np.abs(a["s"] - b["s"]) / s)

    def damp(a, b):
        return np.max(np.stack([np.abs(a[f] - b[f]) for f in
                                ("as_re", "as_im", "ap_re", "ap_im")]), axis=0)

    amp_bar = AMP_ABS * np.maximum(1, events_on_path(r))
    spread, aspread = dpos(p, r), damp(p, r)
    stable = ((spread <= 1e-12) & (aspread <= 0.1 * amp_bar)
              & (p["n_acc"] == r["n_acc"]) & (p["n_rej"] == r["n_rej"]))
    well = {f: a[stable] for f, a in g.items()}
    well_ref = {f: a[stable] for f, a in r.items()}
    summ = compare(well, well_ref, tol, label=label + "/well-conditioned",
                   amp_dir_sens=amp_dir_sens)
    dg, ag = dpos(g, r), damp(g, r)
    ill = ~stable
    summ.update(well_conditioned=int(stable.sum()), ill_conditioned=int(ill.sum()),
                ill_max_rel=float(dg[ill].max(initial=0.0)),
                ill_max_spread=float(spread[ill].max(initial=0.0)),
                ill_max_amp=float(ag[ill].max(initial=0.0)),
                ill_max_amp_spread=float(aspread[ill].max(initial=0.0)))
    if ill.any():
        summ.update(ill_median_rel=float(np.median(dg[ill])),
                    ill_median_spread=float(np.median(spread[ill])),
                    ill_median_amp=float(np.median(ag[ill])),
                    ill_median_amp_spread=float(np.median(aspread[ill])))
        assert summ["ill_max_rel"] <= ill_cap, f"{label}: ill-conditioned ray beyond cap {summ}"
        assert summ["ill_max_amp"] <= amp_cap, f"{label}: ill-conditioned amplitude {summ}"
        assert summ["ill_median_rel"] <= ill_factor * max(summ["ill_median_spread"], POS_REL), \
            f"{label}: GPU deviates more than the oracle's own sensitivity {summ}"
        assert summ["ill_median_amp"] <= ill_factor * max(summ["ill_median_amp_spread"],
                                                          AMP_ABS), \
            f"{label}: GPU amplitudes deviate more than the oracle's own sensitivity {summ}"
    return summ


# largest |grad n| of the analytic media used in the tests (firn profile
# 0.43 / 75 m at the surface), to turn a position tolerance into one on n
GRAD_N_MAX = 6e-3


def event_pairs(ev):
    return ev["key"].astype(np.uint64) * np.uint64(256) + ev["ordinal"].astype(np.uint64)


def compare_events(got_ev, ref_ev, got_rec, ref_rec, label="", amp_dir_sens=0.0):
    """Event records of the GPU against the oracle's, matched by (key,
    ordinal), for the rays whose step counts agree (see compare): the same
    events exist; boundary, outcome, generation and media are equal; the
    crossing point, path length and travel time meet the record bars; the
    incidence direction and cosine, the indices (through the position) and
    the incident amplitudes and coefficients (through the direction) follow
    from those."""
    g = sort_by_key(got_rec)
    r = ref_rec
    common, gi, ri = np.intersect1d(g["key"], r["key"], assume_unique=True, return_indices=True)
    same = (g["n_acc"][gi] == r["n_acc"][ri]) & (g["n_rej"][gi] == r["n_rej"][ri])
    good = set(common[same].tolist())
    gsel = np.array([int(k) in good for k in got_ev["key"]], dtype=bool)
    rsel = np.array([int(k) in good for k in ref_ev["key"]], dtype=bool)
    gp, rp = event_pairs(got_ev)[gsel], event_pairs(ref_ev)[rsel]
    assert np.array_equal(gp, rp), f"{label}: event sets differ ({len(gp)} vs {len(rp)})"
    G = {f: a[gsel] for f, a in got_ev.items()}
    R = {f: a[rsel] for f, a in ref_ev.items()}
    for f in ("boundary", "outcome", "gen", "region_in", "region_out"):
        assert np.array_equal(G[f], R[f]), f"{label}: event {f} differs"
    s = np.maximum(R["s"], 1.0)
    dpos = np.linalg.norm(G["pos"] - R["pos"], axis=1) / s
    ds = np.abs(G["s"] - R["s"]) / s
    dt = np.abs(G["t"] - R["t"]) / np.maximum(np.abs(R["t"]), 1e-300)
    du = np.linalg.norm(G["dir"] - R["dir"], axis=1)
    dn = np.maximum(np.abs(G["n1"] - R["n1"]), np.abs(G["n2"] - R["n2"]))
    dci = np.abs(G["cos_i"] - R["cos_i"])
    damp = np.max(np.abs(G["amp"] - R["amp"]), axis=1)
    dcoef = np.max(np.abs(G["coef"] - R["coef"]), axis=1)
    summary = dict(events=len(rp), of=len(ref_ev["key"]), pos=float(dpos.max(initial=0)),
                   s=float(ds.max(initial=0)), t=float(dt.max(initial=0)),
                   dir=float(du.max(initial=0)), n=float(dn.max(initial=0)),
                   cos_i=float(dci.max(initial=0)), amp=float(damp.max(initial=0)),
                   coef=float(dcoef.max(initial=0)))
    assert summary["pos"] <= POS_REL and summary["s"] <= POS_REL and summary["t"] <= POS_REL, \
        f"{label}: event position / path / time {summary}"
    assert np.all(dn <= GRAD_N_MAX * POS_REL * s + 1e-14), f"{label}: event indices {summary}"
    # the normal turns by |dpos| / R between two nearby points of a surface of
    # curvature radius R (25 m for the smallest, the spherical void)
    assert np.all(dci <= du + dpos * s / 25.0 + 1e-14), f"{label}: incidence cosine {summary}"
    # the incident amplitude is the product of the Fresnel factors of the
    # events before this one on the ray's path: 1e-12 per such event
    prior = {"key": R["key"], "n_ev": R["ordinal"] - 1}
    bar = AMP_ABS * np.maximum(1, events_on_path(prior)) + amp_dir_sens * du
    assert np.all(damp <= bar), f"{label}: incident amplitudes {summary}"
    bar = AMP_ABS + amp_dir_sens * du
    # Fresnel coefficients are steep functions of the incidence near the
    # critical angle: their bar adds how far the oracle's coefficients move
    # between the two sides' inputs (n1, n2, cos_i)
    sens = np.array([_coef_shift(G["n1"][i], G["n2"][i], G["cos_i"][i],
                                 R["n1"][i], R["n2"][i], R["cos_i"][i])
                     for i in range(len(rp))])
    assert np.all(dcoef <= bar + 2.0 * sens), f"{label}: coefficients {summary}"
    return summary


def _coef_shift(n1a, n2a, cia, n1b, n2b, cib):
    import oracle
    fa = oracle.fresnel(float(n1a), float(n2a), float(cia))[:4]
    fb = oracle.fresnel(float(n1b), float(n2b), float(cib))[:4]
    return max(max(abs(x.real - y.real), abs(x.imag - y.imag)) for x, y in zip(fa, fb))
