"""Pins of the oracle's curved boundaries (spheres, paraboloids): straight
lines in constant media meet them where elementary geometry says, reflection
at a sphere keeps a ray's angular momentum about the centre, a paraboloid's
reflected rays pass through its focus, and the reflected and refracted
directions at the hit point follow the law of reflection and vector Snell
with the local normal."""
import math

import numpy as np
import pytest

from paper_1810_01780_amd import workloads as W


def scene(regions, surfaces, src, dirs, s_max=1000.0, G=1, model=W.MODEL_EXACT, tol=1e-10):
    src = np.atleast_2d(np.asarray(src, float))
    dirs = np.atleast_2d(np.asarray(dirs, float))
    return W.Scene(name="curved", regions=regions, planes=surfaces, sources=src,
                   ray_src=np.zeros(len(dirs), np.int32), dirs=dirs,
                   limits=W.Limits(tol=tol, h_min=1e-3, h_max=10.0, s_max=s_max,
                                   max_generations=G, model=model))


def const(n, z_top=-np.inf, z_bot=np.inf):
    return W.Region(a=n, z_top=z_top, z_bot=z_bot)


def sphere(c, R, pos, neg, kind=W.PLANE_FRESNEL):
    return W.Plane(point=tuple(c), normal=(0.0, 0.0, 1.0), region_pos=pos, region_neg=neg,
                   kind=kind, shape=W.SHAPE_SPHERE, param=R)


def unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


@pytest.mark.parametrize("model", [W.MODEL_PAPER, W.MODEL_EXACT])
def test_line_meets_sphere(oracle_lib, model):
    c, R = np.array([0.0, 0.0, 60.0]), 20.0
    o = np.array([1.0, 2.0, 50.0])
    rng = np.random.default_rng(0)
    u = unit(rng.standard_normal((16, 3)))
    sc = scene([const(1.3)], [sphere(c, R, 0, 0, kind=W.PLANE_ABSORB)], o, u, model=model)
    rec, st = oracle_lib.trace(sc)
    assert np.all(rec["status"] == 5)  # absorbed on the sphere
    d = o - c
    b = u @ d
    t = -b + np.sqrt(b * b - (d @ d - R * R))
    order = (rec["key"] >> np.uint64(24)).astype(int)
    hit = o + t[order, None] * u[order]
    P = np.stack([rec["x"], rec["y"], rec["z"]], 1)
    assert np.abs(P - hit).max() <= 1e-9 * R
    assert np.allclose(rec["s"], t[order], rtol=1e-12, atol=1e-10)
    assert np.allclose(rec["t"], 1.3 * t[order] / 299792458.0, rtol=1e-12)


def test_reflection_in_sphere_keeps_angular_momentum(oracle_lib):
    """Inside a reflecting sphere (constant medium) a ray runs along chords
    of equal length 2 sqrt(R^2 - L^2), L = |(r - c) x u| being conserved."""
    c, R = np.array([0.0, 0.0, 200.0]), 30.0
    o = c + np.array([0.0, 12.0, 0.0])
    u = unit([[1.0, 0.3, 0.2]])
    L0 = np.linalg.norm(np.cross(o - c, u[0]))
    sc = scene([const(1.0), const(1.5)], [sphere(c, R, 0, 1)], o, u, s_max=700.0, G=1)
    rec, st = oracle_lib.trace(sc)
    assert st["records"] == 1 and rec["status"][0] == 1
    r = np.array([rec["x"][0], rec["y"][0], rec["z"][0]])
    uf = np.array([rec["ux"][0], rec["uy"][0], rec["uz"][0]])
    assert np.linalg.norm(r - c) <= R + 1e-9
    assert np.linalg.norm(np.cross(r - c, uf)) == pytest.approx(L0, abs=1e-8)
    # events: first chord from o, then chords of length 2 sqrt(R^2 - L^2)
    d = o - c
    b = u[0] @ d
    t1 = -b + math.sqrt(b * b - (d @ d - R * R))
    chord = 2 * math.sqrt(R * R - L0 * L0)
    assert rec["n_ev"][0] == 1 + int((700.0 - t1) // chord)


def test_paraboloid_reflections_pass_through_the_focus(oracle_lib):
    """Rays parallel to the axis of z = z_v + k rho^2 reflect along lines
    through the focus (0, 0, z_v + 1/(4k))."""
    zv, k = 100.0, 0.01
    F = np.array([0.0, 0.0, zv + 1.0 / (4 * k)])
    par = W.Plane(point=(0.0, 0.0, zv), normal=(0.0, 0.0, 1.0), region_pos=0, region_neg=0,
                  shape=W.SHAPE_PARABOLOID, param=k)
    offs = np.array([[5.0, 0.0], [0.0, 10.0], [14.0, -14.0], [-30.0, 4.0]])
    src = np.column_stack([offs, np.zeros(len(offs))])
    for j in range(len(offs)):
        sc = scene([const(1.0)], [par], src[j], [[0.0, 0.0, 1.0]], s_max=150.0)
        rec, st = oracle_lib.trace(sc)
        r = np.array([rec["x"][0], rec["y"][0], rec["z"][0]])
        u = np.array([rec["ux"][0], rec["uy"][0], rec["uz"][0]])
        # distance from F to the line through r along u
        dist = np.linalg.norm(np.cross(F - r, u))
        assert dist <= 1e-9 * 150.0, (j, dist)
        assert rec["n_ev"][0] == 1


def test_refraction_and_reflection_at_a_sphere(oracle_lib):
    """A ray from outside hits a sphere of n = 1.5: the reflected parent and
    the refracted secondary leave the hit point along u + 2 cos(i) N and
    eta u + (eta cos(i) - cos(t)) N with the outward normal N there."""
    c, R = np.array([0.0, 0.0, 100.0]), 20.0
    o = np.array([5.0, 0.0, 50.0])
    u = np.array([0.0, 0.0, 1.0])
    s_max = 60.0
    sc = scene([const(1.0), const(1.5)], [sphere(c, R, 0, 1)], o, [u], s_max=s_max, G=2)
    rec, st = oracle_lib.trace(sc)
    assert st["records"] == 2
    zP = c[2] - math.sqrt(R * R - 25.0)
    P = np.array([5.0, 0.0, zP])
    tP = zP - o[2]
    N = (P - c) / R
    ci = -(u @ N)
    eta = 1.0 / 1.5
    ct = math.sqrt(1 - eta * eta * (1 - ci * ci))
    ur = u + 2 * ci * N
    ut = eta * u + (eta * ci - ct) * N
    gen = rec["gen"]
    par, sec = np.argmax(gen == 0), np.argmax(gen == 1)
    for i, dvec in ((par, ur), (sec, ut)):
        want = P + (s_max - tP) * dvec
        got = np.array([rec["x"][i], rec["y"][i], rec["z"][i]])
        assert np.abs(got - want).max() <= 1e-9 * s_max, i
        assert np.allclose([rec["ux"][i], rec["uy"][i], rec["uz"][i]], dvec, atol=1e-12)
    # Fresnel at the local incidence angle: A_s of the secondary is t_s
    ts = 2 * ci / (ci + 1.5 * ct)
    assert rec["as_re"][sec] == pytest.approx(ts, abs=1e-12)
