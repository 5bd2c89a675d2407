"""Small seeded scenes shared by the oracle and GPU tests: one that uses
every slot of the descriptor tables at once (RT_MAX_REGIONS media,
RT_MAX_PLANES boundaries plus the six box faces and the travel-time limit,
RT_MAX_ANOMALIES anomalies), and a single ray crossing a spherical void
along a chord shorter than its step."""
import numpy as np

from paper_1810_01780_amd import workloads as W


def maximal(n_rays=256, anomalies=False, model=W.MODEL_PAPER, seed=7):
    """Air over seven firn layers (8 media) separated by the surface and six
    horizontal Fresnel interfaces; nine vertical planes (four Fresnel
    between the same medium on both sides, five absorbing) make 16
    boundaries; a box, a travel-time and an amplitude limit; four
    generations; with anomalies=True also 8 Gaussian anomalies spread over
    the layers (the general kernel)."""
    rng = np.random.default_rng(seed)
    depths = [0.0, 20.0, 45.0, 80.0, 120.0, 170.0, 230.0]
    regions = [W.air_region()]
    for i, top in enumerate(depths):
        bot = depths[i + 1] if i + 1 < len(depths) else np.inf
        regions.append(W.Region(a=1.78 + 0.004 * i, dn=0.43, z0=75.0, z_top=top, z_bot=bot))
    planes = [W.surface_plane(ice=1, air=0)]
    for i, z in enumerate(depths[1:]):
        planes.append(W.Plane(point=(0.0, 0.0, z), normal=(0.0, 0.0, 1.0),
                              region_pos=i + 2, region_neg=i + 1))
    # vertical planes x = const: Fresnel ones join a layer to itself (n1 = n2:
    # full transmission, no reflection), absorbing ones end the ray
    for j, x in enumerate((-300.0, -220.0, -150.0, 160.0, 240.0, 310.0, 380.0, 450.0, 520.0)):
        kind = W.PLANE_FRESNEL if j % 2 == 0 and j < 8 else W.PLANE_ABSORB
        planes.append(W.Plane(point=(x, 0.0, 0.0), normal=(1.0, 0.0, 0.0), region_pos=3,
                              region_neg=3, kind=kind))
    assert len(planes) == 16 and len(regions) == 8
    anoms = []
    if anomalies:
        for k in range(8):
            anoms.append(W.Anomaly(centre=(rng.uniform(-200, 200), rng.uniform(-50, 50),
                                           rng.uniform(30, 260)),
                                   amplitude=float(rng.choice([-1, 1]) * rng.uniform(0.005, 0.03)),
                                   sigma=float(rng.uniform(10, 30)), region=1 + k % 7))
    sources = np.array([[0.0, 0.0, 100.0], [30.0, 10.0, 200.0]])
    dirs = W.isotropic(rng, n_rays)
    ray_src = (np.arange(n_rays) % 2).astype(np.int32)
    return W.Scene(name="maximal", regions=regions, planes=planes, sources=sources,
                   ray_src=ray_src, dirs=dirs, anomalies=anoms,
                   limits=W.Limits(tol=1e-6, h_min=1e-3, h_max=10.0, s_max=1500.0,
                                   t_max=6e-6, amp_min=1e-4, max_generations=4, model=model),
                   box_lo=(-1000.0, -1000.0, -800.0), box_hi=(1000.0, 1000.0, 1000.0))


def void_chord(model, theta_deg=40.0, radius=10.0):
    """Ice of constant n = 1.5 holding a spherical void (n = 1, radius 10 m,
    centre at 100 m depth); one ray travels straight down at the impact
    parameter R sin(theta) and meets the void at incidence theta."""
    b = radius * np.sin(np.radians(theta_deg))
    regions = [W.Region(a=1.5, z_top=-np.inf, z_bot=np.inf),
               W.Region(a=1.0, z_top=np.inf, z_bot=np.inf)]
    planes = [W.Plane(point=(0.0, 0.0, 100.0), normal=(0.0, 0.0, 1.0), region_pos=0,
                      region_neg=1, shape=W.SHAPE_SPHERE, param=radius)]
    return W.Scene(name="void-chord", regions=regions, planes=planes,
                   sources=np.array([[b, 0.0, 50.0]]), ray_src=np.zeros(1, np.int32),
                   dirs=np.array([[0.0, 0.0, 1.0]]),
                   limits=W.Limits(tol=1e-6, h_min=1e-3, h_max=10.0, s_max=60.0,
                                   max_generations=2, model=model))


def slab(model=W.MODEL_PAPER, angles_deg=(5.0, 15.0, 25.0, 35.0, 40.0, 45.0, 60.0),
         amp_min=0.05, max_generations=2, s_max=400.0, n_slab=1.5, thickness=10.0):
    """A slab of constant index n_slab between z = 0 and z = thickness with air
    (n = 1) above and below, both faces Fresnel; one source at mid-depth;
    rays in the x-z plane at the given angles from the downward vertical.
    Inside, a ray bounces between the faces along straight segments, its
    amplitudes multiplied by the same reflection coefficients at every
    bounce, and each bounce below the critical angle casts a secondary
    into the air."""
    regions = [W.Region(a=1.0, z_bot=0.0), W.Region(a=n_slab, z_top=0.0, z_bot=thickness),
               W.Region(a=1.0, z_top=thickness)]
    planes = [W.Plane(point=(0.0, 0.0, 0.0), normal=(0.0, 0.0, 1.0), region_pos=1,
                      region_neg=0),
              W.Plane(point=(0.0, 0.0, thickness), normal=(0.0, 0.0, 1.0), region_pos=2,
                      region_neg=1)]
    th = np.radians(np.asarray(angles_deg, dtype=np.float64))
    dirs = np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], axis=1)
    return W.Scene(name="slab", regions=regions, planes=planes,
                   sources=np.array([[0.0, 0.0, 0.5 * thickness]]),
                   ray_src=np.zeros(len(th), np.int32), dirs=dirs,
                   limits=W.Limits(tol=1e-6, h_min=1e-3, h_max=10.0, s_max=s_max,
                                   amp_min=amp_min, max_generations=max_generations,
                                   model=model))


def linear_grid(model=W.MODEL_EXACT, n_rays=64, analytic=False, seed=11):
    """A field linear in x, y and z, n = 1.25 + 2^-12 x - 2^-13 y + 2^-10 z,
    sampled on 9 x 9 x 9 FP32 nodes at 8 m spacing (every node value and
    difference exact), or its analytic form (a linear medium along the
    gradient's axis); isotropic rays from the centre run until they leave a
    box 1 m inside the grid, so each one crosses an edge cell of the grid
    while no stage of its steps (at most 0.5 m) reaches beyond the grid, where
    clamping would hold n constant."""
    B = np.array([2.0 ** -12, -(2.0 ** -13), 2.0 ** -10])
    a, sp, m = 1.25, 8.0, 9
    origin = (-32.0, -32.0, 0.0)
    ax = [origin[i] + sp * np.arange(m) for i in range(3)]
    zz, yy, xx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    vals = a + B[0] * xx + B[1] * yy + B[2] * zz
    g = vals.astype(np.float32)
    assert np.array_equal(g.astype(np.float64), vals)
    rng = np.random.default_rng(seed)
    dirs = W.isotropic(rng, n_rays)
    if analytic:
        regions = [W.Region(a=a, b=float(np.linalg.norm(B)), axis=tuple(B))]
        grid = None
    else:
        regions = [W.Region(a=0.0, use_grid=True)]
        grid = W.Grid(n=np.ascontiguousarray(g), origin=origin, spacing=(sp, sp, sp))
    return W.Scene(name="linear-grid", regions=regions, planes=[],
                   sources=np.array([[0.0, 0.0, 32.0]]), ray_src=np.zeros(n_rays, np.int32),
                   dirs=dirs, grid=grid, box_lo=(-31.0, -31.0, 1.0), box_hi=(31.0, 31.0, 63.0),
                   limits=W.Limits(tol=1e-8, h_min=1e-3, h_max=0.5, s_max=500.0, model=model))


def step_limits(model=W.MODEL_PAPER):
    """Three scenes whose rays end on the step limits, by name:
    'steps': two rays in air whose steps grow five-fold from 1 mm (closed-form
    positions) and run into max_steps_per_ray = 5;
    'overflow': a ray launched at x = 1.7e308 whose first 1e307 m step
    overflows the position (NONFINITE), beside an ordinary ray;
    'events': a ray totally reflected between the faces of an n = 1.5 slab
    in air until its 256th event (STEPCAP)."""
    air = [W.Region(a=1.0)]
    steps = W.Scene(name="stepcap-steps", regions=air, planes=[],
                    sources=np.array([[0.0, 0.0, 40.0]]), ray_src=np.zeros(2, np.int32),
                    dirs=np.array([[0.6, 0.0, 0.8], [0.0, 1.0, 0.0]]),
                    limits=W.Limits(tol=1e-6, h_min=1e-3, h_max=10.0, h_init=1e-3,
                                    s_max=5000.0, model=model, max_steps_per_ray=5))
    overflow = W.Scene(name="nonfinite", regions=[W.Region(a=1.31)], planes=[],
                       sources=np.array([[1.7e308, 0.0, 40.0], [0.0, 0.0, 40.0]]),
                       ray_src=np.array([0, 1], np.int32),
                       dirs=np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]),
                       limits=W.Limits(tol=1e-6, h_min=1e-3, h_max=1e307, h_init=1e307,
                                       s_max=1e308, model=model))
    sl = slab(model=model, angles_deg=(45.0,), amp_min=0.0, max_generations=1, s_max=5000.0)
    sl.name = "stepcap-events"
    return {"steps": steps, "overflow": overflow, "events": sl}
