"""Seeded synthetic scenes for the ray tracer.

This module only *describes* inputs: media, boundary planes, sources, launch
directions, step limits and (for the gridded medium) the FP32 refractive-index
grid.  It holds none of the tracing arithmetic; both the HIP path and the CPU
oracle consume the same ``Scene`` objects, so the two sides see bit-identical
inputs.

Media (paper §2, worked example and accuracy study): a region is stratified in
depth ``z`` (z positive downward, surface at z = 0, air above) with

    n(z) = a + b*z - dn*exp(-z/z0)          (analytic region)

or takes n from the grid (``use_grid``).  The paper's firn profile is
n0 - dn*exp(-depth/z0); with a = n0, b = 0 it is the first form.  b != 0 with
dn = 0 gives the linear profile used by the closed-form tests.

Every random quantity is drawn from ``numpy.random.SeedSequence(181001780)``,
one spawned child per named workload, so a workload is fully determined by its
name and sizes.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

MASTER_SEED = 181001780

# model flags
MODEL_PAPER = 0   # locally paraxial form of the eikonal (paper §2, eq. 2)
MODEL_EXACT = 1   # full eikonal (paper §2, eq. 1)

# plane kinds
PLANE_FRESNEL = 0  # reflect + refracted secondary, Fresnel amplitudes
PLANE_ABSORB = 1   # terminate the ray on contact
SHAPE_PLANE, SHAPE_SPHERE, SHAPE_PARABOLOID = 0, 1, 2  # boundary surface shapes


@dataclasses.dataclass
class Region:
    a: float
    b: float = 0.0
    dn: float = 0.0
    z0: float = 1.0
    z_top: float = -np.inf   # launch-region lookup: z_top <= z < z_bot
    z_bot: float = np.inf
    use_grid: bool = False
    # stratification axis: n = a + b zeta - dn exp(-zeta / z0), zeta = k . r
    # with k = axis / |axis|; all zero means depth, zeta = z
    axis: Sequence[float] = (0.0, 0.0, 0.0)


@dataclasses.dataclass
class Anomaly:
    """Gaussian index anomaly: amplitude exp(-|r - centre|^2 / (2 sigma^2))
    added to the refractive index of one region."""
    centre: Sequence[float]
    amplitude: float
    sigma: float
    region: int


@dataclasses.dataclass
class Plane:
    """A boundary surface: a plane (point, normal), a sphere (centre = point,
    radius = param; region_pos outside) or a paraboloid z = z_v + param
    ((x - x_v)^2 + (y - y_v)^2) with vertex = point (region_pos below)."""
    point: Sequence[float]
    normal: Sequence[float]
    region_pos: int       # region on the side the normal points to
    region_neg: int
    kind: int = PLANE_FRESNEL
    shape: int = 0        # SHAPE_PLANE, SHAPE_SPHERE, SHAPE_PARABOLOID
    param: float = 0.0


@dataclasses.dataclass
class Grid:
    n: np.ndarray          # float32 [nz, ny, nx], x fastest
    origin: Sequence[float]
    spacing: Sequence[float]


@dataclasses.dataclass
class Limits:
    tol: float = 1e-6
    h_min: float = 1e-3
    h_max: float = 10.0
    h_init: float = 0.0      # 0 -> h_max
    s_max: float = 2000.0
    t_max: float = 0.0       # 0 -> off
    amp_min: float = 0.0     # 0 -> off
    max_generations: int = 1
    model: int = MODEL_PAPER
    max_steps_per_ray: int = 1_000_000
    max_steps_per_launch: int = 0    # GPU launches only: 0 = no step budget


@dataclasses.dataclass
class Scene:
    name: str
    regions: List[Region]
    planes: List[Plane]
    sources: np.ndarray           # float64 [S, 3]
    ray_src: np.ndarray           # int32 [N]
    dirs: np.ndarray              # float64 [N, 3] (need not be unit length)
    limits: Limits
    box_lo: Optional[Sequence[float]] = None
    box_hi: Optional[Sequence[float]] = None
    grid: Optional[Grid] = None
    anomalies: List[Anomaly] = dataclasses.field(default_factory=list)

    @property
    def n_rays(self) -> int:
        return int(self.dirs.shape[0])

    def capacity_hint(self) -> int:
        """Record capacity large enough for every workload in this module."""
        g = self.limits.max_generations
        return max(16, self.n_rays * (1 if g <= 1 else 8) + 64)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx, dtype=np.int64)
        return dataclasses.replace(self, ray_src=self.ray_src[idx].copy(),
                                   dirs=self.dirs[idx].copy())


def _rng(workload: int) -> np.random.Generator:
    child = np.random.SeedSequence(MASTER_SEED).spawn(5)[workload]
    return np.random.default_rng(child)


def isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniform on the sphere: cos(theta) = 1 - 2 xi1, phi = 2 pi xi2."""
    xi = rng.random((n, 2))
    ct = 1.0 - 2.0 * xi[:, 0]
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * np.pi * xi[:, 1]
    return np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)


# --- media used by the workloads --------------------------------------------
FIRN = dict(a=1.78, dn=0.43, z0=75.0)           # n(z) = 1.78 - 0.43 exp(-z/75 m)
PAPER_FIRN = dict(a=1.788, dn=0.463, z0=71.4)   # paper §2 worked example


def air_region(z_bot: float = 0.0) -> Region:
    return Region(a=1.0, z_top=-np.inf, z_bot=z_bot)


def surface_plane(ice: int, air: int, kind: int = PLANE_FRESNEL) -> Plane:
    # normal +z points into the ice (depth grows downward)
    return Plane(point=(0.0, 0.0, 0.0), normal=(0.0, 0.0, 1.0),
                 region_pos=ice, region_neg=air, kind=kind)


def point_source_fan(n_rays: int = 1024, depth: float = 200.0,
                     tol: float = 1e-6, s_max: float = 2000.0,
                     generations: int = 2, model: int = MODEL_PAPER,
                     surface_kind: int = PLANE_FRESNEL) -> Scene:
    """1,024 rays from one point source at 200 m depth in one vertical plane.

    Launch angles are the midpoints theta_k = (k + 1/2) * 180 deg / N measured
    from the upward vertical in the x-z plane, u = (sin th, 0, -cos th).  Air
    above z = 0, firn 1.78 - 0.43 exp(-z/75 m) below; the surface reflects with
    one refracted secondary (two generations).  Rays end at the path limit or
    on a face of a 3 km cube centred on the source's surface point.
    """
    th = (np.arange(n_rays, dtype=np.float64) + 0.5) * (np.pi / n_rays)
    dirs = np.stack([np.sin(th), np.zeros_like(th), -np.cos(th)], axis=1)
    regions = [air_region(), Region(**FIRN, z_top=0.0, z_bot=np.inf)]
    planes = [surface_plane(ice=1, air=0, kind=surface_kind)]
    return Scene(name="fan1024", regions=regions, planes=planes,
                 sources=np.array([[0.0, 0.0, depth]]),
                 ray_src=np.zeros(n_rays, dtype=np.int32), dirs=dirs,
                 limits=Limits(tol=tol, h_min=1e-3, h_max=10.0, s_max=s_max,
                               max_generations=generations, model=model),
                 box_lo=(-1500.0, -1500.0, -1500.0),
                 box_hi=(1500.0, 1500.0, 1500.0))


def two_layer(rays_per_source: int = 16384, n_sources: int = 64,
              generations: int = 4, model: int = MODEL_PAPER,
              s_max: float = 5000.0, tol: float = 1e-6) -> Scene:
    """Isotropic rays from seeded sources in the two-layer firn model.

    Sources at x = y = 0, depths uniform in 10-1500 m (64 sources x 16,384 rays
    = 1,048,576 rays at full size).  The firn profile holds down to the layer
    plane at 150 m; below it the same profile continues with +0.01 added.  The
    surface and the layer plane both reflect and spawn refracted secondaries,
    up to four generations.  Rays end at 5 km path length.
    """
    rng = _rng(1)
    depths = rng.uniform(10.0, 1500.0, size=n_sources)
    sources = np.stack([np.zeros(n_sources), np.zeros(n_sources), depths], axis=1)
    dirs = isotropic(rng, n_sources * rays_per_source)
    ray_src = np.repeat(np.arange(n_sources, dtype=np.int32), rays_per_source)
    regions = [air_region(),
               Region(**FIRN, z_top=0.0, z_bot=150.0),
               Region(a=FIRN["a"] + 0.01, dn=FIRN["dn"], z0=FIRN["z0"],
                      z_top=150.0, z_bot=np.inf)]
    planes = [surface_plane(ice=1, air=0),
              Plane(point=(0.0, 0.0, 150.0), normal=(0.0, 0.0, 1.0),
                    region_pos=2, region_neg=1)]
    return Scene(name="twolayer", regions=regions, planes=planes,
                 sources=sources, ray_src=ray_src, dirs=dirs,
                 limits=Limits(tol=tol, h_min=1e-3, h_max=10.0, s_max=s_max,
                               max_generations=generations, model=model))


def gaussian_random_field(rng: np.random.Generator, shape, spacing: float,
                          sigma: float, corr_len: float) -> np.ndarray:
    """Periodic Gaussian random field by FFT spectral synthesis (float64).

    Covariance sigma^2 exp(-r^2 / (2 l^2)); the amplitude spectrum is the square
    root of its Fourier transform, exp(-k^2 l^2 / 4) up to a constant, which the
    final renormalisation to the sample standard deviation fixes.
    """
    white = rng.standard_normal(shape)
    ks = [2.0 * np.pi * np.fft.fftfreq(m, d=spacing) for m in shape]
    kz, ky, kx = np.meshgrid(*ks, indexing="ij")
    amp = np.exp(-(kx * kx + ky * ky + kz * kz) * corr_len * corr_len / 4.0)
    f = np.fft.ifftn(np.fft.fftn(white) * amp).real
    f -= f.mean()
    return f * (sigma / f.std())


def gridded(rays_per_source: int = 16384, n_sources: int = 256,
            nx: int = 256, ny: int = 256, nz: int = 128, spacing: float = 10.0,
            generations: int = 1, model: int = MODEL_PAPER,
            s_max: float = 3000.0, tol: float = 1e-7) -> Scene:
    """Gridded firn: 256 x 256 x 128 FP32 nodes at 10 m.

    n = 1.78 - 0.43 exp(-z/75 m) plus a Gaussian random field (sigma 1e-3,
    correlation length 50 m), covering x, y in [-1275, 1275] m and depth in
    [0, 1270] m.  256 sources (x, y uniform in +-500 m, depth 20-1200 m) with
    16,384 isotropic rays each (4,194,304 rays at full size).  The surface
    reflects; with one generation the transmitted air rays are suppressed.  The
    box is the grid's horizontal extent and depth range, with air up to -1270 m.
    """
    rng = _rng(2)
    ox, oy = -(nx - 1) * spacing / 2.0, -(ny - 1) * spacing / 2.0
    z = np.arange(nz, dtype=np.float64) * spacing
    prof = FIRN["a"] - FIRN["dn"] * np.exp(-z / FIRN["z0"])
    grf = gaussian_random_field(rng, (nz, ny, nx), spacing, 1e-3, 50.0)
    n = (prof[:, None, None] + grf).astype(np.float32)
    # sources at x, y within +-500 m (or 40 % of a smaller grid), depth 20-1200 m
    half = min(500.0, 0.4 * min(-ox, -oy))
    xs = rng.uniform(-half, half, size=(n_sources, 2))
    depths = rng.uniform(20.0, min(1200.0, 0.9 * (nz - 1) * spacing), size=n_sources)
    sources = np.concatenate([xs, depths[:, None]], axis=1)
    dirs = isotropic(rng, n_sources * rays_per_source)
    ray_src = np.repeat(np.arange(n_sources, dtype=np.int32), rays_per_source)
    regions = [air_region(), Region(a=0.0, use_grid=True, z_top=0.0, z_bot=np.inf)]
    planes = [surface_plane(ice=1, air=0)]
    zmax = (nz - 1) * spacing
    return Scene(name="grid256", regions=regions, planes=planes,
                 sources=sources, ray_src=ray_src, dirs=dirs,
                 limits=Limits(tol=tol, h_min=1e-3, h_max=10.0, s_max=s_max,
                               max_generations=generations, model=model),
                 box_lo=(ox, oy, -zmax), box_hi=(-ox, -oy, zmax),
                 grid=Grid(n=n, origin=(ox, oy, 0.0), spacing=(spacing,) * 3))


def paper_example(n_rays: int = 512, generations: int = 4,
                  model: int = MODEL_PAPER) -> Scene:
    """The worked example of the paper (section 2, Fig. 1).

    Air above z = 0; a top layer of constant n = 1.5 from 0 to 10 m depth;
    below it the profile 1.788 - 0.463 exp(-z/71.4 m).  Rays leave a point at
    240 m depth in all directions of the x-z plane; they end after 5 us of
    travel time, or when their amplitude falls below 0.05 of the initial one.
    Both interfaces reflect and cast refracted secondaries.
    """
    th = (np.arange(n_rays, dtype=np.float64) + 0.5) * (2.0 * np.pi / n_rays)
    dirs = np.stack([np.sin(th), np.zeros_like(th), -np.cos(th)], axis=1)
    regions = [air_region(),
               Region(a=1.5, z_top=0.0, z_bot=10.0),
               Region(**PAPER_FIRN, z_top=10.0, z_bot=np.inf)]
    planes = [surface_plane(ice=1, air=0),
              Plane(point=(0.0, 0.0, 10.0), normal=(0.0, 0.0, 1.0),
                    region_pos=2, region_neg=1)]
    return Scene(name="paper_example", regions=regions, planes=planes,
                 sources=np.array([[0.0, 0.0, 240.0]]),
                 ray_src=np.zeros(n_rays, dtype=np.int32), dirs=dirs,
                 limits=Limits(tol=1e-6, h_min=1e-3, h_max=10.0, s_max=1e4,
                               t_max=5e-6, amp_min=0.05,
                               max_generations=generations, model=model))


@dataclasses.dataclass
class SolvePairs:
    """Emitter -> receiver pairs: source at (0, 0, zs), receiver at
    (dist, 0, zr); scene gives the medium (planes[0] is the surface)."""
    scene: Scene
    zs: np.ndarray
    zr: np.ndarray
    dist: np.ndarray

    @property
    def n(self) -> int:
        return int(self.zs.shape[0])


def solve_pairs(n_pairs: int = 65536, model: int = MODEL_PAPER) -> SolvePairs:
    """Seeded source/receiver pairs in the two-layer firn model: source depth
    50-2000 m, receiver depth 0-200 m, horizontal distance 10 m-3 km, all
    uniform.  Each pair is solved for its direct and its surface-reflected
    ray."""
    rng = _rng(3)
    zs = rng.uniform(50.0, 2000.0, size=n_pairs)
    zr = rng.uniform(0.0, 200.0, size=n_pairs)
    dist = rng.uniform(10.0, 3000.0, size=n_pairs)
    scene = two_layer(rays_per_source=1, n_sources=1, generations=1, model=model)
    return SolvePairs(scene=scene, zs=zs, zr=zr, dist=dist)


WORKLOADS = {
    "fan1024": point_source_fan,
    "twolayer": two_layer,
    "grid256": gridded,
    "paper_example": paper_example,
}


# --- surrogate network inputs -----------------------------------------------
MLP_DIMS = [(5, 256), (256, 256), (256, 256), (256, 256), (256, 12)]


def mlp_init_params(seed: int = 0) -> np.ndarray:
    """Seeded initial parameters of the surrogate network, FP32, in the
    layout of the C header (per layer W [n_out][n_in], then b [n_out]):
    normal weights with variance 2 / n_in (He), zero biases."""
    rng = np.random.default_rng(np.random.SeedSequence([MASTER_SEED, 4, seed]))
    parts = []
    for n_in, n_out in MLP_DIMS:
        parts.append((rng.standard_normal(n_in * n_out) * np.sqrt(2.0 / n_in)).astype(np.float32))
        parts.append(np.zeros(n_out, np.float32))
    return np.concatenate(parts)


def two_layer_medium(z0: float = FIRN["z0"], dn: float = FIRN["dn"], model: int = MODEL_PAPER,
                     tol: float = 1e-6) -> Scene:
    """The two-layer firn medium of the solve workloads with the firn
    profile a - dn exp(-z/z0) (a = 1.78) scaled by (z0, dn): firn down to the
    150 m plane, the same profile + 0.01 below, Fresnel surface and layer."""
    regions = [air_region(),
               Region(a=FIRN["a"], dn=dn, z0=z0, z_top=0.0, z_bot=150.0),
               Region(a=FIRN["a"] + 0.01, dn=dn, z0=z0, z_top=150.0, z_bot=np.inf)]
    planes = [surface_plane(ice=1, air=0),
              Plane(point=(0.0, 0.0, 150.0), normal=(0.0, 0.0, 1.0),
                    region_pos=2, region_neg=1)]
    return Scene(name="twolayer-medium", regions=regions, planes=planes,
                 sources=np.zeros((1, 3)), ray_src=np.zeros(1, np.int32),
                 dirs=np.array([[1.0, 0.0, 0.0]]),
                 limits=Limits(tol=tol, h_min=1e-3, h_max=10.0, s_max=5000.0,
                               max_generations=1, model=model))


def surrogate_training_set(n_profiles: int, pairs_per_profile: int, seed: int = 0):
    """Seeded training pairs for the solve surrogate: per profile, the scale
    depth z0 ~ U(40, 120) m and the contrast dn ~ U(0.35, 0.5), then pairs
    as in solve_pairs (source 50-2000 m, receiver 0-200 m, distance
    10 m - 3 km).  Returns a list of (z0, dn, zs, zr, dist)."""
    rng = np.random.default_rng(np.random.SeedSequence([MASTER_SEED, 5, seed]))
    out = []
    for _ in range(n_profiles):
        z0 = rng.uniform(40.0, 120.0)
        dn = rng.uniform(0.35, 0.5)
        zs = rng.uniform(50.0, 2000.0, pairs_per_profile)
        zr = rng.uniform(0.0, 200.0, pairs_per_profile)
        dist = rng.uniform(10.0, 3000.0, pairs_per_profile)
        out.append((z0, dn, zs, zr, dist))
    return out


def curved(n_sources: int = 4, rays_per_source: int = 256, model: int = MODEL_PAPER,
           generations: int = 3, s_max: float = 1500.0, tol: float = 1e-6,
           bed_kind: int = PLANE_ABSORB) -> Scene:
    """Curved boundaries in firn: an air-filled spherical void (radius 25 m,
    centre at 150 m depth) with Fresnel walls, a paraboloidal bed
    z = 400 m - 0.0005 rho^2 (absorbing, or a Fresnel interface to rock of
    n = 2.5 below it), the flat Fresnel surface; isotropic rays from
    sources 40 m off the axis at 180 and 220 m depth; amplitude cut 1e-3
    (bounds the bounces inside the void)."""
    rng = _rng(4)
    offs = np.array([[40.0, 0.0, 180.0], [-40.0, 0.0, 180.0], [0.0, 40.0, 220.0],
                     [0.0, -40.0, 220.0]])[:n_sources]
    dirs = isotropic(rng, n_sources * rays_per_source)
    ray_src = np.repeat(np.arange(n_sources, dtype=np.int32), rays_per_source)
    regions = [air_region(),
               Region(**FIRN, z_top=0.0, z_bot=np.inf),
               Region(a=1.0, z_top=np.inf, z_bot=np.inf),       # inside the void
               Region(a=2.5, z_top=np.inf, z_bot=np.inf)]       # rock below the bed
    below = 3 if bed_kind == PLANE_FRESNEL else 1
    planes = [surface_plane(ice=1, air=0),
              Plane(point=(0.0, 0.0, 150.0), normal=(0.0, 0.0, 1.0), region_pos=1,
                    region_neg=2, shape=SHAPE_SPHERE, param=25.0),
              Plane(point=(0.0, 0.0, 400.0), normal=(0.0, 0.0, 1.0), region_pos=below,
                    region_neg=1, kind=bed_kind, shape=SHAPE_PARABOLOID, param=-5e-4)]
    return Scene(name="curved", regions=regions, planes=planes, sources=offs,
                 ray_src=ray_src, dirs=dirs,
                 limits=Limits(tol=tol, h_min=1e-3, h_max=10.0, s_max=s_max, amp_min=1e-3,
                               max_generations=generations, model=model))


def field3d(n_sources: int = 4, rays_per_source: int = 256, model: int = MODEL_PAPER,
            generations: int = 2, s_max: float = 1500.0, tol: float = 1e-6,
            tilt_deg: float = 8.0) -> Scene:
    """Firn that is not stratified in depth: the profile of FIRN along an axis
    tilted by tilt_deg from the vertical toward +x, a high-index lens
    (+0.04, sigma 20 m, centre at 120 m depth) and a low-index pocket
    (-0.15, sigma 8 m, at (30, 20, 60) m) in it, under the flat Fresnel
    surface; isotropic rays from sources 40 m off the axis at 180 and 220 m
    depth."""
    rng = _rng(4)
    offs = np.array([[40.0, 0.0, 180.0], [-40.0, 0.0, 180.0], [0.0, 40.0, 220.0],
                     [0.0, -40.0, 220.0]])[:n_sources]
    dirs = isotropic(rng, n_sources * rays_per_source)
    ray_src = np.repeat(np.arange(n_sources, dtype=np.int32), rays_per_source)
    t = np.radians(tilt_deg)
    regions = [air_region(),
               Region(**FIRN, z_top=0.0, z_bot=np.inf, axis=(np.sin(t), 0.0, np.cos(t)))]
    anomalies = [Anomaly(centre=(0.0, 0.0, 120.0), amplitude=0.04, sigma=20.0, region=1),
                 Anomaly(centre=(30.0, 20.0, 60.0), amplitude=-0.15, sigma=8.0, region=1)]
    return Scene(name="field3d", regions=regions, planes=[surface_plane(ice=1, air=0)],
                 sources=offs, ray_src=ray_src, dirs=dirs, anomalies=anomalies,
                 limits=Limits(tol=tol, h_min=1e-3, h_max=10.0, s_max=s_max,
                               max_generations=generations, model=model))
