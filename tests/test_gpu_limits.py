"""GPU parity for the limits of a ray: the travel-time limit, the amplitude
cut, the per-ray step cap, the event cap and overflow, plus the gridded
field's edge cells.  Each scene is the one the oracle's closed-form pins use
(tests/test_oracle_limits.py), traced through the C ABI and compared record
by record with the oracle at the standard bars."""
import sys

import numpy as np
import pytest

from paper_1810_01780_amd import workloads as W

from . import scenes
from .parity import compare
from .test_oracle_pins import launch, scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_01780_amd import binding
    binding.lib()
    return binding


def run(gpu, oracle_lib, sc, name):
    print(f"\n[gpu-case] {name}: {sc.n_rays} rays, model {sc.limits.model}", flush=True)
    sys.stdout.flush()
    got, gst = gpu.trace(sc)
    ref, rst = oracle_lib.trace(sc)
    summ = compare(got, ref, sc.limits.tol, label=name)
    print(f"[gpu-case] {name}: {summ}", flush=True)
    for f in ("accepted", "rejected", "events", "spawned", "suppressed_gen", "suppressed_amp",
              "records", "nonfinite"):
        assert gst[f] == rst[f], (name, f, gst[f], rst[f])
    return got, ref


@pytest.mark.parametrize("model", [W.MODEL_PAPER, W.MODEL_EXACT])
@pytest.mark.parametrize("amp_min", [0.05, 0.01, 0.3])
def test_amplitude_cut_slab(gpu, oracle_lib, model, amp_min):
    sc = scenes.slab(model=model, amp_min=amp_min)
    got, ref = run(gpu, oracle_lib, sc, f"slab-amp{amp_min}-m{model}")
    assert np.sum(ref["status"] == oracle_lib.ST_AMP) > 0


@pytest.mark.parametrize("model", [W.MODEL_PAPER, W.MODEL_EXACT])
def test_time_limit(gpu, oracle_lib, model):
    """Constant medium and the firn profile, rays ending at t_max."""
    const = scene([W.Region(a=1.31)], dirs=[(0.3, -0.4, 0.5), (-1.0, 0.0, 0.2)],
                  s_max=1000.0, t_max=1e-6, model=model)
    got, ref = run(gpu, oracle_lib, const, f"time-constant-m{model}")
    assert np.all(got["status"] == oracle_lib.ST_TIME)
    firn = scene([W.Region(a=1.78, dn=0.43, z0=75.0)], src=(0.0, 0.0, 40.0),
                 dirs=[launch(t) for t in (60.0, 120.0, 150.0, 175.0)], model=model,
                 tol=1e-8, s_max=5000.0, t_max=1.5e-6)
    got, ref = run(gpu, oracle_lib, firn, f"time-firn-m{model}")
    assert np.all(got["status"] == oracle_lib.ST_TIME)
    assert np.all(np.abs(got["t"] - 1.5e-6) <= 1e-12 * 1.5e-6)


@pytest.mark.parametrize("model", [W.MODEL_PAPER, W.MODEL_EXACT])
def test_grid_edge_cells(gpu, oracle_lib, model):
    """The linear field on a 9^3 grid, rays through the edge cells of every
    axis (one-sided node differences) on the general kernel."""
    got, ref = run(gpu, oracle_lib, scenes.linear_grid(model=model), f"grid-edges-m{model}")
    assert np.all(got["status"] == oracle_lib.ST_BOX)


@pytest.mark.parametrize("model", [W.MODEL_PAPER, W.MODEL_EXACT])
@pytest.mark.parametrize("which", ["steps", "events", "overflow"])
def test_step_limits(gpu, oracle_lib, model, which):
    """STEPCAP from max_steps_per_ray and from the 255-event cap, and
    NONFINITE from a position overflow, as the oracle ends them."""
    sc = scenes.step_limits(model)[which]
    got, ref = run(gpu, oracle_lib, sc, f"limits-{which}-m{model}")
    want = {"steps": oracle_lib.ST_STEPCAP, "events": oracle_lib.ST_STEPCAP,
            "overflow": oracle_lib.ST_NONFINITE}[which]
    g = got["status"][np.argsort(got["key"])]
    assert g[0] == want
