"""raytrace_launch_static, the launch for callers that cannot allocate:
through the C ABI, its records and statistics equal raytrace_launch's on
the same scene, on two calls in a row (the second smaller, so stale
contents of the static scratch must not leak into it), in both models; a
launch whose scratch exceeds the static array is refused."""
import sys

import numpy as np
import pytest

from paper_1810_01780_amd import workloads as W

from .parity import sort_by_key

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_01780_amd import binding
    binding.lib()
    return binding


def _trace(gpu, sc, static):
    ds = gpu.DeviceScene(sc, static_scratch=static)
    ds.launch()
    rec, st = ds.collect()
    assert (ds.workspace is None) == static
    return sort_by_key(rec), st


@pytest.mark.parametrize("model", [W.MODEL_PAPER, W.MODEL_EXACT])
def test_static_scratch_matches_workspace_launch(gpu, model):
    big = W.two_layer(rays_per_source=64, model=model)          # 4,096 primaries
    small = W.two_layer(rays_per_source=8, n_sources=16, model=model)
    for name, sc in (("large", big), ("smaller", small)):
        print(f"\n[gpu-case] static-scratch {name} m{model}: {sc.n_rays} rays", flush=True)
        sys.stdout.flush()
        a, sa = _trace(gpu, sc, static=True)
        b, sb = _trace(gpu, sc, static=False)
        assert sa["records"] > sc.n_rays
        for f in b:
            assert np.array_equal(a[f], b[f]), (name, f)
        for f in ("accepted", "rejected", "relocation", "events", "spawned", "records",
                  "needed", "max_gen", "sched_errors"):
            assert sa[f] == sb[f], (name, f)


def test_static_scratch_size_limit(gpu):
    sc = W.two_layer(rays_per_source=8)
    ds = gpu.DeviceScene(sc, capacity=9_000_000, static_scratch=True)
    assert ds.ws_bytes > gpu.RT_STATIC_SCRATCH_BYTES
    with pytest.raises(gpu.RTError) as e:
        ds.launch()
    assert e.value.status == gpu.RT_ERR_UNSUPPORTED
    assert "static scratch" in gpu.rt_last_error()
