"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The host side of the C ABI (descriptor validation, workspace sizes,
  statistics -> status; csrc/rt_host.cpp) built with g++ and both sanitizers
  into tests/host_checks.cpp's driver: valid and invalid descriptors, every
  table full, fake device pointers that must never be read.
* The oracle built with gcc and both sanitizers, loaded into a Python child
  process with the ASan runtime preloaded: small traces (both models, every
  kind of surface, a grid, the step and event caps, an overflow), events,
  shots, solves and seeded solves; its results must equal those of the plain
  build bit for bit (the same IEEE arithmetic, no contraction).
A sanitizer report aborts the program, so a non-zero exit fails the test.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _tool(name):
    if shutil.which(name) is None:
        pytest.skip(f"{name} not available")
    return name


def test_host_abi_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_checks")
    cmd = [_tool("g++"), "-std=c++17", "-O1", "-g", *SAN,
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1810_01780_amd", "csrc"), "-I", "/opt/rocm/include",
           os.path.join(ROOT, "tests", "host_checks.cpp"),
           os.path.join(ROOT, "paper_1810_01780_amd", "csrc", "rt_host.cpp"),
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    subprocess.run(cmd, check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env={**os.environ, **ENV},
                       timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks ok" in r.stdout


CHILD = r'''
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
from paper_1810_01780_amd import workloads as W
from tests import scenes


def run(lib):
    oracle._LIB, oracle._lib = lib, None
    out = []
    for model in (W.MODEL_PAPER, W.MODEL_EXACT):
        for sc in (W.point_source_fan(n_rays=64, model=model),
                   W.two_layer(rays_per_source=8, n_sources=4, model=model),
                   W.curved(n_sources=2, rays_per_source=8, model=model),
                   scenes.maximal(n_rays=32, model=model),
                   scenes.maximal(n_rays=16, anomalies=True, model=model),
                   scenes.linear_grid(model=model, n_rays=16),
                   scenes.slab(model=model),
                   *scenes.step_limits(model=model).values()):
            rec, st = oracle.trace(sc, threads=2)
            out += [rec[f] for f in sorted(rec)] + [np.array(sorted(st.items()), dtype=object)]
        ev_rec, ev_st, ev = oracle.trace(W.two_layer(rays_per_source=4, n_sources=2,
                                                     model=model), threads=2, events=True)
        out += [ev[f] for f in sorted(ev)]
    sp = W.solve_pairs(16)
    s = oracle.solve(sp.scene, sp.zs, sp.zr, sp.dist, threads=2)
    out += [s[f] for f in sorted(s)]
    seed = np.where(s["found"] == 1, s["theta"] + 1e-3, 1.0)
    q = oracle.solve_seeded(sp.scene, sp.zs, sp.zr, sp.dist, seed, np.ones_like(s["found"]),
                            threads=2)
    out += [q[f] for f in sorted(q)]
    return out


a = run(sys.argv[2])
b = run(sys.argv[3])
assert len(a) == len(b)
for x, y in zip(a, b):
    assert np.array_equal(x, y, equal_nan=True) if x.dtype != object else \
        list(x.ravel()) == list(y.ravel())
print("oracle under sanitizers ok:", len(a), "arrays equal")
'''


def test_oracle_under_sanitizers(tmp_path):
    import oracle
    plain = oracle.build(force=False)
    san = str(tmp_path / "liboracle_san.so")
    src = os.path.join(ROOT, "oracle", "raytrace_oracle.c")
    subprocess.run([_tool("gcc"), "-O1", "-g", "-std=gnu11", "-ffp-contract=off",
                    "-fno-fast-math", *SAN, "-shared", "-fPIC", "-o", san, src, "-lm",
                    "-lpthread"], check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True, check=True).stdout.strip()
    script = tmp_path / "child.py"
    script.write_text(CHILD)
    env = {**os.environ, **ENV, "LD_PRELOAD": asan}
    r = subprocess.run([sys.executable, str(script), ROOT, san, plain], capture_output=True,
                       text=True, env=env, timeout=600, cwd=ROOT)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "oracle under sanitizers ok" in r.stdout
