"""Training and use of the solve surrogate, through the C ABI only.

Data: the tracer's full solves (raytrace_solve) of seeded pairs in seeded
firn profiles; features and targets are formed on the GPU by
rt_surrogate_features / rt_surrogate_targets.  Training: rt_mlp_gradients
and rt_mlp_adam (BF16 matrix cores, FP32 Adam) on minibatches of the
shuffled set, cosine learning-rate decay.  Use: raytrace_solve_surrogate,
which seeds every entry with the network, verifies each seed by shooting and
hands the pairs it cannot verify to the tracer.
"""
from __future__ import annotations

import math
import time
from typing import Dict, Optional

import numpy as np

from . import binding as B
from . import workloads as W


def generate(n_profiles: int, pairs_per_profile: int, seed: int = 0,
             model: int = W.MODEL_PAPER, log=None) -> Dict[str, "torch.Tensor"]:
    """Training set on the GPU: x [N][5], t [N][8], m [N][2] (FP32), rows
    shuffled with a seeded permutation; N = n_profiles * pairs_per_profile."""
    import torch
    dev = torch.device("cuda")
    N = n_profiles * pairs_per_profile
    x = torch.empty((N, 5), dtype=torch.float32, device=dev)
    t = torch.empty((N, 8), dtype=torch.float32, device=dev)
    m = torch.empty((N, 2), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    t0 = time.perf_counter()
    found = 0
    for k, (z0, dn, zs, zr, dist) in enumerate(
            W.surrogate_training_set(n_profiles, pairs_per_profile, seed)):
        ds = B.DeviceSolve(W.two_layer_medium(z0, dn, model=model), zs, zr, dist)
        ds.launch()
        r0 = k * pairs_per_profile
        st = B.rt_surrogate_features(ds.pairs, z0, dn, x[r0:].data_ptr(), stream)
        st = st or B.rt_surrogate_targets(ds.out, ds.n, t[r0:].data_ptr(), m[r0:].data_ptr(),
                                          stream)
        if st != B.RT_OK:
            raise B.RTError(st, B.rt_last_error())
        torch.cuda.synchronize()
        found += int(ds.stats()["found"])
        del ds
    perm = torch.as_tensor(np.random.default_rng(seed).permutation(N), device=dev)
    data = {"x": x.index_select(0, perm).contiguous(), "t": t.index_select(0, perm).contiguous(),
            "m": m.index_select(0, perm).contiguous()}
    if log:
        log(f"training set: {N} pairs in {n_profiles} profiles, {found} of {2 * N} entries "
            f"solved, {time.perf_counter() - t0:.1f} s")
    return data


def train(data, steps: int, batch: int = 4096, lr: float = 2e-3, lr_final: float = 2e-5,
          seed: int = 0, log=None, net: Optional[B.DeviceMLP] = None):
    """Train the network; returns (DeviceMLP, list of (step, loss))."""
    import torch
    N = int(data["x"].shape[0])
    batch = min(batch, N)
    if net is None:
        net = B.DeviceMLP(W.mlp_init_params(seed), max_batch=batch, training=True)
    losses = []
    nb = N // batch
    t0 = time.perf_counter()
    for step in range(steps):
        j = (step % nb) * batch
        a = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * step / max(1, steps)))
        net.train_step(data["x"][j:j + batch], data["t"][j:j + batch], data["m"][j:j + batch], a)
        if step % 500 == 0 or step == steps - 1:
            torch.cuda.synchronize()
            losses.append((step, float(net.loss.cpu().numpy()[0])))
            if log:
                log(f"step {step}: loss {losses[-1][1]:.5f} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return net, losses


def default_model(seed: int = 0, n_profiles: int = 128, pairs_per_profile: int = 8192,
                  steps: int = 6000, log=None):
    """The training recipe used by the tests and the benchmark."""
    data = generate(n_profiles, pairs_per_profile, seed=seed, log=log)
    net, losses = train(data, steps, seed=seed, log=log)
    return net, losses
