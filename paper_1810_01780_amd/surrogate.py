"""Training and use of the solve surrogate, through the C ABI only.

Data: the tracer's full solves (raytrace_solve) of seeded pairs in seeded
firn profiles; features, targets and labels (a solution exists; more than
one root) are formed on the GPU by rt_surrogate_features /
rt_surrogate_targets.  Training: rt_mlp_gradients
and rt_mlp_adam (BF16 matrix cores, FP32 Adam) on minibatches of the
shuffled set, cosine learning-rate decay.  Use: raytrace_solve_surrogate,
which seeds the entries the network predicts to have one root, verifies each
seed by shooting and hands every other entry to the tracer.
"""
from __future__ import annotations

import math
import time
from typing import Dict, Optional

import numpy as np

from . import binding as B
from . import workloads as W


class _SolveSlot:
    """Outputs and workspace of one profile solve in flight on its own
    stream (default priority); reused for the next profile on that stream."""

    def __init__(self, n: int, field, params, dev):
        import torch
        self.torch = torch
        self.stream = torch.cuda.Stream(device=dev)
        self.n = n
        self.res = {f: torch.zeros(2 * n, dtype=torch.int32, device=dev) for f in B.SOLVE_I32}
        self.res.update({f: torch.zeros(2 * n, dtype=torch.float64, device=dev)
                         for f in B.SOLVE_F64})
        self.stats = torch.zeros(len(B.SOLVE_STAT_FIELDS), dtype=torch.int64, device=dev)
        self.out = B.rt_solve_outputs(*([self.res[f].data_ptr() for f in B.SOLVE_I32 + B.SOLVE_F64]
                                        + [self.stats.data_ptr()]))
        self.params = params
        self.ws_bytes = B.rt_solve_workspace_bytes(field, n, params)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)

    def run(self, scene, z0, dn, zs, zr, dist, x, t, m):
        """Enqueue the tracer's solve of the pairs (device views) in the
        profile's medium, then the features and targets of its rows."""
        desc = B.HostDescriptors(scene)
        pairs = B.rt_pairs(zs.data_ptr(), zr.data_ptr(), dist.data_ptr(), self.n)
        h = self.stream.cuda_stream
        st = B.raytrace_solve(desc.field, desc.bnd, desc.tol, desc.limits, pairs, self.params,
                              self.out, self.ws.data_ptr(), self.ws_bytes, h, None)
        st = st or B.rt_surrogate_features(pairs, z0, dn, x.data_ptr(), h)
        st = st or B.rt_surrogate_targets(self.out, self.n, t.data_ptr(), m.data_ptr(), h)
        if st != B.RT_OK:
            raise B.RTError(st, B.rt_last_error())


def generate(n_profiles: int, pairs_per_profile: int, seed: int = 0,
             model: int = W.MODEL_PAPER, streams: int = 4, log=None) -> Dict[str, "torch.Tensor"]:
    """Training set on the GPU: x [N][5], t [N][8], labels m [N][4] (FP32),
    rows shuffled with a seeded permutation; N = n_profiles *
    pairs_per_profile.  Each profile is one tracer solve (raytrace_solve);
    'streams' profiles are solved at a time, each on a stream of its own, so
    that the latency-bound tails of their refinements overlap."""
    import torch
    dev = torch.device("cuda")
    N = n_profiles * pairs_per_profile
    x = torch.empty((N, 5), dtype=torch.float32, device=dev)
    t = torch.empty((N, 8), dtype=torch.float32, device=dev)
    m = torch.empty((N, 4), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    profiles = W.surrogate_training_set(n_profiles, pairs_per_profile, seed)
    cols = [torch.as_tensor(np.concatenate([p[i] for p in profiles]), device=dev)
            for i in (2, 3, 4)]  # zs, zr, dist of every row
    torch.cuda.synchronize()
    params = B.solve_params()
    field0 = B.HostDescriptors(W.two_layer_medium(model=model)).field
    slots = [_SolveSlot(pairs_per_profile, field0, params, dev) for _ in range(streams)]
    torch.cuda.synchronize()  # the slots' buffers are cleared on the current stream
    for k, (z0, dn, _, _, _) in enumerate(profiles):
        r0, r1 = k * pairs_per_profile, (k + 1) * pairs_per_profile
        slots[k % streams].run(W.two_layer_medium(z0, dn, model=model), z0, dn,
                               *(c[r0:r1] for c in cols), x[r0:r1], t[r0:r1], m[r0:r1])
    torch.cuda.synchronize()
    found = int(m[:, :2].sum().item())
    multi = int(m[:, 2:].sum().item())
    perm = torch.as_tensor(np.random.default_rng(seed).permutation(N), device=dev)
    data = {"x": x.index_select(0, perm).contiguous(), "t": t.index_select(0, perm).contiguous(),
            "m": m.index_select(0, perm).contiguous()}
    if log:
        log(f"training set: {N} pairs in {n_profiles} profiles, {found} of {2 * N} entries "
            f"solved ({multi} with more than one root), {time.perf_counter() - t0:.1f} s")
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


def default_model(seed: int = 0, n_profiles: int = 2048, pairs_per_profile: int = 8192,
                  steps: int = 8000, batch: int = 16384, log=None):
    """The training recipe: 2,048 seeded profiles x 8,192 pairs (16.8 M
    tracer-solved pairs), 8,000 Adam steps of 16,384 rows (about 8 passes);
    the tests use fewer profiles and steps."""
    data = generate(n_profiles, pairs_per_profile, seed=seed, log=log)
    net, losses = train(data, steps, batch=batch, seed=seed, log=log)
    return net, losses
