"""GPU parity of the surrogate network's kernels (BF16 matrix cores, FP32
accumulation) against the FP64 reference in oracle/mlp.py.

Bars.  The reference is evaluated at the GPU's BF16-rounded weights and
inputs, and (``emulate``) rounds to BF16 exactly what the GPU stores in BF16:
hidden activations and the gradients w.r.t. pre-activations.  What remains is
FP32 accumulation (relative ~1e-7 over K <= 8192 products) and the rare BF16
rounding that lands on the other side of a tie because of it: one BF16 ulp
(2^-8 relative) in a small fraction of elements, each carried to the outputs
with the network's gain.  Outputs: RMS difference <= 1e-3 of the outputs'
RMS (flips are rare), largest difference <= 2e-2 of it (a few flips in one
row).  Gradients: per layer, norm of the difference <= 3e-3 of the layer's
gradient norm.  Without emulation (FP64 activations) the same measures must
hold to 1e-2 / 6e-2 / 3e-2: four layers of up to 2^-9 relative rounding.
A wrong operand layout or a missing term gives differences of order one.
"""
import numpy as np
import pytest

from oracle import mlp as M
from paper_1810_01780_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_01780_amd import binding
    binding.lib()
    return binding


def _data(B, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, 5)).astype(np.float32)
    t = rng.standard_normal((B, 8)).astype(np.float32)
    m = (rng.random((B, 4)) < 0.6).astype(np.float32)
    return x, t, m


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("B", [1, 127, 128, 129, 1000, 65536 + 77])
def test_fused_forward_equals_layer_launches(gpu, B):
    """The one-launch forward (activations kept in LDS per 128-row tile)
    against one launch per layer: the same MFMA products in the same order
    and the same epilogues, so every output bit for bit, for batches below,
    at and above one tile and a ragged last tile."""
    import torch
    print(f"\n[gpu-case] mlp-fused B={B}", flush=True)
    p = W.mlp_init_params(11)
    p[-12:] = 0.05
    net = gpu.DeviceMLP(p, max_batch=B, training=False)
    x, _, _ = _data(B, seed=B + 3)
    xd = _dev(x * 2.0)
    y1 = torch.full((B, 12), -7.0, dtype=torch.float32, device="cuda")
    y2 = torch.full((B, 12), -9.0, dtype=torch.float32, device="cuda")
    net.forward(xd, y1)
    net.forward(xd, y2, layers=True)
    torch.cuda.synchronize()
    a, b = y1.cpu().numpy(), y2.cpu().numpy()
    assert np.isfinite(a).all()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), np.abs(a - b).max()


@pytest.mark.parametrize("B", [1, 37, 1000, 4096])
def test_forward_matches_reference(gpu, B):
    import torch
    print(f"\n[gpu-case] mlp-forward B={B}", flush=True)
    p = W.mlp_init_params(7)
    p[-12:] = 0.1  # non-zero output biases
    net = gpu.DeviceMLP(p, max_batch=B, training=False)
    x, _, _ = _data(B, seed=B)
    y = torch.zeros((B, 12), dtype=torch.float32, device="cuda")
    net.forward(_dev(x), y)
    torch.cuda.synchronize()
    g = y.cpu().numpy().astype(np.float64)
    ref_e, _ = M.forward(p, x, bf16=True, act_bf16=True)
    ref, _ = M.forward(p, x, bf16=True)
    rms = np.sqrt(np.mean(ref ** 2))
    rms_e, max_e = np.sqrt(np.mean((g - ref_e) ** 2)) / rms, np.abs(g - ref_e).max() / rms
    rms_f, max_f = np.sqrt(np.mean((g - ref) ** 2)) / rms, np.abs(g - ref).max() / rms
    print(f"[gpu-case] mlp-forward B={B}: rms {rms:.3g}; emulated rms {rms_e:.2e} max "
          f"{max_e:.2e}; fp64 rms {rms_f:.2e} max {max_f:.2e}", flush=True)
    assert rms_e <= 1e-3 and max_e <= 2e-2
    assert rms_f <= 1e-2 and max_f <= 6e-2


@pytest.mark.parametrize("B", [48, 1000, 4096, 16384])
def test_gradients_match_reference(gpu, B):
    print(f"\n[gpu-case] mlp-gradients B={B}", flush=True)
    p = W.mlp_init_params(8)
    net = gpu.DeviceMLP(p, max_batch=B, training=True)
    x, t, m = _data(B, seed=100 + B)
    net.gradients(_dev(x), _dev(t), _dev(m))
    import torch
    torch.cuda.synchronize()
    gg = net.grad.cpu().numpy().astype(np.float64)
    gl = float(net.loss.cpu().numpy()[0])
    le, ge = M.gradients(p, x, t, m, bf16=True, emulate=True)
    lf, gf = M.gradients(p, x, t, m, bf16=True, emulate=False)
    assert gl == pytest.approx(le, rel=1e-4)
    lay, _ = M.layout()
    worst_e = worst_f = 0.0
    for w, b, ni, no in lay:
        sl = slice(w, b + no)
        n = np.linalg.norm(ge[sl])
        worst_e = max(worst_e, np.linalg.norm(gg[sl] - ge[sl]) / n)
        worst_f = max(worst_f, np.linalg.norm(gg[sl] - gf[sl]) / np.linalg.norm(gf[sl]))
    print(f"[gpu-case] mlp-gradients B={B}: loss {gl:.6g} vs {le:.6g}; layer-norm rel. error "
          f"emulated {worst_e:.2e}, fp64 {worst_f:.2e}", flush=True)
    assert worst_e <= 3e-3 and worst_f <= 3e-2


def test_adam_matches_reference(gpu):
    import torch
    print("\n[gpu-case] mlp-adam", flush=True)
    p = W.mlp_init_params(9)
    net = gpu.DeviceMLP(p, max_batch=16, training=True)
    rng = np.random.default_rng(1)
    n = p.size
    pr, mr, vr = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 4):
        g = (rng.standard_normal(n) * 10.0 ** rng.uniform(-6, 0, n)).astype(np.float32)
        net.grad.copy_(_dev(g))
        net.adam(lr=1e-3)
        pr, mr, vr = M.adam(pr, mr, vr, g.astype(np.float64), step, 1e-3)
    torch.cuda.synchronize()
    pg = net.params.cpu().numpy().astype(np.float64)
    assert np.abs(pg - pr).max() <= 1e-6 * np.abs(pr).max() + 1e-8


def test_training_reduces_loss(gpu):
    """A smooth synthetic regression task: 300 Adam steps on the GPU cut the
    loss by more than 5x."""
    import torch
    print("\n[gpu-case] mlp-train", flush=True)
    B = 2048
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (B * 4, 5)).astype(np.float32)
    t = np.stack([np.sin(2 * x[:, 0]) * x[:, 1], x[:, 2] ** 2, np.cos(x[:, 3]), x[:, 4],
                  x[:, 0] * x[:, 4], np.tanh(x[:, 1] + x[:, 2]), x[:, 3] - x[:, 0], x[:, 1]],
                 axis=1).astype(np.float32)
    m = np.stack([x[:, 0] > -0.5, x[:, 1] + x[:, 2] > 0, x[:, 3] > 0.5, x[:, 4] < -0.5],
                 axis=1).astype(np.float32)
    net = gpu.DeviceMLP(W.mlp_init_params(10), max_batch=B, training=True)
    xd, td, md = _dev(x), _dev(t), _dev(m)
    losses = []
    for step in range(300):
        i = (step % 4) * B
        net.train_step(xd[i:i + B], td[i:i + B], md[i:i + B], lr=2e-3)
        if step % 50 == 0 or step == 299:
            torch.cuda.synchronize()
            losses.append(float(net.loss.cpu().numpy()[0]))
    print(f"[gpu-case] mlp-train: losses {losses}", flush=True)
    assert losses[-1] < losses[0] / 5
