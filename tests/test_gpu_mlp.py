"""GPU parity of the warm-start network's kernels against the FP64 oracle
(forward, gradients, one Adam step) and of the THC pair gather/scatter.

Tolerances: FP32 weights, activations and accumulation -> forward outputs
within 2e-5 of the FP64 reference relative to their largest value, gradients
within 1e-4 relative to the largest gradient entry of each parameter.
"""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from paper_2404_17744_amd import thcsox, warmstart

pytestmark = pytest.mark.gpu


def _case(m=64, H=128, B=300, seed=3):
    rng = np.random.default_rng(seed)
    p = warmstart.init_params(m, H, seed)
    p["W3"] = p["W3"] * 30.0   # a non-trivial residual branch
    p32 = {k: v.astype(np.float32) for k, v in p.items()}
    x = rng.standard_normal((B, m)).astype(np.float32)
    t = (x + 0.1 * rng.standard_normal((B, m))).astype(np.float32)
    return p32, x, t


def test_mlp_forward_matches_oracle(dev):
    p32, x, t = _case()
    print("case mlp forward m64 H128 B300", flush=True)
    net = thcsox.MLP(64, 128, p32, max_batch=128)   # exercises the batch chunking
    y = net.forward(torch.from_numpy(x).to(dev)).cpu().numpy()
    net.close()
    ref, _ = omlp.forward({k: v.astype(np.float64) for k, v in p32.items()}, x.astype(np.float64))
    assert np.abs(y - ref).max() / np.abs(ref).max() < 2e-5


def test_mlp_gradients_match_oracle(dev):
    p32, x, t = _case()
    print("case mlp gradients m64 H128 B300", flush=True)
    net = thcsox.MLP(64, 128, p32, max_batch=512)
    loss, g = net.gradients(torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev))
    net.close()
    lref, gref = omlp.loss_and_grads({k: v.astype(np.float64) for k, v in p32.items()},
                                     x.astype(np.float64), t.astype(np.float64))
    assert abs(loss - lref) < 1e-5 * lref
    for k in gref:
        err = np.abs(g[k] - gref[k]).max() / np.abs(gref[k]).max()
        assert err < 1e-4, (k, err)


def test_mlp_adam_step_matches_oracle(dev):
    p32, x, t = _case()
    print("case mlp adam m64 H128 B300", flush=True)
    net = thcsox.MLP(64, 128, p32, max_batch=512)
    xd, td = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    _, g = net.gradients(xd, td)
    net.train_step(xd, td, 1e-3)
    after = net.params()
    net.close()
    p64 = {k: v.astype(np.float64) for k, v in p32.items()}
    omlp.adam_step(p64, {k: v.astype(np.float64) for k, v in g.items()}, {}, lr=1e-3)
    for k in p64:
        step_ref = p64[k] - p32[k]
        step = after[k].astype(np.float64) - p32[k]
        # first Adam step moves each parameter by ~lr * sign(g): compare the steps
        assert np.abs(step - step_ref).max() < 2e-6, k


def test_mlp_adam_four_steps_match_oracle(dev):
    """Four training steps in a row: the moment accumulation and the bias
    correction at t >= 2.  Each step's gradients are read back from the GPU at
    the GPU's current parameters and fed to the oracle's Adam, so the check
    isolates the update rule from the FP32 gradient rounding.  The first two
    steps are long (lr 0.05) so that the parameters move and later gradients
    differ from the first; the moments then mix gradients of both signs."""
    p32, x, t = _case()
    print("case mlp adam x4 m64 H128 B300", flush=True)
    net = thcsox.MLP(64, 128, p32, max_batch=512)
    xd, td = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    p64 = {k: v.astype(np.float64) for k, v in p32.items()}
    state = {}
    for step in range(4):
        before = net.params()
        _, g = net.gradients(xd, td)
        lr = 0.05 if step < 2 else 1e-3
        net.train_step(xd, td, lr)
        after = net.params()
        omlp.adam_step(p64, {k: v.astype(np.float64) for k, v in g.items()}, state, lr=lr)
        for k in p64:
            # compare this step's update, taken from the same starting point
            step_gpu = after[k].astype(np.float64) - before[k]
            step_ref = p64[k] - before[k]
            assert np.abs(step_gpu - step_ref).max() < 2e-6 * max(1.0, lr / 1e-3), (step, k)
            p64[k] = after[k].astype(np.float64)   # follow the GPU's FP32 parameters
    assert state["t"] == 4
    net.close()


def test_pair_gather_scatter_roundtrip(dev):
    m, A = 8, 40
    rng = np.random.default_rng(0)
    S = torch.from_numpy(rng.standard_normal((m, A, A))).to(dev)
    S[:, 3, 7] = 0.0                                  # an all-zero pair keeps scale 1
    scale = warmstart.pair_scale(S)
    Sn = S.cpu().numpy().reshape(m, -1)
    ref_scale = np.abs(Sn).max(0)
    ref_scale[ref_scale == 0] = 1.0
    np.testing.assert_allclose(scale.cpu().numpy(), ref_scale)
    x = warmstart.pair_profiles(S, scale)
    assert x.shape == (A * A, m)
    ref = (Sn / ref_scale[None, :]).T
    assert np.abs(x.cpu().numpy() - ref).max() < 1e-7
    assert np.abs(x.cpu().numpy()).max() <= 1.0
    back = torch.empty_like(S)
    thcsox.thcsox_pair_scatter(m, A, x.data_ptr(), scale.data_ptr(), back.data_ptr(),
                               torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert (back - S).abs().max().item() < 1e-6 * S.abs().max().item()
    pairs = torch.tensor([0, 5, A * A - 1], dtype=torch.int64, device=dev)
    xs = warmstart.pair_profiles(S, scale, pairs).cpu().numpy()
    assert np.abs(xs - ref[[0, 5, A * A - 1]]).max() < 1e-7


@pytest.mark.parametrize("m,H,B", [(64, 512, 300), (32, 128, 77), (64, 256, 64)])
def test_mlp_forward_bf16_matches_oracle(dev, m, H, B):
    """The fused bf16 inference kernel against the oracle's forward_bf16 (the
    same roundings, exact sums): FP32 accumulation, the device exp in silu and
    the rare bf16 rounding flip of a hidden value that these cause keep the
    difference under half a bf16 unit of the residual branch; the full-precision
    forward is farther away (the bf16 roundings themselves)."""
    p32, x, _ = _case(m=m, H=H, B=B)
    rng = np.random.default_rng(m + H)
    for k in ("b1", "b2", "b3"):   # non-zero biases
        p32[k] = (0.3 * rng.standard_normal(p32[k].shape)).astype(np.float32)
    print(f"case mlp forward bf16 m{m} H{H} B{B}", flush=True)
    net = thcsox.MLP(m, H, p32, max_batch=64)
    xd = torch.from_numpy(x).to(dev)
    y = net.forward_bf16(xd).cpu().numpy()
    net.close()
    p64 = {k: v.astype(np.float64) for k, v in p32.items()}
    ref = omlp.forward_bf16(p64, x.astype(np.float64))
    full, _ = omlp.forward(p64, x.astype(np.float64))
    branch = np.abs(full - x).max()
    err, dist = np.abs(y - ref).max(), np.abs(full - ref).max()
    print(f"  max |gpu - oracle bf16| {err / branch:.2e}, |oracle bf16 - FP64 forward| "
          f"{dist / branch:.2e} (relative to the branch)")
    assert err <= 2.0 ** -9 * branch
    assert dist > 4 * err


def test_mlp_forward_bf16_edges_and_refresh(dev):
    """Batch 0 is a no-op, unsupported widths are refused, a large ragged batch
    matches the FP32 forward to bf16 accuracy, and after a training step the
    bf16 copy follows the new parameters."""
    from paper_2404_17744_amd.thcsox import ThcsoxError
    p32, x, t = _case(m=64, H=512, B=256)
    net = thcsox.MLP(64, 512, p32, max_batch=256)
    print("case mlp forward bf16 edges", flush=True)
    empty = torch.empty((0, 64), dtype=torch.float32, device=dev)
    assert net.forward_bf16(empty).shape == (0, 64)
    rng = np.random.default_rng(9)
    big = torch.from_numpy(rng.standard_normal((100003, 64)).astype(np.float32)).to(dev)
    yb, yf = net.forward_bf16(big), net.forward(big)
    branch = (yf - big).abs().max().item()
    assert (yb - yf).abs().max().item() <= 8 * 2.0 ** -8 * branch
    sel = [0, 63, 64, 50000, 100002]
    ref = omlp.forward_bf16({k: v.astype(np.float64) for k, v in p32.items()},
                            big[sel].cpu().numpy().astype(np.float64))
    assert np.abs(yb[sel].cpu().numpy() - ref).max() <= 2.0 ** -9 * branch
    xd, td = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    net.train_step(xd, td, 1e-2)
    p_new = {k: v.astype(np.float64) for k, v in net.params().items()}
    y2 = net.forward_bf16(xd).cpu().numpy()
    ref2 = omlp.forward_bf16(p_new, x.astype(np.float64))
    assert np.abs(y2 - ref2).max() <= 2.0 ** -9 * branch
    net.close()
    with pytest.raises(ThcsoxError):
        odd = thcsox.MLP(48, 128, {k: v for k, v in _case(m=48, H=128, B=4)[0].items()})
        try:
            odd.forward_bf16(torch.zeros((4, 48), dtype=torch.float32, device=dev))
        finally:
            odd.close()
