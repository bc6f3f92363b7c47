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
