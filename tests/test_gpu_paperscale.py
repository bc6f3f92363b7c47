"""The paper-scale one-GPU share (n=1100, naux=5500, 100 tau points, seed 0).

The FP64 oracle cannot run here at this size (U alone is 53 GB in FP64), so the
checks are properties that hold at any size, with the GPU FP64 path as the
reference (it matches the oracle to 1e-10 at n=8, 100 and 300):

* the fp16x2 path (in the configuration the throughput measurement uses)
  against the FP64 path on two tau points: 1e-6 relative in Sigma;
* the FP32 and bf16x3 paths against the FP64 path on the same points, 1e-6
  (their fused kernels with FP64 partial tiles over ranges of more than 8 v,
  and the A stage's kernels for ldk > 320);
* Sigma(tau) symmetric for the symmetric inputs;
* the symmetric-D path against the full path;
* homogeneity Sigma[c G] = c^3 Sigma[G] (c a power of two, so exact up to the
  rounding of the contraction);
* sampled Sig_thc elements of the fp16x2 path against the oracle's sequence
  evaluated one (R, P) pair at a time (which needs only the P and R slices of
  U), across tile boundaries, both triangles and the ragged last tile
  (5500 = 42 * 128 + 124): 1e-6 of the largest sampled magnitude.
"""
import numpy as np
import pytest
import torch

from oracle import sox as osox
from paper_2404_17744_amd import synth, thcsox

pytestmark = pytest.mark.gpu
NAME = "sox_n1100_naux5500_ntau100"
KS = (0, 37)


@pytest.fixture(scope="module")
def case(dev):
    print(f"case {NAME} seed 0: generating inputs", flush=True)
    s, tau, w, G, beta = synth.workload(NAME, seed=0)
    return dict(s=s, tau=tau, w=w, beta=beta, G=torch.from_numpy(G).to(dev),
                X=torch.from_numpy(s.X).to(dev), V=torch.from_numpy(s.V).to(dev))


def _sigma(case, precision, sym="auto", scale=1.0):
    plan = thcsox.Plan(case["X"], case["V"], case["tau"], case["w"], case["beta"],
                       precision=precision)
    info = plan.info()
    # ranges of 8 v would need 144 partial tiles of 5500^2 (17 GB in FP32): the plan
    # falls back to longer ranges with FP64 partial tiles flushed every 8 v
    assert info["partial_f32"] == 0 and info["vrange"] > 8
    plan.set_symmetry(sym)
    G = case["G"] * scale if scale != 1.0 else case["G"]
    out = torch.zeros_like(case["G"])
    for k in KS:
        plan.sigma(G, k, k + 1, out=out)
    torch.cuda.synchronize()
    plan.close()
    return out[list(KS)].cpu().numpy()


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_paperscale_mixed_vs_fp64(case):
    print(f"case {NAME} fp64 k={KS}", flush=True)
    S64 = _sigma(case, "fp64")
    print(f"case {NAME} fp16x2 k={KS}", flush=True)
    S16 = _sigma(case, "fp16x2")
    err = _rel(S16, S64)
    print(f"  fp16x2 vs fp64 max rel {err:.2e}")
    assert err <= 1e-6
    assert _rel(S64, np.transpose(S64, (0, 2, 1))) <= 1e-12
    assert _rel(S16, np.transpose(S16, (0, 2, 1))) <= 1e-6
    case["S16"] = S16
    case["S64"] = S64


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_paperscale_fp32_bf16x3_vs_fp64(case, precision):
    S64 = case.get("S64")
    if S64 is None:
        print(f"case {NAME} fp64 k={KS}", flush=True)
        S64 = case["S64"] = _sigma(case, "fp64")
    print(f"case {NAME} {precision} k={KS}", flush=True)
    S = _sigma(case, precision)
    err = _rel(S, S64)
    print(f"  {precision} vs fp64 max rel {err:.2e}")
    assert err <= 1e-6


def test_paperscale_symmetric_path_and_homogeneity(case):
    print(f"case {NAME} fp16x2 full path", flush=True)
    S_full = _sigma(case, "fp16x2", sym="off")
    S_sym = case.get("S16")
    if S_sym is None:
        S_sym = _sigma(case, "fp16x2")
    assert _rel(S_sym, S_full) <= 1e-6
    print(f"case {NAME} fp16x2 G scaled by 2", flush=True)
    S2 = _sigma(case, "fp16x2", scale=2.0)
    # the per-tau power-of-two scaling absorbs the factor: the same bits, times 8
    assert _rel(S2, 8.0 * S_sym) <= 1e-12


def test_paperscale_sampled_sig_thc_vs_oracle(case):
    s, m = case["s"], len(case["tau"])
    naux = s.naux
    print(f"case {NAME} fp16x2 Sig_thc k=0,1 vs oracle elements", flush=True)
    plan = thcsox.Plan(case["X"], case["V"], case["tau"], case["w"], case["beta"],
                       precision="fp16x2")
    out = torch.zeros_like(case["G"])
    St = torch.zeros((2, naux, naux), dtype=torch.float64, device=case["G"].device)
    plan.sigma(case["G"], 0, 2, thc=True, out=out, out_thc=St)
    torch.cuda.synchronize()
    plan.close()
    last = naux - 1
    pairs = [(0, 0), (last, last), (last, 0), (0, last), (127, 128), (128, 127),
             (5376, 17), (17, 5376), (2750, 2750), (1000, 4000), (4000, 1000)]
    rng = np.random.default_rng(9)
    pairs += [tuple(int(x) for x in rng.integers(0, naux, 2)) for _ in range(5)]
    G = case["G"].cpu().numpy()
    for k in range(2):
        ref = osox.sig_thc_elements(s.X, s.V, G[k], G[m - 1 - k], pairs)
        got = St[k].cpu().numpy()
        vals = np.array([got[R, P] for R, P in pairs])
        err = float(np.abs(vals - ref).max() / np.abs(ref).max())
        print(f"  k={k}: rel err {err:.2e} over {len(pairs)} elements")
        assert err <= 1e-6
