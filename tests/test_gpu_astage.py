"""GPU parity of the fp16x2, bf16x3 and FP32 A stages, A_Pqv = sum_s U_Pqs G_sv(beta - tau), at the
orbital counts that select each of its kernels, through Sigma (every element
of A enters it) against the oracle's THC-SOX sequence.

The A stage keeps G(beta - tau) in registers while the padded orbital count
ldk = 64 ceil(n / 64) is at most 320 (one kernel per number of 32-wide k
chunks, 2 .. 10), and streams both operands through LDS beyond that:

* n = 200 and n = 256: eight k chunks (n = 256 with no padding: every column
  and row of the last chunk is real);
* n = 320: ten chunks, no padding (the last 32-row step of every P is full);
* n = 321: ldk = 384, the streaming kernel (one padded chunk of 31 columns
  past its first 320-column block).

An odd tau count leaves the last A-stage launch with a single tau point (the
launch forms two at a time).  naux = 3 (in every mode) leaves most of the
persistent workers without a step and some XCDs without a range.  The smaller counts (n = 1 .. 150 and 300) are in
the edge, parity and full-size tests.  Bar: 2e-6 of max |Sigma|, as the other
split-precision parity tests.

The bf16x3 A stage keeps G(beta - tau) in registers while ldk = 32 ceil(n / 32)
is at most 320: one kernel per chunk count 1 .. 10, with the 16-column tiles in
one block of up to 12 (n <= 192: 1, 2 or 3 tiles per wave) or in two blocks
(12 tiles and 1 or 2 tiles per wave).  The cases cover every chunk count, both
block splits, a block of exactly 12 tiles (n = 192), full and ragged last
tiles, steps wholly past n (32 ceil(n / 32) - n >= 16) and the streaming kernel
beyond (n = 321).  Bar: 2e-7 of max |Sigma| (the bf16x3 path reaches 1e-8 to
5e-8 at these sizes, a few 1e-9 at naux = 1800; one dropped plane product or a
wrong plane costs about 2^-16), and 2e-6 at naux = 3, where no sum over THC
points averages the FP32 accumulation's rounding: there fp16x2, FP32 and bf16x3
all measure about 1e-7 (the floor every split mode shares; their other tests
hold 2e-6).

The FP32 A stage runs the fp16x2 register kernel's FP32 form while ldk =
32 ceil(n / 32) is a multiple of 64 up to 320 (2, 4, 6, 8 or 10 k chunks),
and the streaming kernel otherwise (n = 150: ldk = 160; n = 321).  Bar: 2e-6
of max |Sigma|, as the other FP32 parity tests.
"""
import numpy as np
import pytest
import torch

from oracle import sox as osox
from paper_2404_17744_amd import synth, thcsox

pytestmark = pytest.mark.gpu

TOL = 2e-6
BETA = 100.0
CASES = [(200, 72, 3), (256, 40, 2), (320, 56, 3), (321, 48, 3), (300, 3, 3)]


@pytest.mark.parametrize("case", CASES, ids=[f"n{a}_naux{b}_ntau{c}" for a, b, c in CASES])
def test_astage_kernels_fp16x2(dev, case):
    n, naux, ntau = case
    print(f"case n{n} naux{naux} ntau{ntau} fp16x2 A stage", flush=True)
    s = synth.make_system(n, naux, seed=40 + n)
    tau, w = synth.cheb_tau_grid(ntau, BETA)
    G = synth.g0_tau(s, tau, BETA)
    ref = osox.sigma_all_tau(osox.sigma_thc_paper, G, s.X, s.V)
    plan = thcsox.Plan(torch.from_numpy(s.X).to(dev), torch.from_numpy(s.V).to(dev), tau, w,
                       BETA, precision="fp16x2")
    S = plan.sigma(torch.from_numpy(G).to(dev))
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    plan.close()
    assert np.isfinite(S).all()
    for k in range(ntau):
        err = float(np.abs(S[k] - ref[k]).max() / np.abs(ref[k]).max())
        print(f"  tau {k}: rel err {err:.2e}", flush=True)
        assert err <= TOL


BF3_TOL = 2e-7
BF3_CASES = [(20, 37, 2), (50, 40, 2), (96, 44, 2), (128, 40, 2), (150, 48, 2), (192, 40, 2),
             (200, 52, 2), (256, 40, 2), (270, 46, 2), (289, 40, 2), (320, 56, 2), (321, 48, 2),
             (300, 3, 2)]


@pytest.mark.parametrize("case", BF3_CASES, ids=[f"n{a}_naux{b}_ntau{c}" for a, b, c in BF3_CASES])
def test_astage_kernels_bf16x3(dev, case):
    n, naux, ntau = case
    print(f"case n{n} naux{naux} ntau{ntau} bf16x3 A stage", flush=True)
    s = synth.make_system(n, naux, seed=60 + n)
    tau, w = synth.cheb_tau_grid(ntau, BETA)
    G = synth.g0_tau(s, tau, BETA)
    ref = osox.sigma_all_tau(osox.sigma_thc_paper, G, s.X, s.V)
    plan = thcsox.Plan(torch.from_numpy(s.X).to(dev), torch.from_numpy(s.V).to(dev), tau, w,
                       BETA, precision="bf16x3")
    S = plan.sigma(torch.from_numpy(G).to(dev))
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    plan.close()
    assert np.isfinite(S).all()
    for k in range(ntau):
        err = float(np.abs(S[k] - ref[k]).max() / np.abs(ref[k]).max())
        print(f"  tau {k}: rel err {err:.2e}", flush=True)
        assert err <= (BF3_TOL if naux >= 32 else 2e-6)


F32_TOL = 2e-6
F32_CASES = [(40, 37, 2), (100, 44, 3), (150, 40, 2), (180, 48, 2), (250, 40, 2), (300, 52, 2),
             (320, 40, 2), (321, 44, 2), (300, 3, 2)]


@pytest.mark.parametrize("case", F32_CASES, ids=[f"n{a}_naux{b}_ntau{c}" for a, b, c in F32_CASES])
def test_astage_kernels_fp32(dev, case):
    n, naux, ntau = case
    print(f"case n{n} naux{naux} ntau{ntau} fp32 A stage", flush=True)
    s = synth.make_system(n, naux, seed=80 + n)
    tau, w = synth.cheb_tau_grid(ntau, BETA)
    G = synth.g0_tau(s, tau, BETA)
    ref = osox.sigma_all_tau(osox.sigma_thc_paper, G, s.X, s.V)
    plan = thcsox.Plan(torch.from_numpy(s.X).to(dev), torch.from_numpy(s.V).to(dev), tau, w,
                       BETA, precision="fp32")
    S = plan.sigma(torch.from_numpy(G).to(dev))
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    plan.close()
    assert np.isfinite(S).all()
    for k in range(ntau):
        err = float(np.abs(S[k] - ref[k]).max() / np.abs(ref[k]).max())
        print(f"  tau {k}: rel err {err:.2e}", flush=True)
        assert err <= F32_TOL
