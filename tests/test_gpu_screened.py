"""GPU parity of the screened exchange terms (thcsox_static_screening and
thcsox_sigma_screened) against the oracle (oracle/screened.py): the statically
screened core W, SOSEX (one line screened, both placements) and G3W2 (both
lines) in all four plan precisions, on sizes that span several fused tiles and
a ragged one, with symmetric and non-symmetric G, the unscreened limit (W = V
reproduces SOX) and the end-to-end chain G -> W -> Sigma -> E.

Bars: FP64 1e-10 relative in Sigma and W (1e-12 for W from the same G), 1e-8
relative in energy; the mixed precisions 1e-6 relative in Sigma and energy, as
for the SOX path.
"""
import numpy as np
import pytest
import torch

from oracle import energy as oen
from oracle import screened as osc
from oracle import sox as osox
from paper_2404_17744_amd import synth, thcsox

pytestmark = pytest.mark.gpu
BETA = 100.0
TOL = {"fp64": 1e-10, "fp32": 1e-6, "bf16x3": 1e-6, "fp16x2": 1e-6}


def _case(n, naux, m, seed, general=False):
    s = synth.make_system(n, naux, seed=seed)
    tau, w = synth.cheb_tau_grid(m, BETA)
    G = synth.random_general_g(n, m, seed=seed + 1) if general else synth.g0_tau(s, tau, BETA)
    return s, tau, w, G


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("n,naux,m,general", [(8, 32, 12, False), (37, 150, 16, False),
                                              (23, 97, 8, True)])
def test_static_screening_matches_oracle(dev, n, naux, m, general):
    print(f"case static screening n{n} naux{naux} m{m} general={general}", flush=True)
    s, tau, w, G = _case(n, naux, m, seed=11, general=general)
    plan = thcsox.Plan(torch.from_numpy(s.X).to(dev), torch.from_numpy(s.V).to(dev), tau, w,
                       BETA, precision="fp64")
    W = plan.static_screening(torch.from_numpy(G).to(dev)).cpu().numpy()
    plan.close()
    ref = osc.screened_core(s.V, osc.static_polarization(s.X, G, w))
    err = _rel(W, ref)
    print(f"  W rel err {err:.2e}")
    assert err <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "fp16x2"])
@pytest.mark.parametrize("kind", ["sosex", "g3w2"])
def test_screened_sigma_matches_oracle(dev, precision, kind):
    n, naux, m = 37, 150, 16
    print(f"case screened {kind} {precision} n{n} naux{naux} m{m}", flush=True)
    s, tau, w, G = _case(n, naux, m, seed=5)
    W = osc.screened_core(s.V, osc.static_polarization(s.X, G, w))
    fn = osc.sigma_sosex if kind == "sosex" else (lambda X, V, W_, g, gb: osc.sigma_g3w2(X, W_, g, gb))
    ref = np.stack([fn(s.X, s.V, W, G[k], G[m - 1 - k]) for k in range(m)])
    plan = thcsox.Plan(torch.from_numpy(s.X).to(dev), torch.from_numpy(s.V).to(dev), tau, w,
                       BETA, precision=precision)
    Gd = torch.from_numpy(G).to(dev)
    S = plan.sigma_screened(Gd, torch.from_numpy(W).to(dev), kind)
    E = plan.energy(Gd, S)
    plan.close()
    Sn = S.cpu().numpy()
    E_ref = oen.energy_tau(G, ref, w)
    err = _rel(Sn, ref)
    print(f"  Sigma rel err {err:.2e}  E {E:.12f} oracle {E_ref:.12f}")
    assert err <= TOL[precision]
    assert abs(E - E_ref) <= (1e-8 if precision == "fp64" else 1e-6) * max(1.0, abs(E_ref))
    assert np.abs(Sn - Sn.transpose(0, 2, 1)).max() <= TOL[precision] * np.abs(Sn).max()


@pytest.mark.parametrize("kind", ["sosex", "g3w2"])
def test_screened_sigma_nonsymmetric_g(dev, kind):
    """A non-symmetric G: both placements differ beyond a transpose, and the
    symmetric-D path must stay off."""
    n, naux, m = 23, 97, 8
    print(f"case screened {kind} fp64 non-symmetric G n{n} naux{naux} m{m}", flush=True)
    s, tau, w, G = _case(n, naux, m, seed=3, general=True)
    rng = np.random.default_rng(4)
    L = rng.standard_normal((naux, naux))
    W = osc.screened_core(s.V, L @ L.T / naux)
    W = 0.5 * (W + W.T)
    fn = osc.sigma_sosex if kind == "sosex" else (lambda X, V, W_, g, gb: osc.sigma_g3w2(X, W_, g, gb))
    ref = np.stack([fn(s.X, s.V, W, G[k], G[m - 1 - k]) for k in range(m)])
    plan = thcsox.Plan(torch.from_numpy(s.X).to(dev), torch.from_numpy(s.V).to(dev), tau, w,
                       BETA, precision="fp64")
    S = plan.sigma_screened(torch.from_numpy(G).to(dev), torch.from_numpy(W).to(dev), kind)
    plan.close()
    err = _rel(S.cpu().numpy(), ref)
    print(f"  Sigma rel err {err:.2e}")
    assert err <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp16x2"])
def test_unscreened_limit_reproduces_sox(dev, precision):
    n, naux, m = 37, 150, 16
    print(f"case screened W = V {precision}", flush=True)
    s, tau, w, G = _case(n, naux, m, seed=6)
    plan = thcsox.Plan(torch.from_numpy(s.X).to(dev), torch.from_numpy(s.V).to(dev), tau, w,
                       BETA, precision=precision)
    Gd = torch.from_numpy(G).to(dev)
    Vd = torch.from_numpy(s.V).to(dev)
    S_sox = plan.sigma(Gd)
    S_g3 = plan.sigma_screened(Gd, Vd, "g3w2")
    S_so = plan.sigma_screened(Gd, Vd, "sosex")
    torch.cuda.synchronize()
    plan.close()
    # G3W2 with W = V runs the SOX kernels on an identical second U
    assert torch.equal(S_g3, S_sox)
    err = (S_so - S_sox).abs().max().item() / S_sox.abs().max().item()
    print(f"  SOSEX(W=V) vs SOX rel {err:.2e}")
    assert err <= (1e-12 if precision == "fp64" else 1e-6)


def test_end_to_end_chain(dev):
    """G -> W (library) -> SOSEX and G3W2 (library) -> energies, against the
    oracle's own chain, on the n = 8 / naux = 32 / 12-point workload and a
    tau slice that splits mirror pairs."""
    s, tau, w, G, beta = synth.workload("sox_n8_naux32_ntau12", seed=0)
    m = len(tau)
    print("case screened end-to-end n8 naux32 m12", flush=True)
    W_ref = osc.screened_core(s.V, osc.static_polarization(s.X, G, w))
    plan = thcsox.Plan(torch.from_numpy(s.X).to(dev), torch.from_numpy(s.V).to(dev), tau, w,
                       beta, precision="fp64")
    Gd = torch.from_numpy(G).to(dev)
    W = plan.static_screening(Gd)
    for kind, fn in (("sosex", lambda g, gb: osc.sigma_sosex(s.X, s.V, W_ref, g, gb)),
                     ("g3w2", lambda g, gb: osc.sigma_g3w2(s.X, W_ref, g, gb))):
        ref = np.stack([fn(G[k], G[m - 1 - k]) for k in range(m)])
        S = plan.sigma_screened(Gd, W, kind)
        part = torch.zeros_like(S)
        plan.sigma_screened(Gd, W, kind, 3, 8, out=part)
        E = plan.energy(Gd, S)
        Sn = S.cpu().numpy()
        assert _rel(Sn, ref) <= 1e-10
        assert np.array_equal(part.cpu().numpy()[3:8], Sn[3:8])
        assert abs(E - oen.energy_tau(G, ref, w)) <= 1e-10 * max(1.0, abs(E))
        E_sox = oen.energy_tau(G, osox.sigma_all_tau(osox.sigma_thc_paper, G, s.X, s.V), w)
        print(f"  {kind}: E {E:.10f}  (SOX {E_sox:.10f})")
    plan.close()
