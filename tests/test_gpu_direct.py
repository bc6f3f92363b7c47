"""GPU parity of the GF2 direct (bubble) self-energy against the oracle's THC
form (itself pinned to the six-index definition and to the MP2 Coulomb limit)."""
import numpy as np
import pytest
import torch

from oracle import direct as od
from oracle import energy as oenergy
from oracle import sox as osox
from paper_2404_17744_amd import synth, thcsox

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _plan(dev, s, tau, w, beta, precision="fp64"):
    return thcsox.Plan(torch.from_numpy(s.X).to(dev), torch.from_numpy(s.V).to(dev), tau, w,
                       beta, precision=precision)


def test_direct_general_g_ragged(dev):
    """n=40, naux=150 (partial 32-wide transpose tiles), non-symmetric G, 8 tau."""
    s = synth.make_system(40, 150, seed=21)
    tau, w = synth.cheb_tau_grid(8, 100.0)
    G = synth.random_general_g(40, 8, seed=22)
    print("case direct n40 naux150 ntau8 general G", flush=True)
    ref = osox.sigma_all_tau(od.sigma_direct_thc, G, s.X, s.V)
    plan = _plan(dev, s, tau, w, 100.0)
    Gd = torch.from_numpy(G).to(dev)
    S = plan.sigma_direct(Gd)
    # tau slices compose
    S2 = torch.zeros_like(S)
    plan.sigma_direct(Gd, 0, 3, out=S2)
    plan.sigma_direct(Gd, 3, 8, out=S2)
    torch.cuda.synchronize()
    plan.close()
    assert _rel(S.cpu().numpy(), ref) <= 1e-12
    assert torch.equal(S, S2)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "fp16x2"])
def test_direct_and_full_gf2_energy(dev, precision):
    """G0 of the n=90, naux=400 system (12 tau): Sigma^dir (FP64 in every plan
    precision), its energy, and the full second-order energy with SOX."""
    s = synth.make_system(90, 400, seed=11)
    tau, w = synth.cheb_tau_grid(12, 100.0)
    G = synth.g0_tau(s, tau, 100.0)
    print(f"case direct n90 naux400 ntau12 G0 plan {precision}", flush=True)
    ref = osox.sigma_all_tau(od.sigma_direct_thc, G, s.X, s.V)
    ref_x = osox.sigma_all_tau(osox.sigma_thc_paper, G, s.X, s.V)
    plan = _plan(dev, s, tau, w, 100.0, precision)
    Gd = torch.from_numpy(G).to(dev)
    Sd = plan.sigma_direct(Gd)
    Sx = plan.sigma(Gd)
    E_d = plan.energy(Gd, Sd)
    plan.sigma_direct(Gd, out=Sx, accumulate=True)   # Sx now holds direct + SOX
    E_tot = plan.energy(Gd, Sx)
    plan.close()
    Ed_ref = oenergy.energy_tau(G, ref, w)
    Ex_ref = oenergy.energy_tau(G, ref_x, w)
    assert _rel(Sd.cpu().numpy(), ref) <= 1e-12
    assert abs(E_d - Ed_ref) <= 1e-10 * max(1.0, abs(Ed_ref))
    assert E_d < 0.0
    tol = 1e-10 if precision == "fp64" else 1e-6
    assert abs(E_tot - (Ed_ref + Ex_ref)) <= tol * max(1.0, abs(Ed_ref + Ex_ref))


def test_direct_fullsize_sampled(dev):
    """n=300, naux=1800, 100 tau (the throughput workload): two tau points against
    the oracle's THC form."""
    name = "sox_n300_naux1800_ntau100"
    s, tau, w, G, beta = synth.workload(name, seed=0)
    print(f"case direct {name} k=0,37", flush=True)
    plan = _plan(dev, s, tau, w, beta, "fp16x2")
    Gd = torch.from_numpy(G).to(dev)
    S = torch.zeros_like(Gd)
    for k in (0, 37):
        plan.sigma_direct(Gd, k, k + 1, out=S)
    torch.cuda.synchronize()
    plan.close()
    m = len(tau)
    for k in (0, 37):
        ref = od.sigma_direct_thc(s.X, s.V, G[k], G[m - 1 - k])
        assert _rel(S[k].cpu().numpy(), ref) <= 1e-11, k


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "fp16x2"])
def test_single_spin_orbital_direct_cancels_sox(dev, precision):
    """n = 1 (one v, a k row padded to the full stage width, v ranges left empty),
    naux = 37 (one ragged tile): the SOX term against the oracle, and the direct
    term equal to minus the SOX term (Pauli: one spin-orbital holds one electron)."""
    X, V = synth.thc_factors(1, 37, seed=11)
    G = synth.random_general_g(1, 8, seed=1)
    tau, w = synth.cheb_tau_grid(8, 100.0)
    print(f"case n1 naux37 ntau8 {precision}", flush=True)
    ref = osox.sigma_all_tau(osox.sigma_thc_paper, G, X, V)
    plan = thcsox.Plan(torch.from_numpy(X).to(dev), torch.from_numpy(V).to(dev), tau, w, 100.0,
                       precision=precision)
    Gd = torch.from_numpy(G).to(dev)
    Sx = plan.sigma(Gd).cpu().numpy()
    Sd = plan.sigma_direct(Gd).cpu().numpy()
    plan.close()
    ex = np.abs(Sx - ref).max() / np.abs(ref).max()
    canc = np.abs(Sx + Sd).max() / np.abs(ref).max()
    print(f"  SOX rel err {ex:.2e}  |SOX + direct| / |SOX| {canc:.2e}")
    tol = 1e-12 if precision == "fp64" else 2e-6
    assert ex <= tol and canc <= tol
