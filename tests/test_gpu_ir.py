"""GPU parity on the IR sampling grids (beta = 1000, Lambda = 1e5, the paper's
production grid, and beta = 100, Lambda = 1e4): the library's grids and tables drive the Dyson step, the SOX
evaluation and the energy; the oracle runs the same steps on its own grids.

The two grids are the same to the accuracy an FP64 singular value expansion
fixes them (tau points ~1e-8 relative; the frequency sets agree except for up
to four points where a sign change of the highest basis functions' transform
is decided at their noise level, either choice being a valid sampling point;
checked on the CPU), so results are compared as functions: the oracle's fitted result is
evaluated at the library's tau points, and energies (integrals) directly.
Bars: the transforms are accurate to ~1e-8 (eps = 1e-10 times the fit's
condition number, a few hundred), so 1e-7 absolute on G, 1e-8 relative on
FP64 energies, 1e-6 Ha on the fp16x2 energy.
"""
import numpy as np
import pytest
import torch

from oracle import ir as oir
from oracle import sox as osox
from paper_2404_17744_amd import synth, thcsox

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[(1000.0, 100.0), (100.0, 100.0)],
                ids=["beta1000_L1e5", "beta100_L1e4"])
def grids(request):
    beta, wmax = request.param
    g = thcsox.thcsox_ir_grid(beta, wmax, 1e-10)
    b = oir.IRBasis(beta, wmax, 1e-10)
    tau_o, nf_o = b.tau_points(), b.matsubara_points()
    Wf_o, Wb_o = oir.transforms(b, tau_o, nf_o)
    return g, dict(b=b, tau=tau_o, nf=nf_o, Wf=Wf_o, Wb=Wb_o, beta=beta)


def test_ir_dyson_sigma0_is_g0(dev, grids):
    g, o = grids
    BETA = o["beta"]
    s = synth.make_system(12, 48, seed=4)
    print(f"case IR dyson sigma=0 n12 L{len(g['tau'])} nf{len(g['freq_n'])}", flush=True)
    F = torch.from_numpy(s.F).to(dev)
    d = thcsox.Dyson(F, s.mu, g["tau"], BETA, grid=g)
    S = torch.zeros((len(g["tau"]), 12, 12), dtype=torch.float64, device=dev)
    G, gamma = d.step(S)
    torch.cuda.synchronize()
    d.close()
    G0 = synth.g0_tau(s, g["tau"], BETA)
    err = np.abs(G.cpu().numpy() - G0).max()
    occ = 0.5 * (1.0 - np.tanh(0.5 * BETA * (s.eps - s.mu)))
    dn = abs(np.trace(gamma.cpu().numpy()) - occ.sum())
    print(f"  |G - G0| {err:.2e}  |Tr gamma - N| {dn:.2e}")
    assert err <= 1e-7 and dn <= 1e-6


def test_ir_dyson_step_vs_oracle(dev, grids):
    g, o = grids
    BETA = o["beta"]
    s = synth.make_system(16, 64, seed=5)
    print("case IR dyson pole-sum sigma n16 seed 5", flush=True)
    S_lib = synth.pole_sigma(16, g["tau"], BETA, seed=6)
    S_ora = synth.pole_sigma(16, o["tau"], BETA, seed=6)
    G_o, gam_o = oir.dyson_step_sampled(s.F, s.mu, BETA, S_ora, o["Wf"], o["Wb"], o["nf"])
    G_ref = oir.evaluate_at(o["b"], o["tau"], G_o, g["tau"])
    d = thcsox.Dyson(torch.from_numpy(s.F).to(dev), s.mu, g["tau"], BETA, grid=g)
    G, gamma = d.step(torch.from_numpy(S_lib).to(dev))
    G2, gamma2, mu, ev = d.step_mu(torch.from_numpy(S_lib).to(dev), s.n_occ, s.mu, tol=1e-6)
    torch.cuda.synchronize()
    d.close()
    err = np.abs(G.cpu().numpy() - G_ref).max()
    derr = np.abs(gamma.cpu().numpy() - gam_o).max()
    print(f"  |G - oracle| {err:.2e}  |gamma - oracle| {derr:.2e}  mu search: mu {mu:.6f} "
          f"({ev} solves), Tr gamma {np.trace(gamma2.cpu().numpy()):.8f}")
    assert err <= 1e-7 and derr <= 1e-7
    assert abs(np.trace(gamma2.cpu().numpy()) - s.n_occ) <= 1e-6


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "fp16x2"])
def test_ir_sox_energy_vs_oracle(dev, grids, precision):
    g, o = grids
    BETA = o["beta"]
    s = synth.make_system(20, 80, seed=7, lam=0.2)
    print(f"case IR SOX energy n20 naux80 seed 7 {precision}", flush=True)
    G_lib = synth.g0_tau(s, g["tau"], BETA)
    G_ora = synth.g0_tau(s, o["tau"], BETA)
    S_ora = osox.sigma_all_tau(osox.sigma_thc_paper, G_ora, s.X, s.V)
    M = oir.energy_matrix(o["b"], o["tau"])
    E_ref = -0.5 * float(np.sum(M * np.einsum("apq,bqp->ab", G_ora, S_ora)))
    plan = thcsox.Plan(torch.from_numpy(s.X).to(dev), torch.from_numpy(s.V).to(dev), g["tau"],
                       np.zeros(len(g["tau"])), BETA, precision=precision)
    Gd = torch.from_numpy(G_lib).to(dev)
    S = plan.sigma(Gd)
    E = plan.energy_basis(Gd, S, g)
    torch.cuda.synchronize()
    plan.close()
    S_ref = oir.evaluate_at(o["b"], o["tau"], S_ora, g["tau"])
    serr = np.abs(S.cpu().numpy() - S_ref).max() / np.abs(S_ref).max()
    print(f"  E {E:.12f} oracle {E_ref:.12f} dE {E - E_ref:.2e}  Sigma rel {serr:.2e}")
    if precision == "fp64":
        assert abs(E - E_ref) <= 1e-8 * abs(E_ref) and serr <= 1e-7
    else:
        assert abs(E - E_ref) <= 1e-6 and serr <= 1e-6
