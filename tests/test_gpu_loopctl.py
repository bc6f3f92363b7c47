"""GPU parity of the loop-control entry points (chemical-potential search in the
Dyson step, damping, Pulay DIIS) against the oracle and closed forms."""
import numpy as np
import pytest
import torch
from scipy.optimize import brentq

from oracle import loopctl as olc
from oracle import sox as osox
from oracle import transforms as otr
from paper_2404_17744_amd import synth, thcsox

pytestmark = pytest.mark.gpu
BETA = 100.0


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_mu_search_zero_sigma_matches_fermi_root(dev):
    """Sigma = 0: the mu that puts n_occ - 1/2 electrons in the system is the root
    of the Fermi sum over the one-body levels (closed form)."""
    s = synth.make_system(20, 40, seed=2)
    tau, w = synth.cheb_tau_grid(64, BETA)
    print("case mu search n20 Sigma=0 nelec n_occ-1/2", flush=True)
    nelec = s.n_occ - 0.5
    d = thcsox.Dyson(torch.from_numpy(s.F).to(dev), s.mu, tau, BETA, 256)
    G, gam, mu, evals = d.step_mu(torch.zeros((64, 20, 20), dtype=torch.float64, device=dev),
                                  nelec, s.mu, tol=1e-10)
    d.close()
    f = lambda x: np.sum(1.0 / (1.0 + np.exp(np.clip(BETA * (s.eps - x), -700, 700)))) - nelec
    mu_exact = brentq(f, -3.0, 3.0, xtol=1e-15)
    print(f"  mu {mu:.12f} closed form {mu_exact:.12f} evaluations {evals}")
    assert abs(float(torch.trace(gam)) - nelec) <= 1e-10
    assert abs(mu - mu_exact) <= 5e-8


def test_mu_search_matches_oracle(dev):
    """SOX self-energy at G0 (n=30, naux=120, 64 tau, 256 frequencies)."""
    s = synth.make_system(30, 120, seed=8, lam=0.5)
    tau, w = synth.cheb_tau_grid(64, BETA)
    G0 = synth.g0_tau(s, tau, BETA)
    S = osox.sigma_all_tau(osox.sigma_thc_paper, G0, s.X, s.V)
    Tm = otr.cheb_to_matsubara(64, 256, BETA)
    nelec = s.n_occ - 0.5
    print("case mu search n30 naux120 SOX Sigma nelec n_occ-1/2", flush=True)
    G_ref, gam_ref, mu_ref, ev_ref = olc.loop_step_mu(s.F, s.mu, BETA, S, Tm, nelec, tol=1e-10)
    d = thcsox.Dyson(torch.from_numpy(s.F).to(dev), s.mu, tau, BETA, 256)
    G, gam, mu, evals = d.step_mu(torch.from_numpy(S).to(dev), nelec, s.mu, tol=1e-10)
    # the plan keeps the new chemical potential for plain steps
    G2, _ = d.step(torch.from_numpy(S).to(dev))
    d.close()
    print(f"  mu {mu:.12f} oracle {mu_ref:.12f}; evaluations {evals} / {ev_ref}")
    assert abs(mu - mu_ref) <= 1e-9
    assert _rel(G.cpu().numpy(), G_ref) <= 1e-10
    assert _rel(gam.cpu().numpy(), gam_ref) <= 1e-10
    assert abs(float(torch.trace(gam)) - nelec) <= 1e-10
    assert torch.equal(G, G2)


def test_mix_is_the_damping_formula(dev):
    rng = np.random.default_rng(3)
    a = rng.standard_normal((7, 11, 11))
    b = rng.standard_normal((7, 11, 11))
    io = torch.from_numpy(a.copy()).to(dev)
    thcsox.mix(0.3, torch.from_numpy(b).to(dev), io)
    torch.cuda.synchronize()
    assert np.abs(io.cpu().numpy() - olc.damp(a, b, 0.3)).max() <= 1e-15


def test_diis_matches_oracle(dev):
    """Five steps of a noisy contraction on (m, n, n) arrays, depth 4 (the
    history wraps), against the oracle's extrapolation over the same window."""
    rng = np.random.default_rng(5)
    shape = (16, 24, 24)
    target = rng.standard_normal(shape)
    ins, outs = [], []
    x = np.zeros(shape)
    xd = torch.zeros(shape, dtype=torch.float64, device=dev)
    nxt = torch.empty_like(xd)
    diis = thcsox.Diis(xd, depth=4)
    for it in range(5):
        out = 0.6 * x + 0.4 * target + 1e-3 * rng.standard_normal(shape)
        ins.append(x.copy())
        outs.append(out)
        used = diis.step(torch.from_numpy(x).to(dev), torch.from_numpy(out).to(dev), nxt)
        ref = olc.diis_next(ins[-4:], outs[-4:])
        got = nxt.cpu().numpy()
        assert used == min(it + 1, 4)
        assert _rel(got, ref) <= 1e-11, (it, _rel(got, ref))
        x = ref
    diis.close()


def test_diis_exact_on_linear_map_and_errors(dev):
    d = 6
    rng = np.random.default_rng(1)
    M = rng.standard_normal((d, d))
    M *= 0.8 / np.abs(np.linalg.eigvals(M)).max()
    b = rng.standard_normal(d)
    x_star = np.linalg.solve(np.eye(d) - M, b)
    x = torch.zeros(d, dtype=torch.float64, device=dev)
    nxt = torch.empty_like(x)
    diis = thcsox.Diis(x, depth=8)
    for _ in range(d + 1):
        out = torch.from_numpy(M @ x.cpu().numpy() + b).to(dev)
        diis.step(x, out, nxt)
        x = nxt.clone()
    diis.close()
    assert np.abs(x.cpu().numpy() - x_star).max() <= 1e-10 * np.abs(x_star).max()
    with pytest.raises(thcsox.ThcsoxError):
        thcsox.Diis(x, depth=0)
    s = synth.make_system(6, 12, seed=0)
    tau, _ = synth.cheb_tau_grid(8, BETA)
    dd = thcsox.Dyson(torch.from_numpy(s.F).to(dev), s.mu, tau, BETA, 16)
    with pytest.raises(thcsox.ThcsoxError):
        dd.step_mu(torch.zeros((8, 6, 6), dtype=torch.float64, device=dev), 7.0, s.mu)
    dd.close()
