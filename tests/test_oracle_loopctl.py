"""Pins for the oracle's loop control (chemical-potential search, damping,
Pulay DIIS), each against something other than the oracle itself:

* with Sigma = 0, N(mu) is the Fermi sum over the one-body levels, so the mu
  that the search finds (through the Dyson solve and the Chebyshev fit) must
  match the root of that closed form, found by a bracketing scalar solver;
  N_el = n_occ - 1/2 puts the root at a steep point of N(mu) (half an electron in
  the highest occupied level);
* Pulay DIIS on a linear fixed-point map x = M x + b is a Krylov method: with
  depth > dim it reaches (1 - M)^-1 b after at most dim + 1 extrapolations;
* damping keeps the fixed point of a linear map and converges to it.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import loopctl, transforms as tr
from paper_2404_17744_amd import synth

BETA = 100.0


def _fermi_root(eps, nelec):
    f = lambda mu: np.sum(1.0 / (1.0 + np.exp(np.clip(BETA * (eps - mu), -700, 700)))) - nelec
    return brentq(f, eps.min() - 1.0, eps.max() + 1.0, xtol=1e-15, rtol=1e-15)


@pytest.mark.parametrize("seed", [2, 5])
def test_find_mu_matches_fermi_closed_form(seed):
    s = synth.make_system(20, 40, seed=seed)
    Tm = tr.cheb_to_matsubara(64, 256, BETA)
    nelec = s.n_occ - 0.5
    mu, N, evals = loopctl.find_mu(s.F, BETA, np.zeros((64, 20, 20)), Tm, nelec, s.mu,
                                   tol=1e-10)
    mu_exact = _fermi_root(s.eps, nelec)
    assert abs(N - nelec) <= 1e-10
    # the Chebyshev fit (m = 64) carries ~1e-7 in N, dN/dmu ~ beta/4
    assert abs(mu - mu_exact) <= 5e-8, (mu, mu_exact)
    assert evals < 40
    # a start above the root walks down to the same mu
    mu2, _, _ = loopctl.find_mu(s.F, BETA, np.zeros((64, 20, 20)), Tm, nelec, s.mu + 1.0,
                                tol=1e-10)
    assert abs(mu2 - mu) <= 1e-9


def test_find_mu_with_sigma_conserves_electrons():
    s = synth.make_system(12, 40, seed=3)
    Tm = tr.cheb_to_matsubara(32, 64, BETA)
    rng = np.random.default_rng(4)
    S = 0.05 * rng.standard_normal((32, 12, 12))
    S = 0.5 * (S + S.transpose(0, 2, 1))
    nelec = s.n_occ + 0.25
    G, gam, mu, _ = loopctl.loop_step_mu(s.F, s.mu, BETA, S, Tm, nelec, tol=1e-10)
    assert abs(np.trace(gam) - nelec) <= 1e-10
    # N(mu) increases with mu
    S_iw = tr.tau_to_matsubara(S, Tm)
    Ns = [loopctl.electron_number(s.F, mu + d, BETA, S_iw, Tm) for d in (-0.05, 0.0, 0.05)]
    assert Ns[0] < Ns[1] < Ns[2]


def _linear_map(d, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((d, d))
    M *= 0.8 / np.abs(np.linalg.eigvals(M)).max()
    b = rng.standard_normal(d)
    return M, b, np.linalg.solve(np.eye(d) - M, b)


def test_diis_is_exact_on_a_linear_map():
    d = 6
    M, b, x_star = _linear_map(d, 1)
    ins, outs = [], []
    x = np.zeros(d)
    for it in range(d + 1):
        ins.append(x)
        outs.append(M @ x + b)
        x = loopctl.diis_next(ins, outs)
    assert np.abs(x - x_star).max() <= 1e-10 * np.abs(x_star).max()


def test_damping_keeps_the_fixed_point():
    M, b, x_star = _linear_map(5, 2)
    assert np.allclose(loopctl.damp(x_star, M @ x_star + b, 0.6), x_star, rtol=0, atol=1e-14)
    x = np.zeros(5)
    for _ in range(400):
        x = loopctl.damp(x, M @ x + b, 0.5)
    assert np.abs(x - x_star).max() <= 1e-10


# Planted slips in copies of the loop-control steps must fail the pins above.
def _diis_mutant(inputs, outputs, slip):
    k = len(inputs)
    res = [o - i for i, o in zip(inputs, outputs)]
    B = np.zeros((k + 1, k + 1))
    for i in range(k):
        for j in range(k):
            B[i, j] = float(np.dot(res[i].ravel(), res[j].ravel()))
    B[k, :k] = 1.0
    B[:k, k] = 1.0
    rhs = np.zeros(k + 1)
    rhs[k] = 1.0
    if slip == "rhs_zero":          # lose the sum-to-one constraint
        rhs[k] = 0.0
        rhs[0] = 1.0
    c = np.linalg.lstsq(B, rhs, rcond=None)[0][:k]
    base = inputs if slip == "extrapolate_inputs" else outputs
    out = np.zeros_like(outputs[0])
    for ci, o in zip(c, base):
        out += ci * o
    return out


@pytest.mark.parametrize("slip", ["rhs_zero", "extrapolate_inputs"])
def test_diis_mutants_are_caught(slip):
    d = 6
    M, b, x_star = _linear_map(d, 1)
    ins, outs = [], []
    x = np.zeros(d)
    for _ in range(d + 1):
        ins.append(x)
        outs.append(M @ x + b)
        x = _diis_mutant(ins, outs, slip)
    assert np.abs(x - x_star).max() > 1e-6 * np.abs(x_star).max()


def test_density_sign_slip_is_caught():
    """gamma = +G(beta^-) instead of -G(beta^-): no bracket for a positive N_el."""
    s = synth.make_system(20, 40, seed=2)
    Tm = tr.cheb_to_matsubara(64, 256, BETA)
    S_iw = tr.tau_to_matsubara(np.zeros((64, 20, 20)), Tm)

    def n_wrong(mu):
        cG = tr.fit_coeffs_from_matsubara(tr.dyson(s.F, mu, S_iw, BETA), Tm)
        return float(np.trace(np.sum(cG, axis=0)))

    # -N(mu) <= 0 up to the fit noise (1e-4 far below every level): no target of
    # half an electron or more can be bracketed
    assert max(n_wrong(mu) for mu in (-2.0, s.mu, 2.0)) < 0.5


# Commutator DIIS (reading in oracle/loopctl.py).
def _sym_profiles(m, n, seed, scale):
    rng = np.random.default_rng(seed)
    S = scale * rng.standard_normal((m, n, n))
    return S + S.transpose(0, 2, 1)


def test_commutator_residual_forms_agree():
    """[G_in, F + Sigma_out] = [G_in, Sigma_out - Sigma_in] because G_in inverts
    (i w + mu) - F - Sigma_in; a G taken from Sigma_out breaks the identity."""
    s = synth.make_system(12, 36, seed=3)
    m = 32
    Tm = tr.cheb_to_matsubara(m, 128, BETA)
    S_in = tr.tau_to_matsubara(_sym_profiles(m, 12, 1, 0.02), Tm)
    S_out = tr.tau_to_matsubara(_sym_profiles(m, 12, 2, 0.02), Tm)
    G_in = tr.dyson(s.F, s.mu, S_in, BETA)
    e = loopctl.commutator_residual(G_in, S_out - S_in)
    ref = loopctl.commutator_residual_definition(G_in, s.F, S_out)
    assert np.abs(e - ref).max() <= 1e-10 * np.abs(ref).max()
    G_bad = tr.dyson(s.F, s.mu, S_out, BETA)
    bad = loopctl.commutator_residual(G_bad, S_out - S_in)
    assert np.abs(bad - ref).max() > 1e-3 * np.abs(ref).max()


def test_commutator_vanishes_along_the_inverse():
    """A step D = c G^-1 commutes with G: the commutator residual is zero where
    the Pulay residual is not (the two measure different things)."""
    s = synth.make_system(10, 30, seed=4)
    m = 16
    Tm = tr.cheb_to_matsubara(m, 64, BETA)
    S_in = tr.tau_to_matsubara(_sym_profiles(m, 10, 3, 0.02), Tm)
    G = tr.dyson(s.F, s.mu, S_in, BETA)
    D = 0.3 * np.linalg.inv(G)
    e = loopctl.commutator_residual(G, D)
    assert np.abs(e).max() <= 1e-12 * np.abs(D).max()
    assert np.abs(D).max() > 0.1


def test_commutator_diis_loop_reaches_the_plain_fixed_point():
    """The oracle's loop (SOX at lambda = 0.3, n = 12, fixed mu) from the same
    start: plain iteration and commutator DIIS(4) reach the same energy, the
    DIIS run in fewer iterations (measured: 14 plain, 9 commutator DIIS, 10
    Pulay DIIS)."""
    from oracle import energy as oen, sox as osox
    s = synth.make_system(12, 36, seed=5, lam=0.3)
    m, nw = 32, 128
    tau, w = synth.cheb_tau_grid(m, BETA)
    Tm = tr.cheb_to_matsubara(m, nw, BETA)
    U = osox.precontract_u(s.X, s.V)

    def sox(G):
        return np.stack([osox.sigma_thc_paper(s.X, s.V, G[k], G[m - 1 - k], U=U)
                         for k in range(m)])

    def run(cdiis):
        S_in = np.zeros((m, 12, 12))
        G, gam, G_iw = tr.loop_step(s.F, s.mu, BETA, S_in, Tm)
        E_prev, hist_e, hist_o = None, [], []
        for it in range(60):
            S_out = sox(G)
            E = float(np.sum(s.F * gam.T)) + oen.energy_tau(G, S_out, w)
            if E_prev is not None and abs(E - E_prev) < 1e-9:
                return it + 1, E
            E_prev = E
            if cdiis:
                D = tr.tau_to_matsubara(S_out - S_in, Tm)
                hist_e.append(loopctl.commutator_residual(G_iw, D))
                hist_o.append(S_out)
                hist_e, hist_o = hist_e[-4:], hist_o[-4:]
                S_in = loopctl.cdiis_next(hist_e, hist_o)
            else:
                S_in = S_out
            G, gam, G_iw = tr.loop_step(s.F, s.mu, BETA, S_in, Tm)
        raise AssertionError("no convergence")

    it_plain, E_plain = run(False)
    it_cd, E_cd = run(True)
    assert abs(E_plain - E_cd) <= 1e-8
    assert it_cd < it_plain, (it_cd, it_plain)


def test_electron_number_across_the_gap_sox_alone_and_full_second_order():
    """Why the chemical-potential search suits the full second-order loop and not
    the exchange term alone (n = 16, lambda = 0.5, 32 tau points, fixed mu): at
    the converged Sigma, N(mu) with Sigma held fixed rises across the one-body gap
    for Sigma^dir + Sigma^SOX, one root, but falls for Sigma^SOX alone, whose
    spectral weight is not of one sign; N(mu) = N_el then has several roots and
    the search hops between them from one iteration to the next."""
    from oracle import direct as odir, sox as osox
    n, m, nw = 16, 32, 256
    s = synth.make_system(n, 3 * n, seed=0, lam=0.5)
    Tm = tr.cheb_to_matsubara(m, nw, BETA)
    U = osox.precontract_u(s.X, s.V)
    ev = np.sort(s.eps)
    mus = np.linspace(ev[s.n_occ - 1] + 0.02, ev[s.n_occ] - 0.02, 9)
    slopes = {}
    for terms in ("sox", "gf2"):
        S = np.zeros((m, n, n))
        for _ in range(40):
            G, _, _ = tr.loop_step(s.F, s.mu, BETA, S, Tm)
            S_new = np.stack([osox.sigma_thc_paper(s.X, s.V, G[k], G[m - 1 - k], U=U)
                              for k in range(m)])
            if terms == "gf2":
                S_new += np.stack([odir.sigma_direct_thc(s.X, s.V, G[k], G[m - 1 - k])
                                   for k in range(m)])
            done = np.abs(S_new - S).max() < 1e-10
            S = S_new
            if done:
                break
        assert done
        S_iw = tr.tau_to_matsubara(S, Tm)
        slopes[terms] = np.diff([loopctl.electron_number(s.F, mu, BETA, S_iw, Tm) for mu in mus])
    assert np.all(slopes["gf2"] > 0.0)
    assert np.all(slopes["sox"][1:-1] < 0.0)
