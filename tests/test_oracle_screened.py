"""Pins for the oracle's screened-exchange self-energies (oracle/screened.py):
the static polarization against its Lindhard closed form, the screened core
against its series and the screening inequality, the two-core THC sequence
against the six-index definition with both integral tensors assembled, the
unscreened limit (SOSEX = G3W2 = SOX), and planted slips."""
import numpy as np
import pytest

from oracle import screened as osc
from oracle import sox as osox
from paper_2404_17744_amd import synth

BETA = 100.0


def _system(n=6, naux=20, seed=4):
    s = synth.make_system(n, naux, seed=seed)
    tau, w = synth.cheb_tau_grid(100, BETA)
    return s, tau, w, synth.g0_tau(s, tau, BETA)


def test_static_polarization_matches_lindhard_closed_form():
    s, tau, w, G = _system()
    P = osc.static_polarization(s.X, G, w)
    ref = osc.static_polarization_g0(s.X, s.Q, s.eps, s.mu, BETA)
    assert np.abs(P - ref).max() <= 1e-10 * np.abs(ref).max()
    # positive semidefinite: the physical (negative) polarization is -Pi0
    assert np.linalg.eigvalsh(0.5 * (ref + ref.T)).min() >= -1e-12 * np.abs(ref).max()


def test_lindhard_weight_limits():
    """Two orbitals, one occupied and one virtual, at low temperature.  In the
    orbital basis (psi = I) the mixed products psi_jQ psi_kQ vanish, so Pi0 is
    diagonal with beta (1 - f) f, which vanishes at low temperature.  In a
    rotated basis both time orderings of the particle-hole pair contribute
    1 / (xi_virt - xi_occ) each, the textbook static weight 2 / (e_a - e_i)."""
    X = np.eye(2)
    eps = np.array([-0.5, 0.7])
    P = osc.static_polarization_g0(X, np.eye(2), eps, 0.1, 1000.0)
    f = np.array([osc._f(x, 1000.0) for x in eps - 0.1])
    assert np.allclose(P, np.diag(1000.0 * (1 - f) * f), rtol=0, atol=1e-200)
    c, s_ = np.cos(0.3), np.sin(0.3)
    Qr = np.array([[c, -s_], [s_, c]])
    P2 = osc.static_polarization_g0(X, Qr, eps, 0.1, 1000.0)
    v = Qr[:, 1] * Qr[:, 0]          # psi_virt * psi_occ per THC point
    assert np.allclose(P2, 2.0 / (eps[1] - eps[0]) * np.outer(v, v), rtol=1e-12, atol=1e-14)


def test_screened_core_series_and_inequality():
    s, tau, w, G = _system()
    P = osc.static_polarization(s.X, G, w)
    V = s.V
    for eps_ in (1e-3, 1e-4):
        W = osc.screened_core(V, eps_ * P)
        series = V - eps_ * V @ P @ V + eps_ ** 2 * V @ P @ V @ P @ V
        assert np.abs(W - series).max() <= 10 * eps_ ** 3 * np.abs(V @ P @ V @ P @ V @ P @ V).max()
    W = osc.screened_core(V, P)
    assert np.abs(W - W.T).max() <= 1e-12 * np.abs(W).max()
    # screening lowers the interaction: V - W = W Pi0 V is positive semidefinite
    lam = np.linalg.eigvalsh(0.5 * ((V - W) + (V - W).T))
    assert lam.min() >= -1e-10 * np.abs(V).max()


@pytest.mark.parametrize("symmetric", [False, True])
def test_two_core_sequence_matches_six_index_definition(symmetric):
    n, naux = 6, 20
    s = synth.make_system(n, naux, seed=7)
    if symmetric:
        tau, w = synth.cheb_tau_grid(4, BETA)
        G = synth.g0_tau(s, tau, BETA)
    else:
        G = synth.random_general_g(n, 4, seed=8)
    rng = np.random.default_rng(9)
    L = rng.standard_normal((naux, naux))
    Pi0 = L @ L.T / naux
    W = osc.screened_core(s.V, Pi0)
    for k in range(4):
        for Va, Vc in ((s.V, W), (W, s.V), (W, W)):
            got = osc.sigma_two_cores(s.X, Va, Vc, G[k], G[3 - k])
            ref = osc.sigma_two_cores_bruteforce(s.X, Va, Vc, G[k], G[3 - k])
            assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        if symmetric:
            a = osc.sigma_two_cores(s.X, s.V, W, G[k], G[3 - k])
            b = osc.sigma_two_cores(s.X, W, s.V, G[k], G[3 - k])
            assert np.abs(a.T - b).max() <= 1e-12 * np.abs(a).max()
            so = osc.sigma_sosex(s.X, s.V, W, G[k], G[3 - k])
            assert np.abs(so - so.T).max() <= 1e-12 * np.abs(so).max()


def test_unscreened_limit_is_sox():
    s, tau, w, G = _system(n=6, naux=24, seed=2)
    W = osc.screened_core(s.V, np.zeros_like(s.V))
    assert np.array_equal(W, np.linalg.solve(np.eye(24), s.V))
    for k in (0, 37, 99):
        ref = osox.sigma_thc_paper(s.X, s.V, G[k], G[99 - k])
        for got in (osc.sigma_sosex(s.X, s.V, W, G[k], G[99 - k]),
                    osc.sigma_g3w2(s.X, W, G[k], G[99 - k])):
            assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_screening_lowers_the_exchange_energy_magnitude():
    """With W <= V the screened exchange terms are smaller than SOX: |E^G3W2| <
    |E^SOSEX| < |E^SOX| for the independent-particle G (all three positive, the
    sign of the exchange term)."""
    from oracle import energy as oen
    s, tau, w, G = _system(n=6, naux=24, seed=2)
    P = osc.static_polarization(s.X, G, w)
    W = osc.screened_core(s.V, P)
    m = len(tau)
    S_sox = np.stack([osox.sigma_thc_paper(s.X, s.V, G[k], G[m - 1 - k]) for k in range(m)])
    S_so = np.stack([osc.sigma_sosex(s.X, s.V, W, G[k], G[m - 1 - k]) for k in range(m)])
    S_g3 = np.stack([osc.sigma_g3w2(s.X, W, G[k], G[m - 1 - k]) for k in range(m)])
    E = [oen.energy_tau(G, S, w) for S in (S_sox, S_so, S_g3)]
    assert E[0] > E[1] > E[2] > 0.0, E


def test_planted_slips_are_caught():
    s, tau, w, G = _system()
    ref = osc.static_polarization_g0(s.X, s.Q, s.eps, s.mu, BETA)
    m = len(tau)
    # the bubble closed on G(tau) twice instead of its mirror
    bad = sum(w[k] * osc.polarization_tau(s.X, G[k], G[k]) for k in range(m))
    assert np.abs(bad - ref).max() > 1e-3 * np.abs(ref).max()
    # anti-screening sign: V (1 - Pi0 V)^-1 breaks the series pin
    P = 1e-3 * ref
    anti = np.linalg.solve(np.eye(s.naux) - s.V @ P, s.V)
    V = s.V
    series = V - V @ P @ V + V @ P @ V @ P @ V
    assert np.abs(anti - series).max() > 100 * np.abs(osc.screened_core(V, P) - series).max()
