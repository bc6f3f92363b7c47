"""Pins for the oracle's second-order direct (bubble) self-energy:

* the THC form against the six-index definition on a non-symmetric G, so a
  dropped transpose or a swapped G / G(beta - tau) fails;
* E[G0] at low temperature -> 2 x the spin-orbital MP2 Coulomb term (negative),
  with the same energy functional that gives 2 x the exchange term for SOX;
  together with that pin, E_dir + E_SOX -> 2 x the spin-orbital MP2 energy;
* planted slips in copies of the THC form are caught by the first pin.
"""
import numpy as np
import pytest

from oracle import direct as od
from oracle import energy as oenergy
from oracle import sox as osox
from paper_2404_17744_amd import synth


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def general_case():
    s = synth.make_system(6, 20, seed=2)
    G = synth.random_general_g(6, 4, seed=3)
    return s, G, osox.thc_eri(s.X, s.V)


def test_thc_form_matches_definition(general_case):
    s, G, v = general_case
    for k in range(4):
        ref = od.sigma_direct_bruteforce(v, G[k], G[3 - k])
        assert _rel(od.sigma_direct_thc(s.X, s.V, G[k], G[3 - k]), ref) < 1e-13


def test_energy_is_twice_mp2_coulomb():
    s = synth.make_system(6, 24, seed=1)
    vmo = oenergy.to_mo(osox.thc_eri(s.X, s.V), s.Q)
    occ = np.arange(s.n) < s.n_occ
    EJ = od.mp2_coulomb(vmo, s.eps, occ)
    Ex = oenergy.mp2_exchange(vmo, s.eps, occ)
    tau, w = synth.cheb_tau_grid(128, 100.0)
    G = synth.g0_tau(s, tau, 100.0)
    Ed = oenergy.energy_tau(G, osox.sigma_all_tau(od.sigma_direct_thc, G, s.X, s.V), w)
    Es = oenergy.energy_tau(G, osox.sigma_all_tau(osox.sigma_thc_paper, G, s.X, s.V), w)
    assert EJ < 0
    assert abs(Ed / (2 * EJ) - 1.0) < 1e-8
    # full second order: the spin-orbital MP2 energy is E_J + E_x (E_x as defined, positive)
    assert abs((Ed + Es) / (2 * (EJ + Ex)) - 1.0) < 1e-8


def _mutant(X, V, G, Gb, slip):
    Gt = X.T @ G @ X
    Gbt = X.T @ (G if slip == "no_mirror" else Gb) @ X
    Pi = Gt * (Gbt if slip == "no_transpose" else Gbt.T)
    W = V @ Pi @ V
    H = W * (Gt.T if slip == "transposed_outer_g" else Gt)
    out = X @ H @ X.T
    return -out if slip == "exchange_sign" else out


@pytest.mark.parametrize("slip", ["no_mirror", "no_transpose", "transposed_outer_g",
                                  "exchange_sign"])
def test_mutants_are_caught(general_case, slip):
    s, G, v = general_case
    errs = [_rel(_mutant(s.X, s.V, G[k], G[3 - k], slip),
                 od.sigma_direct_bruteforce(v, G[k], G[3 - k])) for k in range(4)]
    assert max(errs) > 1e-3


def test_single_spin_orbital_terms_cancel():
    """One spin-orbital cannot hold two electrons: at second order the direct and
    the exchange diagrams cancel exactly (Sigma^dir = -Sigma^SOX for n = 1, any G).
    Pins the relative sign of the two oracles to the Pauli principle."""
    X, V = synth.thc_factors(1, 37, seed=11)
    G = synth.random_general_g(1, 8, seed=1)
    for k in range(8):
        a = osox.sigma_thc_paper(X, V, G[k], G[7 - k])
        b = od.sigma_direct_thc(X, V, G[k], G[7 - k])
        assert abs(a[0, 0] + b[0, 0]) <= 1e-13 * abs(a[0, 0])
