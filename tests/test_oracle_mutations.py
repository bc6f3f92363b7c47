"""Planted mistakes in (copies of) the oracle must be caught by the pins.

Each mutant is a one-line slip a transcription of the paper could make.  For
every mutant at least one pin -- brute force on a non-symmetric G, the
zero-temperature MP2-exchange limit, the sign of the energy -- must fail.
"""
import numpy as np
import pytest

from oracle import energy as oenergy
from oracle import sox as osox
from paper_2404_17744_amd import synth


def paper_sequence(X, V, G, Gb, slip=None):
    """The oracle's THC sequence with an optional planted slip."""
    U = osox.precontract_u(X, V)
    GR = X.T @ (G.T if slip == "transpose_first_projection" else G)
    GwP = G @ X
    if slip == "no_mirror":
        Gb = G
    A = U @ Gb
    if slip == "swap_A_indices":
        A = A.transpose(0, 2, 1)
    B = np.matmul(GR, A)
    C = U @ GwP
    D = np.einsum("RvP,PRv->PR", C, B)
    sig = -D.T if slip != "drop_sign" else D.T
    if slip == "no_transpose_D":
        sig = -D
    return X @ sig @ X.T


def pins(slip, energy_half=True):
    """Return {pin: passed} for a mutant."""
    out = {}
    s = synth.make_system(6, 20, seed=2)
    G = synth.random_general_g(6, 4, seed=3)
    v = osox.thc_eri(s.X, s.V)
    ref = osox.sigma_all_tau(osox.sigma_bruteforce, G, v)
    got = np.stack([paper_sequence(s.X, s.V, G[k], G[3 - k], slip) for k in range(4)])
    out["bruteforce"] = np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    s6 = synth.make_system(6, 24, seed=1)
    tau, w = synth.cheb_tau_grid(100, 100.0)
    G6 = synth.g0_tau(s6, tau, 100.0)
    S6 = np.stack([paper_sequence(s6.X, s6.V, G6[k], G6[99 - k], slip) for k in range(100)])
    E = oenergy.energy_tau(G6, S6, w) * (1.0 if energy_half else 2.0)
    vmo = oenergy.to_mo(osox.thc_eri(s6.X, s6.V), s6.Q)
    Ex = oenergy.mp2_exchange(vmo, s6.eps, np.arange(6) < s6.n_occ)
    out["mp2_limit"] = abs(E / (2 * Ex) - 1) < 1e-6
    out["sign"] = E > 0
    return out


def test_unmutated_passes_all():
    assert all(pins(None).values())


@pytest.mark.parametrize("slip", ["transpose_first_projection", "no_mirror", "swap_A_indices",
                                  "drop_sign", "no_transpose_D"])
def test_mutant_is_caught(slip):
    res = pins(slip)
    assert not all(res.values()), f"mutant {slip} passed every pin: {res}"


def test_energy_without_half_is_caught():
    res = pins(None, energy_half=False)
    assert not all(res.values())
