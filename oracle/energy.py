"""Galitskii-Migdal energies in FP64 (test infrastructure only).

Paper: Sec. "Definitions", Eqs. E1b and E2b, and the density matrix defined
just above them.

Reading of Eq. E2b used throughout (the printed form has no 1/2 and no
frequency range): the dynamic energy of spin-orbitals is

    E_dyn = 1/2 * (1/beta) sum_{n in Z} Tr[G(i w_n) Sigma(i w_n)]
          = -1/2 * int_0^beta Tr[G(beta - tau) Sigma(tau)] dtau

(the second line follows from the antiperiodic inverse transform).
"""
from __future__ import annotations

import numpy as np


def energy_tau(G: np.ndarray, Sigma: np.ndarray, w: np.ndarray) -> float:
    """E = -1/2 sum_k w_k Tr[G(beta - tau_k) Sigma(tau_k)] on a mirror-symmetric
    grid (G(beta - tau_k) is G[m-1-k]); w are the quadrature weights on [0, beta].
    Tr[A B] = sum_pq A_qp B_pq."""
    m = G.shape[0]
    tot = 0.0
    for k in range(m):
        tot += w[k] * np.sum(G[m - 1 - k].T * Sigma[k])
    return -0.5 * float(tot)


def fermi(xi: np.ndarray, beta: float) -> np.ndarray:
    """f(xi) = 1 / (1 + exp(beta xi)), evaluated without overflow."""
    out = np.empty_like(xi, dtype=float)
    pos = xi >= 0
    e = np.exp(-beta * np.abs(xi))
    out[pos] = e[pos] / (1.0 + e[pos])
    out[~pos] = 1.0 / (1.0 + e[~pos])
    return out


def sox_energy_g0_closed_form(v_mo: np.ndarray, xi: np.ndarray, beta: float) -> float:
    """E_SOX at the independent-particle G, integrated over tau analytically.

    In the orbital basis that diagonalises the Fock operator G0 is diagonal,
    g_p(tau) = -exp(-xi_p tau) (1 - f_p).  Inserting it into the SOX expression
    and the energy reading above,

        E = 1/2 sum_{pqst} (pt|qs)(tq|sp) int_0^beta g_p(t) g_q(t) g_s(b-t) g_t(b-t) dt

    and the integral of the four exponentials is
        [f_p f_q (1-f_s)(1-f_t) - (1-f_p)(1-f_q) f_s f_t] / (xi_s + xi_t - xi_p - xi_q),
    written below in the expm1 form that stays finite when the denominator
    vanishes.  At zero temperature this is twice the MP2 exchange energy.
    """
    f = fermi(xi, beta)
    h = 1.0 - f
    a = xi[:, None] + xi[None, :]            # a[p, q] = xi_p + xi_q
    ff = f[:, None] * f[None, :]             # f_p f_q
    hh = h[:, None] * h[None, :]             # (1-f_p)(1-f_q)
    # d[p,q,s,t] = b - a with b = xi_s + xi_t
    d = a[None, None, :, :] - a[:, :, None, None]
    num_pos = ff[:, :, None, None] * hh[None, None, :, :]     # f_p f_q (1-f_s)(1-f_t)
    num_neg = hh[:, :, None, None] * ff[None, None, :, :]     # (1-f_p)(1-f_q) f_s f_t
    ad = np.abs(d)
    small = ad < 1e-300
    safe = np.where(small, 1.0, ad)
    kern = np.where(small, beta, -np.expm1(-beta * safe) / safe)
    integ = np.where(d >= 0, num_pos, num_neg) * kern
    # (pt|qs)(tq|sp) with v_mo[a,b,c,d] = (ab|cd)
    pref = np.einsum("ptqs,tqsp->pqst", v_mo, v_mo, optimize=True)
    return 0.5 * float(np.sum(pref * integ))


def mp2_exchange(v_mo: np.ndarray, eps: np.ndarray, occ: np.ndarray) -> float:
    """Spin-orbital MP2 exchange term at zero temperature:
    E_x = 1/2 sum_{ij occ, ab virt} (ia|jb)(ib|ja) / (e_a + e_b - e_i - e_j)."""
    o = np.where(occ)[0]
    vv = np.where(~occ)[0]
    iajb = v_mo[np.ix_(o, vv, o, vv)]                      # (ia|jb)
    ibja = np.transpose(iajb, (0, 3, 2, 1))                 # (ib|ja)[i,a,j,b]
    den = (eps[vv][None, :, None, None] + eps[vv][None, None, None, :]
           - eps[o][:, None, None, None] - eps[o][None, None, :, None])
    return 0.5 * float(np.sum(iajb * ibja / den))


def to_mo(v: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """(ab|cd) in the orbital basis Q (columns are orbitals)."""
    return np.einsum("pqrs,pa,qb,rc,sd->abcd", v, Q, Q, Q, Q, optimize=True)
