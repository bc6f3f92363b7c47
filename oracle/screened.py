"""Exchange self-energies with screened interaction lines, FP64 (test
infrastructure only: imported by tests, the smoke check and the CPU baseline).

The paper notes that contractions of the SOX type also appear when one
interaction line of the exchange diagram is screened (second-order screened
exchange, SOSEX) or both are (G3W2), and names these as its next step
(closing paragraph of Sec. "THC-scGF2: algorithm and implementation details";
Sec. "Conclusions and future work").  It prints no formula for them.  The
readings used here:

* Polarization in the THC basis: the bubble of the direct term,
      Pi(tau)_QS = Gt_QS(tau) Gbt_SQ(tau),   Gt = X^T G(tau) X,  Gbt = X^T G(beta - tau) X
  (positive semidefinite for the independent-particle G: the physical,
  negative irreducible polarization is -Pi, consistent with the + sign of the
  direct term, which is the second-order GW term).
* Static screening: the interaction line is the random-phase-screened
  interaction at zero bosonic frequency,
      Pi0 = int_0^beta Pi(tau) dtau     (the grid's quadrature weights),
      W   = V (1 + Pi0 V)^-1            (= V - V Pi0 V + V Pi0 V Pi0 V - ...),
  instantaneous like the bare line, so the SOX time reduction applies
  unchanged and the contraction is literally the SOX one with a second core
  matrix.  (The dynamically screened line would turn each tau point into a
  convolution over a second time; not done.)
* Which line: with cores Va on the line (pr|qs) and Vc on the line (tu|vw),
      Sigma[Va; Vc]_tr = - sum (pr|qs)_Va (tu|vw)_Vc G_wp(tau) G_uq(tau) G_sv(-tau);
  SOSEX screens one line and is symmetrised over the two choices,
      Sigma^SOSEX = (Sigma[V; W] + Sigma[W; V]) / 2,
  G3W2 screens both, Sigma^G3W2 = Sigma[W; W].  For symmetric G,
  Sigma[W; V] = Sigma[V; W]^T.
Pins (tests): W against the series and the screening inequality W <= V, Pi0
against its closed form for the independent-particle G, both self-energies
against the six-index definition with the screened integrals assembled, and
Pi0 = 0 (W = V) reproducing SOX.
"""
from __future__ import annotations

import numpy as np

from . import sox as _sox


def polarization_tau(X: np.ndarray, G: np.ndarray, Gb: np.ndarray) -> np.ndarray:
    """Pi(tau)_QS = Gt_QS Gbt_SQ with Gt = X^T G X, Gbt = X^T Gb X (Gb = G(beta - tau))."""
    Gt = X.T @ G @ X
    Gbt = X.T @ Gb @ X
    return Gt * Gbt.T


def static_polarization(X: np.ndarray, G: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Pi0 = sum_k w_k Pi(tau_k) on a mirror-symmetric grid (G(beta - tau_k) = G[m-1-k])."""
    m = G.shape[0]
    naux = X.shape[1]
    P = np.zeros((naux, naux))
    for k in range(m):
        P += w[k] * polarization_tau(X, G[k], G[m - 1 - k])
    return P


def static_polarization_g0(X, Q, eps, mu, beta) -> np.ndarray:
    """Closed form of int_0^beta Pi(tau) dtau for the independent-particle
    G0(tau) = -Q diag((1 - f) e^{-xi tau}) Q^T (0 < tau < beta), whose mirror is
    G0(beta - tau) = -Q diag(f e^{xi tau}) Q^T.  With psi = X^T Q (the THC image
    of the orbitals), xi = eps - mu and f the Fermi function,
        Pi0_QS = sum_jk c_jk (psi_jQ psi_kQ) (psi_jS psi_kS),
        c_jk = (1 - f_j) f_k int_0^beta e^{-(xi_j - xi_k) tau} dtau
             = (f_k - f_j) / (xi_j - xi_k)          (xi_j != xi_k)
             = beta (1 - f_j) f_j                    (xi_j == xi_k)
    (the Lindhard weights; (1 - f_j) f_k e^{-beta (xi_j - xi_k)} = f_j (1 - f_k))."""
    xi = np.asarray(eps, dtype=float) - mu
    f = np.array([_f(x, beta) for x in xi])
    psi = (X.T @ Q).T                      # psi[j, Q]
    n = len(xi)
    Pi0 = np.zeros((X.shape[1], X.shape[1]))
    for j in range(n):
        for k in range(n):
            d = xi[j] - xi[k]
            c = beta * (1.0 - f[j]) * f[j] if abs(d) < 1e-12 else (f[k] - f[j]) / d
            v = psi[j] * psi[k]
            Pi0 += c * np.outer(v, v)
    return Pi0


def _f(x, beta):
    """Fermi function 1 / (1 + e^{beta x}) without overflow."""
    if x >= 0:
        e = np.exp(-beta * x)
        return e / (1.0 + e)
    return 1.0 / (1.0 + np.exp(beta * x))


def screened_core(V: np.ndarray, Pi0: np.ndarray) -> np.ndarray:
    """W = V (1 + Pi0 V)^-1 (a linear solve: (1 + V Pi0) W = V, the same matrix)."""
    naux = V.shape[0]
    return np.linalg.solve(np.eye(naux) + V @ Pi0, V)


def sigma_two_cores(X: np.ndarray, Va: np.ndarray, Vc: np.ndarray, G: np.ndarray,
                    Gb: np.ndarray) -> np.ndarray:
    """Sigma[Va; Vc] by the paper's THC sequence with the line (pr|qs) on core Va
    (its U enters A) and the line (tu|vw) on core Vc (its U enters C):
        A_Pqv = sum_s Ua_Pqs G_sv(-tau),  B_PRv = sum_q G_Rq A_Pqv,
        C_RvP = sum_w Uc_Rvw G_wP,        D_PR  = sum_v C_RvP B_PRv,
        Sigma = X (-D^T) X^T."""
    Ua = _sox.precontract_u(X, Va)
    Uc = _sox.precontract_u(X, Vc)
    GR = X.T @ G
    GwP = G @ X
    A = Ua @ Gb                                # [P, q, v]
    B = np.matmul(GR, A)                       # [P, R, v]
    C = Uc @ GwP                               # [R, v, P]
    D = np.einsum("RvP,PRv->PR", C, B, optimize=True)
    return X @ (-D.T) @ X.T


def sigma_two_cores_bruteforce(X, Va, Vc, G, Gb) -> np.ndarray:
    """The six-index definition with both ERI tensors assembled (n <= 8):
    Sigma_tr = - sum (pr|qs)_Va (tu|vw)_Vc G_wp G_uq Gb_sv."""
    va = _sox.thc_eri(X, Va)
    vc = _sox.thc_eri(X, Vc)
    n = G.shape[0]
    out = np.empty((n, n))
    for t in range(n):
        for r in range(n):
            out[t, r] = -np.einsum("pqs,uvw,wp,uq,sv->", va[:, r, :, :], vc[t, :, :, :],
                                   G, G, Gb, optimize=False)
    return out


def sigma_sosex(X, V, W, G, Gb, two=sigma_two_cores) -> np.ndarray:
    """(Sigma[V; W] + Sigma[W; V]) / 2: one line screened, both placements."""
    return 0.5 * (two(X, V, W, G, Gb) + two(X, W, V, G, Gb))


def sigma_g3w2(X, W, G, Gb, two=sigma_two_cores) -> np.ndarray:
    """Sigma[W; W]: both lines screened."""
    return two(X, W, W, G, Gb)
