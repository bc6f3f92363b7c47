"""Second-order direct (bubble) self-energy of GF2 in FP64 (test infrastructure
only: imported by tests, the smoke check and the CPU baseline).

The paper includes the GF2 direct term (Sec. "Self-energy functionals", the
diagram figure; full scGF2 = direct + SOX) and states that its THC treatment
follows the THC-GW work it cites, without printing a formula.  The readings
used here:

* Definition, in the spin-orbital convention of the SOX term, with the same
  instantaneous-interaction time reduction and the same reading of G(-tau) as
  the value stored at beta - tau; the closed fermion loop of the bubble flips
  the sign relative to the exchange term:
      Sigma^dir_tr = + sum_{pqsuvw} (tu|vw) (pr|qs) G_up(tau) G_wq(tau) G_sv(-tau)
* THC form (expanding both ERIs with X and V):
      Gt = X^T G(tau) X,  Gbt = X^T G(beta - tau) X,
      Pi_QS = Gt_QS Gbt_SQ,  W = V Pi V,  Sigma^dir = X (W o Gt) X^T
  (o: elementwise product), 2 naux^3 + O(naux^2 n) work per tau.
Pins (tests): the THC form against the six-index definition on a non-symmetric
G, and E[G0] -> 2 x the spin-orbital MP2 Coulomb term at low temperature (the
same functional that gives 2 x the exchange term for SOX).
"""
from __future__ import annotations

import numpy as np


def sigma_direct_bruteforce(v: np.ndarray, G: np.ndarray, Gb: np.ndarray) -> np.ndarray:
    """The six-index definition, one (t, r) element at a time (n <= 8)."""
    n = G.shape[0]
    out = np.empty((n, n))
    for t in range(n):
        for r in range(n):
            out[t, r] = np.einsum("uvw,pqs,up,wq,sv->", v[t, :, :, :], v[:, r, :, :],
                                  G, G, Gb, optimize=False)
    return out


def sigma_direct_thc(X: np.ndarray, V: np.ndarray, G: np.ndarray, Gb: np.ndarray) -> np.ndarray:
    """Gt = X^T G X, Pi = Gt o Gbt^T, W = V Pi V, Sigma = X (W o Gt) X^T."""
    Gt = X.T @ G @ X
    Gbt = X.T @ Gb @ X
    Pi = Gt * Gbt.T
    W = V @ Pi @ V
    return X @ (W * Gt) @ X.T


def mp2_coulomb(v_mo: np.ndarray, eps: np.ndarray, occ: np.ndarray) -> float:
    """Spin-orbital MP2 Coulomb (direct) term at zero temperature:
    E_J = -1/2 sum_{ij occ, ab virt} (ia|jb)^2 / (e_a + e_b - e_i - e_j)."""
    o = np.where(occ)[0]
    vv = np.where(~occ)[0]
    iajb = v_mo[np.ix_(o, vv, o, vv)]
    den = (eps[vv][None, :, None, None] + eps[vv][None, None, None, :]
           - eps[o][:, None, None, None] - eps[o][None, None, :, None])
    return -0.5 * float(np.sum(iajb * iajb / den))
