"""SOX self-energy in FP64, four independent ways (test infrastructure only).

Paper: Sec. "THC-scGF2: algorithm and implementation details".

All functions work on one imaginary-time point: ``G`` is G(tau) [n, n] and
``Gb`` is the value used for G(-tau), i.e. G(beta - tau) (the mirrored grid
point).  ``sigma_all_tau`` applies one of them over a mirror-symmetric grid.

Index convention: G[p, q] = G_pq(tau).  The electron-repulsion integrals are
in chemists' notation, v[p, r, q, s] = (pr|qs).
"""
from __future__ import annotations

import numpy as np


def thc_eri(X: np.ndarray, V: np.ndarray) -> np.ndarray:
    """(ij|kl) = sum_PQ X_iP X_jP V_PQ X_kQ X_lQ  (Eq. THC_ERI, real X).

    Assembled in two steps: the pair density X_iP X_jP for every P, then the
    contraction with V and the second pair density.
    """
    pair = np.einsum("iP,jP->ijP", X, X)            # [n, n, naux]
    half = pair @ V                                    # [n, n, naux]: sum_P pair_ijP V_PQ
    return np.einsum("ijQ,klQ->ijkl", half, pair)


def sigma_bruteforce(v: np.ndarray, G: np.ndarray, Gb: np.ndarray) -> np.ndarray:
    """Literal definition, one (t, r) element at a time:

        Sigma_tr = - sum_{pqsuvw} (pr|qs) (tu|vw) G_wp(tau) G_uq(tau) G_sv(-tau)

    (the final SOX expression after the instantaneous-interaction time
    reduction).  No factorisation at all: the whole six-index sum is evaluated
    for every output element.  Only for n <= 8.
    """
    n = G.shape[0]
    out = np.empty((n, n))
    for t in range(n):
        for r in range(n):
            # all six summation indices at once, no intermediate contraction
            out[t, r] = -np.einsum("pqs,uvw,wp,uq,sv->", v[:, r, :, :], v[t, :, :, :],
                                   G, G, Gb, optimize=False)
    return out


def sigma_eri_chain(v: np.ndarray, G: np.ndarray, Gb: np.ndarray) -> np.ndarray:
    """Conventional O(n^5) route: contract one Green's function at a time, the
    way standard ERI transformations do (described after the SOX expression).

        I1[w,r,q,s] = sum_p G_wp (pr|qs)
        I2[w,r,u,s] = sum_q G_uq I1[w,r,q,s]
        I3[w,r,u,v] = sum_s G_sv(-tau) I2[w,r,u,s]
        Sigma_tr    = - sum_{uvw} (tu|vw) I3[w,r,u,v]
    """
    I1 = np.einsum("wp,prqs->wrqs", G, v, optimize=True)
    I2 = np.einsum("uq,wrqs->wrus", G, I1, optimize=True)
    I3 = np.einsum("sv,wrus->wruv", Gb, I2, optimize=True)
    return -np.einsum("tuvw,wruv->tr", v, I3, optimize=True)


def sigma_thc_basis(X: np.ndarray, V: np.ndarray, G: np.ndarray,
                    Gb: np.ndarray) -> np.ndarray:
    """The definition with v = THC(X, V) substituted and every orbital sum done
    first (quartic in the number of THC points, used only as a cross-check):

        Sigma_tr = - sum_{PQRS} X_tR X_rP V_PQ V_RS  Gw_SP  Gw_RQ  Gbw_QS
        with Gw = X^T G X (the six orbital sums pair up into three projected G).

    The pairing: (pr|qs)(tu|vw) = X_pP X_rP V_PQ X_qQ X_sQ . X_tR X_uR V_RS X_vS X_wS;
    G_wp pairs X_wS with X_pP, G_uq pairs X_uR with X_qQ, G_sv pairs X_sQ with X_vS.
    """
    Gw = X.T @ G @ X         # Gw[S, P] = sum_wp X_wS G_wp X_pP
    Gbw = X.T @ Gb @ X       # Gbw[Q, S] = sum_sv X_sQ Gb_sv X_vS
    naux = X.shape[1]
    D = np.empty((naux, naux))   # D[P, R]
    for R in range(naux):
        # H[Q, P] = sum_S Gbw[Q, S] V[R, S] Gw[S, P]
        H = (Gbw * V[R][None, :]) @ Gw
        # D[P, R] = sum_Q V[P, Q] Gw[R, Q] H[Q, P]
        D[:, R] = np.einsum("PQ,Q,QP->P", V, Gw[R], H)
    return -(X @ D.T @ X.T)


def sigma_thc_paper(X: np.ndarray, V: np.ndarray, G: np.ndarray, Gb: np.ndarray,
                    U: np.ndarray | None = None, return_thc: bool = False,
                    p_block: int = 256):
    """The paper's THC-SOX contraction sequence (Eq. U_contraction and the
    eight equations after it), conjugates dropped (real inputs):

        U_Pqs    = sum_Q  V_PQ X_qQ X_sQ                 (once per system)
        G_Rq     = sum_u  X_uR G_uq(tau)                 (printed "sum_uq": sum over u)
        G_wP     = sum_p  G_wp(tau) X_pP                 (printed "sum_uq": sum over p)
        A_Pqv    = sum_s  U_Pqs G_sv(-tau)
        B_PRv    = sum_q  A_Pqv G_Rq
        C_RvP    = sum_w  U_Rvw G_wP
        D_PR     = sum_v  C_RvP B_PRv
        Sig_RP   = -D_PR
        Sigma_tr = sum_PR X_tR Sig_RP X_rP

    Each equation is evaluated as written.  To bound memory, the equations for
    A, B, C and D are evaluated for one block of P at a time (P is a free index
    of all four, so this changes no sum).
    """
    n, naux = X.shape
    if U is None:
        U = precontract_u(X, V)
    GR = X.T @ G                       # G_Rq   [naux, n]
    GwP = G @ X                        # G_wP   [n, naux]
    D = np.empty((naux, naux))         # D[P, R]
    for p0 in range(0, naux, p_block):
        p1 = min(naux, p0 + p_block)
        A = U[p0:p1] @ Gb              # A[P, q, v] = sum_s U[P, q, s] Gb[s, v]
        B = np.matmul(GR, A)           # B[P, R, v] = sum_q G_Rq A[P, q, v]
        C = U @ GwP[:, p0:p1]          # C[R, v, P] = sum_w U[R, v, w] G_wP
        D[p0:p1] = np.einsum("RvP,PRv->PR", C, B, optimize=True)   # sum over v
    sig_thc = -D.T                     # Sig[R, P] = -D[P, R]
    sigma = X @ sig_thc @ X.T          # Sigma[t, r] = sum_RP X_tR Sig_RP X_rP
    if return_thc:
        return sigma, sig_thc
    return sigma


def sig_thc_elements(X: np.ndarray, V: np.ndarray, G: np.ndarray, Gb: np.ndarray,
                     pairs) -> np.ndarray:
    """Selected elements Sig_RP = -D_PR of the paper's sequence (the equations
    listed in ``sigma_thc_paper``) for a list of (R, P) pairs, without forming
    U, A, B, C or D whole -- for sizes where those do not fit in host memory.

    For one pair only the slices with first index P or R enter:
        U_Pqs = sum_Q V_PQ X_qQ X_sQ     (Eq. U_contraction: X diag(V_P) X^T)
        A_Pqv = sum_s U_Pqs G_sv(-tau)
        B_PRv = sum_q A_Pqv G_Rq,  G_Rq = sum_u X_uR G_uq(tau)
        C_RvP = sum_w U_Rvw G_wP,  G_wP = sum_p G_wp(tau) X_pP
        D_PR  = sum_v C_RvP B_PRv
    """
    out = np.empty(len(pairs))
    for i, (R, P) in enumerate(pairs):
        U_P = (X * V[P]) @ X.T             # U[P, q, s]
        U_R = (X * V[R]) @ X.T             # U[R, v, w]
        A_P = U_P @ Gb                     # A[P, q, v]
        G_R = X[:, R] @ G                  # G_Rq
        G_P = G @ X[:, P]                  # G_wP
        B = G_R @ A_P                      # B[P, R, v]
        C = U_R @ G_P                      # C[R, v, P]
        out[i] = -float(C @ B)             # Sig_RP = -sum_v C_RvP B_PRv
    return out


def precontract_u(X: np.ndarray, V: np.ndarray) -> np.ndarray:
    """U_Pqs = sum_Q V_PQ X_qQ X_sQ (Eq. U_contraction); shape [naux, n, n]."""
    n, naux = X.shape
    pair = np.einsum("qQ,sQ->Qqs", X, X).reshape(naux, n * n)
    return (V @ pair).reshape(naux, n, n)


def sigma_all_tau(fn, G: np.ndarray, *args, taus=None, **kw) -> np.ndarray:
    """Apply a single-point SOX function at grid points ``taus`` (default all).

    On a mirror-symmetric grid G(beta - tau_k) is stored at index m-1-k.
    Returns an array [len(taus), n, n] (plus the THC-basis array when asked).
    """
    m = G.shape[0]
    ks = range(m) if taus is None else taus
    outs = [fn(*args, G[k], G[m - 1 - k], **kw) for k in ks]
    if outs and isinstance(outs[0], tuple):
        return tuple(np.stack(z) for z in zip(*outs))
    return np.stack(outs)
