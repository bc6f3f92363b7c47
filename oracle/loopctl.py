"""Loop control for the self-consistency iterations, in FP64 (test
infrastructure only: imported by tests, the smoke check and the CPU baseline).

Paper: Sec. "Definitions" (fully self-consistent Dyson solution "with the update
of the chemical potential") and the size-consistency appendix ("Case 2:
optimized chemical potential": mu is chosen every iteration so that the average
electron number stays fixed; damping and DIIS-type linear combinations of
self-energies are allowed).  The paper uses frequency-dependent commutator DIIS
from a companion paper and does not print it; two variants are built here:
plain Pulay DIIS on the self-energy residual, and a commutator DIIS whose
residual lives on the Matsubara grid (the reading below).

* N(mu) = Tr gamma(mu), gamma = -G(beta^-) from one Dyson solve at mu with the
  given Sigma (N increases with mu).
* find_mu: bracket the root of N(mu) - N_el by steps from the starting mu, then
  the Illinois variant of regula falsi (Dowell & Jarratt 1971) until
  |N(mu) - N_el| <= tol or the bracket is narrower than 1e-14 (1 + |mu|).
* damping: Sigma_next = alpha Sigma_in + (1 - alpha) Sigma_out.
* Pulay DIIS: residuals r_i = Sigma_out_i - Sigma_in_i of the last `depth`
  iterations; coefficients c minimise |sum_i c_i r_i|^2 subject to sum_i c_i = 1
  ((k+1) x (k+1) bordered system with B_ij = <r_i, r_j>); Sigma_next =
  sum_i c_i Sigma_out_i.
* Commutator DIIS (reading): at self-consistency G(i w) commutes with the
  matrix it inverts, so with G_i = Dyson(Sigma_in_i) the frequency-dependent
  error of iteration i is the commutator with the new self-energy,
      e_i(i w_n) = [G_i(i w_n), F + Sigma_out_i(i w_n)]
                 = G_i D_i - D_i G_i,    D_i = Sigma_out_i(i w_n) - Sigma_in_i(i w_n)
  (the two forms agree because G_i commutes with F + Sigma_in_i), on the kept
  frequencies n >= 0 (the n < 0 ones are complex conjugates); B_ij =
  Re sum_n Tr[e_i(i w_n)^H e_j(i w_n)], the same bordered system, Sigma_next =
  sum_i c_i Sigma_out_i.
"""
from __future__ import annotations

import numpy as np

from . import transforms as tr


def electron_number(F: np.ndarray, mu: float, beta: float, S_iw: np.ndarray,
                    Tmat: np.ndarray) -> float:
    """Tr gamma after one Dyson solve at chemical potential mu (S_iw fixed)."""
    G_iw = tr.dyson(F, mu, S_iw, beta)
    cG = tr.fit_coeffs_from_matsubara(G_iw, Tmat)
    return float(np.trace(tr.density_matrix_from_coeffs(cG)))


def find_mu(F: np.ndarray, beta: float, Sigma_tau: np.ndarray, Tmat: np.ndarray,
            nelec: float, mu0: float, tol: float = 1e-10, step: float = 0.1,
            max_eval: int = 80):
    """Chemical potential with Tr gamma = nelec; returns (mu, N(mu), evaluations)."""
    S_iw = tr.tau_to_matsubara(Sigma_tau, Tmat)

    def f(mu):
        return electron_number(F, mu, beta, S_iw, Tmat) - nelec

    evals = 1
    a, fa = mu0, f(mu0)
    if abs(fa) <= tol:
        return a, fa + nelec, evals
    # bracket: walk from mu0 against the sign of f, doubling the step
    d = -step if fa > 0 else step
    b, fb = a + d, f(a + d)
    evals += 1
    while fa * fb > 0 and evals < max_eval:
        a, fa = b, fb
        d *= 2.0
        b, fb = a + d, f(a + d)
        evals += 1
    if abs(fb) <= tol:
        return b, fb + nelec, evals
    if fa * fb > 0:
        raise RuntimeError("no bracket for the chemical potential")
    # Illinois: regula falsi on the bracket (a, b); when the new point falls on
    # the same side as b, the end a is kept and its value halved
    while evals < max_eval:
        c = (a * fb - b * fa) / (fb - fa)
        fc = f(c)
        evals += 1
        if abs(fc) <= tol or abs(b - a) <= 1e-14 * (1.0 + abs(c)):
            return c, fc + nelec, evals
        if fc * fb < 0:
            a, fa = b, fb
        else:
            fa *= 0.5
        b, fb = c, fc
    raise RuntimeError("chemical potential search did not converge")


def loop_step_mu(F: np.ndarray, mu0: float, beta: float, Sigma_tau: np.ndarray,
                 Tmat: np.ndarray, nelec: float, tol: float = 1e-10):
    """find_mu, then the Dyson step at that mu: (G_tau, gamma, mu, evaluations)."""
    mu, _, evals = find_mu(F, beta, Sigma_tau, Tmat, nelec, mu0, tol)
    G_tau, gam, _ = tr.loop_step(F, mu, beta, Sigma_tau, Tmat)
    return G_tau, gam, mu, evals


def damp(sigma_in: np.ndarray, sigma_out: np.ndarray, alpha: float) -> np.ndarray:
    """alpha Sigma_in + (1 - alpha) Sigma_out."""
    return alpha * sigma_in + (1.0 - alpha) * sigma_out


def diis_next(inputs: list, outputs: list) -> np.ndarray:
    """Pulay extrapolation over the given (Sigma_in, Sigma_out) history."""
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
    c = np.linalg.solve(B, rhs)[:k]
    out = np.zeros_like(outputs[0])
    for ci, o in zip(c, outputs):
        out += ci * o
    return out


def commutator_residual(G_iw: np.ndarray, D_iw: np.ndarray) -> np.ndarray:
    """e(i w_n) = G(i w_n) D(i w_n) - D(i w_n) G(i w_n) for every kept n."""
    return np.matmul(G_iw, D_iw) - np.matmul(D_iw, G_iw)


def commutator_residual_definition(G_iw: np.ndarray, F: np.ndarray,
                                   Sout_iw: np.ndarray) -> np.ndarray:
    """[G(i w_n), F + Sigma_out(i w_n)] written out (the defining form)."""
    H = F[None, :, :] + Sout_iw
    return np.matmul(G_iw, H) - np.matmul(H, G_iw)


def cdiis_next(residuals: list, outputs: list) -> np.ndarray:
    """Extrapolation with B_ij = Re sum Tr[e_i^H e_j] over the given history of
    frequency-dependent residuals and output self-energies (tau)."""
    k = len(residuals)
    B = np.zeros((k + 1, k + 1))
    for i in range(k):
        for j in range(k):
            B[i, j] = float(np.real(np.vdot(residuals[i].ravel(), residuals[j].ravel())))
    B[k, :k] = 1.0
    B[:k, k] = 1.0
    rhs = np.zeros(k + 1)
    rhs[k] = 1.0
    c = np.linalg.solve(B, rhs)[:k]
    out = np.zeros_like(outputs[0])
    for ci, o in zip(c, outputs):
        out += ci * o
    return out
