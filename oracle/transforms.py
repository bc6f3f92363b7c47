"""Imaginary-time <-> Matsubara transforms, Dyson equation and one
self-consistency iteration, in FP64 (test infrastructure only).

Paper: Sec. "Definitions" (Dyson equation, Eq. Dyson, and the density matrix).
The paper runs on intermediate-representation grids and cites Chebyshev grids
as an alternative; the readings used here are:

* tau grid: roots of T_m mapped to [0, beta], x_k = 2 tau_k / beta - 1.
* forward transform: interpolate F(tau) by the Chebyshev series through the
  roots, F(tau) = sum_l c_l T_l(x), and integrate each term exactly against
  exp(i w_n tau): F(i w_n) = sum_l T_nl c_l with
  T_nl = int_0^beta exp(i w_n tau) T_l(2 tau/beta - 1) dtau, w_n = (2n+1) pi / beta.
* backward transform: the real coefficients c that minimise
  sum_n |sum_l T_nl c_l - F(i w_n)|^2 over the n >= 0 frequencies kept.
* Dyson in an orthonormal basis: G(i w_n) = [(i w_n + mu) 1 - F - Sigma(i w_n)]^-1.
* density matrix gamma = -G(beta^-) = -sum_l c_l (T_l(1) = 1).
"""
from __future__ import annotations

import numpy as np


def cheb_nodes(m: int) -> np.ndarray:
    """Ascending roots of T_m: x_k = -cos((2k+1) pi / 2m)."""
    k = np.arange(m)
    return -np.cos((2 * k + 1) * np.pi / (2 * m))


def cheb_vander(x: np.ndarray, L: int) -> np.ndarray:
    """V[k, l] = T_l(x_k) by the three-term recurrence."""
    V = np.empty((len(x), L))
    V[:, 0] = 1.0
    if L > 1:
        V[:, 1] = x
    for l in range(2, L):
        V[:, l] = 2 * x * V[:, l - 1] - V[:, l - 2]
    return V


def cheb_coeffs(F_tau: np.ndarray) -> np.ndarray:
    """Interpolating Chebyshev coefficients through the m roots:
    c_l = (2 - delta_l0)/m sum_k F(tau_k) T_l(x_k)  (discrete orthogonality)."""
    m = F_tau.shape[0]
    T = cheb_vander(cheb_nodes(m), m)                 # [k, l]
    scale = np.full(m, 2.0 / m); scale[0] = 1.0 / m
    return np.einsum("kl,k...->l...", T, F_tau) * scale.reshape((m,) + (1,) * (F_tau.ndim - 1))


def matsubara_freqs(nw: int, beta: float) -> np.ndarray:
    return (2 * np.arange(nw) + 1) * np.pi / beta


def cheb_to_matsubara(m: int, nw: int, beta: float, panels: int = 2048,
                      order: int = 16) -> np.ndarray:
    """T[n, l] = int_0^beta exp(i w_n tau) T_l(2 tau/beta - 1) dtau by composite
    Gauss-Legendre quadrature (``panels`` equal panels of ``order`` points)."""
    gx, gw = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(-1.0, 1.0, panels + 1)
    half = 0.5 * (edges[1:] - edges[:-1])
    mid = 0.5 * (edges[1:] + edges[:-1])
    x = (mid[:, None] + half[:, None] * gx[None, :]).ravel()
    wx = (half[:, None] * gw[None, :]).ravel()
    tau = 0.5 * beta * (1.0 + x)
    wt = 0.5 * beta * wx
    Tl = cheb_vander(x, m)                            # [pts, l]
    wn = matsubara_freqs(nw, beta)
    E = np.exp(1j * np.outer(wn, tau)) * wt[None, :]  # [n, pts]
    return E @ Tl


def tau_to_matsubara(F_tau: np.ndarray, Tmat: np.ndarray) -> np.ndarray:
    """F(i w_n) = sum_l T_nl c_l with c the interpolating coefficients."""
    c = cheb_coeffs(F_tau)
    return np.einsum("nl,l...->n...", Tmat, c)


def fit_coeffs_from_matsubara(F_iw: np.ndarray, Tmat: np.ndarray) -> np.ndarray:
    """Real least-squares Chebyshev coefficients from F(i w_n), n = 0..nw-1:
    stack real and imaginary parts, solve min ||[Re T; Im T] c - [Re F; Im F]||."""
    nw, m = Tmat.shape
    A = np.concatenate([Tmat.real, Tmat.imag], axis=0)            # [2nw, m]
    rhs = np.concatenate([F_iw.real, F_iw.imag], axis=0).reshape(2 * nw, -1)
    c, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    return c.reshape((m,) + F_iw.shape[1:])


def coeffs_to_tau(c: np.ndarray) -> np.ndarray:
    m = c.shape[0]
    T = cheb_vander(cheb_nodes(m), m)
    return np.einsum("kl,l...->k...", T, c)


def dyson(F: np.ndarray, mu: float, Sigma_iw: np.ndarray, beta: float) -> np.ndarray:
    """G(i w_n) = [(i w_n + mu) 1 - F - Sigma(i w_n)]^-1 for every kept n."""
    nw, n, _ = Sigma_iw.shape
    wn = matsubara_freqs(nw, beta)
    out = np.empty_like(Sigma_iw, dtype=complex)
    eye = np.eye(n)
    for i in range(nw):
        out[i] = np.linalg.inv((1j * wn[i] + mu) * eye - F - Sigma_iw[i])
    return out


def density_matrix_from_coeffs(cG: np.ndarray) -> np.ndarray:
    """gamma = -G(beta^-) = -sum_l c_l T_l(1)."""
    return -np.sum(cG, axis=0)


def loop_step(F: np.ndarray, mu: float, beta: float, Sigma_tau: np.ndarray,
              Tmat: np.ndarray):
    """Sigma(tau) -> Sigma(i w_n) -> Dyson -> fitted G(tau) and gamma."""
    S_iw = tau_to_matsubara(Sigma_tau, Tmat)
    G_iw = dyson(F, mu, S_iw, beta)
    cG = fit_coeffs_from_matsubara(G_iw, Tmat)
    return coeffs_to_tau(cG), density_matrix_from_coeffs(cG), G_iw
