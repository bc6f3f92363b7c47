"""Intermediate-representation (IR) basis and sparse sampling in FP64 (test
infrastructure only: imported by tests, the smoke check and the CPU baseline).

The paper runs its loop on IR grids with sparse sampling in tau and in
Matsubara frequency (computational-details section; the basis and the sampling
method are those of the references it cites).  Written here from their
definitions:

* Fermionic kernel, tau in [0, beta], omega in [-wmax, wmax], Lambda = beta wmax:
      K(tau, omega) = exp(-tau omega) / (1 + exp(-beta omega)),
  so a Green's function with spectral function rho is G(tau) = -int K rho.
  In x = 2 tau / beta - 1, y = omega / wmax it is
      K(x, y) = exp(-Lambda y (x + 1) / 2) / (1 + exp(-Lambda y)).
* Its singular value expansion on [-1, 1]^2, K(x, y) = sum_l s_l u_l(x) v_l(y),
  truncated at s_l / s_0 >= eps, gives the basis u_l.  Here: piecewise
  Gauss-Legendre quadrature (segments graded geometrically towards the edges
  of x and the centre of y, where K varies on the scale 1 / Lambda), the SVD of
  sqrt(w_x) K sqrt(w_y), and Nystrom evaluation away from the nodes,
      u_l(x) = (1 / s_l) int K(x, y) v_l(y) dy.
* The Matsubara transform of each Nystrom term is closed form: the transform
  of K(., omega) at i w_n = (2n + 1) pi / beta is 1 / (omega - i w_n).
* Sampling: the tau points are the L roots of u_L (the first basis function
  past the cut), mirror-symmetric by parity; the Matsubara points are the
  n >= 0 where one of the last four functions u_{L-3} .. u_L changes sign in
  frequency (each transform is purely real or purely imaginary by parity),
  plus n = 0.  For real G(tau) the negative frequencies are the complex
  conjugates; the real and the imaginary parts each fix the coefficients of
  one parity, so about L/2 frequencies are the least a fit needs.  At low n the
  highest functions' transforms sit at their FP64 noise level, and the sign
  changes of u_{L-1} and u_L alone left some (Lambda, eps) fits with condition
  numbers of 1e7 and more; the four functions' union (about four times the
  minimum) keeps them below 1e3.
"""
from __future__ import annotations

import numpy as np

Q = 16   # Gauss-Legendre nodes per segment


def _segments(smallest: float, centre: bool) -> np.ndarray:
    """Breakpoints on [-1, 1], halving towards +-1 (centre=False) or towards 0
    (centre=True) down to `smallest`."""
    d = [1.0]
    while d[-1] > smallest:
        d.append(d[-1] / 2)
    d = np.array(d)
    if centre:
        half = np.concatenate([d[::-1], ])            # smallest .. 1
        return np.concatenate([-half[::-1], [0.0], half])
    # towards the edges: -1, -1 + smallest, ..., 0, ..., 1 - smallest, 1
    left = -1.0 + d[::-1][:-1]                        # -1 + smallest .. -1 + 1/2
    return np.concatenate([[-1.0], left, [0.0], -left[::-1], [1.0]])


def _gauss(breaks: np.ndarray):
    t, wt = np.polynomial.legendre.leggauss(Q)
    a, b = breaks[:-1, None], breaks[1:, None]
    x = (0.5 * (b - a) * t[None, :] + 0.5 * (a + b)).ravel()
    w = (0.5 * (b - a) * wt[None, :]).ravel()
    return x, w


def kernel_xy(x: np.ndarray, y: np.ndarray, lam: float) -> np.ndarray:
    """K(x, y) in the scaled variables, evaluated without overflow."""
    x = np.asarray(x, dtype=float)[:, None]
    y = np.asarray(y, dtype=float)[None, :]
    # exp(-lam y (x+1)/2) / (1 + exp(-lam y)); for y < 0 divide through by exp(-lam y)
    pos = y >= 0
    a = np.where(pos, -lam * y * (x + 1) / 2, lam * y * (1 - x) / 2)
    b = np.where(pos, np.exp(-lam * np.abs(y)), np.exp(-lam * np.abs(y)))
    return np.exp(a) / (1.0 + b)


class IRBasis:
    """Fermionic IR basis for Lambda = beta wmax, cut at s_l / s_0 >= eps."""

    def __init__(self, beta: float, wmax: float, eps: float = 1e-10):
        self.beta, self.wmax = float(beta), float(wmax)
        self.lam = self.beta * self.wmax
        small = 0.25 / self.lam
        self.x, self.wx = _gauss(_segments(small, centre=False))
        self.y, self.wy = _gauss(_segments(small, centre=True))
        A = np.sqrt(self.wx)[:, None] * kernel_xy(self.x, self.y, self.lam) * np.sqrt(self.wy)[None, :]
        Um, s, Vt = np.linalg.svd(A, full_matrices=False)
        L = int(np.sum(s / s[0] >= eps))
        self.s_all = s
        self.L = L
        self.s = s[:L + 1]                       # one past the cut (for the tau sampling)
        self.vw = Vt[:L + 1].T * np.sqrt(self.wy)[:, None]   # sqrt(w_y) V: [Ny, L+1]
        # sign convention: u_l(x -> 1) > 0
        sgn = np.sign(self.u_x(np.array([1.0]), all_=True)[0])
        self.vw *= sgn[None, :]

    # ---- real-axis functions -------------------------------------------------
    def u_x(self, x: np.ndarray, all_: bool = False) -> np.ndarray:
        """u_l(x) by Nystrom, [len(x), L] (or L + 1 with all_)."""
        K = kernel_xy(x, self.y, self.lam)
        out = (K @ self.vw) / self.s[None, :]
        return out if all_ else out[:, :self.L]

    def u_tau(self, tau: np.ndarray, all_: bool = False) -> np.ndarray:
        """u_l(tau) normalised on [0, beta]: sqrt(2 / beta) u_l(x(tau))."""
        x = 2.0 * np.asarray(tau) / self.beta - 1.0
        return np.sqrt(2.0 / self.beta) * self.u_x(x, all_)

    def uhat(self, n: np.ndarray, all_: bool = False) -> np.ndarray:
        """int_0^beta exp(i w_n tau) u_l(tau) dtau, w_n = (2n + 1) pi / beta: [len(n), L]."""
        wn = (2 * np.asarray(n, dtype=float) + 1) * np.pi / self.beta
        om = self.wmax * self.y
        ft = 1.0 / (om[None, :] - 1j * wn[:, None])           # transform of K(., omega_j)
        # u_l(tau) = sqrt(2/beta) (1/s_l) sum_j K(tau, omega_j) sqrt(w_j) V_jl
        out = np.sqrt(2.0 / self.beta) * (ft @ self.vw) / self.s[None, :]
        return out if all_ else out[:, :self.L]

    # ---- sampling --------------------------------------------------------------
    def tau_points(self) -> np.ndarray:
        """The L roots of u_L on (0, beta), ascending, mirror-symmetric."""
        L = self.L

        def f(x):
            return self.u_x(np.atleast_1d(x), all_=True)[:, L]

        # bracket on the quadrature nodes of the positive half (u_L has parity (-1)^L)
        xs = np.concatenate([[0.0], self.x[self.x > 0], [1.0]])
        fs = f(xs)
        roots = []
        for a, b, fa, fb in zip(xs[:-1], xs[1:], fs[:-1], fs[1:]):
            if fa == 0.0 and a == 0.0:
                continue
            if fa * fb < 0:
                for _ in range(200):                 # bisection to the last bit
                    mid = 0.5 * (a + b)
                    if mid == a or mid == b:
                        break
                    fm = f(mid)[0]
                    if fa * fm <= 0:
                        b, fb = mid, fm
                    else:
                        a, fa = mid, fm
                roots.append(0.5 * (a + b))
        pos = np.array(roots)
        xr = np.concatenate([-pos[::-1], [0.0], pos]) if L % 2 == 1 else \
            np.concatenate([-pos[::-1], pos])
        assert len(xr) == L, (len(xr), L)
        return self.beta * (xr + 1.0) / 2.0

    def matsubara_points(self, nmax: int | None = None) -> np.ndarray:
        """n >= 0 where one of uhat_{L-3} .. uhat_L (the last three kept functions
        and the first past the cut) changes sign in frequency -- the larger index
        of each change -- together with n = 0, ascending.  Each transform is
        purely real or purely imaginary (parity), so its sign is that of the
        non-zero part."""
        if nmax is None:
            nmax = int(10 * self.lam / (2 * np.pi)) + 10
        n = np.arange(nmax + 1)
        u = np.concatenate([self.uhat(n[c:c + 20000], all_=True)[:, self.L - 3:self.L + 1]
                            for c in range(0, len(n), 20000)])
        pts = [np.array([0])]
        for l in range(4):
            f = u[:, l]
            part = f.real if (self.L - 3 + l) % 2 == 1 else f.imag
            sgn = np.sign(part)
            pts.append(np.nonzero(sgn[1:] * sgn[:-1] < 0)[0] + 1)
        return np.unique(np.concatenate(pts))

def transforms(b: IRBasis, tau: np.ndarray, nfreq: np.ndarray):
    """Real matrices of the tau <-> i w transforms on the sampling points:
    Wf [2 nf, m]: [Re; Im] F(i w_n) = Wf F(tau_k) (fit on tau, evaluate in w);
    Wb [m + 1, 2 nf]: F(tau_k) and, last row, F(beta^-) from the least-squares
    fit of the coefficients to [Re; Im] F(i w_n)."""
    Ut = b.u_tau(tau)                         # [m, L]
    Uh = b.uhat(nfreq)                        # [nf, L]
    coef_from_tau = np.linalg.solve(Ut, np.eye(len(tau)))      # [L, m]
    F = Uh @ coef_from_tau
    Wf = np.vstack([F.real, F.imag])
    Uri = np.vstack([Uh.real, Uh.imag])      # [2 nf, L]
    fit = np.linalg.pinv(Uri)                # [L, 2 nf]
    ends = b.u_tau(np.array([b.beta]))       # u_l(beta^-)
    Wb = np.vstack([Ut @ fit, ends @ fit])
    return Wf, Wb


def energy_matrix(b: IRBasis, tau: np.ndarray) -> np.ndarray:
    """M [m, m] with int_0^beta A(beta - tau) B(tau) dtau = sum_kk' A(tau_k') M[k', k] B(tau_k)
    for A, B in the span of the basis: with a = Ut^-1 A, b = Ut^-1 B and
    u_l(beta - tau) = (-1)^l u_l(tau), the integral is sum_l (-1)^l a_l b_l."""
    Ut = b.u_tau(tau)
    Ui = np.linalg.solve(Ut, np.eye(len(tau)))
    par = (-1.0) ** np.arange(b.L)
    return Ui.T @ (par[:, None] * Ui)


def dyson_step_sampled(F: np.ndarray, mu: float, beta: float, Sigma_tau: np.ndarray,
                       Wf: np.ndarray, Wb: np.ndarray, nf: np.ndarray):
    """One Dyson step on the sampling grids (Sec. "Definitions", Eq. Dyson in an
    orthonormal basis): Sigma(i w_n) = Wf Sigma(tau) on the sampled n >= 0,
    G(i w_n) = [(i w_n + mu) 1 - F - Sigma(i w_n)]^-1, then G(tau_k) and
    gamma = -G(beta^-) from the least-squares fit (rows of Wb).
    Returns (G_tau [m, n, n], gamma [n, n])."""
    m, n, _ = Sigma_tau.shape
    nfr = len(nf)
    S = np.tensordot(Wf, Sigma_tau, axes=(1, 0))          # [2 nf, n, n]
    Siw = S[:nfr] + 1j * S[nfr:]
    wn = (2 * np.asarray(nf, dtype=float) + 1) * np.pi / beta
    Giw = np.stack([np.linalg.inv((1j * w + mu) * np.eye(n) - F - Siw[j])
                    for j, w in enumerate(wn)])
    Gri = np.concatenate([Giw.real, Giw.imag])            # [2 nf, n, n]
    out = np.tensordot(Wb, Gri, axes=(1, 0))              # [m + 1, n, n]
    return out[:m], -out[m]


def evaluate_at(b: IRBasis, tau: np.ndarray, F_tau: np.ndarray, tau_new: np.ndarray) -> np.ndarray:
    """The basis expansion fitted to F on the sampling points tau, evaluated at
    tau_new: F(tau_new) = U(tau_new) Ut^-1 F(tau).  F_tau: [m, ...]."""
    coef = np.linalg.solve(b.u_tau(tau), F_tau.reshape(len(tau), -1))
    return (b.u_tau(np.asarray(tau_new)) @ coef).reshape((len(tau_new),) + F_tau.shape[1:])
