"""Seeded synthetic inputs for the THC-SOX self-energy.

This module only draws inputs.  It holds none of the self-energy, energy,
transform or Dyson arithmetic, so both the GPU path and the FP64 CPU oracle can
consume exactly the same arrays without sharing any code of the method.

What is drawn (one ``numpy.random.default_rng(seed)`` stream, in this order):

1. ``A ~ N(0,1)[n,n]`` -> QR -> ``Q * sign(diag R)``: a Haar-random orthogonal
   matrix whose columns are the molecular orbitals of a model Fock operator.
2. ``eps_occ ~ U(-1.5,-0.3)[n_occ]`` and ``eps_virt ~ U(0.1,2.0)[n-n_occ]``
   orbital energies in Hartree; ``mu`` sits at mid-gap.
3. ``X ~ N(0, 1/n)[n, naux]``: the collocation matrix of the THC factorisation
   (paper, Sec. "Tensor hypercontraction", Eq. THC_ERI).  The variance is 1/n.
4. ``L ~ N(0,1)[naux,naux]`` and ``V = lam * L L^T / naux``: a symmetric
   positive semi-definite core matrix, the same Gram structure as the LS-THC
   core ``U_PQ = sum_C A^C_P A^C_Q`` of the paper.

The imaginary-time grid is the set of roots of the Chebyshev polynomial T_m
mapped to [0, beta]; it is mirror symmetric, so G(beta - tau_k) is stored at
index m-1-k.  Its quadrature weights are Fejer's first rule.  The starting
Green's function is the independent-particle one in closed form, written so
that no exponential overflows (exp(+beta*xi) never appears).

Nothing here depends on torch or on the compiled library.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

# Workload shapes (orbitals n, THC points naux, tau points m, inverse temperature beta).
WORKLOADS = {
    # tiny case, brute-force checkable
    "sox_n8_naux32_ntau12": dict(n=8, naux=32, m=12, beta=100.0),
    # one self-consistency iteration case (256 Matsubara points)
    "sox_n100_naux500_ntau64": dict(n=100, naux=500, m=64, beta=100.0, nw=256),
    # the mixed-precision throughput case
    "sox_n300_naux1800_ntau100": dict(n=300, naux=1800, m=100, beta=100.0),
    # one-GPU share at paper scale
    "sox_n1100_naux5500_ntau100": dict(n=1100, naux=5500, m=100, beta=100.0),
    # the paper's largest system size with its interpolation ratio naux / n = 10
    "sox_n1127_naux11270_ntau100": dict(n=1127, naux=11270, m=100, beta=100.0),
}


@dataclasses.dataclass
class System:
    """One generated system: model Fock operator, THC factors and grid."""

    n: int
    naux: int
    n_occ: int
    Q: np.ndarray        # [n, n] orthogonal, columns = orbitals
    eps: np.ndarray      # [n] orbital energies (occupied first)
    mu: float            # chemical potential at mid-gap
    X: np.ndarray        # [n, naux]
    V: np.ndarray        # [naux, naux] symmetric PSD
    lam: float = 1.0     # interaction scale already folded into V

    @property
    def F(self) -> np.ndarray:
        return (self.Q * self.eps) @ self.Q.T

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.Q, self.eps, self.X, self.V):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]


def make_system(n: int, naux: int, seed: int, n_occ: int | None = None,
                lam: float = 1.0) -> System:
    """Draw one system in the fixed order described in the module docstring."""
    if n_occ is None:
        n_occ = n // 2
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    Qm, R = np.linalg.qr(A)
    Qm = Qm * np.sign(np.diag(R))
    eps_occ = rng.uniform(-1.5, -0.3, size=n_occ)
    eps_virt = rng.uniform(0.1, 2.0, size=n - n_occ)
    X = rng.normal(0.0, math.sqrt(1.0 / n), size=(n, naux))
    L = rng.standard_normal((naux, naux))
    V = (L @ L.T) / naux
    V = 0.5 * (V + V.T) * lam
    eps = np.concatenate([eps_occ, eps_virt])
    mu = 0.5 * (eps_occ.max() + eps_virt.min())
    return System(n=n, naux=naux, n_occ=n_occ, Q=Qm, eps=eps, mu=float(mu),
                  X=np.ascontiguousarray(X), V=np.ascontiguousarray(V), lam=lam)


def cheb_tau_grid(m: int, beta: float):
    """Chebyshev-root grid on [0, beta] (ascending) and Fejer-1 weights.

    x_k = -cos((2k+1) pi / 2m); tau_k = beta (1 + x_k) / 2.  The weights
    integrate every polynomial of degree < m exactly on [-1, 1] and are scaled
    by beta/2 for [0, beta].
    """
    k = np.arange(m)
    theta = (2 * k + 1) * np.pi / (2 * m)
    x = -np.cos(theta)
    tau = 0.5 * beta * (1.0 + x)
    # Fejer's first rule on the roots, in the ascending order used above
    # (theta -> pi - theta maps cos(2 j theta) onto itself).
    s = np.zeros(m)
    for j in range(1, m // 2 + 1):
        s += np.cos(2 * j * theta) / (4 * j * j - 1)
    w = (2.0 / m) * (1.0 - 2.0 * s)
    return tau, w * (0.5 * beta)


def g0_tau(sys_: System, tau: np.ndarray, beta: float) -> np.ndarray:
    """Independent-particle G(tau) = Q diag(g(xi, tau)) Q^T, tau in (0, beta).

    g(xi, tau) = -exp(-xi tau) / (1 + exp(-beta xi))         for xi >= 0
               = -exp(xi (beta - tau)) / (1 + exp(beta xi))  for xi <  0
    Both branches only exponentiate non-positive numbers.
    """
    xi = sys_.eps - sys_.mu
    out = np.empty((len(tau), sys_.n, sys_.n))
    for k, t in enumerate(tau):
        g = np.where(xi >= 0,
                     -np.exp(-np.abs(xi) * t) / (1.0 + np.exp(-beta * np.abs(xi))),
                     -np.exp(-np.abs(xi) * (beta - t)) / (1.0 + np.exp(-beta * np.abs(xi))))
        out[k] = (sys_.Q * g) @ sys_.Q.T
    return out


def workload(name: str, seed: int = 0, lam: float = 1.0):
    """(system, tau, weights, G0[m,n,n], beta) for one named workload."""
    cfg = WORKLOADS[name]
    s = make_system(cfg["n"], cfg["naux"], seed, lam=lam)
    tau, w = cheb_tau_grid(cfg["m"], cfg["beta"])
    G = g0_tau(s, tau, cfg["beta"])
    return s, tau, w, G, cfg["beta"]


def pole_sigma(n: int, tau: np.ndarray, beta: float, seed: int, npoles: int = 4,
               scale: float = 0.05) -> np.ndarray:
    """A self-energy-like input with a closed form at any tau: a sum of poles,
    Sigma(tau) = -sum_j A_j K(tau, w_j), K(tau, w) = exp(-tau w) / (1 + exp(-beta w)),
    A_j random symmetric (n x n, entries ~ scale), w_j = +-U(0.2, 3) Ha.
    Returns [len(tau), n, n]."""
    rng = np.random.default_rng(seed)
    out = np.zeros((len(tau), n, n))
    for _ in range(npoles):
        A = rng.normal(0.0, scale, (n, n))
        A = 0.5 * (A + A.T)
        w = rng.uniform(0.2, 3.0) * (1 if rng.random() < 0.5 else -1)
        t = np.asarray(tau)
        k = (np.exp(-t * w) / (1 + np.exp(-beta * w)) if w >= 0
             else np.exp(w * (beta - t)) / (1 + np.exp(beta * w)))
        out -= k[:, None, None] * A[None]
    return out


def thc_factors(n: int, naux: int, seed: int):
    """X ~ N(0, 1/n) [n, naux] and V = L L^T / naux (L ~ N(0, 1)) alone, for
    cases without an orbital spectrum (e.g. a single spin-orbital)."""
    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, math.sqrt(1.0 / n), size=(n, naux))
    L = rng.standard_normal((naux, naux))
    V = (L @ L.T) / naux
    return np.ascontiguousarray(X), np.ascontiguousarray(0.5 * (V + V.T))


def random_general_g(n: int, m: int, seed: int, scale: float = 0.3) -> np.ndarray:
    """Non-symmetric dense G[m,n,n] for checks that must not lean on G = G^T."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((m, n, n))


def block_diag_system(parts: list[System]) -> System:
    """Non-interacting supersystem: orbitals and THC points of each fragment
    stay on that fragment (X, V, Q block diagonal)."""
    n = sum(p.n for p in parts)
    naux = sum(p.naux for p in parts)
    Q = np.zeros((n, n)); X = np.zeros((n, naux)); V = np.zeros((naux, naux))
    eps = np.concatenate([p.eps for p in parts])
    io = ia = 0
    for p in parts:
        Q[io:io + p.n, io:io + p.n] = p.Q
        X[io:io + p.n, ia:ia + p.naux] = p.X
        V[ia:ia + p.naux, ia:ia + p.naux] = p.V
        io += p.n; ia += p.naux
    mu = parts[0].mu
    return System(n=n, naux=naux, n_occ=sum(p.n_occ for p in parts), Q=Q, eps=eps,
                  mu=mu, X=X, V=V)


def warmstart_system(seed: int, lam: float, n_range=(40, 160)):
    """One system of the learned-warm-start set: n uniform in n_range (drawn from
    its own stream), naux = 5 n, n_occ = n // 2, interaction scale lam."""
    n = int(np.random.default_rng(seed + 10**6).integers(n_range[0], n_range[1] + 1))
    return make_system(n, 5 * n, seed, lam=lam)
