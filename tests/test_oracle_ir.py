"""Pins of the IR-basis oracle (oracle/ir.py) to facts other than itself (CPU).

* Single poles: G(tau) = -K(tau, xi) has the closed-form transform
  1 / (i w_n - xi); the tau -> i w map on the sampling points must give it, and
  the least-squares fit back from the sampled frequencies must give G(tau) on
  the tau points and G(beta^-) -- for poles inside the window |xi| <= wmax.
* The energy form integrates A(beta - tau) B(tau) over [0, beta] exactly for a
  particle and a hole pole (closed form).
* Orthonormality and parity of the leading basis functions, the number of
  tau sampling points (the L roots of u_L, mirror-symmetric).
* The SOX energy of G0 on the IR grid equals that on a converged Chebyshev grid
  (the same integral by an independent quadrature; the Chebyshev rule is pinned
  to the MP2-exchange limit elsewhere).
* Planted slips (a dropped conjugate/sign in the transform, the parity factor
  of the energy form) are caught.
* Re-expansion at other tau points (``evaluate_at``) gives a single pole's
  closed form between the sampling points and near both ends.
"""
import numpy as np
import pytest

from oracle import energy as oenergy
from oracle import ir
from oracle import sox as osox
from paper_2404_17744_amd import synth


def _kt(tau, w, beta):
    """K(tau, w) = exp(-tau w) / (1 + exp(-beta w)) without overflow."""
    if w >= 0:
        return np.exp(-tau * w) / (1 + np.exp(-beta * w))
    return np.exp(w * (beta - tau)) / (1 + np.exp(beta * w))


@pytest.fixture(scope="module", params=[(100.0, 10.0), (1000.0, 100.0)],
            ids=["beta100_L1e3", "beta1000_L1e5"])
def grid(request):
    beta, wmax = request.param
    b = ir.IRBasis(beta, wmax)
    tau = b.tau_points()
    nf = b.matsubara_points()
    Wf, Wb = ir.transforms(b, tau, nf)
    return b, tau, nf, Wf, Wb


def test_sampling_points(grid):
    b, tau, nf, _, _ = grid
    assert len(tau) == b.L
    assert np.all(np.diff(tau) > 0) and tau[0] > 0 and tau[-1] < b.beta
    assert np.abs(tau + tau[::-1] - b.beta).max() <= 1e-12 * b.beta
    assert nf[0] == 0 and np.all(np.diff(nf) > 0)
    # enough frequencies for each parity class: ceil(L / 2) equations at least
    assert len(nf) >= (b.L + 1) // 2


def test_orthonormal_and_parity(grid):
    b = grid[0]
    U = b.u_x(b.x)[:, :20]
    O = (U * b.wx[:, None]).T @ U
    assert np.abs(O - np.eye(20)).max() < 1e-12
    xs = np.linspace(-0.99, 0.99, 37)
    par = (-1.0) ** np.arange(20)
    assert np.abs(b.u_x(-xs)[:, :20] - b.u_x(xs)[:, :20] * par).max() < 1e-9 * np.abs(U).max()


@pytest.mark.parametrize("frac", [-0.9, -0.05, 0.003, 0.02, 0.5])
def test_single_pole_transforms(grid, frac):
    b, tau, nf, Wf, Wb = grid
    xi = frac * b.wmax
    beta = b.beta
    G = -_kt(tau, xi, beta)
    wn = (2 * nf + 1) * np.pi / beta
    Giw = 1.0 / (1j * wn - xi)
    F = Wf @ G
    nfr = len(nf)
    assert np.abs(F[:nfr] + 1j * F[nfr:] - Giw).max() <= 1e-8 * np.abs(Giw).max()
    back = Wb @ np.concatenate([Giw.real, Giw.imag])
    assert np.abs(back[:-1] - G).max() <= 1e-7
    assert abs(back[-1] - (-_kt(beta, xi, beta))) <= 1e-7


def test_energy_form_particle_hole_pair(grid):
    b, tau = grid[0], grid[1]
    M = ir.energy_matrix(b, tau)
    beta = b.beta
    for w1, w2 in [(0.3, -0.5), (-0.2, 1.1), (0.05, -0.05)]:
        A, B = _kt(tau, w1, beta), _kt(tau, w2, beta)
        # int_0^beta K(beta - t, w1) K(t, w2) dt for opposite signs: the product is
        # pref exp(-c s) with s = beta - t (w1 > 0) or s = t (w1 < 0), c = |w1 - w2|
        c = abs(w1 - w2)
        pref = 1.0 / ((1 + np.exp(-beta * abs(w1))) * (1 + np.exp(-beta * abs(w2))))
        ex = pref * (-np.expm1(-beta * c)) / c
        assert abs(A @ M @ B - ex) <= 1e-9 * abs(ex), (w1, w2, A @ M @ B, ex)


def test_energy_form_parity_slip_caught(grid):
    b, tau = grid[0], grid[1]
    Ut = b.u_tau(tau)
    Ui = np.linalg.solve(Ut, np.eye(len(tau)))
    M_bad = Ui.T @ Ui                           # parity factor dropped
    A, B = _kt(tau, 0.3, b.beta), _kt(tau, -0.5, b.beta)
    assert abs(A @ M_bad @ B - A @ ir.energy_matrix(b, tau) @ B) > 1e-3


def test_transform_conjugation_slip_caught(grid):
    b, tau, nf, Wf, _ = grid
    G = -_kt(tau, 0.3, b.beta)
    wn = (2 * nf + 1) * np.pi / b.beta
    nfr = len(nf)
    F = Wf @ G
    bad = F[:nfr] - 1j * F[nfr:]                # i w_n -> -i w_n
    assert np.abs(bad - 1.0 / (1j * wn - 0.3)).max() > 1e-3


def test_sox_energy_ir_equals_chebyshev():
    """E_SOX[G0] of the 8-orbital system at beta = 100: IR grid (52 points) vs
    a 100-point Chebyshev grid (converged to ~1e-15 at this beta)."""
    s = synth.make_system(8, 32, seed=0, lam=0.2)
    beta = 100.0
    tc, wc = synth.cheb_tau_grid(100, beta)
    Gc = synth.g0_tau(s, tc, beta)
    Sc = osox.sigma_all_tau(osox.sigma_thc_paper, Gc, s.X, s.V)
    E_cheb = oenergy.energy_tau(Gc, Sc, wc)
    b = ir.IRBasis(beta, 10.0)
    ti = b.tau_points()
    Gi = synth.g0_tau(s, ti, beta)
    Si = osox.sigma_all_tau(osox.sigma_thc_paper, Gi, s.X, s.V)
    M = ir.energy_matrix(b, ti)
    # E = -1/2 int Tr[G(beta - tau) Sigma(tau)] dtau = -1/2 sum_k'k M[k', k] T[k', k]
    T = np.einsum("apq,bqp->ab", Gi, Si)       # T[k', k] = sum_pq G_pq(tau_k') Sigma_qp(tau_k)
    E_ir = -0.5 * float(np.sum(M * T))
    assert abs(E_ir - E_cheb) <= 1e-8 * abs(E_cheb), (E_ir, E_cheb)


def test_dyson_step_sampled_reproduces_g0():
    """Sigma = 0: the sampled Dyson step returns the closed-form G0(tau) on the IR
    points and Tr gamma = the Fermi sum (beta = 1000, the paper's Lambda)."""
    s = synth.make_system(12, 48, seed=4)
    b = ir.IRBasis(1000.0, 100.0)
    tau, nf = b.tau_points(), b.matsubara_points()
    Wf, Wb = ir.transforms(b, tau, nf)
    G, gamma = ir.dyson_step_sampled(s.F, s.mu, 1000.0, np.zeros((len(tau), 12, 12)), Wf, Wb, nf)
    G0 = synth.g0_tau(s, tau, 1000.0)
    assert np.abs(G - G0).max() <= 1e-7
    occ = 0.5 * (1.0 - np.tanh(500.0 * (s.eps - s.mu)))      # Fermi function, no overflow
    assert abs(np.trace(gamma) - occ.sum()) <= 1e-6


@pytest.mark.parametrize("frac", [-0.7, -0.01, 0.004, 0.3])
def test_evaluate_at_reproduces_single_pole(grid, frac):
    """Re-expanding sampled data at other tau points: a single pole sampled on
    the IR points and evaluated at points between them (and near both ends)
    gives the closed form -K(tau, xi); a pole pair in a matrix-valued F keeps
    each element apart."""
    b, tau = grid[0], grid[1]
    beta, xi = b.beta, frac * b.wmax
    tau_new = np.concatenate([[1e-6 * beta, 0.5 * beta, beta * (1 - 1e-6)],
                              0.5 * (tau[:-1] + tau[1:])[::7]])
    got = ir.evaluate_at(b, tau, -np.array([_kt(t, xi, beta) for t in tau]), tau_new)
    ex = -np.array([_kt(t, xi, beta) for t in tau_new])
    assert np.abs(got - ex).max() <= 1e-8
    F = np.array([[[-_kt(t, xi, beta), 0.0], [0.5 * _kt(t, -xi, beta), -_kt(t, 2 * xi, beta)]]
                  for t in tau])
    got = ir.evaluate_at(b, tau, F, tau_new)
    assert got.shape == (len(tau_new), 2, 2)
    assert np.abs(got[:, 0, 1]).max() <= 1e-12
    assert np.abs(got[:, 1, 0] - 0.5 * np.array([_kt(t, -xi, beta) for t in tau_new])).max() <= 1e-8
