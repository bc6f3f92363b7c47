"""GPU parity at the edges of the shape space and at the method's degenerate
inputs, against the FP64 oracle (the paper's THC-SOX sequence, pinned to the
literal six-index definition elsewhere).

* Shapes: a single THC point (naux = 1: one row of every tile), a single
  orbital with a single point, one tau point (the grid's middle point is its
  own mirror: G(beta - tau) is G(tau)), an odd tau count, naux one past a
  128-row tile, n one past the 64-wide fp16x2 k stage (a second stage of
  padding), and n smaller than the number of v ranges (most ranges empty).
  Each for the four precisions, on the full path (general G) and the
  symmetric one (G = G^T at every tau point).
* G = 0 at one tau point: Sigma there and at its mirror is exactly zero (every
  term carries G(tau) or takes it as G(beta - tau)); the other points match the
  oracle and nothing turns into NaN (a zero maximum sets no scale).  G = 0
  everywhere gives Sigma = 0 and E = 0 exactly.
* The GF2 direct term on the same shapes (FP64, 1e-12), and the Dyson step at
  n = 1, 2 and 9 against the oracle's transforms and inversion (1e-10, as the
  other Dyson tests).

Bars as in the other parity tests: 1e-12 of max |Sigma| in FP64 (these sums have
at most a few hundred terms), 2e-6 on the split paths; energies to the same
fraction of the sum of their terms' magnitudes.  The random general G cancels
heavily at n = 65, naux = 5 (the same sequence on |X|, |V|, |G| reaches 2e5 times
max |Sigma|): fp16x2 lands at 1.0e-6 there, every other case below 6e-7; the
kernels reduce in a fixed order, so the figure is the same on every run.
"""
import numpy as np
import pytest
import torch

from oracle import direct as od
from oracle import energy as oenergy
from oracle import sox as osox
from oracle import transforms as otr
from paper_2404_17744_amd import synth, thcsox

pytestmark = pytest.mark.gpu

PRECISIONS = ["fp64", "fp32", "bf16x3", "fp16x2"]
TOL = {"fp64": 1e-12, "fp32": 2e-6, "bf16x3": 2e-6, "fp16x2": 2e-6}
# (n, naux, ntau)
SHAPES = [(1, 1, 1), (3, 1, 5), (1, 7, 3), (2, 129, 3), (65, 5, 1), (5, 33, 2)]
BETA = 50.0


def _inputs(n, naux, ntau, sym, seed):
    X, V = synth.thc_factors(n, naux, seed=seed)
    G = synth.random_general_g(n, ntau, seed=seed + 1)
    if sym:
        G = 0.5 * (G + G.transpose(0, 2, 1))
    tau, w = synth.cheb_tau_grid(ntau, BETA)
    return X, V, G, tau, w


def _gpu(dev, X, V, G, tau, w, precision):
    plan = thcsox.Plan(torch.from_numpy(X).to(dev), torch.from_numpy(V).to(dev), tau, w, BETA,
                       precision=precision)
    Gd = torch.from_numpy(G).to(dev)
    S = plan.sigma(Gd)
    E = plan.energy(Gd, S)
    flags = list(plan.symmetric_flags())
    torch.cuda.synchronize()
    out = S.cpu().numpy()
    plan.close()
    return out, E, flags


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("sym", [False, True], ids=["general", "symmetric"])
@pytest.mark.parametrize("shape", SHAPES, ids=[f"n{a}_naux{b}_ntau{c}" for a, b, c in SHAPES])
def test_edge_shapes(dev, shape, sym, precision):
    n, naux, ntau = shape
    print(f"case n{n} naux{naux} ntau{ntau} {'sym' if sym else 'general'} {precision}", flush=True)
    X, V, G, tau, w = _inputs(n, naux, ntau, sym, seed=20 + n + naux)
    ref = osox.sigma_all_tau(osox.sigma_thc_paper, G, X, V)
    E_ref = oenergy.energy_tau(G, ref, w)
    S, E, flags = _gpu(dev, X, V, G, tau, w, precision)
    assert np.isfinite(S).all()
    err = float(np.abs(S - ref).max() / np.abs(ref).max())
    print(f"  rel err {err:.2e}  E {E:.6e} (oracle {E_ref:.6e})  symmetric {flags}", flush=True)
    assert err <= TOL[precision]
    # scale of the energy: its terms' magnitudes, sum_k w_k sum_pq |G_qp(beta - tau_k) Sigma_pq|
    escale = sum(abs(w[k]) * float(np.abs(G[ntau - 1 - k].T * ref[k]).sum()) for k in range(ntau))
    assert abs(E - E_ref) <= TOL[precision] * escale
    # a 1 x 1 G is symmetric whatever its value
    assert all(flags) == (sym or n == 1)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_zero_g_at_one_tau_point(dev, precision):
    n, naux, ntau, k0 = 20, 70, 6, 1
    print(f"case n{n} naux{naux} ntau{ntau} G(tau_{k0}) = 0 {precision}", flush=True)
    X, V, G, tau, w = _inputs(n, naux, ntau, False, seed=7)
    G[k0] = 0.0
    ref = osox.sigma_all_tau(osox.sigma_thc_paper, G, X, V)
    S, E, _ = _gpu(dev, X, V, G, tau, w, precision)
    assert np.isfinite(S).all() and np.isfinite(E)
    zero = [k0, ntau - 1 - k0]
    assert not S[zero].any()
    rest = [k for k in range(ntau) if k not in zero]
    err = float(np.abs(S[rest] - ref[rest]).max() / np.abs(ref[rest]).max())
    print(f"  rel err {err:.2e}", flush=True)
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_zero_g_everywhere(dev, precision):
    print(f"case n12 naux40 ntau4 G = 0 {precision}", flush=True)
    X, V, G, tau, w = _inputs(12, 40, 4, False, seed=9)
    G[:] = 0.0
    S, E, _ = _gpu(dev, X, V, G, tau, w, precision)
    assert not S.any() and E == 0.0


# the GF2 direct term (FP64 in every plan precision) on the same shapes
@pytest.mark.parametrize("shape", SHAPES, ids=[f"n{a}_naux{b}_ntau{c}" for a, b, c in SHAPES])
def test_direct_edge_shapes(dev, shape):
    n, naux, ntau = shape
    print(f"case direct n{n} naux{naux} ntau{ntau} general", flush=True)
    X, V, G, tau, w = _inputs(n, naux, ntau, False, seed=40 + n + naux)
    ref = osox.sigma_all_tau(od.sigma_direct_thc, G, X, V)
    plan = thcsox.Plan(torch.from_numpy(X).to(dev), torch.from_numpy(V).to(dev), tau, w, BETA,
                       precision="fp64")
    S = plan.sigma_direct(torch.from_numpy(G).to(dev))
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    plan.close()
    err = float(np.abs(S - ref).max() / np.abs(ref).max())
    print(f"  rel err {err:.2e}", flush=True)
    assert err <= 1e-12


# the Dyson step: a single orbital, two, and n = 9 (one 8-column panel and a
# 1-column one); a random Sigma 20 times the spread of F forces row interchanges
@pytest.mark.parametrize("n", [1, 2, 9])
def test_dyson_edge_sizes(dev, n):
    ntau, nw = 8, 16
    rng = np.random.default_rng(60 + n)
    A = rng.standard_normal((n, n))
    F = 0.5 * (A + A.T)
    mu = 0.05
    tau, _ = synth.cheb_tau_grid(ntau, BETA)
    S = 20.0 * max(1.0, np.abs(F).max()) * rng.standard_normal((ntau, n, n))
    print(f"case dyson n{n} ntau{ntau} nw{nw} random Sigma", flush=True)
    Tm = otr.cheb_to_matsubara(ntau, nw, BETA)
    G_ref, gam_ref, _ = otr.loop_step(F, mu, BETA, S, Tm)
    d = thcsox.Dyson(torch.from_numpy(F).to(dev), mu, tau, BETA, nw)
    G, gam = d.step(torch.from_numpy(S).to(dev))
    torch.cuda.synchronize()
    G, gam = G.cpu().numpy(), gam.cpu().numpy()
    d.close()
    eg = float(np.abs(G - G_ref).max() / np.abs(G_ref).max())
    ea = float(np.abs(gam - gam_ref).max() / np.abs(gam_ref).max())
    print(f"  G rel err {eg:.2e}  gamma rel err {ea:.2e}", flush=True)
    assert eg < 1e-10 and ea < 1e-10
