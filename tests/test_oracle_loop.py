"""Pins of the oracle's transforms, Dyson step and warm-start network (CPU)."""
import numpy as np
import pytest

from oracle import mlp as omlp
from oracle import transforms as otr
from paper_2404_17744_amd import synth

BETA = 100.0


@pytest.fixture(scope="module")
def tmat64():
    return otr.cheb_to_matsubara(64, 256, BETA)


def test_transform_closed_forms(tmat64):
    """T_n0 = int exp(i w tau) = 2i/w_n and T_n1 = -4 / (beta w_n^2) exactly."""
    wn = otr.matsubara_freqs(256, BETA)
    assert np.abs(tmat64[:, 0] - 2j / wn).max() < 1e-12
    assert np.abs(tmat64[:, 1] - (-4.0 / (BETA * wn ** 2))).max() < 1e-12


def test_transform_panel_convergence(tmat64):
    finer = otr.cheb_to_matsubara(64, 256, BETA, panels=4096)
    assert np.abs(finer - tmat64).max() < 1e-11


def test_forward_transform_exact_for_polynomials(tmat64):
    """F(tau) = tau^2 is reproduced by the interpolant; its transform is
    i beta^2/w - 2 beta/w^2 - 4i/w^3 (antiperiodic endpoints)."""
    tau, _ = synth.cheb_tau_grid(64, BETA)
    F = otr.tau_to_matsubara(tau ** 2, tmat64)
    wn = otr.matsubara_freqs(256, BETA)
    exact = 1j * BETA ** 2 / wn - 2 * BETA / wn ** 2 - 4j / wn ** 3
    assert np.abs(F - exact).max() < 1e-9 * np.abs(exact).max()


def test_zero_sigma_round_trip(tmat64):
    """Sigma = 0: Dyson + least-squares fit returns the closed-form G0 and the
    density matrix holds n_occ electrons."""
    s = synth.make_system(20, 40, seed=2)
    tau, _ = synth.cheb_tau_grid(64, BETA)
    G0 = synth.g0_tau(s, tau, BETA)
    G, gam, _ = otr.loop_step(s.F, s.mu, BETA, np.zeros_like(G0), tmat64)
    assert np.abs(G - G0).max() < 5e-9
    assert abs(np.trace(gam) - s.n_occ) < 1e-8
    assert np.abs(gam - gam.T).max() < 1e-12


def test_mlp_gradients_match_finite_differences():
    m, H = 6, 8
    rng = np.random.default_rng(0)
    p = omlp.init_params(m, H, seed=1)
    for k in p:
        p[k] = p[k] + 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((5, m)); t = rng.standard_normal((5, m))
    _, g = omlp.loss_and_grads(p, x, t)
    for k in p:
        flat = p[k].reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[idx]
            flat[idx] = old + 1e-6; lp, _ = omlp.loss_and_grads(p, x, t)
            flat[idx] = old - 1e-6; lm, _ = omlp.loss_and_grads(p, x, t)
            flat[idx] = old
            fd = (lp - lm) / 2e-6
            assert abs(fd - g[k].reshape(-1)[idx]) < 1e-7 * max(1.0, abs(fd)), (k, idx)


def test_adam_first_step_is_signed_lr():
    """With bias correction the first Adam step is -lr * g / (|g| + eps)."""
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    st = {}
    omlp.adam_step(p, g, st, lr=0.01)
    assert np.allclose(p["w"], np.array([1.0, -2.0, 3.0]) - 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8))


def test_adam_three_steps_hand_derived():
    """Three Adam steps written out by hand (b1 = 0.9, b2 = 0.999, eps -> 0).

    Constant gradient g for two steps: m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2,
    so the bias-corrected step is exactly -lr sign(g) both times.  Then the
    gradient flips to -g: m_3 = b1 m_2 - (1 - b1) g = (0.9 * 0.19 - 0.1) g = 0.071 g,
    mhat = 0.071 g / (1 - 0.9^3) = (0.071 / 0.271) g, and v_3 = (1 - b2^3) g^2 gives
    vhat = g^2: the momentum still points along g, so the third step is
    -lr (0.071 / 0.271) sign(g), about a quarter of the first.  A second entry
    changes magnitude instead (g = 1, then 3): m_2 = 0.9 * 0.1 + 0.1 * 3 = 0.39,
    v_2 = 0.999 * 0.001 + 0.001 * 9 = 0.009999, so the second step is
    -lr (0.39 / 0.19) / sqrt(0.009999 / 0.001999).
    """
    lr = 0.01
    p = {"w": np.array([2.0, -1.0, 0.5])}
    st = {}
    gs = [np.array([0.25, -3.0, 1.0]), np.array([0.25, -3.0, 3.0]), np.array([-0.25, 3.0, 3.0])]
    hist = [p["w"].copy()]
    for g in gs:
        omlp.adam_step(p, {"w": g}, st, lr=lr, eps=0.0)
        hist.append(p["w"].copy())
    steps = np.diff(np.array(hist), axis=0)
    # entries 0 and 1: constant gradient, then a sign flip
    for e, sg in ((0, 1.0), (1, -1.0)):
        assert abs(steps[0, e] - (-lr * sg)) < 1e-15
        assert abs(steps[1, e] - (-lr * sg)) < 1e-15
        assert abs(steps[2, e] - (-lr * sg * 0.071 / 0.271)) < 1e-15
    # entry 2: magnitude change at step 2
    assert abs(steps[0, 2] - (-lr)) < 1e-15
    want2 = -lr * (0.39 / 0.19) / np.sqrt(0.009999 / 0.001999)
    assert abs(steps[1, 2] - want2) < 1e-14
    assert st["t"] == 3


def test_bf16_round_values():
    """Nearest with ties to even on the 8-bit significand: 1 + 2^-8 lies halfway
    between 1 and 1 + 2^-7 and goes to 1 (even); 1 + 3 2^-8 lies halfway between
    1 + 2^-7 (odd) and 1 + 2^-6 and goes up; just above a tie rounds up; signs
    and powers of two pass; and it agrees with torch's bfloat16 conversion."""
    import torch
    cases = {1.0: 1.0, 1 + 2 ** -8: 1.0, 1 + 3 * 2 ** -8: 1 + 2 ** -6,
             1 + 2 ** -8 + 2 ** -20: 1 + 2 ** -7, -(1 + 3 * 2 ** -8): -(1 + 2 ** -6),
             2.0 ** -30: 2.0 ** -30, 3.0: 3.0, 0.0: 0.0}
    for a, want in cases.items():
        assert omlp.bf16_round(a) == want, (a, omlp.bf16_round(a), want)
    rng = np.random.default_rng(0)
    v = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-6, 6, 20000)).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(omlp.bf16_round(v), ref)


def test_forward_bf16_within_the_rounding_bound():
    """bf16 weights and layer inputs move the output of the residual branch by
    a few bf16 units of it (relative 2^-8 per rounding, four roundings per
    path) on random data; and on a network whose weights and inputs are already
    bf16 values (one-hot inputs, identity W2) the only roundings left are those
    of h1 and h2, written out here by hand."""
    m, H = 16, 32
    p = omlp.init_params(m, H, seed=2)
    p["W3"] *= 30.0
    rng = np.random.default_rng(3)
    x = rng.standard_normal((200, m))
    ref, _ = omlp.forward(p, x)
    got = omlp.forward_bf16(p, x)
    branch = np.abs(ref - x).max()
    assert 0.0 < np.abs(got - ref).max() <= 8 * 2.0 ** -8 * branch
    # exact case: W, x bf16 values; one-hot rows make every product a single term
    q = {k: omlp.bf16_round(v) for k, v in p.items()}
    q["W2"] = np.eye(H)
    xe = np.zeros((m, m)); xe[np.arange(m), np.arange(m)] = 1.0
    # then z1 = W1 column + b1 (bf16 values), h1 = silu(z1) is rounded once in
    # both; the difference from forward is exactly the rounding of h1 and h2
    h1 = omlp.silu(q["W1"].T + q["b1"])
    h2 = omlp.silu(omlp.bf16_round(h1) + q["b2"])
    want = xe + omlp.bf16_round(h2) @ q["W3"].T + q["b3"]
    assert np.allclose(omlp.forward_bf16(q, xe), want, rtol=0, atol=1e-15)
