"""FP64 reference of the warm-start network (test infrastructure only).

The paper has no learned component; this network exists only to give the
self-consistency loop a better starting self-energy.  It is a residual MLP
applied independently to every THC pair (R, P): its input is the vector of a
pair's first-iteration self-energy over the tau grid (m values, already
normalised per tau point), its output the same vector of the converged one:

    h1  = silu(W1 x + b1)          W1: [H, m]
    h2  = silu(W2 h1 + b2)         W2: [H, H]
    out = x + W3 h2 + b3           W3: [m, H]
    loss = mean over batch and m of (out - target)^2

silu(z) = z / (1 + exp(-z)).  Rows of ``x`` are samples.
"""
from __future__ import annotations

import numpy as np


def init_params(m: int, H: int, seed: int) -> dict:
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.standard_normal((H, m)) / np.sqrt(m), "b1": np.zeros(H),
        "W2": rng.standard_normal((H, H)) / np.sqrt(H), "b2": np.zeros(H),
        "W3": rng.standard_normal((m, H)) * (0.1 / np.sqrt(H)), "b3": np.zeros(m),
    }


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p: dict, x: np.ndarray):
    z1 = x @ p["W1"].T + p["b1"]
    h1 = silu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = silu(z2)
    out = x + h2 @ p["W3"].T + p["b3"]
    return out, (x, z1, h1, z2, h2)


def bf16_round(a) -> np.ndarray:
    """Nearest bf16 value of each element (returned as float64): the value is
    first taken to FP32 (nearest), then its 32-bit pattern is rounded to the
    top 16 bits, to nearest with ties to the even pattern (the bf16 format is
    FP32 with the low 16 significand bits dropped).  Finite inputs only."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(p: dict, x: np.ndarray) -> np.ndarray:
    """The network with bf16 weights and bf16 layer inputs: every weight matrix
    and each layer's input (x, h1, h2) rounded by bf16_round, products summed
    exactly (FP64 here), biases, silu and the residual add on the unrounded x
    as in forward."""
    W1, W2, W3 = (bf16_round(p[k]) for k in ("W1", "W2", "W3"))
    h1 = silu(bf16_round(x) @ W1.T + p["b1"])
    h2 = silu(bf16_round(h1) @ W2.T + p["b2"])
    return x + (bf16_round(h2) @ W3.T + p["b3"])


def loss_and_grads(p: dict, x: np.ndarray, target: np.ndarray):
    """Mean-squared loss and its exact gradients by the chain rule."""
    out, (x, z1, h1, z2, h2) = forward(p, x)
    r = out - target
    N = r.size
    loss = float(np.sum(r * r) / N)
    dout = 2.0 * r / N                                  # d loss / d out
    g = {"W3": dout.T @ h2, "b3": dout.sum(0)}
    dh2 = dout @ p["W3"]
    dz2 = dh2 * dsilu(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * dsilu(z1)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return loss, g


def adam_step(p: dict, g: dict, state: dict, lr: float, b1: float = 0.9,
              b2: float = 0.999, eps: float = 1e-8) -> None:
    """One Adam update (Kingma & Ba), bias-corrected, in place."""
    t = state.get("t", 0) + 1
    state["t"] = t
    for k in p:
        mk = state.setdefault("m_" + k, np.zeros_like(p[k]))
        vk = state.setdefault("v_" + k, np.zeros_like(p[k]))
        mk *= b1; mk += (1 - b1) * g[k]
        vk *= b2; vk += (1 - b2) * g[k] * g[k]
        mhat = mk / (1 - b1 ** t)
        vhat = vk / (1 - b2 ** t)
        p[k] -= lr * mhat / (np.sqrt(vhat) + eps)
