"""Learned warm start for the SOX self-consistency loop.

The paper iterates G -> Sigma[G] -> Dyson -> G from a Hartree-Fock start.  The
warm start replaces the first Dyson step's input by a predicted converged
self-energy: the first SOX evaluation (at the Hartree-Fock G) gives
Sigma^(1) in the THC basis; a residual MLP maps the tau-profile of every THC
pair (R, P) of Sigma^(1) to that of the converged Sigma; the prediction is
back-projected to the orbital basis and fed to the Dyson step, after which the
plain loop runs as usual and judges it (the converged answer does not depend
on the start; only the number of iterations does).

All arithmetic runs in libthcsox: SOX, energy, back-projection, Dyson step,
pair gather/scatter, the network's FP32 forward, backward and Adam kernels
(training) and its fused bf16 inference kernel (the learned starts: weights and
layer inputs rounded to bf16, FP32 accumulation).  Torch provides device
buffers and index tensors only.

    python -m paper_2404_17744_amd.warmstart --train 200 --eval 56
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import synth, thcsox

M_TAU, BETA, N_MATSUBARA = 64, 100.0, 256


class SCF:
    """Plain SOX self-consistency for one system (fixed mu, fixed F)."""

    def __init__(self, sys_, precision="fp16x2", tol=1e-7, max_iter=60, damping=1.0, dev=None):
        import torch
        self.torch = torch
        self.dev = dev or torch.device("cuda:0")
        self.s = sys_
        self.tau, self.w = synth.cheb_tau_grid(M_TAU, BETA)
        X = torch.from_numpy(sys_.X).to(self.dev)
        V = torch.from_numpy(sys_.V).to(self.dev)
        self.plan = thcsox.Plan(X, V, self.tau, self.w, BETA, precision=precision)
        self.dyson = thcsox.Dyson(torch.from_numpy(sys_.F).to(self.dev), sys_.mu, self.tau, BETA,
                                  N_MATSUBARA)
        self.tol, self.max_iter, self.damping = tol, max_iter, damping
        n, A = sys_.n, sys_.naux
        self.S = torch.zeros((M_TAU, n, n), dtype=torch.float64, device=self.dev)
        self.Sthc = torch.zeros((M_TAU, A, A), dtype=torch.float64, device=self.dev)

    def first_sigma_thc(self):
        """Sigma^(1) in the THC basis at the Hartree-Fock start (one SOX evaluation)."""
        G, _ = self.dyson.step(self.S.zero_())
        self.plan.sigma(G, out=self.S, thc=True, out_thc=self.Sthc)
        return G

    def run(self, Sigma_start=None, count_start=0):
        """Iterate from Dyson(Sigma_start) (Hartree-Fock start if None) until
        |dE| < tol.  Returns (evaluations, energies, converged).

        A start that is unusable -- the Dyson step refuses it (a non-finite or
        singular matrix) or the first energy from it is not finite -- falls back
        to the Hartree-Fock start; the evaluations already spent stay counted
        and ``self.fell_back`` records it."""
        self.fell_back = False
        if Sigma_start is None:
            return self._iterate(None, count_start)
        try:
            evals, energies, ok = self._iterate(Sigma_start, count_start)
            if energies and np.isfinite(energies[0]):
                return evals, energies, ok
        except thcsox.ThcsoxError:
            evals, energies = count_start, []
        self.fell_back = True
        ev, E, ok = self._iterate(None, evals)
        return ev, energies + E, ok

    def _iterate(self, Sigma_start, count_start):
        S0 = self.S.zero_() if Sigma_start is None else Sigma_start
        G, gam = self.dyson.step(S0)
        energies, Sold = [], None
        evals = count_start
        for it in range(self.max_iter):
            self.plan.sigma(G, out=self.S, thc=True, out_thc=self.Sthc)
            evals += 1
            if Sold is not None and self.damping < 1.0:
                self.S.mul_(self.damping).add_(Sold, alpha=1.0 - self.damping)
            E = self.dyson.onebody(gam) + self.plan.energy(G, self.S)
            energies.append(E)
            if not np.isfinite(E):
                return evals, energies, False
            if len(energies) > 1 and abs(energies[-1] - energies[-2]) < self.tol:
                return evals, energies, True
            Sold = self.S.clone() if self.damping < 1.0 else None
            G, gam = self.dyson.step(self.S)
        return evals, energies, False

    def close(self):
        self.plan.close()
        self.dyson.close()


def pair_profiles(Sthc, scale, pairs=None, out=None):
    """x[b][k] = Sthc[k][pair_b] / scale[pair_b] via thcsox_pair_gather."""
    torch = __import__("torch")
    m, A = Sthc.shape[0], Sthc.shape[1]
    npairs = A * A if pairs is None else pairs.numel()
    if out is None:
        out = torch.empty((npairs, m), dtype=torch.float32, device=Sthc.device)
    thcsox.thcsox_pair_gather(m, A, Sthc.data_ptr(), scale.data_ptr(),
                              None if pairs is None else pairs.data_ptr(), npairs,
                              out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return out


def pair_scale(Sthc):
    """scale[p] = max_k |Sthc[k][p]|: each pair's largest magnitude over tau."""
    torch = __import__("torch")
    m, A = Sthc.shape[0], Sthc.shape[1]
    scale = torch.empty(A * A, dtype=torch.float64, device=Sthc.device)
    thcsox.thcsox_pair_scale(m, A, Sthc.data_ptr(), scale.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
    return scale


def collect(seeds, lam, samples_per_system, rng, precision="fp16x2", damping=1.0, log=print,
            n_range=(40, 160)):
    """Run the plain loop on each system; keep sampled pair profiles of
    Sigma^(1) (inputs) and of the converged Sigma (targets)."""
    torch = __import__("torch")
    xs, ts, stats = [], [], []
    for sd in seeds:
        t0 = time.time()
        s = synth.warmstart_system(sd, lam, n_range)
        scf = SCF(s, precision=precision, damping=damping)
        scf.first_sigma_thc()
        S1 = scf.Sthc.clone()
        evals, E, ok = scf.run(count_start=0)
        A = s.naux
        scale = pair_scale(S1)
        pairs = torch.from_numpy(rng.choice(A * A, size=min(samples_per_system, A * A),
                                            replace=False).astype(np.int64)).to(S1.device)
        xs.append(pair_profiles(S1, scale, pairs))
        ts.append(pair_profiles(scf.Sthc, scale, pairs))
        stats.append({"seed": sd, "n": s.n, "evals": evals, "converged": ok, "E": E[-1]})
        log(f"  system {sd}: n={s.n} loop evals={evals} converged={ok} E={E[-1]:.9f} "
            f"({time.time() - t0:.1f} s)")
        scf.close()
    return torch.cat(xs), torch.cat(ts), stats


def init_params(m, H, seed):
    """Deterministic initial weights (scaled Gaussians; the output layer small
    so the untrained network is close to the identity map)."""
    rng = np.random.default_rng(seed)
    return {"W1": rng.standard_normal((H, m)) / np.sqrt(m), "b1": np.zeros(H),
            "W2": rng.standard_normal((H, H)) / np.sqrt(H), "b2": np.zeros(H),
            "W3": rng.standard_normal((m, H)) * (0.01 / np.sqrt(H)), "b3": np.zeros(m)}


def train(x, t, hidden=512, epochs=30, batch=4096, lr=1e-3, seed=0, log=print):
    torch = __import__("torch")
    net = thcsox.MLP(x.shape[1], hidden, init_params(x.shape[1], hidden, seed), max_batch=batch)
    g = torch.Generator(device="cpu").manual_seed(seed)
    N = x.shape[0]
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g).to(x.device)
        lr_ep = lr * 0.5 * (1 + np.cos(np.pi * ep / epochs))   # cosine decay
        tot, nb = 0.0, 0
        for b0 in range(0, N - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb, tb = x.index_select(0, idx).contiguous(), t.index_select(0, idx).contiguous()
            tot += net.train_step(xb, tb, float(lr_ep))
            nb += 1
        losses.append(tot / max(1, nb))
        if ep % 5 == 0 or ep == epochs - 1:
            log(f"  epoch {ep}: loss {losses[-1]:.3e}")
    return net, losses


def warm_sigma(scf, net, bf16=True):
    """Predicted converged Sigma(tau) in the orbital basis for scf's system."""
    return warm_sigmas([scf], net, bf16)[0]


def warm_sigmas(scfs, net, bf16=True):
    """Predicted converged Sigma(tau) for several systems at once: the first
    SOX evaluation of each, then ONE network forward over the THC pairs of all
    of them (a ragged batch: system i contributes its naux_i^2 pair profiles;
    with bf16 the fused bf16 inference kernel, else the FP32 layers), then the
    scatter back to each system's THC basis and the back-projection."""
    torch = __import__("torch")
    xs, scales = [], []
    for scf in scfs:
        scf.first_sigma_thc()
        scale = pair_scale(scf.Sthc)
        xs.append(pair_profiles(scf.Sthc, scale))
        scales.append(scale)
    x = xs[0] if len(xs) == 1 else torch.cat(xs)
    y = net.forward_bf16(x) if bf16 else net.forward(x)
    out, o = [], 0
    for scf, scale in zip(scfs, scales):
        m, A = scf.Sthc.shape[0], scf.Sthc.shape[1]
        pred = torch.empty_like(scf.Sthc)
        thcsox.thcsox_pair_scatter(m, A, y[o:o + A * A].data_ptr(), scale.data_ptr(),
                                   pred.data_ptr(), torch.cuda.current_stream().cuda_stream)
        o += A * A
        out.append(scf.plan.backproject(pred))
    return out


def inference_net(net, max_batch=65536):
    """A copy of a trained network sized for large inference batches."""
    p = net.params()
    return thcsox.MLP(net.m, net.H, p, max_batch=max_batch)


def evaluate(seeds, lam, net, precision="fp16x2", damping=1.0, log=print, n_range=(40, 160),
             bf16=True):
    """SOX evaluations to |dE| < 1e-7 from the Hartree-Fock start and from the
    learned start, for every system, and the wall time of each.  The learned
    starts of all systems are predicted as one ragged batch (warm_sigmas); the
    warm wall time of a system is its own iteration time plus its share (by
    pair count) of the batched first evaluations and inference."""
    torch = __import__("torch")
    systems = [synth.warmstart_system(sd, lam, n_range) for sd in seeds]
    scfs = [SCF(s, precision=precision, damping=damping) for s in systems]
    rows = []
    for sd, s, scf in zip(seeds, systems, scfs):
        torch.cuda.synchronize(); t0 = time.time()
        ev_hf, E_hf, ok_hf = scf.run()
        torch.cuda.synchronize(); t1 = time.time()
        rows.append({"seed": sd, "n": s.n, "hf_evals": ev_hf, "hf_converged": ok_hf,
                     "E_hf": E_hf[-1], "hf_s": t1 - t0})
    torch.cuda.synchronize(); t0 = time.time()
    preds = warm_sigmas(scfs, net, bf16)
    torch.cuda.synchronize(); t_pred = time.time() - t0
    pairs = np.array([s.naux ** 2 for s in systems], dtype=float)
    for r, s, scf, Sw in zip(rows, systems, scfs, preds):
        torch.cuda.synchronize(); t0 = time.time()
        ev_w, E_w, ok_w = scf.run(Sigma_start=Sw, count_start=1)
        torch.cuda.synchronize(); t1 = time.time()
        r.update({"warm_evals": ev_w, "warm_converged": ok_w, "E_warm": E_w[-1],
                  "warm_fell_back": scf.fell_back,
                  "warm_s": (t1 - t0) + t_pred * s.naux ** 2 / pairs.sum()})
        log(f"  eval {r['seed']}: n={s.n} HF {r['hf_evals']} evals ({r['hf_s']:.2f} s)  "
            f"warm {ev_w} evals ({r['warm_s']:.2f} s)  dE_final {E_w[-1] - r['E_hf']:.2e}")
    for scf in scfs:
        scf.close()
    return rows


def fp32_inference_check(net, x, t, ev, a, nr, hf):
    """The same held-out systems with the FP32 forward instead of the bf16
    inference kernel, and the loss of both forwards on the first training
    samples (the loss of the bf16 forward from the oracle-parity kernel)."""
    nb = min(65536, x.shape[0])
    xs, ts = x[:nb].contiguous(), t[:nb].contiguous()
    tn = ts.cpu().numpy().astype(np.float64)
    loss32 = float(((net.forward(xs).cpu().numpy() - tn) ** 2).mean())
    loss16 = float(((net.forward_bf16(xs).cpu().numpy() - tn) ** 2).mean())
    inet = inference_net(net)
    rows = evaluate(ev, a.lam, inet, a.precision, a.damping, n_range=nr, bf16=False)
    inet.close()
    wm = np.array([r["warm_evals"] for r in rows])
    return {"fp32_inference": {"loss_fp32_forward": loss32, "loss_bf16_forward": loss16,
                               "warm_evals_mean": float(wm.mean()),
                               "warm_time_mean_s": float(np.mean([r["warm_s"] for r in rows])),
                               "systems_saved": int((wm < hf).sum()),
                               "systems_worse": int((wm > hf).sum())}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--eval", type=int, default=56)
    ap.add_argument("--first-seed", type=int, default=1000)
    ap.add_argument("--lam", type=float, default=0.2)
    ap.add_argument("--damping", type=float, default=1.0)
    ap.add_argument("--samples", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--hidden", type=int, default=512)
    ap.add_argument("--precision", default="fp16x2")
    ap.add_argument("--out", default=None)
    ap.add_argument("--nmin", type=int, default=40)
    ap.add_argument("--nmax", type=int, default=160)
    ap.add_argument("--fp32-inference-check", action="store_true",
                    help="also evaluate the held-out systems with the FP32 forward (the "
                         "default inference rounds weights and layer inputs to bf16)")
    a = ap.parse_args()
    nr = (a.nmin, a.nmax)
    rng = np.random.default_rng(7)
    tr = list(range(a.first_seed, a.first_seed + a.train))
    ev = list(range(a.first_seed + a.train, a.first_seed + a.train + a.eval))
    t0 = time.time()
    x, t, st = collect(tr, a.lam, a.samples, rng, a.precision, a.damping, n_range=nr)
    t_collect = time.time() - t0
    t0 = time.time()
    net, losses = train(x, t, hidden=a.hidden, epochs=a.epochs)
    t_train = time.time() - t0
    inet = inference_net(net)
    rows = evaluate(ev, a.lam, inet, a.precision, a.damping, n_range=nr)
    inet.close()
    hf = np.array([r["hf_evals"] for r in rows]); wm = np.array([r["warm_evals"] for r in rows])
    res = {"lam": a.lam, "damping": a.damping, "train_systems": len(tr), "eval_systems": len(ev),
           "n_range": list(nr), "train_loop_evals_mean": float(np.mean([r["evals"] for r in st])),
           "samples_per_system": a.samples, "epochs": a.epochs, "hidden": a.hidden,
           "final_loss": losses[-1], "identity_loss": float(((x - t) ** 2).mean().item()),
           "collect_s": t_collect, "train_s": t_train,
           "hf_evals_mean": float(hf.mean()), "warm_evals_mean": float(wm.mean()),
           "hf_time_mean_s": float(np.mean([r["hf_s"] for r in rows])),
           "warm_time_mean_s": float(np.mean([r["warm_s"] for r in rows])),
           "max_final_energy_diff": float(max(abs(r["E_warm"] - r["E_hf"]) for r in rows)),
           "systems_saved": int(sum(r["warm_evals"] < r["hf_evals"] for r in rows)),
           "systems_worse": int(sum(r["warm_evals"] > r["hf_evals"] for r in rows)),
           "fell_back": int(sum(r["warm_fell_back"] for r in rows)),
           "all_converged": bool(all(r["hf_converged"] and r["warm_converged"] for r in rows)),
           "rows": rows}
    if a.fp32_inference_check:
        res.update(fp32_inference_check(net, x, t, ev, a, nr, hf))
    print(json.dumps({k: v for k, v in res.items() if k != "rows"}), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
