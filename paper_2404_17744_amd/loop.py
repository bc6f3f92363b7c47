"""SOX-only self-consistency loop on one GPU (fixed F and mu):

    G0 (independent particles) -> Sigma^SOX[G] -> Dyson on the Matsubara grid -> G -> ...

Every step runs in libthcsox (SOX evaluation, energy, tau -> i omega transform,
batched Dyson inversion, least-squares fit back to tau, one-body energy);
torch only provides device buffers.  Prints one JSON line per iteration and a
summary line, e.g. for the paper-scale one-GPU share:

    python -m paper_2404_17744_amd.loop --workload sox_n1100_naux5500_ntau100 --iters 10
"""
from __future__ import annotations

import argparse
import json
import time

from . import synth, thcsox


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="sox_n1100_naux5500_ntau100")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--lam", type=float, default=1.0)
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--precision", default="fp16x2")
    ap.add_argument("--matsubara", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-7)
    a = ap.parse_args()

    import torch
    dev = torch.device("cuda:0")
    t0 = time.time()
    s, tau, w, G0, beta = synth.workload(a.workload, seed=a.seed, lam=a.lam)
    t_gen = time.time() - t0
    X = torch.from_numpy(s.X).to(dev)
    V = torch.from_numpy(s.V).to(dev)
    G = torch.from_numpy(G0).to(dev)
    torch.cuda.synchronize()
    t0 = time.time()
    plan = thcsox.Plan(X, V, tau, w, beta, precision=a.precision)
    dyson = thcsox.Dyson(torch.from_numpy(s.F).to(dev), s.mu, tau, beta, a.matsubara)
    torch.cuda.synchronize()
    t_plan = time.time() - t0
    S = torch.zeros_like(G)
    E_prev, iters = None, []
    for it in range(a.iters):
        torch.cuda.synchronize()
        t1 = time.time()
        plan.sigma(G, out=S)
        E_sox = plan.energy(G, S)
        t2 = time.time()
        G, gamma = dyson.step(S, G_out=G)
        E1 = dyson.onebody(gamma)
        t3 = time.time()
        E = E1 + E_sox
        row = {"iter": it + 1, "E_total": E, "E_sox": E_sox, "E_onebody": E1,
               "dE": None if E_prev is None else E - E_prev,
               "sox_s": t2 - t1, "dyson_s": t3 - t2,
               "symmetric_tau_points": int(plan.symmetric_flags().sum()),
               "tau_points_per_s": len(tau) / (t2 - t1)}
        print(json.dumps(row), flush=True)
        iters.append(row)
        if E_prev is not None and abs(E - E_prev) < a.tol:
            break
        E_prev = E
    plan.close()
    dyson.close()
    sox = [r["sox_s"] for r in iters]
    print(json.dumps({"workload": a.workload, "n": s.n, "naux": s.naux, "ntau": len(tau),
                      "lam": a.lam, "precision": a.precision, "iterations": len(iters),
                      "generate_s": t_gen, "plan_s": t_plan,
                      "sox_s_mean": sum(sox) / len(sox),
                      "dyson_s_mean": sum(r["dyson_s"] for r in iters) / len(iters),
                      "tau_points_per_s": len(tau) * len(sox) / sum(sox)}), flush=True)


if __name__ == "__main__":
    main()
