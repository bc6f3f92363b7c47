"""Self-consistency loop (SOX, or full second order: direct + SOX) on one GPU, fixed F:

    G0 (independent particles) -> Sigma[G] -> (damping or DIIS on Sigma)
       -> Dyson on the Matsubara grid (optionally with the chemical potential
          that conserves the electron number) -> G -> ...

Every step runs in libthcsox (SOX evaluation, energy, tau -> i omega transform,
batched Dyson inversion, chemical-potential search, least-squares fit back to
tau, one-body energy, damping, DIIS and its commutator residual); torch only
provides device buffers.
Prints one JSON line per iteration and a summary line, e.g. for the paper-scale
one-GPU share:

    python -m paper_2404_17744_amd.loop --workload sox_n1100_naux5500_ntau100 --iters 10
    python -m paper_2404_17744_amd.loop --workload sox_n300_naux1800_ntau100 --diis 6 --mu-search
    python -m paper_2404_17744_amd.loop --workload sox_n300_naux1800_ntau100 --diis 6 \
        --diis-kind commutator

With --grid ir the loop runs on the IR sparse-sampling grids (tau points and
Matsubara frequencies of the basis at --beta and Lambda = beta --wmax), with
the energy from the basis expansion; the workload then only sets n and naux.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

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
    ap.add_argument("--terms", default="sox", choices=["sox", "gf2"],
                    help="self-energy: the SOX term, or full second order (direct + SOX)")
    ap.add_argument("--damping", type=float, default=0.0,
                    help="Sigma_in <- d Sigma_in + (1 - d) Sigma_out (0: none)")
    ap.add_argument("--diis", type=int, default=0, help="DIIS depth on Sigma (0: none)")
    ap.add_argument("--diis-kind", default="pulay", choices=["pulay", "commutator"],
                    help="residual: Sigma_out - Sigma_in, or the frequency-dependent "
                         "commutator [G(i w), F + Sigma_out(i w)]")
    ap.add_argument("--mu-search", action="store_true",
                    help="chemical potential that keeps n_occ electrons at every Dyson step "
                         "(meant for --terms gf2: with the exchange term alone N(mu) falls "
                         "across the gap and has several roots, so the search hops between them)")
    # The target has to sit above the grid's accuracy in N: with Sigma != 0 the
    # density fitted on 64 Chebyshev points at beta = 100 is off by up to ~5e-4
    # (128 points, or the IR grid, bring it below 1e-7); in a gap N(mu) is nearly
    # flat, so a tighter target moves mu far across the gap to absorb that error
    ap.add_argument("--mu-tol", type=float, default=None,
                    help="electron-number tolerance (default 1e-3 on the Chebyshev grid, "
                         "1e-5 on the IR grid)")
    ap.add_argument("--grid", default="cheb", choices=["cheb", "ir"],
                    help="Chebyshev roots (the workload's grid) or IR sparse sampling")
    ap.add_argument("--beta", type=float, default=1000.0, help="inverse temperature (--grid ir)")
    ap.add_argument("--wmax", type=float, default=100.0, help="frequency window (--grid ir)")
    ap.add_argument("--ir-eps", type=float, default=1e-10, help="basis cut s_l / s_0 (--grid ir)")
    a = ap.parse_args()
    mu_tol = a.mu_tol if a.mu_tol is not None else (1e-3 if a.grid == "cheb" else 1e-5)

    import torch
    dev = torch.device("cuda:0")
    t0 = time.time()
    s, tau, w, G0, beta = synth.workload(a.workload, seed=a.seed, lam=a.lam)
    grid = None
    if a.grid == "ir":
        grid = thcsox.thcsox_ir_grid(a.beta, a.wmax, a.ir_eps)
        beta, tau = a.beta, grid["tau"]
        w = np.zeros(len(tau))            # the energy comes from the basis expansion
        G0 = synth.g0_tau(s, tau, beta)
    t_gen = time.time() - t0
    X = torch.from_numpy(s.X).to(dev)
    V = torch.from_numpy(s.V).to(dev)
    G = torch.from_numpy(G0).to(dev)
    torch.cuda.synchronize()
    t0 = time.time()
    plan = thcsox.Plan(X, V, tau, w, beta, precision=a.precision)
    dyson = thcsox.Dyson(torch.from_numpy(s.F).to(dev), s.mu, tau, beta, a.matsubara,
                         grid=grid)
    torch.cuda.synchronize()
    t_plan = time.time() - t0
    S_out = torch.zeros_like(G)    # Sigma^SOX of the current G
    S_in = torch.zeros_like(G)     # the Sigma fed to the Dyson step
    S_next = torch.empty_like(G)
    diis, e_buf = None, None
    if a.diis > 0 and a.diis_kind == "commutator":
        nf = dyson.nfreq
        e_buf = torch.empty((2, nf, s.n, s.n), dtype=torch.float64, device=dev)
        diis = thcsox.Diis(S_out, depth=a.diis, residual_like=e_buf)
    elif a.diis > 0:
        diis = thcsox.Diis(S_out, depth=a.diis)
    mu = s.mu
    # the start: G0 and its density matrix from a Dyson step with Sigma = 0, so
    # that every energy pairs E_1 = Tr[F gamma] and E_2 of the same G
    G, gamma = dyson.step(S_in, G_out=G)
    E_prev, iters = None, []
    for it in range(a.iters):
        torch.cuda.synchronize()
        t1 = time.time()
        plan.sigma(G, out=S_out)
        if a.terms == "gf2":
            plan.sigma_direct(G, out=S_out, accumulate=True)   # direct + SOX
        E_2 = plan.energy(G, S_out) if grid is None else plan.energy_basis(G, S_out, grid)
        E1 = dyson.onebody(gamma)   # the density matrix of the G that Sigma came from
        nelec = float(np.trace(gamma.cpu().numpy()))   # host diagnostic
        t2 = time.time()
        used = 1
        if e_buf is not None:
            # the commutator of the G that S_out came from (the last Dyson step's)
            dyson.commutator(S_in, S_out, out=e_buf)
            used = diis.step_res(e_buf, S_out, S_next)
            S_in, S_next = S_next, S_in
        elif it == 0 or (diis is None and a.damping == 0.0):
            S_in.copy_(S_out)
        elif diis is not None:
            used = diis.step(S_in, S_out, S_next)
            S_in, S_next = S_next, S_in
        else:
            thcsox.mix(a.damping, S_out, S_in)
        solves = 1
        if a.mu_search:
            G, gamma, mu, solves = dyson.step_mu(S_in, s.n_occ, mu, tol=mu_tol, G_out=G)
        else:
            G, gamma = dyson.step(S_in, G_out=G)
        t3 = time.time()
        E = E1 + E_2
        row = {"iter": it + 1, "E_total": E, "E_2": E_2, "E_onebody": E1,
               "dE": None if E_prev is None else E - E_prev,
               "mu": mu, "nelec": nelec, "dyson_solves": solves, "diis_used": used,
               "sigma_s": t2 - t1, "dyson_s": t3 - t2,
               "symmetric_tau_points": int(plan.symmetric_flags().sum()),
               "tau_points_per_s": len(tau) / (t2 - t1)}
        print(json.dumps(row), flush=True)
        iters.append(row)
        if E_prev is not None and abs(E - E_prev) < a.tol:
            break
        E_prev = E
    if diis is not None:
        diis.close()
    plan.close()
    dyson.close()
    sig = [r["sigma_s"] for r in iters]
    print(json.dumps({"workload": a.workload, "n": s.n, "naux": s.naux, "ntau": len(tau),
                      "lam": a.lam, "precision": a.precision, "terms": a.terms,
                      "grid": a.grid, "beta": beta,
                      "nfreq": len(grid["freq_n"]) if grid else a.matsubara,
                      "damping": a.damping,
                      "diis": a.diis, "diis_kind": a.diis_kind, "mu_search": a.mu_search, "iterations": len(iters),
                      "converged": len(iters) > 1 and abs(iters[-1]["dE"]) < a.tol,
                      "E_total": iters[-1]["E_total"],
                      "generate_s": t_gen, "plan_s": t_plan,
                      "sigma_s_mean": sum(sig) / len(sig),
                      "dyson_s_mean": sum(r["dyson_s"] for r in iters) / len(iters),
                      "tau_points_per_s": len(tau) * len(sig) / sum(sig)}), flush=True)


if __name__ == "__main__":
    main()
