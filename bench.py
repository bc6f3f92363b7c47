#!/usr/bin/env python3
"""Throughput of the THC-SOX self-energy on one MI355X.

One step = one full Sigma^SOX(tau) evaluation over every tau point of the
workload plus its Galitskii-Migdal energy, inputs resident in HBM (the plan,
i.e. the one-time U precontraction, is built before timing and reported
separately).  The headline runs the mixed-precision path; the FP64 path is
timed beside it and the energy of both is compared with the stored FP64 oracle
value of the same seeded inputs.

    python bench.py [--steps K] [--warmup W] [--precision fp16x2] [--gpus 1]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SOX Σ(τ) τ-points/s + MFMA util at N=300; mixed vs FP64 at ≤1e-6 Ha"
# MI355X published dense peaks (TFLOP/s) of the matrix-core type each mode issues.
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "fp16x2": 2500.0}
PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 6, "fp16x2": 3}
HBM_PEAK_GBS = 8000.0


def fused_flop_per_launch(plan, info, k_end):
    """Algorithmic flops of one fused launch: 2 products of length n for every
    (R, P) pair formed -- all naux^2 pairs, or naux (naux + 1) / 2 where the
    symmetric path applies -- averaged over the tau points 0..k_end-1 of one step."""
    n, na = info["n"], info["naux"]
    flags = plan.symmetric_flags()[:k_end]
    pairs = [na * (na + 1) / 2 if f else na * na for f in flags]
    return 2.0 * 2.0 * n * n * sum(pairs) / k_end, int(sum(flags))


def timed_steps(plan, Gd, S, steps, torch, k_end=None):
    """Run `steps` steps (tau points 0..k_end-1, default all) between two events
    on the plan's stream; returns (ms per step, last energy or None for a tau
    sample, stage times)."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    plan.profile(True)
    e0.record(plan.stream)
    E = None
    for _ in range(steps):
        plan.sigma(Gd, 0, k_end, out=S)
        if k_end is None:
            E = plan.energy(Gd, S)
    e1.record(plan.stream)
    torch.cuda.synchronize()
    st = plan.stage_times()
    plan.profile(False)
    return e0.elapsed_time(e1) / steps, E, st


def fused_source_hash():
    """Hash of the sources that make up the fp16x2 fused kernel: its file, the
    headers it includes and the definition of its argument struct."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2404_17744_amd", "csrc")
    for f in ("fused_f16.hip", "panel.hpp", "mfma.hpp"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "kernels.hpp")) as fh:
        m = re.search(r"struct FusedArgs \{.*?\n\};", fh.read(), re.S)
    h.update(m.group(0).encode())
    return h.hexdigest()[:16]


def measured_traffic(precision, workload, symmetry, info):
    """HBM bytes per fused launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when there is none, the kernel has changed since, or the plan
    launches it differently (symmetry, v split, partial-tile type)."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_fused_{precision}_{workload}.md")
    if not os.path.exists(path):
        return None
    keys = ("traffic_bytes_per_launch", "source_sha256", "symmetry", "vsplit", "partial_tiles")
    kv = {}
    with open(path) as f:
        for line in f:
            key = line.split(":")[0]
            if ":" in line and key in keys:
                kv[key] = line.split(":", 1)[1].strip()
    if kv.get("source_sha256") != fused_source_hash() or "traffic_bytes_per_launch" not in kv:
        return None
    launch = {"symmetry": symmetry, "vsplit": str(info["vsplit"]),
              "partial_tiles": "fp32" if info["partial_f32"] else "fp64"}
    if any(kv.get(k) != v for k, v in launch.items()):
        return None
    return float(kv["traffic_bytes_per_launch"])


def host_details():
    """CPU model, logical CPUs this process may use, and the BLAS behind NumPy."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    blas, threads = "unknown", None
    try:
        from threadpoolctl import threadpool_info
        for t in threadpool_info():
            if t.get("user_api") == "blas":
                blas = f"{t.get('internal_api')} {t.get('version')} ({t.get('architecture')})"
                threads = t.get("num_threads")
                break
    except Exception:
        pass
    return {"cpu_model": model, "nproc": nproc, "blas": blas, "blas_threads": threads}


def cpu_baseline(s, G, taus):
    """The FP64 oracle (the paper's sequence) on a few tau points, host cores."""
    import numpy as np
    from oracle import sox as osox
    host = host_details()
    threads = host["blas_threads"] or host["nproc"]
    t0 = time.time()
    U = osox.precontract_u(s.X, s.V)
    t_u = time.time() - t0
    m = G.shape[0]
    t0 = time.time()
    for k in taus:
        osox.sigma_thc_paper(s.X, s.V, G[k], G[m - 1 - k], U=U)
    dt = time.time() - t0
    return {"value": len(taus) / dt, "unit": "tau-points/s", "cores": threads,
            "kind": "oracle", "host": host,
            "sample": f"{len(taus)} of {m} tau points (k={list(taus)}) of the same workload, "
                      f"FP64 NumPy, {dt:.1f} s; U precontraction excluded ({t_u:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp16x2", choices=list(PEAK))
    ap.add_argument("--workload", default="sox_n300_naux1800_ntau100")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--cpu-taus", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-seed-sweep", action="store_true",
                    help="skip the energy check of the other seeds with stored oracle values")
    ap.add_argument("--symmetry", default="auto", choices=["auto", "off"])
    ap.add_argument("--no-direct", action="store_true",
                    help="skip the GF2 direct-term measurement beside the SOX one")
    ap.add_argument("--tau-sample", type=int, default=0,
                    help="time tau points 0..K-1 only (K > 0), for workloads whose full "
                         "evaluation takes minutes; every tau point costs the same")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU's share only: the SOX self-energy shards over tau "
              "points with no communication, so run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2404_17744_amd import synth, thcsox

    dev = torch.device("cuda:0")
    s, tau, w, G, beta = synth.workload(args.workload, seed=args.seed)
    m = len(tau)
    X = torch.from_numpy(s.X).to(dev)
    V = torch.from_numpy(s.V).to(dev)
    Gd = torch.from_numpy(G).to(dev)
    S = torch.zeros_like(Gd)

    t0 = time.time()
    plan = thcsox.Plan(X, V, tau, w, beta, precision=args.precision)
    plan.set_symmetry(args.symmetry)
    plan_s = time.time() - t0
    info = plan.info()
    k_end = min(args.tau_sample, m) if args.tau_sample > 0 else m
    ksel = None if k_end == m else k_end
    for _ in range(args.warmup):
        plan.sigma(Gd, 0, ksel, out=S)
        if ksel is None:
            plan.energy(Gd, S)
    ms, E_mixed, st = timed_steps(plan, Gd, S, args.steps, torch, ksel)
    S_mixed = S.clone()
    fused_flop, n_sym = fused_flop_per_launch(plan, info, k_end)
    # the GF2 direct (bubble) term on the same plan (FP64), one full evaluation
    direct = None
    if not args.no_direct:
        Sd = torch.zeros_like(Gd)
        plan.sigma_direct(Gd, 0, k_end, out=Sd)   # warm-up; allocates the term's buffers
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(plan.stream)
        plan.sigma_direct(Gd, 0, k_end, out=Sd)
        E_dir = plan.energy(Gd, Sd) if ksel is None else None
        e1.record(plan.stream)
        torch.cuda.synchronize()
        ms_d = e0.elapsed_time(e1)
        na, nn_ = float(s.naux), float(s.n)
        mac_d = 2 * na ** 3 + 3 * na * na * nn_ + 3 * na * nn_ * nn_
        direct = {"tau_points_per_s": k_end / (ms_d * 1e-3), "ms_per_step": ms_d,
                  "E_dir": E_dir, "mac_per_tau": mac_d,
                  "tflops": 2 * mac_d * k_end / (ms_d * 1e-3) / 1e12,
                  "E_gf2_second_order": None if ksel else E_dir + E_mixed}
    plan.close()

    fused_ms, fused_n = st["fused"]
    fused_avg = fused_ms / max(1, fused_n)
    achieved = fused_flop / (fused_avg * 1e-3) / 1e12
    peak = PEAK[args.precision]

    # FP64 path beside it
    fp64 = None
    if args.fp64_steps > 0:
        p64 = thcsox.Plan(X, V, tau, w, beta, precision="fp64")
        p64.set_symmetry(args.symmetry)
        S64 = torch.zeros_like(Gd)
        p64.sigma(Gd, 0, 2, out=S64)
        ms64, E64, st64 = timed_steps(p64, Gd, S64, args.fp64_steps, torch, ksel)
        f64_avg = st64["fused"][0] / max(1, st64["fused"][1])
        fp64 = {"tau_points_per_s": k_end / (ms64 * 1e-3), "ms_per_step": ms64, "E_sox": E64,
                "fused_tflops": fused_flop / (f64_avg * 1e-3) / 1e12,
                "fused_frac_of_fp64_peak": fused_flop / (f64_avg * 1e-3) / 1e12 / PEAK["fp64"]}
        d = (S_mixed - S64).abs().max().item() / S64.abs().max().item()
        fp64["mixed_sigma_rel_err_vs_gpu_fp64"] = d
        fp64["mixed_energy_err_vs_gpu_fp64"] = None if ksel else E_mixed - E64
        p64.close()

    accuracy = {"E_sox": E_mixed}
    gold = os.path.join(ROOT, "tests", "golden", f"oracle_{args.workload}_seed{args.seed}.json")
    if os.path.exists(gold) and ksel is None:
        with open(gold) as f:
            g = json.load(f)
        # inputs may differ in the last bits across hosts (BLAS code paths): ~1e-14 Ha
        accuracy["input_digest_matches_golden"] = g.get("input_digest") == s.digest()
        accuracy["E_oracle"] = g["E_sox"]
        accuracy["energy_err_vs_fp64_oracle_Ha"] = E_mixed - g["E_sox"]
        if fp64:
            accuracy["fp64_path_energy_err_vs_oracle_Ha"] = fp64["E_sox"] - g["E_sox"]
        Sm = S_mixed.cpu().numpy()
        errs = [abs(Sm[k, t, r] - v) for k, t, r, v in g["samples"]]
        accuracy["sigma_sampled_rel_err_vs_oracle"] = max(errs) / g["sigma_absmax"]

    # the same workload at the other seeds that have stored oracle values
    # (untimed: one evaluation each in the headline precision)
    per_seed = {}
    if ksel is None and not args.no_seed_sweep:
        for sd in range(5):
            path = os.path.join(ROOT, "tests", "golden", f"oracle_{args.workload}_seed{sd}.json")
            if not os.path.exists(path):
                continue
            if sd == args.seed:
                Es = E_mixed
            else:
                s2, tau2, w2, G2, beta2 = synth.workload(args.workload, seed=sd)
                X2, V2 = torch.from_numpy(s2.X).to(dev), torch.from_numpy(s2.V).to(dev)
                G2d = torch.from_numpy(G2).to(dev)
                p2 = thcsox.Plan(X2, V2, tau2, w2, beta2, precision=args.precision)
                p2.set_symmetry(args.symmetry)
                Es = p2.energy(G2d, p2.sigma(G2d))
                p2.close()
                del X2, V2, G2d
            with open(path) as f:
                per_seed[str(sd)] = Es - json.load(f)["E_sox"]
        accuracy["energy_err_vs_fp64_oracle_Ha_per_seed"] = per_seed

    out = {
        "metric": METRIC,
        "value": k_end / (ms * 1e-3),
        "unit": "tau-points/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": args.workload, "n": s.n, "naux": s.naux, "ntau": m,
                   "beta": beta, "seed": args.seed, "precision": args.precision,
                   "symmetry": args.symmetry, "vsplit": info["vsplit"],
                   "partial_tiles": "fp32" if info["partial_f32"] else "fp64",
                   "tau_sample": k_end,
                   "parallelism": "none (one GPU; tau points are independent)"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(args.precision, args.workload, args.symmetry,
                                                 info),
                     "kernel": ("fused_f16_kernel" if args.precision == "fp16x2"
                                else f"fused_kernel<{args.precision}>"),
                     "avg_launch_ms": fused_avg, "launches": fused_n,
                     "algorithmic_flop_per_launch": fused_flop,
                     "symmetric_tau_points": n_sym,
                     "plane_products": PRODUCTS[args.precision],
                     "mfma_busy_frac": achieved * PRODUCTS[args.precision] / peak},
        "tflops_whole_step": 2.0 * info["mac_per_tau"] * k_end / (ms * 1e-3) / 1e12,
        "stage_ms_per_step": {k: v[0] / args.steps for k, v in st.items()},
        "plan_s": plan_s,
        "fp64_path": fp64,
        "speedup_vs_fp64_path": (k_end / (ms * 1e-3)) / fp64["tau_points_per_s"] if fp64 else None,
        "gf2_direct_term": direct,
        "accuracy": accuracy,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, G, list(range(args.cpu_taus)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
