"""Write oracle reference values for the full-size workloads (CPU, FP64).

Calls only the oracle package and the seeded input generator.  Output per
workload: tests/golden/oracle_<workload>_seed<seed>.json with the SOX energy,
Tr[G(beta-tau_k) Sigma(tau_k)] for every k, max|Sigma| over all k, and Sigma
at a fixed set of sampled (k, t, r) positions.

    python tests/golden/make_oracle_golden.py sox_n300_naux1800_ntau100 0
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import energy as oenergy  # noqa: E402
from oracle import sox as osox  # noqa: E402
from paper_2404_17744_amd import synth  # noqa: E402


def main(name: str, seed: int) -> None:
    s, tau, w, G, beta = synth.workload(name, seed=seed)
    m = len(tau)
    U = osox.precontract_u(s.X, s.V)
    S = np.empty_like(G)
    t0 = time.time()
    for k in range(m):
        S[k] = osox.sigma_thc_paper(s.X, s.V, G[k], G[m - 1 - k], U=U)
        print(f"{name} seed {seed}: tau {k + 1}/{m} ({time.time() - t0:.0f} s)", flush=True)
    rng = np.random.default_rng(12345)
    ks = np.concatenate([[0, m - 1, m // 2], rng.integers(0, m, 61)])
    ts = rng.integers(0, s.n, len(ks)); rs = rng.integers(0, s.n, len(ks))
    out = {
        "workload": name, "seed": seed, "input_digest": s.digest(),
        "E_sox": oenergy.energy_tau(G, S, w),
        "trace_per_tau": [float(np.sum(G[m - 1 - k].T * S[k])) for k in range(m)],
        "sigma_absmax": float(np.abs(S).max()),
        "sigma_absmax_per_tau": [float(np.abs(S[k]).max()) for k in range(m)],
        "samples": [[int(k), int(t), int(r), float(S[k, t, r])] for k, t, r in zip(ks, ts, rs)],
    }
    path = os.path.join(HERE, f"oracle_{name}_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, "E_sox", out["E_sox"])


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 0)
