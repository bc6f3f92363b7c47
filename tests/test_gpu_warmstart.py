"""The learned warm start, end to end on small systems (n in [40, 56], naux =
5n, 64 tau points, interaction scale 0.2): collect first-iteration and
converged THC-basis self-energies with the plain loop, train the network on
the GPU, then start held-out systems from its prediction (all of them predicted
as one ragged batch).

What is checked: both starts converge to the same energy (the start cannot
change the fixed point); the trained network fits the data better than the
identity map (what it learned); the warm start saves SOX evaluations -- at
least 0.3 on average, on at least one system, and costs none on any (the
evaluation that produces the network's input is counted).  A prediction that
the Dyson step cannot use (forced to NaN on the host) falls back to the
Hartree-Fock start and converges to the same energy.  At the full workload
(200 training and 56 evaluation systems, n in [40, 160]) the learned start
also saves wall time, inference included.
"""
import numpy as np
import pytest
import torch

from paper_2404_17744_amd import synth, warmstart

pytestmark = pytest.mark.gpu


def test_warm_start_gain(dev):
    print("case warm start train 64 eval 24 n 40..56 lam 0.2", flush=True)
    rng = np.random.default_rng(7)
    nr = (40, 56)
    x, t, stats = warmstart.collect(range(1000, 1064), 0.2, 4096, rng, n_range=nr)
    assert all(s["converged"] for s in stats)
    identity = float(((x - t) ** 2).mean().item())
    net, losses = warmstart.train(x, t, hidden=512, epochs=30)
    inet = warmstart.inference_net(net)
    net.close()
    rows = warmstart.evaluate(range(1064, 1088), 0.2, inet, n_range=nr)
    inet.close()
    hf = np.array([r["hf_evals"] for r in rows])
    warm = np.array([r["warm_evals"] for r in rows])
    print(f"  identity loss {identity:.3e} trained {losses[-1]:.3e}; SOX evaluations "
          f"HF {hf.mean():.2f} warm {warm.mean():.2f}; saved on {(warm < hf).sum()}, "
          f"worse on {(warm > hf).sum()} of {len(rows)}; wall time per system HF "
          f"{np.mean([r['hf_s'] for r in rows]):.3f} s warm "
          f"{np.mean([r['warm_s'] for r in rows]):.3f} s")
    assert all(r["hf_converged"] and r["warm_converged"] for r in rows)
    assert not any(r["warm_fell_back"] for r in rows)
    assert max(abs(r["E_warm"] - r["E_hf"]) for r in rows) < 1e-6
    assert losses[-1] < 0.9 * identity
    assert hf.mean() - warm.mean() >= 0.3
    assert (warm < hf).sum() >= 1 and (warm > hf).sum() == 0


def test_unusable_prediction_falls_back_to_hartree_fock(dev):
    print("case warm start NaN prediction n 40", flush=True)
    s = synth.warmstart_system(1100, 0.2, (40, 40))
    scf = warmstart.SCF(s)
    ev_hf, E_hf, ok_hf = scf.run()
    assert ok_hf and not scf.fell_back
    bad = torch.full_like(scf.S, float("nan"))
    ev, E, ok = scf.run(Sigma_start=bad, count_start=1)
    scf.close()
    print(f"  HF {ev_hf} evaluations; NaN start -> fell back, {ev} evaluations")
    assert ok and scf.fell_back
    assert ev == ev_hf + 1            # the spent evaluation stays counted
    assert abs(E[-1] - E_hf[-1]) < 1e-9


def test_warm_start_pays_at_the_full_workload(dev):
    """The 200-training / 56-evaluation workload (n in [40, 160], naux = 5n, 64
    tau points, interaction scale 0.2, seeds 1000-1255): with the fused bf16
    inference the learned start saves SOX evaluations (at least 0.3 on average,
    none worse) and wall time: the batched first evaluations and the inference
    over all 15.4 M THC pairs cost less than the evaluations saved."""
    print("case warm start train 200 eval 56 n 40..160 lam 0.2", flush=True)
    rng = np.random.default_rng(7)
    x, t, stats = warmstart.collect(range(1000, 1200), 0.2, 4096, rng, n_range=(40, 160))
    assert all(s["converged"] for s in stats)
    net, losses = warmstart.train(x, t, hidden=512, epochs=30)
    rows = warmstart.evaluate(range(1200, 1256), 0.2, net, n_range=(40, 160))
    net.close()
    hf = np.array([r["hf_evals"] for r in rows])
    warm = np.array([r["warm_evals"] for r in rows])
    t_hf = np.mean([r["hf_s"] for r in rows])
    t_warm = np.mean([r["warm_s"] for r in rows])
    print(f"  SOX evaluations HF {hf.mean():.3f} warm {warm.mean():.3f}; saved on "
          f"{(warm < hf).sum()}, worse on {(warm > hf).sum()}; wall time per system HF "
          f"{t_hf:.4f} s warm {t_warm:.4f} s")
    assert all(r["hf_converged"] and r["warm_converged"] for r in rows)
    assert max(abs(r["E_warm"] - r["E_hf"]) for r in rows) < 1e-6
    assert hf.mean() - warm.mean() >= 0.3
    assert (warm > hf).sum() == 0
    assert t_warm < t_hf
