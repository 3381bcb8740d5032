"""Benchmark: FP64 gradient evaluations/s of the whitened Fourier-space PTA
log-posterior on the 67-pulsar / 250k-TOA workload (64 HMC chains, leapfrog
length 20), batched form vs plain form, on one GPU.

A step is one HMC trajectory of all chains: momentum draw, 20 leapfrog steps
(each a full log-posterior + gradient evaluation through the batched path)
and the accept test, replayed as one captured HIP graph.  Prints one JSON
line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X dense FP64 (vector and matrix)
HBM_PEAK_GBS = 8000.0


def toa_pass_flops(ds, n_chains):
    """Algorithmic flops of one TOA-pass launch: per TOA and chain,
    F a (2K sin/cos + 3 timing-model columns), F_dm a_dm, the residual,
    g = r/N, chi^2, F^T g and F^T (w g)."""
    K = max(ds["nf_rn"], ds["nf_gw"])
    Kd = ds["nf_dm"]
    per = 2 * (2 * K + 3) + 2 * (2 * Kd) + 3 + 1 + 2 + 2 * (2 * K + 3) + 1 + 2 * (2 * Kd)
    return float(per) * ds["t"].size * n_chains, per


def cpu_baseline(ds, n_chains_sample=8, min_seconds=10.0, seed=204):
    """The oracle timed on the host cores on a bounded sample of the workload."""
    import numpy as np
    import synth
    from oracle import model
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    th = synth.injected_theta(ds, 203)
    X = synth.random_points(ds, n_chains_sample, seed, theta=th, theta_jitter=0.2)
    prep = model.Prepared(ds)
    model.logp_grad(prep, X[:1], with_scale=False)
    n = 0
    t0 = time.perf_counter()
    while True:
        model.logp_grad(prep, X, with_scale=False)
        n += X.shape[0]
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    return dict(value=n / el, unit="grad evals/s", cores=int(threads), kind="oracle",
                sample=f"{n} chain-evaluations ({n_chains_sample} chains per call) of the "
                       f"67 psr / 250k TOA workload, {el:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--chains", type=int, default=64)
    ap.add_argument("--leapfrog", type=int, default=20)
    ap.add_argument("--eps", type=float, default=0.3, help="largest step tried")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(chains shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2607_06834_amd import api, autotune, precond

    torch.cuda.set_device(0)
    ds = synth.cfg2()
    C, L = args.chains, args.leapfrog
    th = synth.injected_theta(ds, 203)
    X0 = synth.random_points(ds, C, 204, theta=th, theta_jitter=0.2)
    g = api.Dataset(ds)
    x = torch.tensor(X0, device="cuda")
    tuning = g.ptafs_get_tuning()
    tune_log = None
    if not args.no_tune:
        tuning, tune_log = autotune.tune(g, x)

    # diagonal inverse mass from the local precision at the injection (App. A),
    # chains moved to the conditional mode of their coefficients, and the
    # largest step whose trial trajectory stays valid (sampler warm-up)
    inv_mass = precond.inverse_mass(g, x[0].clone())
    x = precond.ascend_coefficients(g, x, inv_mass)
    lp, gr, st = g.ptafs_logp_grad(x)
    eps = precond.find_step(g, x, lp, gr, inv_mass, n_leapfrog=L, eps0=args.eps)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        lp, gr, st = g.ptafs_logp_grad(x)
        acc = torch.zeros(C, dtype=torch.int64, device="cuda")
        bad = torch.zeros(C, dtype=torch.int64, device="cuda")
        # warmup (the first call captures the trajectory graph)
        g.ptafs_hmc_run(x, lp, gr, acc, n_traj=max(args.warmup, 1), n_leapfrog=L, eps=eps,
                        seed=203, traj0=0, inv_mass=inv_mass, n_invalid=bad)
        stream.synchronize()
        acc.zero_()
        bad.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.ptafs_hmc_run(x, lp, gr, acc, n_traj=args.steps, n_leapfrog=L, eps=eps,
                        seed=203, traj0=max(args.warmup, 1), inv_mass=inv_mass, n_invalid=bad)
        stream.synchronize()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # every timed leapfrog evaluation must have been a full, valid one
        valid = 1.0 - float(bad.sum().item()) / (C * L * args.steps)
    ms_step = el / args.steps * 1e3
    value = C * L * args.steps / el

    # per-stage timing of the evaluation (HIP events on the launch stream)
    stages = g.ptafs_profile_stages(x, reps=20, stream=stream)
    eval_ms = sum(stages.values())
    flops, per_toa = toa_pass_flops(ds, C)
    achieved = flops / (stages["toa"] * 1e-3) / 1e12
    plain = None
    if not args.no_plain:
        ps = g.ptafs_profile_stages(x, reps=2, plain=True, stream=stream)
        plain = dict(value=C / (sum(ps.values()) * 1e-3), unit="grad evals/s",
                     ms_per_eval=round(sum(ps.values()), 4),
                     toa_ms=round(ps["toa"], 4))
    cpu = None if args.no_cpu else cpu_baseline(ds, min_seconds=args.cpu_seconds)

    out = {
        "metric": "grad evals/s, 67 psr/250k TOA FP64: batched vs plain; serve p50/p99 latency",
        "value": value,
        "unit": "grad evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (NANOGrav-15yr-shaped, seeded)",
        "config": {
            "workload": "67 psr / 250000 TOA over 16 yr; RN 30 + DM 30 + HD common 14 freqs; "
                        f"{C} HMC chains x leapfrog {L}; step = one HIP-graph trajectory",
            "n_psr": int(ds["n_psr"]), "n_toa": int(ds["t"].size), "chains": C,
            "leapfrog": L, "eps": eps, "d": int(g.d),
            "tuning": {"tiles_per_chunk": tuning[0], "waves_per_block": tuning[1],
                       "xcd_map": tuning[2]},
        },
        "roofline": {
            "bound": "mfma",
            "kernel": "k_toa_mfma (TOA pass, FP64 MFMA 16x16x4)",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": None,
            "flop_per_toa_chain": per_toa,
            "avg_launch_ms": stages["toa"],
        },
        "stages_ms": {k: round(v, 5) for k, v in stages.items()},
        "batched_eval": {"value": C / (eval_ms * 1e-3), "unit": "grad evals/s",
                         "ms_per_eval": round(eval_ms, 5)},
        "plain": plain,
        "accept_rate": float(acc.sum().item()) / (C * args.steps),
        "valid_eval_fraction": valid,
        "cpu_baseline": cpu,
    }
    if tune_log is not None:
        out["autotune"] = tune_log
    print(json.dumps(out))
    g.close()


if __name__ == "__main__":
    main()
