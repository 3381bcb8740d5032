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
VALU_PEAK_TFLOPS = 67.3      # FP64 vector FMA as measured by microbench/peaks on MI355X
HBM_PEAK_GBS = 8000.0


def _log(msg):
    """Progress of the run on stderr (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def toa_pass_flops(ds, n_chains):
    """Algorithmic flops of one TOA-pass launch: per TOA and chain,
    F a (2K sin/cos + 3 timing-model columns), F_dm a_dm, the residual,
    g = r/N, chi^2, F^T g and F^T (w g)."""
    K = max(ds["nf_rn"], ds["nf_gw"])
    Kd = ds["nf_dm"]
    per = 2 * (2 * K + 3) + 2 * (2 * Kd) + 3 + 1 + 2 + 2 * (2 * K + 3) + 1 + 2 * (2 * Kd)
    return float(per) * ds["t"].size * n_chains, per


def measured_traffic(tuning):
    """HBM bytes per TOA-pass launch from the committed rocprofv3 counter
    summary (one entry per profiled tuning), if it was taken on the current
    kernel source and covers this tuning."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_toa_mfma_traffic.md")
    if not os.path.exists(path):
        return None
    key = "traffic_bytes_per_launch[" + " ".join(str(int(t)) for t in tuning) + "]"
    fields = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    m = hashlib.sha256()
    for f in ("k_toa.hip", "common.h", "cw_dev.h"):
        m.update(open(os.path.join(ROOT, "paper_2607_06834_amd", "csrc", f), "rb").read())
    if fields.get("source_sha256") != m.hexdigest() or key not in fields:
        return None
    return float(fields[key])


def measured_std_traffic():
    """HBM bytes per launch of k_std_fwd at the 67-pulsar shape from the
    committed counter summary, if it was taken on the current kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "std_form_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    m = hashlib.sha256()
    for f in ("k_std.hip", "std.h", "cw_dev.h"):
        m.update(open(os.path.join(ROOT, "paper_2607_06834_amd", "csrc", f), "rb").read())
    key = "traffic_bytes_per_launch[k_std_fwd 67psr]"
    if fields.get("source_sha256") != m.hexdigest() or key not in fields:
        return None
    return float(fields[key])


def cpu_baseline(ds, n_chains_sample=8, min_seconds=10.0, seed=204, repeats=3, label="67 psr / 250k TOA"):
    """The oracle timed on the host cores on a bounded sample of the workload:
    ``repeats`` timed samples of at least min_seconds / repeats each, the
    median reported (the spread beside it)."""
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
    rates, total_n, total_s = [], 0, 0.0
    for _ in range(repeats):
        n = 0
        t0 = time.perf_counter()
        while True:
            model.logp_grad(prep, X, with_scale=False)
            n += X.shape[0]
            el = time.perf_counter() - t0
            if el >= min_seconds / repeats:
                break
        rates.append(n / el)
        total_n += n
        total_s += el
    return dict(value=float(np.median(rates)), unit="grad evals/s", cores=int(threads), kind="oracle",
                samples=[round(r, 3) for r in rates],
                sample=f"median of {repeats} samples, {total_n} chain-evaluations in all ({n_chains_sample} "
                       f"chains per call) of the {label} workload, {total_s:.1f} s")


def serving_bench(n_traj, rates, n_req, n_chains=16, n_leapfrog=20, quantum=10, max_slots=8,
                  use_graph=True, budget=None, seed0=501, eps=1e-4):
    """Poisson arrivals of independent data sets (20-120 pulsars, 200-8000
    TOAs each, 10-30 frequencies, CW with probability 1/2), each asking for
    n_traj trajectories of n_chains chains, served with continuous batching.
    Every request is first run alone on the idle GPU (its service time); then
    for each rate: p50/p99 of completion - arrival, and p50/p99 of each
    request's slowdown (its latency over its own alone service time)."""
    import numpy as np
    import synth
    from paper_2607_06834_amd import serve

    pool = []
    for i in range(n_req):
        ds = synth.serving_request(seed0 + i)
        th = synth.injected_theta(ds, seed0 + 1000 + i)
        x0 = synth.random_points(ds, n_chains, seed0 + 2000 + i, theta=th, theta_jitter=0.02)
        im = np.ones(x0.shape[1])
        im[: ds["prior_lo"].size] = 1e-8       # hyper-parameters held near their start
        pool.append((ds, x0, im))
    probe = serve.Server(budget_bytes=1 << 40, max_slots=1, quantum=quantum)
    fps = [probe.footprint(ds, n_chains) for ds, _, _ in pool]
    probe.close()
    if budget is None:
        budget = int(6 * np.median(fps))
    evals_per_req = n_traj * n_leapfrog * n_chains

    def run(rate, reqs, slots):
        srv = serve.Server(budget_bytes=budget, max_slots=slots, quantum=quantum, use_graph=use_graph)
        rng = np.random.default_rng(7)
        gaps = rng.exponential(1.0 / rate, len(reqs)) if rate else np.zeros(len(reqs))
        ids = []
        t0 = time.perf_counter()
        t_next = t0
        for g, (ds, x0, im) in zip(gaps, reqs):
            t_next += g
            while time.perf_counter() < t_next:
                time.sleep(min(1e-3, max(0.0, t_next - time.perf_counter())))
            ids.append(srv.submit(ds, x0=x0, n_traj=n_traj, n_leapfrog=n_leapfrog, eps=eps,
                                  seed=11 + len(ids), inv_mass=im))
        res = [srv.wait(i, timeout=3600) for i in ids]
        stats = dict(max_used_bytes=srv.max_used, max_active=srv.max_active)
        srv.close()
        lat = np.array([r["latency"] for r in res])
        t_first = min(r["t_arrival"] for r in res)
        t_last = max(r["t_done"] for r in res)
        bad = sum(int(r["n_invalid"].sum()) for r in res)
        acc = sum(int(r["n_accept"].sum()) for r in res) / (n_chains * n_traj * len(res))
        return lat, dict(rate=rate, completed=len(res), p50_ms=float(np.percentile(lat, 50) * 1e3),
                         p99_ms=float(np.percentile(lat, 99) * 1e3), mean_ms=float(lat.mean() * 1e3),
                         evals_per_s=evals_per_req * len(res) / (t_last - t_first),
                         valid_eval_fraction=1.0 - bad / (evals_per_req * len(res)),
                         accept_rate=acc, **stats)

    run(0.0, pool[:1], 1)                  # warm-up (code objects, first graph capture)
    # service time of every request on an idle GPU (one request at a time)
    alone = np.array([run(0.0, [p], 1)[0][0] for p in pool])
    _log(f"serving: alone service times {np.round(alone * 1e3, 1).tolist()} ms")
    out = []
    for rate in rates:
        lat, r = run(rate, pool, max_slots)
        slow = lat / alone
        r["slowdown_p50"] = float(np.percentile(slow, 50))
        r["slowdown_p99"] = float(np.percentile(slow, 99))
        out.append(r)
        _log(f"serving at {rate} req/s: p50 {r['p50_ms']:.1f} ms, p99 {r['p99_ms']:.1f} ms, "
             f"slowdown p50 {r['slowdown_p50']:.2f} p99 {r['slowdown_p99']:.2f}")
        if r["p50_ms"] > 20 * np.median(alone) * 1e3:
            break                            # saturated
    return dict(
        requests_per_rate=n_req, n_traj=n_traj, n_leapfrog=n_leapfrog, n_chains=n_chains,
        quantum=quantum, max_slots=max_slots, budget_bytes=budget,
        footprint_bytes_median=int(np.median(fps)), footprint_bytes_max=int(max(fps)),
        alone_ms_median=float(np.median(alone) * 1e3), alone_ms_p99=float(np.percentile(alone, 99) * 1e3),
        alone_ms=[round(float(a) * 1e3, 2) for a in alone], rates=out)


def std_flops_fwd(P):
    """Algorithmic flops of k_std_fwd per (pulsar, chain): Cholesky of the
    P x P CURN precision (P^3/3), the triangular inverse (P^3/3) and four
    triangular mat-vecs (X beta d, X^T (t + z), X^T t, L z: 4 P^2)."""
    return 2.0 * P ** 3 / 3.0 + 4.0 * P * P


def std_flops_split(P, PG, PR):
    """Algorithmic flops of the transform stage per (pulsar, chain) with split
    coefficients: the combined factorisation (std_flops_fwd), each set's
    Cholesky and inverse with one mat-vec (2 PB^3 / 3 + PB^2), and S0 a
    (2 P^2)."""
    return std_flops_fwd(P) + 2.0 * (PG ** 3 + PR ** 3) / 3.0 + PG * PG + PR * PR + 2.0 * P * P


def std_bench(n_chains=64, n_leapfrog=20, steps=10, warmup=2, cw=False, split=False):
    """The paper's standardized form (CURN transform on the Gram form, timing
    model marginalised) on the same 67-pulsar / 250k-TOA data set, or (cw)
    on the simulated CW array with the CW in its own Fourier basis, or
    (split) the 67-pulsar set with split common-process / pulsar-noise
    coefficients: HMC trajectories replayed as one HIP graph, per-stage times
    and the roofline of its dominant stage."""
    import numpy as np
    import torch
    import synth
    from paper_2607_06834_amd import api

    ds = synth.cw_array() if cw else synth.cfg2()
    if split:
        ds["split"] = 1
    t0 = time.perf_counter()
    g = api.StdDataset(ds)
    t_create = time.perf_counter() - t0
    lay = g.layout
    th = synth.injected_theta(ds, 203, cw=synth.CW_PAPER if cw else None)
    rng = np.random.default_rng(204)
    th = np.clip(th + rng.uniform(-0.2, 0.2, (n_chains, th.size)), ds["prior_lo"], ds["prior_hi"])
    X0 = np.concatenate([th, rng.standard_normal((n_chains, g.d - int(lay.n_theta)))], axis=1)
    im = torch.ones(g.d, dtype=torch.float64, device="cuda")
    im[: int(lay.n_theta)] = 1e-4
    stream = torch.cuda.Stream()
    eps_used, acc_rate = None, None
    with torch.cuda.stream(stream):
        # the largest step (of a fixed ladder) whose pilot trajectories accept
        # at least 60% and keep every evaluation valid
        for eps in (0.4, 0.2, 0.1, 0.05, 0.02):
            x = torch.tensor(X0, device="cuda")
            lp, gr, st = g.ptafs_std_logp_grad(x, stream=stream)
            acc = torch.zeros(n_chains, dtype=torch.int64, device="cuda")
            bad = torch.zeros(n_chains, dtype=torch.int64, device="cuda")
            g.ptafs_std_hmc_run(x, lp, gr, acc, n_traj=2, n_leapfrog=n_leapfrog, eps=eps, seed=301,
                                inv_mass=im, n_invalid=bad, stream=stream)
            stream.synchronize()
            if acc.sum().item() >= 0.6 * 2 * n_chains and bad.sum().item() == 0:
                eps_used = eps
                break
        eps_used = eps_used or 0.02
        x = torch.tensor(X0, device="cuda")
        lp, gr, st = g.ptafs_std_logp_grad(x, stream=stream)
        acc = torch.zeros(n_chains, dtype=torch.int64, device="cuda")
        bad = torch.zeros(n_chains, dtype=torch.int64, device="cuda")
        g.ptafs_std_hmc_run(x, lp, gr, acc, n_traj=max(warmup, 1), n_leapfrog=n_leapfrog, eps=eps_used,
                            seed=302, inv_mass=im, n_invalid=bad, stream=stream)
        stream.synchronize()
        acc.zero_()
        bad.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.ptafs_std_hmc_run(x, lp, gr, acc, n_traj=steps, n_leapfrog=n_leapfrog, eps=eps_used,
                            seed=302, traj0=max(warmup, 1), inv_mass=im, n_invalid=bad, stream=stream)
        stream.synchronize()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        acc_rate = float(acc.sum().item()) / (n_chains * steps)
        valid = 1.0 - float(bad.sum().item()) / (n_chains * n_leapfrog * steps)
    stages = g.ptafs_std_profile_stages(x, reps=20, stream=stream)
    P = int(lay.p)
    fpp = std_flops_fwd(P)
    kern = "k_std_fwd (per-pulsar CURN factorisation + inverse)"
    if split:
        PG, PR = 2 * int(ds["nf_gw"]), 2 * (int(ds["nf_rn"]) + int(ds["nf_dm"]))
        fpp = std_flops_split(P, PG, PR)
        kern = ("transform stage: k_std_fwd (combined MAP) + k_split_fac x 2 (common, pulsar-noise sets) "
                "+ k_split_comb")
    flops = fpp * n_chains * int(lay.n_psr)
    achieved = flops / (stages["transform"] * 1e-3) / 1e12
    g.close()
    if split:
        wl = ("67 psr / 250000 TOA, RN 30 + DM 30 + HD common 14 with split coefficients (P = 120 combined, "
              f"sets of {PG} and {PR}), {n_chains} chains x leapfrog {n_leapfrog}; "
              "step = one HIP-graph trajectory")
    elif cw:
        wl = (f"{int(lay.n_psr)} psr x 180 TOA over 15 yr, RN 30 + HD common 14 (P = {P}), CW in its own "
              f"basis of 60 frequencies on 2T, {n_chains} chains x leapfrog {n_leapfrog}; "
              "step = one HIP-graph trajectory")
    else:
        wl = ("67 psr / 250000 TOA, RN 30 + DM 30 + HD common 14 (P = 120 coefficients per pulsar), "
              f"{n_chains} chains x leapfrog {n_leapfrog}; step = one HIP-graph trajectory")
    return dict(
        workload=wl,
        value=n_chains * n_leapfrog * steps / el, unit="grad evals/s", ms_per_step=el / steps * 1e3,
        eps=eps_used, accept_rate=acc_rate, valid_eval_fraction=valid, create_s=t_create,
        stages_ms={k: round(v, 5) for k, v in stages.items()},
        ms_per_eval=round(sum(stages.values()), 5),
        roofline={"bound": "mfma", "kernel": kern,
                  "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                  "frac": achieved / FP64_PEAK_TFLOPS, "flop_per_problem": fpp,
                  "problems_per_launch": n_chains * int(lay.n_psr), "avg_launch_ms": stages["transform"],
                  # counted for the shared form at 64 chains (profiles/std_form_traffic.md)
                  "traffic": measured_std_traffic() if not (cw or split) and n_chains == 64 else None})


def cfg4_bench(n_chains=256, n_leapfrog=20, n_traj=10, n_plain=20):
    """The 3-pulsar, 1500-TOA array (config 1) with 256 chains: batched form
    (ragged MFMA TOA pass, HIP-graph trajectories) against the plain form
    (one TOA-pass launch per pulsar, vector ALU, each evaluation launched from
    Python); both checked against the oracle on a sample of chains first."""
    import numpy as np
    import torch
    import synth
    from oracle import model
    from paper_2607_06834_amd import api

    ds = synth.cfg1()
    th = synth.injected_theta(ds, 403, rn=(-14.0, 4.0))
    X0 = synth.random_points(ds, n_chains, 404, theta=th, theta_jitter=0.1)
    g = api.Dataset(ds)
    x = torch.tensor(X0, device="cuda")
    lp_b, gr_b, st_b = g.ptafs_logp_grad(x)
    lp_p, gr_p, st_p = g.ptafs_logp_grad_plain(x)
    idx = np.arange(0, n_chains, 37)
    ref = model.logp_grad(model.Prepared(ds), X0[idx])
    for lp, gr in ((lp_b, gr_b), (lp_p, gr_p)):
        lpn, grn = lp.cpu().numpy()[idx], gr.cpu().numpy()[idx]
        assert np.all(np.abs(lpn - ref["logp"]) <= 1e-9 * np.abs(ref["logp"]))
        assert np.all(np.abs(grn - ref["grad"]) <= 1e-7 * np.maximum(np.abs(ref["grad"]), ref["scale"]))
    lay = model.Prepared(ds).lay
    im = torch.ones(g.d, dtype=torch.float64, device="cuda")
    im[: lay.n_theta] = 1e-4
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        lp, gr, _ = g.ptafs_logp_grad(x, stream=stream)
        acc = torch.zeros(n_chains, dtype=torch.int64, device="cuda")
        g.ptafs_hmc_run(x, lp, gr, acc, n_traj=2, n_leapfrog=n_leapfrog, eps=0.01, seed=403,
                        inv_mass=im, stream=stream)
        stream.synchronize()
        t0 = time.perf_counter()
        g.ptafs_hmc_run(x, lp, gr, acc, n_traj=n_traj, n_leapfrog=n_leapfrog, eps=0.01, seed=403,
                        traj0=2, inv_mass=im, stream=stream)
        stream.synchronize()
        el_b = time.perf_counter() - t0
        out = (torch.empty_like(lp), torch.empty_like(gr), torch.empty(n_chains, dtype=torch.int32,
                                                                        device="cuda"))
        for _ in range(3):
            g.ptafs_logp_grad_plain(x, out=out, stream=stream)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_plain):
            g.ptafs_logp_grad_plain(x, out=out, stream=stream)
        stream.synchronize()
        el_p = time.perf_counter() - t0
        for _ in range(3):
            g.ptafs_logp_grad(x, out=out, stream=stream)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_plain):
            g.ptafs_logp_grad(x, out=out, stream=stream)
        stream.synchronize()
        el_e = time.perf_counter() - t0
    g.close()
    batched = n_chains * n_leapfrog * n_traj / el_b
    plain = n_chains * n_plain / el_p
    return dict(workload="3 psr / 1500 TOA (config 1), 256 chains, leapfrog 20",
                batched_graph_evals_per_s=batched, batched_eager_evals_per_s=n_chains * n_plain / el_e,
                plain_evals_per_s=plain, batched_over_plain=batched / plain,
                parity_checked_chains=int(idx.size))


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
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--tuning", type=int, nargs=3, metavar=("TILES", "WAVES", "XCD"),
                    help="TOA-pass tuning for --no-tune and --profile-evals (default 33 1 1)")
    ap.add_argument("--profile-evals", type=int, default=0,
                    help="only run this many batched evaluations (for profiler passes)")
    ap.add_argument("--serve-full", action="store_true",
                    help="16 requests per rate over 0.25..8 req/s (long)")
    ap.add_argument("--no-cfg4", action="store_true")
    ap.add_argument("--no-std", action="store_true")
    ap.add_argument("--std-only", action="store_true",
                    help="only the standardized-form leg (for profiler passes)")
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
    if args.std_only:
        if args.profile_evals:
            # a fixed number of standardized-form evaluations and nothing else
            import numpy as np
            dss = synth.cfg2()
            gs = api.StdDataset(dss)
            th = synth.injected_theta(dss, 203)
            rng = np.random.default_rng(204)
            th = np.clip(th + rng.uniform(-0.2, 0.2, (args.chains, th.size)), dss["prior_lo"], dss["prior_hi"])
            Xs = np.concatenate([th, rng.standard_normal((args.chains, gs.d - th.shape[1]))], axis=1)
            xs = torch.tensor(Xs, device="cuda")
            for _ in range(args.profile_evals):
                gs.ptafs_std_logp_grad(xs)
            torch.cuda.synchronize()
            print(json.dumps({"std_profile_evals": args.profile_evals, "chains": args.chains}))
            return
        out = {"std_form": std_bench(n_chains=args.chains, n_leapfrog=args.leapfrog,
                                     steps=args.steps, warmup=args.warmup)}
        out["std_form_cw"] = std_bench(n_chains=args.chains, n_leapfrog=args.leapfrog,
                                       steps=args.steps, warmup=args.warmup, cw=True)
        out["std_form_split"] = std_bench(n_chains=args.chains, n_leapfrog=args.leapfrog,
                                          steps=args.steps, warmup=args.warmup, split=True)
        print(json.dumps(out))
        return
    ds = synth.cfg2()
    C, L = args.chains, args.leapfrog
    th = synth.injected_theta(ds, 203)
    X0 = synth.random_points(ds, C, 204, theta=th, theta_jitter=0.2)
    g = api.Dataset(ds)
    x = torch.tensor(X0, device="cuda")
    if args.profile_evals:
        # a fixed number of evaluations at the benchmark's launch configuration
        # and nothing else, for counter passes of a profiler
        g.ptafs_set_tuning(*(args.tuning or (33, 1, 1)))
        for _ in range(args.profile_evals):
            g.ptafs_logp_grad(x)
        torch.cuda.synchronize()
        print(json.dumps({"profile_evals": args.profile_evals, "chains": C,
                          "tuning": g.ptafs_get_tuning()}))
        return
    if args.tuning:
        g.ptafs_set_tuning(*args.tuning)
    tuning = g.ptafs_get_tuning()
    tune_log = None
    if not args.no_tune:
        tuning, tune_log = autotune.tune(g, x)
        _log(f"autotuned {tuning}")

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
    _log(f"{args.steps} trajectories in {el:.3f} s")
    value = C * L * args.steps / el

    # per-stage timing of the evaluation (HIP events on the launch stream)
    stages = g.ptafs_profile_stages(x, reps=20, stream=stream)
    eval_ms = sum(stages.values())
    flops, per_toa = toa_pass_flops(ds, C)
    achieved = flops / (stages["toa"] * 1e-3) / 1e12
    plain = None
    if not args.no_plain:
        # the plain form at its own best chunking (its launches are per pulsar)
        best = None
        for tpc in (2, 4, 8, 16):
            g.ptafs_set_tuning(tpc, 1, 0)
            ps = g.ptafs_profile_stages(x, reps=2, plain=True, stream=stream)
            if best is None or sum(ps.values()) < sum(best[1].values()):
                best = (tpc, ps)
        g.ptafs_set_tuning(*tuning)
        tpc, ps = best
        # the same algorithmic flops as the batched pass, on the vector unit:
        # against the measured FP64 vector-FMA peak (microbench/peaks)
        plain_tf = flops / (ps["toa"] * 1e-3) / 1e12
        plain = dict(value=C / (sum(ps.values()) * 1e-3), unit="grad evals/s",
                     ms_per_eval=round(sum(ps.values()), 4),
                     toa_ms=round(ps["toa"], 4), tiles_per_chunk=tpc,
                     toa_tflops=plain_tf, valu_peak_tflops=VALU_PEAK_TFLOPS,
                     valu_frac=plain_tf / VALU_PEAK_TFLOPS)
    _log("stages and plain form done")
    cpu = None if args.no_cpu else cpu_baseline(ds, min_seconds=args.cpu_seconds)
    if cpu is not None:
        # config 1 beside it (3 psr x 500 TOA): a second point of the oracle's rate
        cpu["config1"] = cpu_baseline(synth.cfg1(), min_seconds=3.0, label="3 psr / 1500 TOA (config 1)")
    _log("cpu baseline done")
    std_form = std_cw = std_split = None
    if not args.no_std:
        std_form = std_bench(n_chains=C, n_leapfrog=L, steps=args.steps, warmup=args.warmup)
        _log(f"standardized form: {std_form['value']:.0f} grad evals/s, stages {std_form['stages_ms']}")
        std_cw = std_bench(n_chains=C, n_leapfrog=L, steps=args.steps, warmup=args.warmup, cw=True)
        _log(f"standardized form with CW: {std_cw['value']:.0f} grad evals/s, stages {std_cw['stages_ms']}")
        std_split = std_bench(n_chains=C, n_leapfrog=L, steps=args.steps, warmup=args.warmup, split=True)
        _log(f"standardized form, split coefficients: {std_split['value']:.0f} grad evals/s, "
             f"stages {std_split['stages_ms']}")
    cfg4 = None
    if not args.no_cfg4:
        cfg4 = cfg4_bench()
        _log(f"config 4: batched {cfg4['batched_graph_evals_per_s']:.0f} vs plain "
             f"{cfg4['plain_evals_per_s']:.0f} grad evals/s")
    serving = None
    if not args.no_serve:
        # config 5: 500 trajectories x 16 chains per request
        if args.serve_full:
            serving = serving_bench(500, (0.25, 0.5, 1, 2, 4, 8), 16)
        else:
            serving = serving_bench(500, (0.25, 1, 4), 8)

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
            "traffic": measured_traffic(tuning),
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
        "std_form": std_form,
        "std_form_cw": std_cw,
        "std_form_split": std_split,
        "cfg4": cfg4,
        "serving": serving,
    }
    if tune_log is not None:
        out["autotune"] = tune_log
    print(json.dumps(out))
    g.close()


if __name__ == "__main__":
    main()
