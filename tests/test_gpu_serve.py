"""Serving (continuous batching of independent data sets on one GPU):
results do not depend on the mix, admission respects the memory budget, and
requests that can never fit are rejected."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_06834_amd import api, serve
    return api, serve


def request(i):
    """Small requests of different shapes (some with CW, some without DM)."""
    rng = np.random.default_rng(600 + i)
    n = int(rng.integers(2, 7))
    counts = rng.integers(20, 120, n)
    k = int(rng.integers(2, 7))
    cw = bool(i % 2)
    ds = synth.make_array(700 + i, n, counts, 9 * synth.YEAR_S, backends_per_psr=rng.integers(1, 3, n),
                          nu_range=(0.4e9, 2e9), nf_rn=k, nf_gw=max(1, k - 1), nf_dm=(k if i % 3 else 0),
                          has_cw=cw)
    th = synth.injected_theta(ds, 800 + i, rn=(-14.0, 3.5), dm=(-14.0, 3.5),
                              cw=(0.3, 1.0, 9.0, -8.0, 1.0, 0.5, 0.7, -14.0) if cw else None)
    x0 = synth.random_points(ds, 8, 900 + i, theta=th, theta_jitter=0.05)
    return ds, x0


def run_requests(serve, reqs, seeds=None, **kw):
    srv = serve.Server(**kw)
    seeds = seeds if seeds is not None else [31 + j for j in range(len(reqs))]
    ids = [srv.submit(ds, x0=x0, n_traj=7, n_leapfrog=4, eps=0.01, seed=s, keep="all")
           for s, (ds, x0) in zip(seeds, reqs)]
    out = [srv.wait(i, timeout=300) for i in ids]
    stats = (srv.max_used, srv.max_active)
    srv.close()
    return out, stats


def test_alone_equals_mix(mods):
    api, serve = mods
    reqs = [request(i) for i in range(6)]
    alone = []
    for j, r in enumerate(reqs):
        o, _ = run_requests(serve, [r], seeds=[31 + j], budget_bytes=1 << 34, max_slots=1, quantum=3)
        alone.append(o[0])
    mix, (used, act) = run_requests(serve, reqs, budget_bytes=1 << 34, max_slots=8, quantum=3)
    assert act > 1
    for a, m in zip(alone, mix):
        for key in ("samples", "logp", "n_accept", "n_invalid", "x"):
            np.testing.assert_array_equal(a[key], m[key])


def test_server_equals_direct_hmc(mods):
    """Quanta of trajectories give the same chain as one uninterrupted run at
    the TOA-pass tuning the server picked for the request."""
    api, serve = mods
    ds, x0 = request(7)
    (res,), _ = run_requests(serve, [(ds, x0)], budget_bytes=1 << 34, max_slots=2, quantum=2)
    assert len(res["tuning"]) == 3
    g = api.Dataset(ds)
    g.ptafs_set_tuning(*res["tuning"])
    x = torch.tensor(x0, device="cuda")
    lp, gr, _ = g.ptafs_logp_grad(x)
    acc = torch.zeros(x.shape[0], dtype=torch.int64, device="cuda")
    smp = torch.empty((7, x.shape[0], g.d), dtype=torch.float64, device="cuda")
    g.ptafs_hmc_run(x, lp, gr, acc, n_traj=7, n_leapfrog=4, eps=0.01, seed=31, traj0=0, samples=smp)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(res["samples"], smp.cpu().numpy())
    np.testing.assert_array_equal(res["n_accept"], acc.cpu().numpy())
    g.close()


def test_admission_by_footprint(mods):
    api, serve = mods
    reqs = [request(i) for i in range(6)]
    probe = serve.Server(budget_bytes=1 << 40, max_slots=1)
    fps = sorted(probe.footprint(ds, x0.shape[0]) for ds, x0 in reqs)
    probe.close()
    budget = fps[-1] + fps[-2]
    out, (used, act) = run_requests(serve, reqs, budget_bytes=budget, max_slots=8, quantum=3)
    assert used <= budget
    assert act >= 2
    assert all(o["t_admit"] >= o["t_arrival"] for o in out)


def test_rejects_what_never_fits(mods):
    api, serve = mods
    ds, x0 = request(0)
    srv = serve.Server(budget_bytes=1 << 20, max_slots=2)
    with pytest.raises(serve.Rejected):
        srv.submit(ds, x0=x0, n_traj=2, eps=0.01, seed=1)
    bad = dict(ds)
    bad["toa_offsets"] = np.array(ds["toa_offsets"])[::-1].copy()
    with pytest.raises(serve.Rejected):
        srv.submit(bad, x0=x0, n_traj=2, eps=0.01, seed=1)
    srv.close()


def test_estimate_matches_created_layout(mods):
    api, serve = mods
    ds, x0 = request(3)
    est = api.ptafs_estimate(ds, 24)
    g = api.Dataset(ds)
    lay = g.ptafs_layout(24)
    for f in ("d", "n_theta", "off_u", "off_z", "off_zdm", "dataset_bytes", "workspace_bytes",
              "hmc_bytes"):
        assert getattr(est, f) == getattr(lay, f), f
    g.close()


def test_cancel_mid_flight_frees_the_request(mods):
    """A request cancelled after its first quantum stops at the next quantum
    boundary, gives back its budget and device state, and the request beside
    it finishes with the result it has alone."""
    import time
    api, serve = mods
    (dsa, xa), (dsb, xb) = request(0), request(1)
    alone, _ = run_requests(serve, [(dsb, xb)], seeds=[77], budget_bytes=1 << 34, max_slots=1, quantum=3)
    srv = serve.Server(budget_bytes=1 << 34, max_slots=8, quantum=3)
    try:
        ra = srv.submit(dsa, x0=xa, n_traj=3000, n_leapfrog=4, eps=0.01, seed=31, keep="all")
        rb = srv.submit(dsb, x0=xb, n_traj=7, n_leapfrog=4, eps=0.01, seed=77, keep="all")
        t_end = time.perf_counter() + 120
        while srv._reqs[ra].done_traj < 3:
            assert time.perf_counter() < t_end, "first quantum of the long request never finished"
            time.sleep(0.01)
        assert srv.cancel(ra)
        with pytest.raises(serve.Cancelled):
            srv.wait(ra, timeout=120)
        got = srv.wait(rb, timeout=300)
        assert 3 <= srv._reqs[ra].done_traj < 3000
        assert srv._reqs[ra].ds is None and srv._reqs[ra].smp is None
        assert srv._used == 0
        assert not srv.cancel(rb)          # already finished
        for key in ("samples", "logp", "n_accept", "n_invalid", "x"):
            np.testing.assert_array_equal(alone[0][key], got[key])
    finally:
        srv.close()


def test_cancel_queued_request(mods):
    """A request cancelled while it waits for a slot is never admitted; the
    one ahead of it completes."""
    api, serve = mods
    (dsa, xa), (dsb, xb) = request(2), request(3)
    srv = serve.Server(budget_bytes=1 << 34, max_slots=1, quantum=3)
    try:
        ra = srv.submit(dsa, x0=xa, n_traj=30, n_leapfrog=4, eps=0.01, seed=31, keep="all")
        rb = srv.submit(dsb, x0=xb, n_traj=7, n_leapfrog=4, eps=0.01, seed=32, keep="all")
        assert srv.cancel(rb)
        with pytest.raises(serve.Cancelled):
            srv.poll(rb)
        got = srv.wait(ra, timeout=300)
        assert got["samples"].shape[0] == 30
        assert srv._reqs[rb].ds is None and np.isnan(srv._reqs[rb].t_admit)
        assert srv._used == 0
    finally:
        srv.close()
