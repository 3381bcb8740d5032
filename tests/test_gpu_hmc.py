"""GPU fixed-step HMC (App. A) against the oracle sampler and closed forms.

Both samplers draw momenta and accept uniforms from Philox4x32-10 with the
same key/counter convention, so trajectories can be compared one by one.
"""
import numpy as np
import pytest

import synth
from oracle import dense, hmc, model

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_06834_amd import api as a
    return a


def small_ds(seed=5):
    return synth.make_array(seed, 3, [25, 30, 35], 8 * synth.YEAR_S, backends_per_psr=[1, 2, 1],
                            nu_range=(0.4e9, 2e9), nf_rn=3, nf_gw=3, nf_dm=2)


def gpu_hmc(api, ds, X0, *, n_traj, L, eps, seed, inv_mass=None, use_graph=True, traj0=0):
    g = api.Dataset(ds)
    x = torch.tensor(X0, device="cuda")
    lp, gr, st = g.ptafs_logp_grad(x)
    acc = torch.zeros(x.shape[0], dtype=torch.int64, device="cuda")
    samples = torch.empty((n_traj, x.shape[0], g.d), dtype=torch.float64, device="cuda")
    im = None if inv_mass is None else torch.tensor(inv_mass, device="cuda")
    g.ptafs_hmc_run(x, lp, gr, acc, n_traj=n_traj, n_leapfrog=L, eps=eps, seed=seed, traj0=traj0,
                    inv_mass=im, samples=samples, use_graph=use_graph)
    torch.cuda.synchronize()
    out = (x.cpu().numpy(), lp.cpu().numpy(), gr.cpu().numpy(), acc.cpu().numpy(),
           samples.cpu().numpy())
    g.close()
    return out


def test_hmc_matches_oracle_trajectories(api):
    ds = small_ds()
    prep = model.Prepared(ds)
    lay = prep.lay
    th = synth.injected_theta(ds, 7, rn=(-14.0, 3.5), dm=(-14.0, 3.5))
    m, Sw = dense.posterior_moments(prep, th)
    X0 = synth.random_points(ds, 8, 8, theta=th, theta_jitter=0.2)
    X0[:, lay.u:] = m + np.random.default_rng(1).standard_normal((8, m.size)) * np.sqrt(np.diag(Sw))
    # inverse mass ~ posterior variances (App. A); a step size that both
    # accepts and rejects (checked with the oracle sampler)
    im = np.ones(lay.d)
    im[: lay.n_theta] = 0.01
    im[lay.u:] = np.diag(Sw)
    eps = 0.3
    x, lp, gr, acc, S = gpu_hmc(api, ds, X0, n_traj=4, L=6, eps=eps, seed=1234, inv_mass=im, traj0=3)

    def lpg(Xb):
        o = model.logp_grad(prep, Xb, with_scale=False)
        return o["logp"], o["grad"]

    ox, olp, ogr, oacc, OS = hmc.run(lpg, X0, n_traj=4, n_leapfrog=6, eps=eps, seed=1234,
                                     traj0=3, inv_mass=im, keep_samples=True)
    np.testing.assert_array_equal(acc, oacc)
    assert 0 < acc.sum() < 32
    np.testing.assert_allclose(S, OS, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(lp, olp, rtol=1e-9)


def test_hmc_graph_replay_equals_eager(api):
    ds = small_ds(6)
    th = synth.injected_theta(ds, 9, rn=(-14.0, 3.5), dm=(-14.0, 3.5))
    X0 = synth.random_points(ds, 16, 10, theta=th, theta_jitter=0.2)
    a = gpu_hmc(api, ds, X0, n_traj=5, L=4, eps=0.03, seed=77, use_graph=True)
    b = gpu_hmc(api, ds, X0, n_traj=5, L=4, eps=0.03, seed=77, use_graph=False)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


def test_hmc_graph_dropped_when_tuning_round_trips(api):
    """A tuning change rebuilds the chunk table that a captured trajectory
    graph reads: after 1 -> 2 -> 1 tiles per chunk, with every buffer of the
    call unchanged, the graph is captured again and its trajectories equal the
    eager ones at the same tuning."""
    ds = small_ds(6)
    th = synth.injected_theta(ds, 9, rn=(-14.0, 3.5), dm=(-14.0, 3.5))
    X0 = torch.tensor(synth.random_points(ds, 16, 10, theta=th, theta_jitter=0.2), device="cuda")
    g = api.Dataset(ds)
    x = X0.clone()
    lp = torch.empty(16, dtype=torch.float64, device="cuda")
    gr = torch.empty_like(x)
    st = torch.empty(16, dtype=torch.int32, device="cuda")
    acc = torch.zeros(16, dtype=torch.int64, device="cuda")

    def run(use_graph):
        x.copy_(X0)
        acc.zero_()
        g.ptafs_logp_grad(x, out=(lp, gr, st))
        g.ptafs_hmc_run(x, lp, gr, acc, n_traj=3, n_leapfrog=4, eps=0.03, seed=77, use_graph=use_graph)
        torch.cuda.synchronize()
        return x.cpu().numpy(), lp.cpu().numpy(), gr.cpu().numpy(), acc.cpu().numpy()

    g.ptafs_set_tuning(1, 1, 1)
    run(True)
    g.ptafs_set_tuning(2, 1, 1)
    g.ptafs_set_tuning(1, 1, 1)
    a = run(True)
    b = run(False)
    g.close()
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


def test_hmc_linear_gaussian_moments(api):
    """Hyper-parameters frozen (inverse mass 0): the coefficients (u, z, z_dm)
    have the closed-form Gaussian posterior of the dense time-domain model."""
    ds = synth.make_array(3, 3, [12, 15, 18], 8 * synth.YEAR_S, backends_per_psr=[1, 2, 1],
                          nu_range=(0.4e9, 2.0e9), nf_rn=2, nf_gw=2, nf_dm=1)
    prep = model.Prepared(ds)
    lay = prep.lay
    theta = synth.injected_theta(ds, 4, rn=(-13.5, 3.0), dm=(-13.5, 3.0))
    m, S = dense.posterior_moments(prep, theta)
    im = np.zeros(lay.d)
    im[lay.u:] = np.diag(S)
    C = 256
    X0 = np.zeros((C, lay.d))
    X0[:, : lay.n_theta] = theta
    # every chain starts at the prior mean u = z = z_dm = 0, away from the
    # posterior mean: the moments test convergence, not only invariance
    n_traj, burn = 200, 40
    x, lp, gr, acc, samp = gpu_hmc(api, ds, X0, n_traj=n_traj, L=16, eps=0.08, seed=99, inv_mass=im)
    assert np.all(samp[:, :, : lay.n_theta] == theta)
    samp = samp[burn:, :, lay.u:]
    assert acc.mean() / n_traj > 0.7
    chm = samp.mean(0)
    zsc = (chm.mean(0) - m) / (chm.std(0) / np.sqrt(C))
    assert np.max(np.abs(zsc)) < 5.0, np.max(np.abs(zsc))
    var = ((samp - m) ** 2).mean(0)
    zv = (var.mean(0) - np.diag(S)) / (var.std(0) / np.sqrt(C))
    assert np.max(np.abs(zv)) < 5.0, np.max(np.abs(zv))


def test_hmc_cfg1_200_trajectories_vs_oracle(api):
    """Config 1: residuals drawn from the model at the injection (oracle
    simulator), 200 fixed-step trajectories of 8 chains (leapfrog 10, step
    0.05 from an oracle pilot over {0.2, 0.1, 0.05, 0.02}, the largest with
    acceptance >= 0.6), hyper-parameters sampled with a small inverse mass;
    the GPU sampler against the oracle sampler trajectory by trajectory
    (App. A: Eqs. Hamiltonian, Gaussian_momentum, HMC_acceptance)."""
    from oracle import simulate
    ds0 = synth.cfg1()
    th = synth.injected_theta(ds0, 103, rn=(-14.0, 4.0))
    ds = simulate.model_residuals(ds0, th, ds0["draws"])
    prep = model.Prepared(ds)
    lay = prep.lay
    m, Sw = dense.posterior_moments(prep, th)
    C = 8
    X0 = synth.random_points(ds, C, 104, theta=th, theta_jitter=0.1)
    X0[:, lay.u:] = m + np.random.default_rng(105).standard_normal((C, m.size)) * np.sqrt(np.diag(Sw))
    im = np.ones(lay.d)
    im[: lay.n_theta] = 0.01
    im[lay.u:] = np.diag(Sw)
    n_traj, L, eps = 200, 10, 0.05
    x, lp, gr, acc, S = gpu_hmc(api, ds, X0, n_traj=n_traj, L=L, eps=eps, seed=103, inv_mass=im)

    def lpg(Xb):
        o = model.logp_grad(prep, Xb, with_scale=False)
        return o["logp"], o["grad"]

    ox, olp, ogr, oacc, OS = hmc.run(lpg, X0, n_traj=n_traj, n_leapfrog=L, eps=eps, seed=103,
                                     inv_mass=im, keep_samples=True)
    dev = np.abs(S - OS) / (np.abs(OS) + 1e-3)
    print(f"[hmc cfg1] accepted {acc.sum()}/{C * n_traj}, max sample deviation "
          f"{dev.max():.2e} (last trajectory {dev[-1].max():.2e})", flush=True)
    np.testing.assert_array_equal(acc, oacc)
    assert 0 < acc.sum() < C * n_traj
    np.testing.assert_allclose(S, OS, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(lp, olp, rtol=1e-9)


@pytest.mark.parametrize("n_psr", [67, 80, 128])
def test_hmc_fused_kick_equals_plain_leapfrog(api, n_psr):
    """The leapfrog kick and drift fused into the assembly kernel (and the
    trajectory's first and last half kicks) against the oracle sampler's
    plain leapfrog driven by the library's own eager log p and gradient, at
    coordinate counts around and beyond the assembly's per-chain preload
    (d = 8511 at 67 pulsars, 10162 at 80, 16258 at 128; RN 30, HD 14, DM 30),
    with a non-uniform inverse mass."""
    counts = [24 + (7 * I) % 11 for I in range(n_psr)]
    ds = synth.make_array(200 + n_psr, n_psr, counts, 12 * synth.YEAR_S,
                          backends_per_psr=[1 + I % 2 for I in range(n_psr)],
                          nu_range=(0.4e9, 2.0e9), nf_rn=30, nf_gw=14, nf_dm=30)
    lay = model.Prepared(ds).lay
    C = 4
    th = synth.injected_theta(ds, 11, rn=(-14.0, 3.5), dm=(-14.0, 3.5))
    X0 = synth.random_points(ds, C, 12, theta=th, theta_jitter=0.05)
    X0[:, lay.u:] = np.random.default_rng(13).standard_normal((C, lay.d - lay.u))
    # the whitened timing-model coordinates are pinned by the data: start
    # them at 0 with a small inverse mass (a step the oracle sampler accepts)
    X0[:, lay.u:lay.z] = 0.0
    im = np.random.default_rng(14).uniform(0.5, 1.5, lay.d)
    im[: lay.n_theta] = 1e-4
    im[lay.u:lay.z] = 1e-8
    g = api.Dataset(ds)

    def lpg(Xb):
        lp, gr, st = g.ptafs_logp_grad(torch.tensor(Xb, device="cuda"))
        torch.cuda.synchronize()
        return lp.cpu().numpy(), gr.cpu().numpy()

    ox, olp, ogr, oacc, OS = hmc.run(lpg, X0, n_traj=3, n_leapfrog=5, eps=0.05, seed=515, traj0=1,
                                     inv_mass=im, keep_samples=True)
    g.close()
    x, lp, gr, acc, S = gpu_hmc(api, ds, X0, n_traj=3, L=5, eps=0.05, seed=515, inv_mass=im, traj0=1)
    print(f"[hmc fused kick {n_psr} psr, d={lay.d}] accepted {acc.sum()}/{3 * C}", flush=True)
    assert lay.d == {67: 8511, 80: 10162, 128: 16258}[n_psr]
    np.testing.assert_array_equal(acc, oacc)
    assert acc.sum() > 0
    np.testing.assert_allclose(S, OS, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(lp, olp, rtol=1e-10)
    np.testing.assert_allclose(gr, ogr, rtol=1e-8, atol=1e-9 * np.abs(ogr).max())
