"""GPU parity of the standardized form (ptafs_std_*, through the C ABI)
against the oracle of oracle/std.py: the CURN standardizing transform on
the Gram form with the timing model marginalised (Sec. IV.B), tempered
likelihoods (App. B) and free spectra (Sec. IV.A).

Bar: log p to 1e-9 relative; per gradient element
|g - g*| <= 1e-7 max(|g*|, S_j) + 10 R_j:
* S_j, for the coefficients, is the oracle's magnitude companion of the
  adjoint (oracle/std.py z_scale, absolute values of every term down to the
  per-TOA sums); for the hyper-parameters, whose autograd gradient has no
  per-term companion, it is 1e-2 of the largest |g*| of that block;
* R_j is the oracle's own rounding sensitivity (oracle/std.py
  rounding_sensitivity): how far g* moves when its per-TOA Gram sums carry
  rounding of their size.  The timing-model projection cancels inside those
  sums, and two FP64 evaluations of them cannot agree more closely;
statuses identical; on the elements that dominate their sums (|g*| >=
S_j/100 and |g*| >= 1e3 R_j) the bar is 1e-7 |g*| with no floor."""
import numpy as np
import pytest

import synth
from oracle import std

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_06834_amd import api as a
    return a


def free_box(ds):
    n, kr, kg, kd = ds["n_psr"], ds["nf_rn"], ds["nf_gw"], ds["nf_dm"]
    m = kg + n * kr + n * kd
    return np.full(m, -20.0), np.full(m, -5.0)


def general_tm(ds):
    t = ds["t"] / ds["tspan"]
    yr = 2 * np.pi * ds["t"] / synth.YEAR_S
    return np.stack([np.ones_like(t), t, t * t, np.sin(yr), np.cos(yr), 2.0 * t], axis=1)


# a CW well inside its box: it does not coalesce within twice a 16-yr span
THETA_CW = np.array([0.3, 1.0, 8.7, -8.2, 0.5, 0.6, 0.9, -14.0])


def make(seed, counts, nf, free=False, tm=False, span=9.0, cw=None):
    """cw: None, or (K_D, T_D / T) of a deterministic CW in its own basis."""
    ds = synth.make_array(seed, len(counts), list(counts), span * synth.YEAR_S,
                          backends_per_psr=[1 + i % 3 for i in range(len(counts))],
                          nu_range=(0.4e9, 2.0e9), nf_rn=nf[0], nf_gw=nf[1], nf_dm=nf[2],
                          has_cw=cw is not None)
    if cw is not None:
        ds["cw_nf"] = int(cw[0])
        ds["cw_tspan"] = float(cw[1]) * ds["tspan"]
    if free:
        ds["spectrum"] = "free"
        lo, hi = free_box(ds)
        if cw is not None:
            lo = np.concatenate([lo, ds["prior_lo"][-8:]])
            hi = np.concatenate([hi, ds["prior_hi"][-8:]])
        ds["prior_lo"], ds["prior_hi"] = lo, hi
    if tm:
        ds["tm"] = general_tm(ds)
    return ds


def points(ds, prep, n, seed, jitter=0.3):
    rng = np.random.default_rng(seed)
    lay = prep.lay
    cw = THETA_CW if lay.has_cw else None
    if prep.free:
        th = rng.uniform(-15.5, -12.5, (n, lay.n_theta))
        if lay.has_cw:
            th[:, lay.cw:] = np.clip(cw + rng.uniform(-jitter, jitter, (n, 8)),
                                     ds["prior_lo"][lay.cw:], ds["prior_hi"][lay.cw:])
    else:
        th0 = synth.injected_theta(ds, seed, rn=(-14.0, 3.5), dm=(-14.0, 3.5), cw=cw)
        th = np.clip(th0 + rng.uniform(-jitter, jitter, (n, th0.size)), ds["prior_lo"], ds["prior_hi"])
    return np.concatenate([th, rng.standard_normal((n, lay.d - lay.n_theta))], axis=1)


def run(api, ds, X, beta=None):
    g = api.StdDataset(ds)
    x = torch.tensor(X, device="cuda")
    b = None if beta is None else torch.tensor(np.asarray(beta, np.float64), device="cuda")
    lp, gr, st = g.ptafs_std_logp_grad(x, beta=b)
    torch.cuda.synchronize()
    out = lp.cpu().numpy(), gr.cpu().numpy(), st.cpu().numpy()
    g.close()
    return out


def check(prep, X, got, beta=None, ref=None, draws=1, strict=True):
    if ref is None:
        ref = std.logp_grad(prep, X, beta=beta)
    lp, gr, st = got
    np.testing.assert_array_equal(st, ref["status"])
    ok = ref["status"] == 0
    assert np.all(lp[~ok] == -np.inf) and np.all(gr[~ok] == 0.0)
    if not ok.any():
        return ref
    rel = np.abs(lp[ok] - ref["logp"][ok]) / np.abs(ref["logp"][ok])
    assert rel.max() <= 1e-9, rel.max()
    lay = prep.lay
    g_ref, g = ref["grad"][ok], gr[ok]
    betas = np.ones(X.shape[0]) if beta is None else np.broadcast_to(np.asarray(beta, np.float64), (X.shape[0],))
    Sc = np.zeros_like(g_ref)
    blocks = [(0, lay.cw), (lay.cw, lay.cw + 8)] if lay.has_cw else [(0, lay.n_theta)]
    for b0, b1 in blocks:
        if b1 > b0:
            Sc[:, b0:b1] = 1e-2 * np.abs(g_ref[:, b0:b1]).max(axis=1, keepdims=True)
    for i, c in enumerate(np.nonzero(ok)[0]):
        Sc[i, lay.z:] = std.z_scale(prep, X[c], float(betas[c])).reshape(-1)
    R = std.rounding_sensitivity(prep, X[ok], betas[ok], draws=draws)
    err = np.abs(g - g_ref)
    tol = 1e-7 * np.maximum(np.abs(g_ref), Sc) + 10.0 * R
    bad = err > tol
    nz = np.abs(g_ref) > 0
    dom = (np.abs(g_ref) >= Sc / 100.0) & (np.abs(g_ref) >= 1e3 * R) & nz
    print(f"[std margins] logp rel {rel.max():.2e}  grad max |g-g*|/|g*| "
          f"{np.max(err[nz] / np.abs(g_ref[nz])):.2e}  max |g-g*|/S {np.max(err / np.maximum(Sc, 1e-300)):.2e}  "
          f"max |g-g*|/R {np.max(err / np.maximum(R, 1e-300)):.2e}  "
          f"dominant ({int(dom.sum())}/{dom.size}) max {np.max(err[dom] / np.abs(g_ref[dom])):.2e}",
          flush=True)
    assert not bad.any(), (np.argwhere(bad)[:5], err[bad][:5], tol[bad][:5])
    if strict:
        # the 1e-7 bar without a floor on the elements that dominate their sums
        assert np.all(err[dom] <= 1e-7 * np.abs(g_ref[dom]))
    return ref


CASES = {
    # name: (counts, (nf_rn, nf_gw, nf_dm), free, tm)
    "small_hd_dm": ([30, 45, 60], (5, 3, 4), False, False),
    "no_dm": ([40, 50, 35], (6, 6, 0), False, False),
    "common_only": ([40, 50, 60], (0, 5, 0), False, False),
    "rn_longer_than_common": ([33, 47, 52, 61], (7, 2, 3), False, False),
    "general_tm": ([44, 38, 51], (4, 4, 2), False, True),
    "free_spectrum": ([35, 42, 48], (4, 3, 2), True, False),
    "single_toa_pulsar": ([1, 60, 45], (3, 3, 2), False, False),
    "one_pulsar": ([120], (8, 8, 4), False, False),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_std_parity(api, name):
    counts, nf, free, tm = CASES[name]
    ds = make(71, counts, nf, free, tm)
    prep = std.StdPrepared(ds)
    X = points(ds, prep, 9, 5)
    check(prep, X, run(api, ds, X))


@pytest.mark.parametrize("beta", [0.3, 1.0])
def test_std_tempered(api, beta):
    """App. B: per-chain temperatures (a ladder mixed in one call)."""
    ds = make(72, [40, 55, 33], (5, 4, 3))
    prep = std.StdPrepared(ds)
    X = points(ds, prep, 8, 6)
    betas = np.array([beta, 1.0, 0.5, 0.1, beta, 0.9, 0.02, 0.7])
    check(prep, X, run(api, ds, X, beta=betas), beta=betas)


@pytest.mark.parametrize("nf", [(8, 8, 0), (8, 8, 1), (16, 16, 0), (8, 8, 9), (30, 14, 30), (30, 30, 30)])
def test_std_coefficient_tiles(api, nf):
    """P = 2 (ka + kdm) across the 16-row tile boundaries of the per-pulsar
    factorisation: 32, 34, 64, 68, 120 (the largest), 120."""
    ds = make(73, [70, 90], nf, span=16.0)
    prep = std.StdPrepared(ds)
    X = points(ds, prep, 5, 7)
    check(prep, X, run(api, ds, X))


@pytest.mark.parametrize("n", [16, 17, 33, 65, 128])
def test_std_pulsar_counts(api, n):
    """N_p across the tile boundaries of the per-frequency factorisation."""
    ds = make(74 + n, [12 + (i % 5) for i in range(n)], (3, 2, 1))
    prep = std.StdPrepared(ds)
    X = points(ds, prep, 3, 8)
    check(prep, X, run(api, ds, X))


def test_std_chain_counts_and_determinism(api):
    ds = make(75, [30, 41, 52], (4, 3, 2))
    prep = std.StdPrepared(ds)
    X = points(ds, prep, 17, 9)
    a = run(api, ds, X)
    b = run(api, ds, X)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    sub = run(api, ds, X[[3]])
    for u, v in zip(a, sub):
        np.testing.assert_array_equal(u[[3]], v)
    check(prep, X, a)


def test_std_status_codes(api):
    ds = make(76, [30, 41, 52], (4, 3, 2))
    lay = std.StdPrepared(ds).lay
    ds["prior_lo"] = ds["prior_lo"].copy()
    amp = [lay.gw] + [lay.rn + 2 * I for I in range(3)] + [lay.dm + 2 * I for I in range(3)]
    ds["prior_lo"][amp] = -400.0
    prep = std.StdPrepared(ds)
    X = points(ds, prep, 6, 10)
    X[0, 1] = 99.0                   # gamma outside the box
    X[1, lay.z + 3] = np.nan         # non-finite coefficient
    X[2, amp] = -300.0               # every spectrum 0: phi_CURN not positive definite
    X[3, lay.dm] = -300.0            # one DM spectrum 0
    got = run(api, ds, X)
    ref = check(prep, X, got)
    assert list(ref["status"]) == [1, 4, 2, 2, 0, 0]


def test_std_coefficients(api):
    """a = a_hat + L z, the map back to the Fourier coefficients."""
    ds = make(77, [30, 41, 52], (4, 3, 2), tm=True)
    prep = std.StdPrepared(ds)
    X = points(ds, prep, 4, 11)
    g = api.StdDataset(ds)
    a = g.ptafs_std_coefficients(torch.tensor(X, device="cuda")).cpu().numpy()
    g.close()
    for c in range(4):
        ref = std.coefficients(prep, X[c])
        np.testing.assert_allclose(a[c], ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


CW_CASES = {
    # name: (counts, (nf_rn, nf_gw, nf_dm), free, tm, (K_D, T_D / T))
    "cw_hd_dm": ([30, 45, 60], (5, 3, 4), False, False, (20, 2.0)),
    "cw_general_tm": ([44, 38, 51], (4, 4, 2), False, True, (12, 2.0)),
    "cw_kd60": ([40, 55], (4, 4, 2), False, False, (60, 2.0)),
    "cw_kd64_short_span": ([35, 41, 29], (3, 3, 0), False, False, (64, 1.5)),
    "cw_free_spectrum": ([35, 42, 48], (4, 3, 2), True, False, (16, 2.0)),
    "cw_one_toa_pulsar": ([1, 60, 45], (3, 3, 2), False, False, (10, 2.0)),
}


@pytest.mark.parametrize("name", sorted(CW_CASES))
def test_std_cw_parity(api, name):
    """The deterministic CW in its own Fourier basis (Sec. IV.C): K_D up to
    the largest 64 (129 samples), extended spans, free spectra, a design
    matrix, a one-TOA pulsar."""
    counts, nf, free, tm, cw = CW_CASES[name]
    ds = make(81, counts, nf, free, tm, cw=cw)
    prep = std.StdPrepared(ds)
    X = points(ds, prep, 9, 15)
    check(prep, X, run(api, ds, X))


def test_std_cw_tempered_and_coefficients(api):
    ds = make(82, [40, 55, 33], (5, 4, 3), cw=(24, 2.0))
    prep = std.StdPrepared(ds)
    X = points(ds, prep, 8, 16)
    betas = np.array([0.3, 1.0, 0.5, 0.1, 1.0, 0.9, 0.02, 0.7])
    check(prep, X, run(api, ds, X, beta=betas), beta=betas)
    g = api.StdDataset(ds)
    a = g.ptafs_std_coefficients(torch.tensor(X[:3], device="cuda")).cpu().numpy()
    g.close()
    for c in range(3):
        ref = std.coefficients(prep, X[c])
        np.testing.assert_allclose(a[c], ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


def test_std_cw_status(api):
    """Status 3 when the CW coalesces before the last sample time of its
    basis; box violations keep status 1 (precedence 1, 4 in, 3, 2, 4 out)."""
    ds = make(83, [30, 41, 52], (4, 3, 2), cw=(16, 2.0))
    lay = std.StdPrepared(ds).lay
    ds["prior_hi"] = ds["prior_hi"].copy()
    ds["prior_hi"][lay.cw + 2], ds["prior_hi"][lay.cw + 3] = 10.5, -7.0
    prep = std.StdPrepared(ds)
    X = points(ds, prep, 5, 17)
    X[0, lay.cw + 2], X[0, lay.cw + 3] = 10.5, -7.0     # coalesces within T_D
    X[1, lay.cw + 2], X[1, lay.cw + 3] = 10.5, -7.0
    X[1, 1] = 99.0                                      # and outside the box
    X[2, lay.cw + 2], X[2, lay.cw + 3] = 10.5, -7.0
    X[2, lay.z + 4] = np.nan                            # and a non-finite input
    ref = check(prep, X, run(api, ds, X))
    assert list(ref["status"]) == [3, 1, 4, 0, 0]


def test_std_hmc_matches_oracle(api):
    """Fixed-step HMC on the standardized density: GPU trajectories against
    the oracle sampler (same Philox draws), tempered chains included."""
    from oracle import hmc
    ds = make(78, [25, 31, 28], (3, 3, 2))
    prep = std.StdPrepared(ds)
    lay = prep.lay
    X0 = points(ds, prep, 6, 12, jitter=0.1)
    betas = np.array([1.0, 1.0, 0.5, 1.0, 0.8, 1.0])
    im = np.ones(lay.d)
    im[:lay.n_theta] = 0.01
    n_traj, L, eps, seed = 4, 6, 0.8, 4321
    g = api.StdDataset(ds)
    x = torch.tensor(X0, device="cuda")
    bt = torch.tensor(betas, device="cuda")
    lp, gr, st = g.ptafs_std_logp_grad(x, beta=bt)
    acc = torch.zeros(6, dtype=torch.int64, device="cuda")
    smp = torch.empty((n_traj, 6, g.d), dtype=torch.float64, device="cuda")
    g.ptafs_std_hmc_run(x, lp, gr, acc, n_traj=n_traj, n_leapfrog=L, eps=eps, seed=seed, traj0=2,
                        inv_mass=torch.tensor(im, device="cuda"), beta=bt, samples=smp)
    torch.cuda.synchronize()
    S = smp.cpu().numpy()
    gacc = acc.cpu().numpy()
    g.close()

    def lpg(Xb):
        o = std.logp_grad(prep, Xb, beta=betas)
        return o["logp"], o["grad"]

    _, _, _, oacc, OS = hmc.run(lpg, X0, n_traj=n_traj, n_leapfrog=L, eps=eps, seed=seed, traj0=2,
                                inv_mass=im, keep_samples=True)
    np.testing.assert_array_equal(gacc, oacc)
    assert 0 < gacc.sum() < 6 * n_traj
    np.testing.assert_allclose(S, OS, rtol=1e-8, atol=1e-10)


def test_std_full_size_sampled(api):
    """The 67-pulsar, 250k-TOA workload (RN 30, DM 30, HD common 14) with
    64 chains; the oracle checks one chain of every 16.  At this size a few
    gradient entries of DM coefficients move by ~1e-8 when the Gram sums
    carry rounding (the timing-model projection leaves the data-dominated
    low-frequency coefficients ill-conditioned, and the red/DM coupling of
    the Gram passes that on); the floor R is the largest shift over four
    draws of both rounding models, and the unfloored 1e-7 |g*| check is
    reported, not asserted."""
    ds = synth.cfg2()
    prep = std.StdPrepared(ds)
    th = synth.injected_theta(ds, 203)
    rng = np.random.default_rng(204)
    th = np.clip(th + rng.uniform(-0.2, 0.2, (64, th.size)), ds["prior_lo"], ds["prior_hi"])
    X = np.concatenate([th, rng.standard_normal((64, prep.lay.d - prep.lay.n_theta))], axis=1)
    got = run(api, ds, X)
    idx = np.array([0, 21, 37, 63])
    assert np.all(got[2] == 0)
    check(prep, X[idx], tuple(v[idx] for v in got), draws=4, strict=False)


def test_std_cw_full_size_sampled(api):
    """The simulated CW array (100 pulsars x 180 TOA, RN 30 + HD common 14,
    CW in 60 frequencies on twice the span) at the paper's injection, 64
    chains; the oracle checks one chain of every 16."""
    ds = synth.cw_array()
    prep = std.StdPrepared(ds)
    th = synth.injected_theta(ds, 203, cw=synth.CW_PAPER)
    rng = np.random.default_rng(204)
    th = np.clip(th + rng.uniform(-0.2, 0.2, (64, th.size)), ds["prior_lo"], ds["prior_hi"])
    X = np.concatenate([th, rng.standard_normal((64, prep.lay.d - prep.lay.n_theta))], axis=1)
    got = run(api, ds, X)
    idx = np.array([0, 21, 37, 63])
    assert np.all(got[2] == 0)
    check(prep, X[idx], tuple(v[idx] for v in got), draws=2, strict=False)
