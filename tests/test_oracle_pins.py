"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
own formula: they use closed forms, printed or hand-derived special values,
structurally different evaluations (dense time-domain Gaussian, Gram form),
finite differences and invariants.
"""
import os

import numpy as np
import pytest

import synth
from oracle import cw as ocw
from oracle import dense, model, philox

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _closed():
    out = {}
    for line in open(os.path.join(GOLD, "closed_forms.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def tiny(seed=7, counts=(15, 20, 25), nf_rn=3, nf_gw=2, nf_dm=2, cw=False, span_yr=8.0):
    n = len(counts)
    return synth.make_array(seed, n, list(counts), span_yr * synth.YEAR_S,
                            backends_per_psr=[2] * n, nu_range=(0.4e9, 2.0e9),
                            nf_rn=nf_rn, nf_gw=nf_gw, nf_dm=nf_dm, has_cw=cw)


def near_points(ds, n, seed, jitter=0.5):
    """Points with hyper-parameters near a plausible injection (so the
    log-density is O(100) and finite differences resolve the gradient)."""
    cw = [0.3, 1.0, 9.0, -8.0, 1.0, 0.4, 0.7, -13.5] if ds["has_cw"] else None
    th = synth.injected_theta(ds, seed, rn=(-14.0, 3.0), dm=(-14.0, 3.0), cw=cw)
    return synth.random_points(ds, n, seed + 1, theta=th, theta_jitter=jitter)


# --------------------------------------------------------------- P7, P6 --

def test_powerlaw_closed_form():
    """Eq. power_law (yr^3 reading): printed-units value and scalings."""
    cf = _closed()
    T = 10.0 * synth.YEAR_S
    rho1 = model.powerlaw(1.0 / T, -14.0, 4.0, T)
    assert np.sqrt(rho1) == pytest.approx(cf["sqrt_rho1_m14_g4_T10yr"], rel=2e-6)
    k = np.arange(1, 11)
    r = model.powerlaw(k / T, -14.0, 13.0 / 3.0, T)
    np.testing.assert_allclose(r / r[0], k ** (-13.0 / 3.0), rtol=1e-13)
    # rho scales with A^2
    assert model.powerlaw(1 / T, -13.0, 4.0, T) / rho1 == pytest.approx(100.0, rel=1e-13)


def test_hd_special_values():
    """Eq. HD: alpha(0+) = 1/2, alpha(pi) = 1/4, minimum -0.1519 at 82.48 deg,
    unit diagonal (alpha_II = 3/2*0 - 0 + 1/2 + 1/2)."""
    cf = _closed()

    def pair(theta):
        p = np.array([[0.0, 0.0, 1.0], [np.sin(theta), 0.0, np.cos(theta)]])
        return model.hd_matrix(p)

    G = pair(1e-9)
    assert G[0, 0] == 1.0 and G[1, 1] == 1.0
    assert G[0, 1] == pytest.approx(cf["hd_at_zero"], abs=1e-9)
    assert pair(np.pi)[0, 1] == pytest.approx(cf["hd_at_pi"], abs=1e-14)
    ang = np.radians(np.linspace(60, 100, 40001))
    vals = np.array([pair(a)[0, 1] for a in ang])
    i = np.argmin(vals)
    assert vals[i] == pytest.approx(cf["hd_min_value"], abs=2e-6)
    assert np.degrees(ang[i]) == pytest.approx(cf["hd_min_angle_deg"], abs=2e-3)
    # identical positions: beta = 0 -> alpha = 1/2 off the diagonal
    G2 = model.hd_matrix(np.array([[1.0, 0, 0], [1.0, 0, 0]]))
    assert G2[0, 1] == 0.5


# --------------------------------------------------------------- P2 -------

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_whitened_prior_identity(seed):
    """Eq. standardized_density (mu = 0, Sigma = phi of Eq. prior_cov):
    the a-prior plus the Jacobian equals the standard normal in z, for any
    hyper-parameters in the box (dense phi, no per-frequency factorisation)."""
    ds = tiny(seed=seed)
    prep = model.Prepared(ds)
    for x in synth.random_points(ds, 3, seed):
        lhs, rhs = dense.whitened_prior(prep, x)
        assert lhs == pytest.approx(rhs, rel=1e-10, abs=1e-8)


# --------------------------------------------------------------- P3 -------

@pytest.mark.parametrize("nf", [(3, 2, 2), (2, 3, 0), (2, 0, 1), (0, 2, 2)])
def test_dense_joint_identity(nf):
    """Eqs. likelihood + a_prior (+ broad Gaussian b prior): at any point the
    per-TOA oracle equals the dense time-domain marginal N(dt; h, C) times the
    conditional N(v; m, S) times |det dv/dw|, with C built across all pulsars
    from the dense prior covariance (HD coupling included)."""
    ds = tiny(seed=11, nf_rn=nf[0], nf_gw=nf[1], nf_dm=nf[2])
    prep = model.Prepared(ds)
    X = np.concatenate([synth.random_points(ds, 3, 5), near_points(ds, 3, 9)])
    out = model.logp_grad(prep, X)
    for c, x in enumerate(X):
        assert out["status"][c] == 0
        ref = dense.dense_joint(prep, x)
        assert out["logp"][c] == pytest.approx(ref, rel=1e-9, abs=1e-7 * out["logp_scale"][c])


def test_dense_joint_identity_cw():
    """Same identity with a deterministic delay h(theta) in the mean."""
    ds = tiny(seed=12, cw=True)
    prep = model.Prepared(ds)
    X = near_points(ds, 3, 4)
    out = model.logp_grad(prep, X)
    lay = prep.lay
    for c, x in enumerate(X):
        h = np.concatenate([ocw.delay(p["t"], p["pos"], x[lay.cw:lay.cw + 8], False)[0]
                            for p in prep.psr])
        ref = dense.dense_joint(prep, x, h=h)
        assert out["logp"][c] == pytest.approx(ref, rel=1e-9, abs=1e-7 * out["logp_scale"][c])


# --------------------------------------------------------------- P1, P8 ---

def test_zero_coefficients_closed_form():
    """z = z_dm = 0 gives a = 0: the likelihood reduces to the white-noise
    Gaussian of dt - M b alone (Eq. likelihood with F a = 0)."""
    ds = tiny(seed=13)
    prep = model.Prepared(ds)
    lay = prep.lay
    x = near_points(ds, 1, 3)[0]
    x[lay.z:] = 0.0
    lp = model.logp_grad(prep, x)["logp"][0]
    u = x[lay.u:lay.u + 3 * prep.n_psr].reshape(-1, 3)
    t = ds["t"]
    off = ds["toa_offsets"]
    chi = 0.0
    for I in range(prep.n_psr):
        tt = t[off[I]:off[I + 1]]
        tau = (tt - 0.5 * (tt.max() + tt.min())) / (0.5 * (tt.max() - tt.min()))
        bI = ds["sigma_b"] * u[I]
        r = ds["dt"][off[I]:off[I + 1]] - (bI[0] + bI[1] * tau + bI[2] * tau ** 2)
        be = ds["backend"][off[I]:off[I + 1]]
        N = (ds["efac"][be] * ds["sigma"][off[I]:off[I + 1]]) ** 2 + ds["equad"][be] ** 2
        chi += -0.5 * np.sum(r * r / N + np.log(2 * np.pi * N))
    rest = -0.5 * np.sum(x[lay.u:] ** 2) - 0.5 * (lay.d - lay.u) * np.log(2 * np.pi)
    rest += -np.sum(np.log(ds["prior_hi"] - ds["prior_lo"]))
    assert lp == pytest.approx(chi + rest, rel=1e-12)


def test_gram_form_equals_per_toa_form():
    """Eq. posterior_implemented (compressed form with precomputed F^T N^-1 F
    and F^T N^-1 dt, constants restored) equals the per-TOA likelihood."""
    ds = tiny(seed=14)
    prep = model.Prepared(ds)
    lay = prep.lay
    X = np.concatenate([synth.random_points(ds, 2, 3), near_points(ds, 2, 5)])
    out = model.logp_grad(prep, X)
    for c, x in enumerate(X):
        prior = -0.5 * np.sum(x[lay.u:] ** 2) - 0.5 * (lay.d - lay.u) * np.log(2 * np.pi) \
            - np.sum(np.log(ds["prior_hi"] - ds["prior_lo"]))
        ref = dense.gram_loglike(prep, x) + prior
        assert out["logp"][c] == pytest.approx(ref, rel=1e-9, abs=1e-9 * out["logp_scale"][c])


# --------------------------------------------------------------- P4 -------

def _fd(prep, x, i, h):
    xp, xm = x.copy(), x.copy()
    xp[i] += h
    xm[i] -= h
    return (model.logp_grad(prep, xp, False)["logp"][0] - model.logp_grad(prep, xm, False)["logp"][0]) / (2 * h)


@pytest.mark.parametrize("cw", [False, True])
def test_gradient_finite_differences(cw):
    """Central differences (h = 1e-6 relative, error estimated from h/2)
    against the hand-derived adjoint, on every coordinate."""
    ds = tiny(seed=21, cw=cw)
    prep = model.Prepared(ds)
    x = near_points(ds, 1, 17, jitter=0.3)[0]
    if cw:
        # a CW loud enough to matter, away from the box edges
        x[prep.lay.cw:prep.lay.cw + 8] = [0.3, 1.0, 9.0, -8.0, 1.0, 0.4, 0.7, -13.5]
    out = model.logp_grad(prep, x)
    g = out["grad"][0]
    assert out["status"][0] == 0
    for i in range(prep.lay.d):
        h = 1e-6 * max(1.0, abs(x[i]))
        f1 = _fd(prep, x, i, h)
        f2 = _fd(prep, x, i, h / 2)
        err = abs(f1 - f2) + 1e-9 * max(abs(g[i]), 1.0)
        assert abs(g[i] - f2) <= 50 * err + 1e-6 * abs(g[i]), (i, g[i], f1, f2)


def test_chol_backward_fd():
    """Cholesky adjoint: <phibar, dphi> equals the directional derivative of
    f(phi) = <A, chol(phi) Z> for random symmetric directions."""
    rng = np.random.default_rng(3)
    n = 6
    B = rng.standard_normal((n, n))
    phi = B @ B.T + n * np.eye(n)
    A = rng.standard_normal((n, 2))
    Z = rng.standard_normal((n, 2))
    L = np.linalg.cholesky(phi)
    pb = model.chol_backward(L, A @ Z.T)

    def f(p):
        return np.sum(A * (np.linalg.cholesky(p) @ Z))

    for _ in range(5):
        D = rng.standard_normal((n, n))
        D = D + D.T
        h = 1e-6
        fd = (f(phi + h * D) - f(phi - h * D)) / (2 * h)
        assert np.sum(pb * D) == pytest.approx(fd, rel=1e-7, abs=1e-9)


# --------------------------------------------------------------- P9 -------

CW0 = np.array([0.3, 1.0, 9.2, -7.8, 0.7, 0.4, 0.9, -13.0])


def test_cw_nonevolving_limit():
    """Eq. phase_evolve_Taylor: for y << 1 the phase advances as w0 t."""
    th = CW0.copy()
    th[2], th[3] = 8.5, -8.5                               # smallest y in the box
    t = np.linspace(0.0, 5 * synth.YEAR_S, 50)
    M = 10 ** th[2] * ocw.T_SUN
    w0 = np.pi * 10 ** th[3]
    y = 256 / 5 * M ** (5 / 3) * w0 ** (8 / 3) * t
    E = -np.expm1(5 / 8 * np.log1p(-y))
    dphi = E / (32 * (M * w0) ** (5 / 3))
    np.testing.assert_allclose(dphi, w0 * t, rtol=1e-5, atol=1e-12)
    assert y.max() < 1e-5


def test_cw_frequency_ode():
    """Eq. CW_evolve solves dw/dt = 96/5 M^(5/3) w^(11/3)."""
    th = CW0.copy()
    th[2], th[3] = 9.5, -7.5                               # largest y in the box
    M = 10 ** th[2] * ocw.T_SUN
    w0 = np.pi * 10 ** th[3]

    def w(t):
        return w0 * (1 - 256 / 5 * M ** (5 / 3) * w0 ** (8 / 3) * t) ** (-3 / 8)

    for t in np.linspace(1e7, 4.5e8, 7):
        h = 1e3
        dw = (w(t + h) - w(t - h)) / (2 * h)
        assert dw == pytest.approx(96 / 5 * M ** (5 / 3) * w(t) ** (11 / 3), rel=1e-6)
    assert ocw.max_y(th, 16 * synth.YEAR_S) < 0.06


def test_cw_symmetries():
    """h is linear in 10^log10h; psi -> psi + pi/2 and Phi0 -> Phi0 + pi/2
    flip its sign; psi -> psi + pi leaves it unchanged."""
    rng = np.random.default_rng(5)
    pos = rng.standard_normal(3)
    pos /= np.linalg.norm(pos)
    t = np.linspace(0, 10 * synth.YEAR_S, 200)
    h0, _ = ocw.delay(t, pos, CW0, False)

    def with_(i, v):
        th = CW0.copy()
        th[i] = v
        return ocw.delay(t, pos, th, False)[0]

    np.testing.assert_allclose(with_(7, CW0[7] + 1.0), 10.0 * h0, rtol=1e-12)
    np.testing.assert_allclose(with_(6, CW0[6] + np.pi / 2), -h0, rtol=1e-9, atol=1e-12 * np.abs(h0).max())
    np.testing.assert_allclose(with_(4, CW0[4] + np.pi / 2), -h0, rtol=1e-9, atol=1e-12 * np.abs(h0).max())
    np.testing.assert_allclose(with_(6, CW0[6] + np.pi), h0, rtol=1e-9, atol=1e-12 * np.abs(h0).max())


def test_cw_gradient_fd():
    """dh/dtheta of the waveform against central differences."""
    rng = np.random.default_rng(6)
    pos = rng.standard_normal(3)
    pos /= np.linalg.norm(pos)
    t = np.linspace(1e6, 12 * synth.YEAR_S, 40)
    for th in (CW0, np.array([-0.6, 4.0, 9.4, -7.6, 5.0, -0.2, 2.5, -12.0])):
        _, g = ocw.delay(t, pos, th, True)
        for i in range(8):
            hh = 1e-6 * max(1.0, abs(th[i]))
            tp, tm = th.copy(), th.copy()
            tp[i] += hh
            tm[i] -= hh
            fd = (ocw.delay(t, pos, tp, False)[0] - ocw.delay(t, pos, tm, False)[0]) / (2 * hh)
            np.testing.assert_allclose(g[:, i], fd, rtol=2e-5, atol=2e-6 * np.abs(fd).max() + 1e-30)


# --------------------------------------------------------------- P10 ------

def test_uncorrelated_limit_factorises():
    """With Gamma = I (CURN) the array density is the product of per-pulsar
    densities, each with the common process added to its own red noise."""
    ds = tiny(seed=31, nf_dm=0)
    prep = model.Prepared(ds)
    prep.Gamma = np.eye(prep.n_psr)
    x = near_points(ds, 1, 2)[0]
    lay = prep.lay
    total = model.logp_grad(prep, x)["logp"][0]
    parts = 0.0
    off = ds["toa_offsets"]
    K = prep.K
    for I in range(prep.n_psr):
        sub = dict(ds)
        sl = slice(off[I], off[I + 1])
        for key in ("t", "sigma", "nu", "backend", "dt"):
            sub[key] = ds[key][sl]
        sub["n_psr"] = 1
        sub["toa_offsets"] = np.array([0, off[I + 1] - off[I]])
        sub["psr_pos"] = ds["psr_pos"][I:I + 1]
        lo, hi = synth.theta_box(1, ds["nf_rn"], ds["nf_gw"], 0, False)
        sub["prior_lo"], sub["prior_hi"] = lo, hi
        sp = model.Prepared(sub)
        xs = np.concatenate([
            x[lay.gw:lay.gw + 2], x[lay.rn + 2 * I:lay.rn + 2 * I + 2],
            x[lay.u + 3 * I:lay.u + 3 * I + 3], x[lay.z + 2 * K * I:lay.z + 2 * K * (I + 1)]])
        parts += model.logp_grad(sp, xs)["logp"][0] + np.sum(np.log(hi - lo))
    # hyper-prior constants: each sub-problem carries its own box, the array once
    parts -= np.sum(np.log(ds["prior_hi"] - ds["prior_lo"]))
    assert total == pytest.approx(parts, rel=1e-11)


def test_pulsar_permutation():
    """Relabelling pulsars leaves the density of the coefficients a unchanged
    (Eq. prior_cov is covariant under relabelling).  With a = L z the same a
    is reached at z' = L'^-1 P L z, L' the factor of the permuted phi, and
    |z'| = |z|, so log p is unchanged; the u and z_dm gradients permute."""
    ds = tiny(seed=41)
    prep = model.Prepared(ds)
    lay = prep.lay
    x = near_points(ds, 1, 8)[0]
    perm = np.array([2, 0, 1])
    off = ds["toa_offsets"]
    ds2 = dict(ds)
    idx = np.concatenate([np.arange(off[p], off[p + 1]) for p in perm])
    for key in ("t", "sigma", "nu", "backend", "dt"):
        ds2[key] = ds[key][idx]
    cnt = np.diff(off)[perm]
    ds2["toa_offsets"] = np.concatenate([[0], np.cumsum(cnt)])
    ds2["psr_pos"] = ds["psr_pos"][perm]
    prep2 = model.Prepared(ds2)
    n, K = prep.n_psr, prep.K

    y = x.copy()
    for blk, w in ((lay.rn, 2), (lay.dm, 2), (lay.u, 3)):
        y[blk:blk + w * n] = x[blk:blk + w * n].reshape(n, w)[perm].ravel()
    y[lay.zdm:] = x[lay.zdm:].reshape(n, -1)[perm].ravel()
    gw, rn, dm, cw, u, z, zdm = prep.split(x[None, :])
    rho, kap, _ = prep.spectra(gw, rn, dm, 1)
    z2 = np.zeros((n, 2 * K))
    Pm = np.eye(n)[perm]
    for k in range(K):
        phi = rho[0, k] * prep.Gamma + np.diag(kap[0, :, k])
        L = np.linalg.cholesky(phi)
        L2 = np.linalg.cholesky(Pm @ phi @ Pm.T)
        for c in range(2):
            z2[:, 2 * k + c] = np.linalg.solve(L2, Pm @ (L @ z[0, :, 2 * k + c]))
    y[lay.z:lay.z + 2 * K * n] = z2.ravel()
    assert np.sum(z2 ** 2) == pytest.approx(np.sum(z ** 2), rel=1e-12)

    a = model.logp_grad(prep, x)
    b = model.logp_grad(prep2, y)
    assert b["logp"][0] == pytest.approx(a["logp"][0], rel=1e-11)
    gu = a["grad"][0][lay.u:lay.u + 3 * n].reshape(n, 3)[perm].ravel()
    np.testing.assert_allclose(b["grad"][0][lay.u:lay.u + 3 * n], gu, rtol=1e-7,
                               atol=1e-9 * np.abs(a["scale"][0][lay.u:lay.z]).max())
    gd = a["grad"][0][lay.zdm:].reshape(n, -1)[perm].ravel()
    np.testing.assert_allclose(b["grad"][0][lay.zdm:], gd, rtol=1e-7,
                               atol=1e-9 * np.abs(a["scale"][0][lay.zdm:]).max())


def test_prior_is_theta_independent_in_z():
    """The whitened prior contributes -z (and -u, -z_dm) to the gradient and
    nothing to the hyper-parameters: with the likelihood switched off
    (infinite white noise) the theta-gradient vanishes."""
    ds = tiny(seed=51)
    ds = dict(ds)
    ds["equad"] = np.full_like(ds["equad"], 1e150)
    prep = model.Prepared(ds)
    lay = prep.lay
    x = synth.random_points(ds, 1, 3)[0]
    out = model.logp_grad(prep, x)
    g = out["grad"][0]
    np.testing.assert_allclose(g[: lay.n_theta], 0.0, atol=1e-200)
    np.testing.assert_allclose(g[lay.u:], -x[lay.u:], rtol=1e-12)


# --------------------------------------------------------------- status ---

def test_status_codes():
    ds = tiny(seed=61, cw=True)
    prep = model.Prepared(ds)
    lay = prep.lay
    X = near_points(ds, 4, 3)
    X[:, lay.cw:lay.cw + 8] = CW0
    X[0, 0] = -25.0                                         # outside the box
    X[1, lay.z] = np.nan                                     # non-finite input
    X[2, lay.cw + 2], X[2, lay.cw + 3] = 9.5, -7.5          # stays inside y < 1
    out = model.logp_grad(prep, X)
    assert list(out["status"]) == [1, 4, 0, 0]
    assert out["logp"][0] == -np.inf and np.all(out["grad"][0] == 0)
    assert np.isfinite(out["logp"][2:]).all()


# --------------------------------------------------------------- RNG ------

def test_philox_known_answers():
    for line in open(os.path.join(GOLD, "philox_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(s, 16) for s in line.split()]
        assert philox.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])
        got = philox.philox_vec([v[0]], [v[1]], [v[2]], [v[3]], v[4], v[5])
        assert tuple(int(g[0]) for g in got) == tuple(v[6:10])


def test_momentum_normals_distribution():
    n = philox.momentum_normals(1234, 3, 7, 200001)
    assert abs(n.mean()) < 0.01 and abs(n.var() - 1.0) < 0.01
    assert np.all(np.isfinite(n))


# ------------------------------------------------- basis and DM weight -----

def _golden_basis():
    rows, chi2 = [], None
    for line in open(os.path.join(GOLD, "basis_rows.txt")):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "row":
            v = [float(s) for s in f[1:]]
            rows.append((int(v[0]), np.array(v[1:5]), np.array(v[5:9]), np.array(v[9:12])))
        elif f[0] == "chi2_forward":
            chi2 = float(f[1])
    return rows, chi2


def _basis_ds(dt):
    """One pulsar, TOAs at T/8, T/4, 3T/8 (the hand-derived data set of
    tests/golden/basis_rows.txt)."""
    T = 10.0 * synth.YEAR_S
    lo, hi = synth.theta_box(1, 2, 0, 2, False)
    return dict(n_psr=1, toa_offsets=np.array([0, 3]), t=np.array([T / 8, T / 4, 3 * T / 8]),
                dt=np.asarray(dt, np.float64), sigma=np.full(3, 1e-6), nu=np.full(3, 1e9),
                backend=np.zeros(3, np.int32), n_backend=1, efac=np.array([1.0]),
                equad=np.array([0.0]), psr_pos=np.array([[0.0, 0.0, 1.0]]), tspan=T,
                nf_rn=2, nf_gw=0, nf_dm=2, dm_scale=1.4e9 ** 2, sigma_b=1e-5, has_cw=0,
                prior_lo=lo, prior_hi=hi)


def test_basis_rows_golden():
    """Sec. III.C (Eqs. Fourier_series, RN=Fa, F_DM) and Eq. TM=Me: the basis
    rows the likelihood uses at three hand-placed TOAs, read off the gradient
    at a = 0 with a one-TOA residual (derivation in the golden file).  A
    cos-before-sin column order, a k = 0..K-1 grid, a shifted time origin,
    a wrong DM weight or a wrong tau normalisation all fail here."""
    rows, _ = _golden_basis()
    rho1 = _closed()["sqrt_rho1_m14_g4_T10yr"]
    for j, gz, gzdm, gu in rows:
        dt = np.zeros(3)
        dt[j] = 1e-12                                        # = N_j
        ds = _basis_ds(dt)
        prep = model.Prepared(ds)
        lay = prep.lay
        x = np.zeros(lay.d)
        x[lay.rn:lay.rn + 2] = [-14.0, 4.0]
        x[lay.dm:lay.dm + 2] = [-14.0, 4.0]
        g = model.logp_grad(prep, x)["grad"][0]
        np.testing.assert_allclose(g[lay.z:lay.z + 4] / rho1, gz, rtol=2e-6, atol=1e-12)
        np.testing.assert_allclose(g[lay.zdm:lay.zdm + 4] / rho1, gzdm, rtol=2e-6, atol=1e-12)
        np.testing.assert_allclose(g[lay.u:lay.u + 3] / ds["sigma_b"], gu, rtol=1e-12, atol=1e-12)


def test_basis_forward_golden():
    """The forward residual with a single nonzero coefficient a_(2,sin) =
    1e-6 s: chi^2 = 2 by hand (golden file); log p is then the a = 0 normal
    constants plus -chi^2/2."""
    _, chi2 = _golden_basis()
    ds = _basis_ds(np.zeros(3))
    prep = model.Prepared(ds)
    lay = prep.lay
    x = np.zeros(lay.d)
    x[lay.rn:lay.rn + 2] = [-14.0, 4.0]
    x[lay.dm:lay.dm + 2] = [-14.0, 4.0]
    sq2 = _closed()["sqrt_rho1_m14_g4_T10yr"] / 4.0          # sqrt(kappa_2) = sqrt(kappa_1)/4
    x[lay.z + 2] = 1e-6 / sq2
    lp = model.logp_grad(prep, x)["logp"][0]
    const = -0.5 * 3 * np.log(2 * np.pi * 1e-12)
    prior = -0.5 * x[lay.z + 2] ** 2 - 0.5 * (lay.d - lay.u) * np.log(2 * np.pi) \
        - np.sum(np.log(ds["prior_hi"] - ds["prior_lo"]))
    assert lp - const - prior == pytest.approx(-0.5 * chi2, rel=5e-6)


# ------------------------------------------------- CW antenna pattern ------

def test_cw_antenna_identity():
    """Sec. III.D (Earth term): with m, n and Omega = -s_hat orthonormal,
    F+^2 + Fx^2 = ((m.p)^2 + (n.p)^2)^2 / (4 (1 + Omega.p)^2)
    = (1 - (Omega.p)^2)^2 / (4 (1 + Omega.p)^2) = (1 + s_hat.p)^2 / 4.
    A sign error in the 1 + Omega.p denominator (or in Omega) breaks it; the
    pattern vanishes for a pulsar at p = Omega."""
    rng = np.random.default_rng(17)
    for _ in range(200):
        p = rng.standard_normal(3)
        p /= np.linalg.norm(p)
        cth, phi = rng.uniform(-1, 1), rng.uniform(0, 2 * np.pi)
        sth = np.sqrt(1 - cth * cth)
        s = np.array([sth * np.cos(phi), sth * np.sin(phi), cth])
        fp, fx, _ = ocw.antenna(p, cth, phi)
        assert fp * fp + fx * fx == pytest.approx(0.25 * (1.0 + s @ p) ** 2, rel=1e-11, abs=1e-15)
        fp0, fx0, _ = ocw.antenna(-s, cth, phi)                # pulsar at p = Omega
        assert abs(fp0) < 1e-15 and abs(fx0) < 1e-15


def test_cw_face_on_amplitude():
    """Face-on source (cos iota = 1): the two polarisations are in quadrature
    with equal amplitude 2 alpha, so as the reference phase Phi0 varies the
    delay at t = 0 is a sinusoid of amplitude 2 alpha sqrt(F+^2 + Fx^2) =
    alpha (1 + s_hat.p), with alpha = h / (2 w0) at t = 0 (w(0) = w0)."""
    rng = np.random.default_rng(23)
    p = rng.standard_normal(3)
    p /= np.linalg.norm(p)
    th = np.array([0.2, 2.0, 9.0, -8.0, 0.0, 1.0, 0.4, -13.0])
    sth = np.sqrt(1 - th[0] ** 2)
    s = np.array([sth * np.cos(th[1]), sth * np.sin(th[1]), th[0]])
    w0 = np.pi * 10 ** th[3]
    amp = 10 ** th[7] / (2 * w0) * (1 + s @ p)
    def h0(ph):
        th[4] = ph
        return ocw.delay(np.array([0.0]), p, th, False)[0][0]

    # a phase shift of pi/4 in Phi0 turns 2 Phi by pi/2: the pair is in
    # quadrature, so h(Phi0)^2 + h(Phi0 + pi/4)^2 is the squared amplitude
    for ph in np.linspace(0, np.pi, 13):
        assert np.hypot(h0(ph), h0(ph + np.pi / 4)) == pytest.approx(amp, rel=1e-12)
    vals = np.abs([h0(ph) for ph in np.linspace(0, np.pi, 721)])
    assert vals.max() == pytest.approx(amp, rel=1e-5)
