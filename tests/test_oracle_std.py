"""Pins of the standardized-posterior oracle (oracle/std.py) against what the
paper and the mathematics fix, each by a route other than the oracle's own
Gram-form arithmetic:

* timing-model marginalisation (Eq. Gmatrix_proj): the G (QR) projection
  against N^-1 - N^-1 M (M^T N^-1 M)^-1 M^T N^-1, and both against the
  infinite-variance limit of a Gaussian prior on the timing-model
  deviations (Sec. IV.A: epsilon ~ N(0, inf));
* the CURN transform (Eqs. PTA_standard_transform_curn,
  standardized_stochastic_posterior): with Gamma = I the CURN posterior of a
  is exactly N(a_hat, Sigma), so the density in z is the standard normal
  times the dense time-domain evidence, for any hyper-parameters and for a
  tempered likelihood (App. B, Eqs. tempered_post, mv_normal_post_temp);
* with HD correlations: the density equals the dense time-domain joint
  p(dt) N(a; m, S) at the transformed a, times the Jacobian;
* free spectrum (Sec. IV.A) against the power law at matching rho_k;
* finite differences of the autograd gradient.
"""
import numpy as np
import pytest

import synth
from oracle import std

LN2PI = np.log(2 * np.pi)


def small(seed=3, counts=(14, 19, 23), nf=(3, 2, 2), tm_cols=None):
    ds = synth.make_array(seed, len(counts), list(counts), 8 * synth.YEAR_S,
                          backends_per_psr=[2] * len(counts), nu_range=(0.4e9, 2.0e9),
                          nf_rn=nf[0], nf_gw=nf[1], nf_dm=nf[2])
    if tm_cols is not None:
        ds["tm"] = tm_cols(ds)
    return ds


def general_tm(ds):
    """A stored design matrix of 5 columns (offset, spin-down-like terms, an
    annual sinusoid pair) with one duplicated column (rank deficient)."""
    t = ds["t"] / ds["tspan"]
    yr = 2 * np.pi * ds["t"] / synth.YEAR_S
    return np.stack([np.ones_like(t), t, t * t, np.sin(yr), np.cos(yr), 2.0 * t], axis=1)


def point(ds, prep, seed, jitter=0.3):
    th = synth.injected_theta(ds, seed, rn=(-14.0, 3.5), dm=(-14.0, 3.5))
    rng = np.random.default_rng(seed)
    th = np.clip(th + rng.uniform(-jitter, jitter, th.size), ds["prior_lo"], ds["prior_hi"])
    return np.concatenate([th, rng.standard_normal(prep.lay.d - prep.lay.n_theta)])


def _psr_arrays(ds, I, prep):
    off = ds["toa_offsets"]
    s, e = off[I], off[I + 1]
    tt = ds["t"][s:e]
    if ds.get("tm") is None:
        c, hs = 0.5 * (tt.min() + tt.max()), 0.5 * (tt.max() - tt.min())
        tau = (tt - c) / hs
        M = np.stack([np.ones_like(tau), tau, tau * tau], 1)
    else:
        M = ds["tm"][s:e]
    K = max(prep.lay.Ka, prep.lay.Kdm)
    arg = 2 * np.pi * np.outer(tt, np.arange(1, K + 1)) / ds["tspan"]
    F = np.empty((tt.size, 2 * K))
    F[:, 0::2], F[:, 1::2] = np.sin(arg), np.cos(arg)
    w = ds["dm_scale"] / ds["nu"][s:e] ** 2
    T = np.concatenate([F[:, :2 * prep.lay.Ka], w[:, None] * F[:, :2 * prep.lay.Kdm]], 1)
    be = ds["backend"][s:e]
    N = (ds["efac"][be] * ds["sigma"][s:e]) ** 2 + ds["equad"][be] ** 2
    return M, T, N, ds["dt"][s:e]


def _G(M):
    """Orthonormal complement of the column space of M (SVD, independent of
    the oracle's QR route)."""
    U, s, _ = np.linalg.svd(M, full_matrices=True)
    r = int(np.sum(s > 1e-10 * s[0]))
    return U[:, r:]


# ------------------------------------------------ timing-model projection --

@pytest.mark.parametrize("tm", [None, general_tm])
def test_projection_forms_agree(tm):
    """Eq. Gmatrix_proj: G (G^T N G)^-1 G^T from an explicit complement basis
    equals the Woodbury-limit form, and ln det(G^T N G) agrees."""
    ds = small(tm_cols=tm)
    a = std.StdPrepared(ds, explicit=True)
    b = std.StdPrepared(ds, explicit=False)
    for I in range(a.n_psr):
        np.testing.assert_allclose(a.S0[I], b.S0[I], rtol=1e-9, atol=1e-9 * np.abs(a.S0[I]).max())
        np.testing.assert_allclose(a.dvec[I], b.dvec[I], rtol=1e-8, atol=1e-9 * np.abs(a.dvec[I]).max())
        assert a.cval[I] == pytest.approx(b.cval[I], rel=1e-9)
        assert a.const[I] == pytest.approx(b.const[I], rel=1e-10)


@pytest.mark.parametrize("tm", [None, general_tm])
def test_projection_is_infinite_variance_limit(tm):
    """Sec. IV.A: the timing-model deviations carry N(0, s^2 I) with s -> inf.
    log N(r; 0, N + s^2 M M^T) + r ln s + (r/2) ln 2 pi + 1/2 ln det(M_r^T M_r)
    tends to -1/2 r^T N~^-1 r - 1/2 ln det(2 pi G^T N G) (the oracle's
    likelihood at a = 0), with M_r the independent columns."""
    ds = small(tm_cols=tm)
    prep = std.StdPrepared(ds)
    for I in range(prep.n_psr):
        M, T, N, dt = _psr_arrays(ds, I, prep)
        G = _G(M)
        r = M.shape[1] - G.shape[1] + (M.shape[0] - M.shape[1])   # rank of M
        r = M.shape[0] - G.shape[1]
        U, sv, _ = np.linalg.svd(M, full_matrices=False)
        Ur = U[:, :r] * sv[:r]                   # same column space, r columns
        target = -0.5 * prep.cval[I] + prep.const[I]
        s = 1e-2                                  # 1e4 x the white-noise level
        Cov = np.diag(N) + s * s * (Ur @ Ur.T)
        Lc = np.linalg.cholesky(Cov)
        y = np.linalg.solve(Lc, dt)
        lg = -0.5 * y @ y - np.sum(np.log(np.diag(Lc))) - 0.5 * dt.size * LN2PI
        lim = lg + r * np.log(s) + 0.5 * r * LN2PI + 0.5 * np.linalg.slogdet(Ur.T @ Ur)[1]
        assert lim == pytest.approx(target, rel=1e-7, abs=1e-6)


# ------------------------------------------------ CURN transform ----------

def _dense_blocks(ds, prep):
    """x = G^T dt, C = G^T N G, T' = G^T T per pulsar (time-domain, dense)."""
    out = []
    for I in range(prep.n_psr):
        M, T, N, dt = _psr_arrays(ds, I, prep)
        G = _G(M)
        out.append((G.T @ dt, G.T @ (N[:, None] * G), G.T @ T))
    return out


def _lognorm(x, C):
    L = np.linalg.cholesky(C)
    y = np.linalg.solve(L, x)
    return -0.5 * y @ y - np.sum(np.log(np.diag(L))) - 0.5 * x.size * LN2PI


@pytest.mark.parametrize("beta", [1.0, 0.37])
def test_curn_identity(beta):
    """With Gamma = I the posterior of a under a (tempered) CURN prior is
    exactly N(a_hat, Sigma): the density in z is N(z; 0, I) times the
    evidence  Z = kappa_beta N(x; 0, C/beta + T' phi T'^T),
    kappa_beta = (2 pi)^(n'(1-beta)/2) det(C)^((1-beta)/2) beta^(-n'/2),
    computed densely in the time domain; the z-gradient is -z."""
    ds = small(seed=5)
    prep = std.StdPrepared(ds)
    prep.Gamma = np.eye(prep.n_psr)
    blocks = _dense_blocks(ds, prep)
    lay = prep.lay
    for seed in (1, 2, 3):
        x = point(ds, prep, seed)
        out = std.logp_grad(prep, x, beta=beta)
        assert out["status"][0] == 0
        import torch
        rho, kap, kdm = (v.numpy() for v in prep.spectra(torch.tensor(x[:lay.n_theta])))
        logZ = 0.0
        for I, (xv, C, Tp) in enumerate(blocks):
            D = np.concatenate([np.repeat(rho + kap[I], 2), np.repeat(kdm[I], 2)])
            npr = xv.size
            kap_b = 0.5 * npr * (1 - beta) * LN2PI + 0.5 * (1 - beta) * np.linalg.slogdet(C)[1] \
                - 0.5 * npr * np.log(beta)
            logZ += kap_b + _lognorm(xv, C / beta + (Tp * D) @ Tp.T)
        z = x[lay.z:]
        ref = -0.5 * z @ z - 0.5 * z.size * LN2PI + logZ - np.sum(np.log(prep.hi - prep.lo))
        assert out["logp"][0] == pytest.approx(ref, rel=1e-10, abs=1e-8)
        np.testing.assert_allclose(out["grad"][0][lay.z:], -z, rtol=1e-8, atol=1e-8)


@pytest.mark.parametrize("beta", [1.0, 0.5])
def test_hd_dense_joint(beta):
    """With HD correlations: beta log L(a) + log N(a; 0, phi) at the
    transformed a equals log Z_beta + log N(a; m_beta, S_beta), the tempered
    joint of the dense time-domain model across all pulsars (HD coupling),
    with S_beta = (beta T'^T C^-1 T' + phi^-1)^-1, m_beta = beta S_beta T'^T C^-1 x;
    the density adds the Jacobian sum_I ln det L_I."""
    ds = small(seed=9)
    prep = std.StdPrepared(ds)
    lay, n = prep.lay, prep.n_psr
    blocks = _dense_blocks(ds, prep)
    import torch
    for seed in (4, 5):
        x = point(ds, prep, seed)
        out = std.logp_grad(prep, x, beta=beta)
        th = torch.tensor(x[:lay.n_theta])
        a, jac, _, spec = prep.transform(th, torch.tensor(x[lay.z:]).reshape(n, lay.P), beta)
        a = a.numpy().reshape(-1)
        rho, kap, kdm = (v.numpy() for v in spec)
        P = lay.P
        Phi = np.zeros((n * P, n * P))
        for I in range(n):
            for J in range(n):
                for k in range(lay.Ka):
                    v = rho[k] * prep.Gamma[I, J] + (kap[I, k] if I == J else 0.0)
                    for c in range(2):
                        Phi[I * P + 2 * k + c, J * P + 2 * k + c] = v
            for k in range(lay.Kdm):
                for c in range(2):
                    j = I * P + 2 * lay.Ka + 2 * k + c
                    Phi[j, j] = kdm[I, k]
        xs = np.concatenate([b[0] for b in blocks])
        nn = xs.size
        C = np.zeros((nn, nn))
        Tp = np.zeros((nn, n * P))
        o = 0
        for I, (xv, Ci, Ti) in enumerate(blocks):
            m = xv.size
            C[o:o + m, o:o + m] = Ci
            Tp[o:o + m, I * P:(I + 1) * P] = Ti
            o += m
        kap_b = 0.5 * nn * (1 - beta) * LN2PI + 0.5 * (1 - beta) * np.linalg.slogdet(C)[1] \
            - 0.5 * nn * np.log(beta)
        logZ = kap_b + _lognorm(xs, C / beta + Tp @ Phi @ Tp.T)
        Ci = np.linalg.inv(C)
        Sinv = beta * Tp.T @ Ci @ Tp + np.linalg.inv(Phi)
        S = np.linalg.inv(Sinv)
        S = 0.5 * (S + S.T)
        mpost = S @ (beta * Tp.T @ Ci @ xs)
        ref = logZ + _lognorm(a - mpost, S) + float(jac) - np.sum(np.log(prep.hi - prep.lo))
        assert out["logp"][0] == pytest.approx(ref, rel=1e-9, abs=1e-7)


def test_cholesky_factor_is_lower_of_sigma():
    """The transform uses the lower Cholesky factor of Sigma_CURN (the paper's
    L with Sigma = L L^T): check a = a_hat + L z against a dense recomputation
    of Sigma and its factor from the stored Gram quantities."""
    ds = small(seed=13)
    prep = std.StdPrepared(ds)
    lay = prep.lay
    x = point(ds, prep, 7)
    a = std.coefficients(prep, x)
    import torch
    rho, kap, kdm = (v.numpy() for v in prep.spectra(torch.tensor(x[:lay.n_theta])))
    for I in range(prep.n_psr):
        D = np.concatenate([np.repeat(rho + kap[I], 2), np.repeat(kdm[I], 2)])
        Sig = np.linalg.inv(prep.S0[I] + np.diag(1 / D))
        L = np.linalg.cholesky(0.5 * (Sig + Sig.T))
        assert np.allclose(np.triu(L, 1), 0.0) and np.all(np.diag(L) > 0)
        z = x[lay.z + I * lay.P: lay.z + (I + 1) * lay.P]
        np.testing.assert_allclose(a[I], Sig @ prep.dvec[I] + L @ z, rtol=1e-9,
                                   atol=1e-12 * np.abs(a[I]).max())


# ------------------------------------------------ free spectrum -----------

def free_box(ds):
    """Free-spectrum box: log10 rho_k in [-20, -5] per frequency (Sec. IV.A)."""
    n, kr, kg, kd = ds["n_psr"], ds["nf_rn"], ds["nf_gw"], ds["nf_dm"]
    m = (kg if kg else 0) + n * (kr if kr else 0) + n * (kd if kd else 0)
    return np.full(m, -20.0), np.full(m, -5.0)


def test_free_spectrum_matches_power_law():
    """At log10 rho_k = log10 P(f_k; A, gamma) the free-spectrum density equals
    the power-law density up to the two hyper-prior normalisations, and the
    power-law gradient is the free-spectrum gradient through d log10 rho_k /
    d log10 A = 2 and d log10 rho_k / d gamma = -log10(f_k yr)."""
    ds = small(seed=17)
    pl = std.StdPrepared(ds)
    dsf = dict(ds)
    dsf["spectrum"] = "free"
    dsf["prior_lo"], dsf["prior_hi"] = free_box(ds)
    fr = std.StdPrepared(dsf)
    x = point(ds, pl, 8)
    import torch
    lay, lf = pl.lay, fr.lay
    rho, kap, kdm = (v.numpy() for v in pl.spectra(torch.tensor(x[:lay.n_theta])))
    th = []
    th += list(np.log10(rho[:ds["nf_gw"]]))
    for I in range(pl.n_psr):
        th += list(np.log10(kap[I, :ds["nf_rn"]]))
    for I in range(pl.n_psr):
        th += list(np.log10(kdm[I]))
    xf = np.concatenate([th, x[lay.z:]])
    a = std.logp_grad(pl, x)
    b = std.logp_grad(fr, xf)
    c_pl = -np.sum(np.log(pl.hi - pl.lo))
    c_fr = -np.sum(np.log(fr.hi - fr.lo))
    assert a["logp"][0] - c_pl == pytest.approx(b["logp"][0] - c_fr, rel=1e-11)
    np.testing.assert_allclose(a["grad"][0][lay.z:], b["grad"][0][lf.z:], rtol=1e-9, atol=1e-12)
    lfy = np.log10(pl.freqs * std.YR)
    gb = b["grad"][0]
    kg = ds["nf_gw"]
    assert a["grad"][0][lay.gw] == pytest.approx(2.0 * gb[lf.gw:lf.gw + kg].sum(), rel=1e-9)
    assert a["grad"][0][lay.gw + 1] == pytest.approx(-(gb[lf.gw:lf.gw + kg] * lfy[:kg]).sum(), rel=1e-9)


# ------------------------------------------------ finite differences ------

@pytest.mark.parametrize("free", [False, True])
def test_gradient_finite_differences(free):
    ds = small(seed=21, tm_cols=general_tm)
    if free:
        ds["spectrum"] = "free"
        ds["prior_lo"], ds["prior_hi"] = free_box(ds)
    prep = std.StdPrepared(ds)
    lay = prep.lay
    if free:
        rng = np.random.default_rng(4)
        x = np.concatenate([rng.uniform(-15.5, -13.5, lay.n_theta), rng.standard_normal(lay.d - lay.n_theta)])
    else:
        x = point(ds, prep, 11)
    g = std.logp_grad(prep, x, beta=0.8)["grad"][0]
    for i in range(lay.d):
        h = 1e-5 * max(1.0, abs(x[i]))
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (std.logp_grad(prep, xp, beta=0.8)["logp"][0] - std.logp_grad(prep, xm, beta=0.8)["logp"][0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=2e-5, abs=2e-6 * max(1.0, np.abs(g).max())), i


def test_status_codes():
    ds = small(seed=23)
    prep = std.StdPrepared(ds)
    lay = prep.lay
    X = np.stack([point(ds, prep, s) for s in (1, 2, 3)])
    X[0, 0] = -25.0                      # outside the box
    X[1, lay.z + 2] = np.nan             # non-finite coefficient
    out = std.logp_grad(prep, X)
    assert list(out["status"]) == [1, 4, 0]
    # spectra underflowing to 0 in a widened box: phi_CURN not positive definite
    ds2 = dict(ds)
    ds2["prior_lo"] = np.full_like(ds["prior_lo"], -400.0)
    prep2 = std.StdPrepared(ds2)
    x = X[2].copy()
    x[lay.gw] = -300.0
    x[lay.rn:lay.rn + 2 * prep.n_psr:2] = -300.0
    assert std.logp_grad(prep2, x)["status"][0] == 2
    assert out["logp"][0] == -np.inf and np.all(out["grad"][0] == 0)
