"""Pins of the standardized-posterior oracle with a deterministic CW signal in
its own Fourier basis (oracle/std.py; Sec. IV.C, Eqs. det_F_basis,
stoch_det_posterior, det_mean, decenter_det_PTA,
standardized_det_posterior), each by a route other than the oracle's stored
products S_D, e_D, Q_D:

* the DFT that maps the sampled delay to a_D against numpy's FFT;
* the basis F_D with the mean reproduces the samples (trigonometric
  interpolation at M = 2 K_D + 1 points);
* the density with the signal equals the density without it on the data
  dt - F_D a_D(theta) (the signal subtracted in the time domain, the Gram
  quantities recomputed from scratch), tempered and not: Eq. det_mean's
  "subtract the deterministic signal, then take the MAP";
* finite differences of the CW coordinates of the autograd gradient;
* status 3 when the CW coalesces within the extended span.
"""
import numpy as np
import pytest

import synth
from oracle import cw as cwmod
from oracle import std

THETA_CW = np.array([0.3, 1.0, 8.7, -8.2, 0.5, 0.6, 0.9, -14.0])


def small_cw(seed=3, counts=(14, 19, 23), nf=(3, 2, 2), kd=12):
    ds = synth.make_array(seed, len(counts), list(counts), 8 * synth.YEAR_S,
                          backends_per_psr=[2] * len(counts), nu_range=(0.4e9, 2.0e9),
                          nf_rn=nf[0], nf_gw=nf[1], nf_dm=nf[2], has_cw=True)
    ds["cw_nf"] = kd
    ds["cw_tspan"] = 2.0 * ds["tspan"]
    return ds


def point(ds, prep, seed, cw=THETA_CW, jitter=0.3):
    th = synth.injected_theta(ds, seed, rn=(-14.0, 3.5), dm=(-14.0, 3.5), cw=cw)
    rng = np.random.default_rng(seed)
    lay = prep.lay
    th[:lay.cw] = np.clip(th[:lay.cw] + rng.uniform(-jitter, jitter, lay.cw),
                          ds["prior_lo"][:lay.cw], ds["prior_hi"][:lay.cw])
    return np.concatenate([th, rng.standard_normal(lay.d - lay.n_theta)])


def test_dft_against_numpy_fft():
    """a_(k,cos) = (2/M) Re X_k and a_(k,sin) = -(2/M) Im X_k with X the FFT
    of the M samples, k = 1..K_D."""
    prep = std.StdPrepared(small_cw())
    rng = np.random.default_rng(1)
    h = rng.standard_normal(prep.Md)
    a = prep.dft @ h
    X = np.fft.rfft(h)
    k = np.arange(1, prep.Kd + 1)
    np.testing.assert_allclose(a[1::2], 2.0 / prep.Md * X[k].real, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(a[0::2], -2.0 / prep.Md * X[k].imag, rtol=1e-12, atol=1e-14)


def test_basis_reproduces_the_samples():
    """With M = 2 K_D + 1 samples, F_D(t_j) a_D plus the mean of the samples
    is the sampled delay itself: pins the sample grid t_j = j T_D / M, the
    frequencies k / T_D and the sin-then-cos order of the basis against the
    transform."""
    ds = small_cw()
    prep = std.StdPrepared(ds)
    t = np.arange(prep.Md) * prep.Td / prep.Md
    arg = 2.0 * np.pi * np.outer(t, np.arange(1, prep.Kd + 1)) / prep.Td
    FD = np.empty((t.size, 2 * prep.Kd))
    FD[:, 0::2], FD[:, 1::2] = np.sin(arg), np.cos(arg)
    for I in range(prep.n_psr):
        h, _ = cwmod.delay(t, prep.pos[I], THETA_CW, want_grad=False)
        np.testing.assert_allclose(FD @ (prep.dft @ h) + h.mean(), h, rtol=0, atol=1e-12 * np.abs(h).max())


def _subtracted(ds, prep, theta_cw):
    """The data set without the CW, its residuals minus F_D a_D(theta_cw) at
    every TOA; a_D from numpy's FFT of the sampled delay."""
    ds0 = dict(ds)
    ds0["has_cw"] = 0
    n_cw = 8
    ds0["prior_lo"] = ds["prior_lo"][:-n_cw]
    ds0["prior_hi"] = ds["prior_hi"][:-n_cw]
    Td, Kd = ds["cw_tspan"], ds["cw_nf"]
    M = 2 * Kd + 1
    ts = np.arange(M) * Td / M
    dt = np.array(ds["dt"], np.float64)
    off = ds["toa_offsets"]
    k = np.arange(1, Kd + 1)
    for I in range(ds["n_psr"]):
        h, _ = cwmod.delay(ts, np.asarray(ds["psr_pos"]).reshape(-1, 3)[I], theta_cw, want_grad=False)
        X = np.fft.rfft(h)
        a_sin, a_cos = -2.0 / M * X[k].imag, 2.0 / M * X[k].real
        tt = ds["t"][off[I]:off[I + 1]]
        arg = 2.0 * np.pi * np.outer(tt, k) / Td
        dt[off[I]:off[I + 1]] -= np.sin(arg) @ a_sin + np.cos(arg) @ a_cos
    ds0["dt"] = dt
    return ds0


@pytest.mark.parametrize("beta", [1.0, 0.4])
def test_density_equals_the_subtracted_data(beta):
    ds = small_cw(seed=5)
    prep = std.StdPrepared(ds)
    lay = prep.lay
    for seed in (2, 3):
        x = point(ds, prep, seed)
        out = std.logp_grad(prep, x, beta=beta)
        assert out["status"][0] == 0
        ds0 = _subtracted(ds, prep, x[lay.cw:lay.cw + 8])
        prep0 = std.StdPrepared(ds0)
        x0 = np.concatenate([x[:lay.cw], x[lay.cw + 8:]])
        ref = std.logp_grad(prep0, x0, beta=beta)
        box = np.sum(np.log(ds["prior_hi"][lay.cw:lay.cw + 8] - ds["prior_lo"][lay.cw:lay.cw + 8]))
        assert out["logp"][0] == pytest.approx(ref["logp"][0] - box, rel=1e-10, abs=1e-8)
        g = np.concatenate([out["grad"][0][:lay.cw], out["grad"][0][lay.cw + 8:]])
        np.testing.assert_allclose(g, ref["grad"][0], rtol=1e-7, atol=1e-9 * np.abs(ref["grad"][0]).max())


def test_cw_gradient_finite_differences():
    ds = small_cw(seed=7)
    prep = std.StdPrepared(ds)
    lay = prep.lay
    x = point(ds, prep, 4)
    out = std.logp_grad(prep, x)
    for j in list(range(lay.cw, lay.cw + 8)) + [0, lay.z + 1]:
        h = 1e-5 * max(abs(x[j]), 1.0)
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (std.logp_grad(prep, xp)["logp"][0] - std.logp_grad(prep, xm)["logp"][0]) / (2 * h)
        assert out["grad"][0][j] == pytest.approx(fd, rel=2e-5, abs=1e-6 * max(1.0, abs(fd)))


def test_status_coalescence():
    """Status 3 when y >= 1 at a sample of the extended span; a point outside
    the box keeps status 1 (precedence)."""
    ds = small_cw(seed=9)
    lay = std.StdPrepared(ds).lay
    ds["prior_hi"] = ds["prior_hi"].copy()
    ds["prior_hi"][lay.cw + 2], ds["prior_hi"][lay.cw + 3] = 10.5, -7.0   # heavier, faster sources
    prep = std.StdPrepared(ds)
    fast = THETA_CW.copy()
    fast[2], fast[3] = 10.5, -7.0        # y reaches 1 within T_D
    assert cwmod.max_y(fast, prep.ts_d[-1]) >= 1.0
    x = point(ds, prep, 1, cw=fast)
    xb = x.copy()
    xb[1] = 99.0
    out = std.logp_grad(prep, np.stack([x, xb, point(ds, prep, 1)]))
    assert list(out["status"]) == [3, 1, 0]
    assert out["logp"][0] == -np.inf and np.all(out["grad"][0] == 0.0)
