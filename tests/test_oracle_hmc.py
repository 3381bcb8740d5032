"""The oracle's fixed-step HMC against analytic posterior moments (App. A).

* Neal's funnel toy of Sec. II.C, sampled in the standardized coordinates of
  Eq. toy_decenter and mapped back: E[y] = 0, Var y = 9, E[x_i] = 9.
* Linear-Gaussian PTA case: with the hyper-parameters frozen (inverse mass 0)
  the coefficients (u, z, z_dm) have the closed-form Gaussian posterior of
  the dense time-domain model (Eqs. likelihood, a_prior).
"""
import os

import numpy as np
import pytest

import synth
from oracle import dense, hmc, model

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _closed():
    out = {}
    for line in open(os.path.join(GOLD, "closed_forms.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def test_funnel_standardized_moments():
    cf = _closed()
    d = 8

    def lpg(X):
        y, z = X[:, 0], X[:, 1:]
        lp = -0.5 * y * y / 9.0 - 0.5 * np.sum(z * z, 1)
        g = np.concatenate([(-y / 9.0)[:, None], -z], 1)
        return lp, g

    C = 64
    x0 = np.zeros((C, d + 1))
    _, _, _, nacc, S = hmc.run(lpg, x0, n_traj=400, n_leapfrog=8, eps=0.35, seed=77,
                               inv_mass=np.concatenate([[9.0], np.ones(d)]), keep_samples=True)
    S = S[50:]
    y = S[:, :, 0]
    x = y[:, :, None] ** 2 + np.exp(y[:, :, None] / 2) * S[:, :, 1:]
    assert nacc.mean() / 400 > 0.8
    ych = y.mean(0)
    assert abs(ych.mean() - cf["funnel_mean_y"]) < 5 * ych.std() / np.sqrt(C)
    vch = ((y - y.mean()) ** 2).mean(0)
    assert abs(vch.mean() - cf["funnel_var_y"]) < 5 * vch.std() / np.sqrt(C)
    xch = x.mean(axis=(0, 2))
    assert abs(xch.mean() - cf["funnel_mean_x"]) < 5 * xch.std() / np.sqrt(C)
    # Var x_i = E[e^y] + Var(y^2) = e^(9/2) + 162: heavy-tailed (e^y), so the
    # per-chain estimates scatter widely; the bound uses their own spread
    vx = ((x - x.mean()) ** 2).mean(axis=(0, 2))
    assert abs(vx.mean() - cf["funnel_var_x"]) < 5 * vx.std() / np.sqrt(C)


def test_linear_gaussian_moments():
    ds = synth.make_array(3, 3, [12, 15, 18], 8 * synth.YEAR_S, backends_per_psr=[1, 2, 1],
                          nu_range=(0.4e9, 2.0e9), nf_rn=2, nf_gw=2, nf_dm=1)
    prep = model.Prepared(ds)
    lay = prep.lay
    theta = synth.injected_theta(ds, 4, rn=(-13.5, 3.0), dm=(-13.5, 3.0))
    m, S = dense.posterior_moments(prep, theta)
    # diagonal inverse mass = posterior variances (App. A, M^-1 = cov(x)); the
    # step is sized to the stiffest correlated direction (eigenvalue ~0.008)
    inv_mass = np.zeros(lay.d)
    inv_mass[lay.u:] = np.diag(S)

    def lpg(X):
        o = model.logp_grad(prep, X, with_scale=False)
        return o["logp"], o["grad"]

    C = 48
    x0 = np.zeros((C, lay.d))
    x0[:, : lay.n_theta] = theta
    # every chain starts at the prior mean u = z = z_dm = 0, away from the
    # posterior mean m: the moments below test convergence to N(m, S), not
    # only that the sampler keeps a distribution it starts in
    n_traj, burn = 200, 40
    _, _, _, nacc, samp = hmc.run(lpg, x0, n_traj=n_traj, n_leapfrog=16, eps=0.08, seed=99,
                                  inv_mass=inv_mass, keep_samples=True)
    # frozen coordinates never move
    assert np.all(samp[:, :, : lay.n_theta] == theta)
    samp = samp[burn:, :, lay.u:]
    assert nacc.mean() / n_traj > 0.7
    chm = samp.mean(0)                                   # (C, dw)
    zsc = (chm.mean(0) - m) / (chm.std(0) / np.sqrt(C))
    assert np.max(np.abs(zsc)) < 5.0, np.max(np.abs(zsc))
    var = ((samp - m) ** 2).mean(0)
    zv = (var.mean(0) - np.diag(S)) / (var.std(0) / np.sqrt(C))
    assert np.max(np.abs(zv)) < 5.0, np.max(np.abs(zv))
