"""Pins of the standardized-posterior oracle with split common-process and
pulsar-noise coefficients (oracle/std.py; App. C, Eqs. separated_post,
split_map_a, split_standardizing_transform), each by a route other than the
oracle's stored Gram quantities:

* the MAP pair (a_hat_G, a_hat_R) solves the linear system of Eq.
  split_map_a, assembled densely in the time domain over the projected
  residuals and solved directly (not through the combined MAP and its
  proportional split), tempered and not;
* a_G = a_hat_G + L_G z_G and a_R = a_hat_R + L_R z_R with L the lower
  Cholesky factors of Sigma_G and Sigma_R recomputed in the time domain;
* the density equals the dense time-domain joint of Eq. separated_post over
  all pulsars (HD-correlated common process, diagonal pulsar noise): the
  tempered evidence times N((a_G, a_R); m, S) at the transformed point,
  plus the Jacobian sum of ln det L_G + ln det L_R;
* finite differences of the autograd gradient;
* status 2 when a prior variance underflows.
Frequency counts are taken unequal both ways, so rows that only one set
covers (common process above the pulsar noise, or the reverse, and the DM
block) are exercised.
"""
import numpy as np
import pytest
import torch

from oracle import std
from test_oracle_std import _dense_blocks, _lognorm, point, small


def split_ds(seed, nf=(3, 2, 2)):
    ds = small(seed=seed, nf=nf)
    ds["split"] = 1
    return ds


def _variances(prep, x):
    lay = prep.lay
    rho, kap, kdm = (v.numpy() for v in prep.spectra(torch.tensor(x[:lay.n_theta])))
    g, r = np.arange(2 * lay.nf_gw), np.concatenate([np.arange(2 * lay.nf_rn), 2 * lay.Ka + np.arange(2 * lay.Kdm)])
    vg = np.repeat(rho[:lay.nf_gw], 2)
    vr = [np.concatenate([np.repeat(kap[I, :lay.nf_rn], 2), np.repeat(kdm[I], 2)]) for I in range(prep.n_psr)]
    return rho, g, r, vg, vr


def _dense_map(blocks, g, r, vg, vr_I, I, beta):
    """Eq. split_map_a for pulsar I, the Gram blocks formed in the time
    domain from the projected basis T' and noise C."""
    xv, C, Tp = blocks[I]
    Ci = np.linalg.inv(C)
    B = Tp.T @ Ci @ Tp
    b = Tp.T @ Ci @ xv
    nG = g.size
    A = np.zeros((nG + r.size, nG + r.size))
    A[:nG, :nG] = beta * B[np.ix_(g, g)] + np.diag(1.0 / vg)
    A[:nG, nG:] = beta * B[np.ix_(g, r)]
    A[nG:, :nG] = beta * B[np.ix_(r, g)]
    A[nG:, nG:] = beta * B[np.ix_(r, r)] + np.diag(1.0 / vr_I)
    sol = np.linalg.solve(A, beta * np.concatenate([b[g], b[r]]))
    SG = np.linalg.inv(beta * B[np.ix_(g, g)] + np.diag(1.0 / vg))
    SR = np.linalg.inv(beta * B[np.ix_(r, r)] + np.diag(1.0 / vr_I))
    return sol[:nG], sol[nG:], np.linalg.cholesky(0.5 * (SG + SG.T)), np.linalg.cholesky(0.5 * (SR + SR.T))


@pytest.mark.parametrize("nf,beta", [((3, 2, 2), 1.0), ((2, 3, 1), 0.45), ((3, 3, 0), 0.8)])
def test_map_and_transform_against_the_joint_system(nf, beta):
    ds = split_ds(31, nf)
    prep = std.StdPrepared(ds)
    lay = prep.lay
    blocks = _dense_blocks(ds, prep)
    for seed in (1, 2):
        x = point(ds, prep, seed)
        _, g, r, vg, vr = _variances(prep, x)
        maps = prep.split_map(torch.tensor(x[:lay.n_theta]), beta)
        coef = std.coefficients(prep, x, beta)
        for I in range(prep.n_psr):
            aG, aR, LG, LR = _dense_map(blocks, g, r, vg, vr[I], I, beta)
            mG, mR = (v.numpy() for v in maps[I])
            sc = max(np.abs(aG).max(), np.abs(aR).max())
            np.testing.assert_allclose(mG, aG, rtol=1e-8, atol=1e-10 * sc)
            np.testing.assert_allclose(mR, aR, rtol=1e-8, atol=1e-10 * sc)
            z = x[lay.z + I * lay.Pz: lay.z + (I + 1) * lay.Pz]
            want = np.concatenate([aG + LG @ z[:lay.PG], aR + LR @ z[lay.PG:]])
            np.testing.assert_allclose(coef[I], want, rtol=1e-8, atol=1e-10 * np.abs(want).max())


@pytest.mark.parametrize("nf,beta", [((3, 2, 2), 1.0), ((2, 3, 1), 0.5)])
def test_density_is_the_dense_split_joint(nf, beta):
    """beta log L(a_G + a_R) + log N(a_G; 0, phi_GWB) + log N(a_R; 0, phi_RN)
    = log Z_beta + log N((a_G, a_R); m, S) with S = (beta B^T C^-1 B +
    Phi^-1)^-1, m = beta S B^T C^-1 x, B = [T'_G | T'_R] over all pulsars and
    Phi the HD (common) and diagonal (pulsar) prior; the density adds the
    Jacobian, recomputed from the time-domain Sigma_G and Sigma_R."""
    ds = split_ds(37, nf)
    prep = std.StdPrepared(ds)
    lay, n = prep.lay, prep.n_psr
    blocks = _dense_blocks(ds, prep)
    PG, PR = lay.PG, lay.PR
    for seed in (4, 5):
        x = point(ds, prep, seed)
        out = std.logp_grad(prep, x, beta=beta)
        assert out["status"][0] == 0
        rho, g, r, vg, vr = _variances(prep, x)
        coef = std.coefficients(prep, x, beta)
        av = np.concatenate([coef[:, :PG].reshape(-1), coef[:, PG:].reshape(-1)])
        NG = n * PG
        Phi = np.zeros((NG + n * PR,) * 2)
        for I in range(n):
            for J in range(n):
                for k in range(lay.nf_gw):
                    for c in range(2):
                        Phi[I * PG + 2 * k + c, J * PG + 2 * k + c] = rho[k] * prep.Gamma[I, J]
            Phi[NG + I * PR: NG + (I + 1) * PR, NG + I * PR: NG + (I + 1) * PR] = np.diag(vr[I])
        xs = np.concatenate([b[0] for b in blocks])
        nn = xs.size
        C = np.zeros((nn, nn))
        B = np.zeros((nn, NG + n * PR))
        o, jac = 0, 0.0
        for I, (xv, Ci, Ti) in enumerate(blocks):
            m = xv.size
            C[o:o + m, o:o + m] = Ci
            B[o:o + m, I * PG:(I + 1) * PG] = Ti[:, g]
            B[o:o + m, NG + I * PR: NG + (I + 1) * PR] = Ti[:, r]
            o += m
            _, _, LG, LR = _dense_map(blocks, g, r, vg, vr[I], I, beta)
            jac += np.sum(np.log(np.diag(LG))) + np.sum(np.log(np.diag(LR)))
        kap_b = 0.5 * nn * (1 - beta) * np.log(2 * np.pi) + 0.5 * (1 - beta) * np.linalg.slogdet(C)[1] \
            - 0.5 * nn * np.log(beta)
        logZ = kap_b + _lognorm(xs, C / beta + B @ Phi @ B.T)
        Ci = np.linalg.inv(C)
        S = np.linalg.inv(beta * B.T @ Ci @ B + np.linalg.inv(Phi))
        S = 0.5 * (S + S.T)
        mpost = S @ (beta * B.T @ Ci @ xs)
        ref = logZ + _lognorm(av - mpost, S) + jac - np.sum(np.log(prep.hi - prep.lo))
        assert out["logp"][0] == pytest.approx(ref, rel=1e-9, abs=1e-7)


def test_split_gradient_finite_differences():
    ds = split_ds(41, (2, 3, 1))
    prep = std.StdPrepared(ds)
    lay = prep.lay
    x = point(ds, prep, 9)
    g = std.logp_grad(prep, x, beta=0.7)["grad"][0]
    for i in range(lay.d):
        h = 1e-5 * max(1.0, abs(x[i]))
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (std.logp_grad(prep, xp, beta=0.7)["logp"][0] - std.logp_grad(prep, xm, beta=0.7)["logp"][0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=2e-5, abs=2e-6 * max(1.0, np.abs(g).max())), i


def test_split_status_codes():
    ds = split_ds(43)
    prep = std.StdPrepared(ds)
    lay = prep.lay
    X = np.stack([point(ds, prep, s) for s in (1, 2)])
    X[0, 0] = -25.0
    out = std.logp_grad(prep, X)
    assert list(out["status"]) == [1, 0]
    ds2 = dict(ds)
    ds2["prior_lo"] = np.full_like(ds["prior_lo"], -400.0)
    prep2 = std.StdPrepared(ds2)
    x = X[1].copy()
    x[lay.gw] = -300.0                  # rho underflows: Sigma_G has no inverse prior
    assert std.logp_grad(prep2, x)["status"][0] == 2


def test_split_needs_both_processes():
    with pytest.raises(ValueError):
        std.StdPrepared(split_ds(47, (0, 2, 1)))
