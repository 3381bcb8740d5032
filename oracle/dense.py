"""Structurally different evaluations used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``gram_loglike``: the compressed form of Eq. posterior_implemented (Sec. V.B),
  with precomputed F^T N^-1 F and F^T N^-1 dt' and with the constants the
  paper drops put back; equals the per-TOA likelihood when h = 0.
* ``dense_joint``: the Gaussian identity
      N(dt; h + Phi v, N) N(v; 0, P) = N(dt; h, N + Phi P Phi^T) N(v; m, S)
  with the dense prior covariance P built directly from Eq. prior_cov (no
  Cholesky) and the full (n x n) time-domain covariance across all pulsars.
  Together with the Jacobian of v = A w it gives log p at any point.
* ``whitened_prior``: -1/2 a^T phi^-1 a - 1/2 ln det 2 pi phi + ln det(da/dz)
  with the dense phi of Eq. prior_cov; must equal -1/2 |z|^2 - d/2 ln 2 pi
  (Eq. standardized_density with mu = 0).
"""
from __future__ import annotations

import numpy as np

from .model import LN2PI, Prepared


def _phi_full(prep: Prepared, rho, kap):
    """Dense prior covariance of the stacked coefficients a (pulsar-major,
    per pulsar k=1 sin, k=1 cos, ...), from Eq. prior_cov."""
    n, K = prep.n_psr, prep.K
    D = n * 2 * K
    P = np.zeros((D, D))
    for I in range(n):
        for J in range(n):
            for k in range(K):
                v = rho[k] * prep.Gamma[I, J] + (kap[I, k] if I == J else 0.0)
                for c in range(2):
                    P[I * 2 * K + 2 * k + c, J * 2 * K + 2 * k + c] = v
    return P


def _transform(prep, x):
    """a, a_dm, b and per-frequency Cholesky factors for one point (oracle
    transform; only used to place v on both sides of the identities)."""
    gw, rn, dm, cw, u, z, zdm = prep.split(x[None, :])
    rho, kap, kdm = prep.spectra(gw, rn, dm, 1)
    n, K = prep.n_psr, prep.K
    a = np.zeros((n, 2 * K))
    Ls = []
    for k in range(K):
        Lk = np.linalg.cholesky(rho[0, k] * prep.Gamma + np.diag(kap[0, :, k]))
        Ls.append(Lk)
        a[:, 2 * k] = Lk @ z[0, :, 2 * k]
        a[:, 2 * k + 1] = Lk @ z[0, :, 2 * k + 1]
    adm = np.repeat(np.sqrt(kdm[0]), 2, axis=1) * zdm[0]
    b = prep.sigma_b * u[0]
    return dict(rho=rho[0], kap=kap[0], kdm=kdm[0], a=a, adm=adm, b=b, Ls=Ls,
                z=z[0], zdm=zdm[0], u=u[0], cw=None if cw is None else cw[0])


def whitened_prior(prep: Prepared, x):
    """Left and right side of the whitened-prior identity for one point."""
    T = _transform(prep, x)
    P = _phi_full(prep, T["rho"], T["kap"])
    a = T["a"].reshape(-1)
    Lp = np.linalg.cholesky(P)
    y = np.linalg.solve(Lp, a)
    logdet_2piP = P.shape[0] * LN2PI + 2.0 * np.sum(np.log(np.diag(Lp)))
    # da/dz is block lower triangular per frequency: det = prod_k det(L_k)^2
    logdet_jac = sum(2.0 * np.sum(np.log(np.diag(Lk))) for Lk in T["Ls"])
    lhs = -0.5 * y @ y - 0.5 * logdet_2piP + logdet_jac
    z = T["z"].reshape(-1)
    rhs = -0.5 * z @ z - 0.5 * z.size * LN2PI
    return lhs, rhs


def _design(prep, T):
    """Block-diagonal Phi = [M, F, w F_dm] over all TOAs, the stacked v and
    the dense prior covariance P of v."""
    n, K, Kdm = prep.n_psr, prep.K, prep.Kdm
    ntot = sum(p["t"].size for p in prep.psr)
    nb, na, nd = 3 * n, 2 * K * n, 2 * Kdm * n
    Phi = np.zeros((ntot, nb + na + nd))
    row = 0
    for I, p in enumerate(prep.psr):
        m = p["t"].size
        Phi[row:row + m, 3 * I:3 * I + 3] = p["M"]
        Phi[row:row + m, nb + 2 * K * I: nb + 2 * K * (I + 1)] = p["F"]
        if Kdm:
            Phi[row:row + m, nb + na + 2 * Kdm * I: nb + na + 2 * Kdm * (I + 1)] = p["w"][:, None] * p["Fdm"]
        row += m
    v = np.concatenate([T["b"].reshape(-1), T["a"].reshape(-1), T["adm"].reshape(-1)])
    P = np.zeros((nb + na + nd, nb + na + nd))
    P[:nb, :nb] = prep.sigma_b ** 2 * np.eye(nb)
    P[nb:nb + na, nb:nb + na] = _phi_full(prep, T["rho"], T["kap"])
    if nd:
        P[nb + na:, nb + na:] = np.diag(np.repeat(T["kdm"], 2, axis=1).reshape(-1))
    return Phi, v, P


def _lognormal(x, mean, cov):
    Lc = np.linalg.cholesky(cov)
    y = np.linalg.solve(Lc, x - mean)
    return -0.5 * y @ y - np.sum(np.log(np.diag(Lc))) - 0.5 * x.size * LN2PI


def dense_joint(prep: Prepared, x, h=None):
    """log p at one point from the dense Gaussian identity (tiny inputs only).

    ``h``: the deterministic delay over all TOAs (zeros if None)."""
    T = _transform(prep, x)
    Phi, v, P = _design(prep, T)
    dt = np.concatenate([p["dt"] for p in prep.psr])
    N = np.concatenate([p["N"] for p in prep.psr])
    if h is None:
        h = np.zeros_like(dt)
    Cov = np.diag(N) + Phi @ P @ Phi.T
    marg = _lognormal(dt, h, Cov)
    Ninv = 1.0 / N
    Sinv = Phi.T @ (Ninv[:, None] * Phi) + np.linalg.inv(P)
    S = np.linalg.inv(Sinv)
    S = 0.5 * (S + S.T)
    m = S @ (Phi.T @ (Ninv * (dt - h)))
    cond = _lognormal(v, m, S)
    n = prep.n_psr
    logdetA = 3 * n * np.log(prep.sigma_b)
    logdetA += sum(2.0 * np.sum(np.log(np.diag(Lk))) for Lk in T["Ls"])
    if prep.Kdm:
        logdetA += np.sum(np.log(np.repeat(np.sqrt(T["kdm"]), 2, axis=1)))
    prior = -np.sum(np.log(prep.hi - prep.lo))
    return marg + cond + logdetA + prior


def gram_loglike(prep: Prepared, x):
    """Log-likelihood in the compressed (Gram) form, h = 0."""
    T = _transform(prep, x)
    out = 0.0
    for I, p in enumerate(prep.psr):
        Ft = np.concatenate([p["F"], p["w"][:, None] * p["Fdm"]], axis=1)
        at = np.concatenate([T["a"][I], T["adm"][I]])
        Ninv = 1.0 / p["N"]
        d1 = p["dt"] - p["M"] @ T["b"][I]
        FNF = Ft.T @ (Ninv[:, None] * Ft)           # computed once per data set
        FNd = Ft.T @ (Ninv * d1)
        out += (-0.5 * d1 @ (Ninv * d1) + FNd @ at - 0.5 * at @ FNF @ at
                - 0.5 * np.sum(np.log(p["N"]) + LN2PI))
    return out


def posterior_moments(prep: Prepared, theta, dt=None):
    """Closed-form Gaussian posterior N(m, S) of w = (u, z, z_dm) at fixed
    hyper-parameters (no CW): the linear-Gaussian case used to check HMC."""
    lay = prep.lay
    x = np.zeros(lay.d)
    x[: lay.n_theta] = theta
    T = _transform(prep, x)
    n, K, Kdm = prep.n_psr, prep.K, prep.Kdm
    Phi, _, _ = _design(prep, T)
    # v = A w with A = blockdiag(sigma_b I, L_full, sqrt(kdm))
    nb, na, nd = 3 * n, 2 * K * n, 2 * Kdm * n
    A = np.zeros((nb + na + nd, nb + na + nd))
    A[:nb, :nb] = prep.sigma_b * np.eye(nb)
    for k in range(K):
        for c in range(2):
            idx = np.array([nb + I * 2 * K + 2 * k + c for I in range(n)])
            A[np.ix_(idx, idx)] = T["Ls"][k]
    if nd:
        A[nb + na:, nb + na:] = np.diag(np.repeat(np.sqrt(T["kdm"]), 2, axis=1).reshape(-1))
    G = Phi @ A
    N = np.concatenate([p["N"] for p in prep.psr])
    if dt is None:
        dt = np.concatenate([p["dt"] for p in prep.psr])
    Sinv = G.T @ (G / N[:, None]) + np.eye(G.shape[1])
    S = np.linalg.inv(Sinv)
    S = 0.5 * (S + S.T)
    m = S @ (G.T @ (dt / N))
    return m, S
