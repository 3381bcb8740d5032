"""Oracle: whitened Fourier-space PTA log-posterior and its gradient (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed, per parameter vector x (Sec. IV with the whitening
a = L(eta) z of Sec. II.B, Eq. standardizing_transform, taken with mu = 0 and
Sigma = phi):

  spectra     rho_k  = P(f_k; gw),  kappa_Ik = P(f_k; rn_I),  kdm_Ik = P(f_k; dm_I)
              P(f; log10A, gamma) = A^2/(12 pi^2) yr^3 (f yr)^-gamma / T
              (Eq. power_law, read with yr^3 so that rho has units s^2)
  correlation Gamma_IJ = 3/2 b ln b - b/4 + 1/2 + 1/2 delta_IJ, b = (1-cos)/2
              (Eq. HD; b ln b -> 0 at b = 0)
  prior cov   phi_k = rho_k Gamma + diag(kappa_.k)            (Eq. prior_cov)
  transform   L_k = chol(phi_k);  a_.k,sin = L_k z_.k,sin;  a_.k,cos = L_k z_.k,cos
              a_dm = sqrt(kdm) z_dm;  b = sigma_b u
  residual    r = dt - M b - F a - w F a_dm - h(theta_cw)
              M = [1, tau, tau^2], tau = (t - c_I)/s_I (mid-point, half span)
              F columns sin/cos(2 pi k t / T), k = 1..K, interleaved
              (Eqs. Fourier_series, RN=Fa); w = dm_scale / nu^2 (F_DM of Sec. III.C)
  likelihood  log L = -1/2 sum_i (r_i^2/N_i + ln N_i + ln 2 pi),
              N_i = (EFAC sigma_i)^2 + EQUAD^2          (Eqs. likelihood, WN_cov)
  posterior   log p = log L - 1/2(|z|^2 + |z_dm|^2 + |u|^2) - d_z/2 ln 2 pi
                      + sum_theta ln 1/(hi - lo)   (uniform hyper-priors, Sec. IV.A)

The gradient is a hand-derived adjoint: with g = r/N,
  dlogL/da = F^T g, dlogL/da_dm = F^T (w g), dlogL/db = M^T g, dlogL/dh = g,
and the per-frequency Cholesky is differentiated with
  phibar = sym(L^-T Phi(L^T Lbar) L^-1),  Lbar = sum_c abar_c z_c^T,
  Phi(X) = lower triangle of X with its diagonal halved,
so that dlogp/drho_k = <phibar_k, Gamma> and dlogp/dkappa_Ik = phibar_k,II.

Per-chain conditions give log p = -inf, gradient 0 and a status:
  1 hyper-parameter outside the prior box, 2 phi_k not positive definite,
  3 CW evolution variable y >= 1 inside the span, 4 non-finite input/output.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

from . import cw as cwmod

YR = 365.25 * 86400.0
LN10 = np.log(10.0)
LN2PI = np.log(2.0 * np.pi)

ST_OK, ST_PRIOR, ST_NOTPD, ST_CW, ST_NONFINITE = 0, 1, 2, 3, 4


def powerlaw(f, log10A, gamma, tspan):
    """Eq. power_law: variance of one Fourier coefficient at frequency f."""
    return 10.0 ** (2.0 * log10A) / (12.0 * np.pi ** 2) * YR ** 3 * (f * YR) ** (-gamma) / tspan


def hd_matrix(pos):
    """Eq. HD: Hellings-Downs correlation of unit vectors ``pos`` (n, 3)."""
    n = pos.shape[0]
    G = np.empty((n, n))
    for I in range(n):
        for J in range(n):
            if I == J:
                G[I, J] = 1.0
                continue
            b = 0.5 * (1.0 - float(np.dot(pos[I], pos[J])))
            blnb = b * np.log(b) if b > 0.0 else 0.0
            G[I, J] = 1.5 * blnb - 0.25 * b + 0.5
    return G


class Layout:
    """Flat parameter vector layout:
    [gw(2) | rn(2 Np) | dm(2 Np) | cw(8) | u(3 Np) | z(Np*2K) | z_dm(Np*2Kdm)],
    absent processes have zero width; z is pulsar-major, per pulsar ordered
    k=1 sin, k=1 cos, k=2 sin, ... (the coefficient order a = [a1, b1, ...]
    of Eq. RN=Fa)."""

    def __init__(self, n_psr, nf_rn, nf_gw, nf_dm, has_cw):
        self.n_psr = n_psr
        self.K = max(nf_rn, nf_gw)
        self.Kdm = nf_dm
        o = 0
        self.gw = o; o += 2 if nf_gw > 0 else 0
        self.rn = o; o += 2 * n_psr if nf_rn > 0 else 0
        self.dm = o; o += 2 * n_psr if nf_dm > 0 else 0
        self.cw = o; o += 8 if has_cw else 0
        self.n_theta = o
        self.u = o; o += 3 * n_psr
        self.z = o; o += n_psr * 2 * self.K
        self.zdm = o; o += n_psr * 2 * self.Kdm
        self.d = o


class Prepared:
    """Dense per-pulsar design matrices and constants of one data set."""

    def __init__(self, ds):
        self.ds = ds
        self.n_psr = n = int(ds["n_psr"])
        self.nf_rn, self.nf_gw, self.nf_dm = int(ds["nf_rn"]), int(ds["nf_gw"]), int(ds["nf_dm"])
        self.has_cw = bool(ds["has_cw"])
        self.lay = Layout(n, self.nf_rn, self.nf_gw, self.nf_dm, self.has_cw)
        self.K, self.Kdm = self.lay.K, self.lay.Kdm
        self.T = float(ds["tspan"])
        self.freqs = np.arange(1, max(self.K, self.Kdm) + 1) / self.T
        self.Gamma = hd_matrix(np.asarray(ds["psr_pos"], np.float64))
        self.lo = np.asarray(ds["prior_lo"], np.float64)
        self.hi = np.asarray(ds["prior_hi"], np.float64)
        self.sigma_b = float(ds["sigma_b"])
        off = np.asarray(ds["toa_offsets"], np.int64)
        t = np.asarray(ds["t"], np.float64)
        self.tmax = float(t.max()) if t.size else 0.0
        self.psr = []
        for I in range(n):
            s, e = int(off[I]), int(off[I + 1])
            tt = t[s:e]
            if tt.size:
                c = 0.5 * (tt.min() + tt.max())
                hs = 0.5 * (tt.max() - tt.min())
            else:
                c, hs = 0.0, 1.0
            if hs == 0.0:
                hs = 1.0                      # single-TOA pulsar: tau = 0
            tau = (tt - c) / hs
            M = np.stack([np.ones_like(tau), tau, tau * tau], axis=1)
            kk = np.arange(1, max(self.K, self.Kdm) + 1)
            arg = 2.0 * np.pi * np.outer(tt, kk) / self.T
            Ffull = np.empty((tt.size, 2 * kk.size))
            Ffull[:, 0::2] = np.sin(arg)
            Ffull[:, 1::2] = np.cos(arg)
            be = np.asarray(ds["backend"][s:e], np.int64)
            sig = np.asarray(ds["sigma"][s:e], np.float64)
            N = (ds["efac"][be] * sig) ** 2 + ds["equad"][be] ** 2
            w = ds["dm_scale"] / np.asarray(ds["nu"][s:e], np.float64) ** 2
            self.psr.append(dict(
                t=tt, dt=np.asarray(ds["dt"][s:e], np.float64), M=M,
                F=Ffull[:, : 2 * self.K], Fdm=Ffull[:, : 2 * self.Kdm],
                N=N, w=w, pos=np.asarray(ds["psr_pos"][I], np.float64)))

    # ------------------------------------------------------------------
    def split(self, x):
        L = self.lay
        n = self.n_psr
        th = x[:, : L.n_theta]
        gw = th[:, L.gw:L.gw + 2] if self.nf_gw > 0 else None
        rn = th[:, L.rn:L.rn + 2 * n].reshape(x.shape[0], n, 2) if self.nf_rn > 0 else None
        dm = th[:, L.dm:L.dm + 2 * n].reshape(x.shape[0], n, 2) if self.nf_dm > 0 else None
        cw = th[:, L.cw:L.cw + 8] if self.has_cw else None
        C = x.shape[0]
        u = x[:, L.u:L.u + 3 * n].reshape(C, n, 3)
        z = x[:, L.z:L.z + n * 2 * self.K].reshape(C, n, 2 * self.K)
        zdm = x[:, L.zdm:L.zdm + n * 2 * self.Kdm].reshape(C, n, 2 * self.Kdm)
        return gw, rn, dm, cw, u, z, zdm

    def spectra(self, gw, rn, dm, C):
        """rho (C, K), kappa (C, Np, K), kdm (C, Np, Kdm) and the frequencies."""
        n, K, Kdm = self.n_psr, self.K, self.Kdm
        f = self.freqs
        rho = np.zeros((C, K))
        kap = np.zeros((C, n, K))
        kdm = np.zeros((C, n, Kdm))
        if self.nf_gw > 0:
            kg = self.nf_gw
            rho[:, :kg] = powerlaw(f[None, :kg], gw[:, 0:1], gw[:, 1:2], self.T)
        if self.nf_rn > 0:
            kr = self.nf_rn
            kap[:, :, :kr] = powerlaw(f[None, None, :kr], rn[:, :, 0:1], rn[:, :, 1:2], self.T)
        if self.nf_dm > 0:
            kdm[:, :, :] = powerlaw(f[None, None, :Kdm], dm[:, :, 0:1], dm[:, :, 1:2], self.T)
        return rho, kap, kdm


def _tril_half(X):
    """Phi(X): lower triangle with the diagonal halved."""
    Y = np.tril(X)
    Y[np.diag_indices_from(Y)] *= 0.5
    return Y


def chol_backward(L, Lbar):
    """Symmetric adjoint phibar of phi = L L^T given Lbar = d f / d L."""
    P = _tril_half(L.T @ Lbar)
    X = solve_triangular(L, P, trans="T", lower=True)          # L^-T P
    S = solve_triangular(L, X.T, trans="T", lower=True).T      # (L^-T P) L^-1
    return 0.5 * (S + S.T)


def logp_grad(prep: Prepared, x, with_scale=True):
    """log p, its gradient, a per-chain status and per-element magnitude
    companions (the same sums taken over absolute values of every term).

    ``x``: (C, d) or (d,).  Returns a dict of arrays with a leading C axis.
    """
    x = np.array(x, dtype=np.float64, copy=True)
    if x.ndim == 1:
        x = x[None, :]
    C, d = x.shape
    lay = prep.lay
    assert d == lay.d, (d, lay.d)
    n, K, Kdm = prep.n_psr, prep.K, prep.Kdm
    status = np.zeros(C, dtype=np.int32)

    # ---- per-chain input checks -------------------------------------
    th = x[:, : lay.n_theta]
    inbox = np.all((th >= prep.lo) & (th <= prep.hi), axis=1) & np.all(np.isfinite(th), axis=1)
    status[~inbox] = ST_PRIOR
    bad_rest = ~np.all(np.isfinite(x[:, lay.n_theta:]), axis=1)
    status[(status == 0) & bad_rest] = ST_NONFINITE
    work = x.copy()
    mid = 0.5 * (prep.lo + prep.hi)
    for c in np.nonzero(status)[0]:
        work[c, : lay.n_theta] = mid
        work[c, lay.n_theta:] = 0.0
    if prep.has_cw:
        for c in range(C):
            if status[c] == 0 and cwmod.max_y(work[c, lay.cw:lay.cw + 8], prep.tmax) >= 1.0:
                status[c] = ST_CW
                work[c, : lay.n_theta] = mid
                work[c, lay.n_theta:] = 0.0

    gw, rn, dm, cwp, u, z, zdm = prep.split(work)
    rho, kap, kdm = prep.spectra(gw, rn, dm, C)
    Gam = prep.Gamma

    # ---- per-frequency transform a = L_k z -------------------------
    Ls = np.zeros((C, K, n, n))
    a = np.zeros((C, n, 2 * K))
    for c in range(C):
        for k in range(K):
            phi = rho[c, k] * Gam + np.diag(kap[c, :, k])
            try:
                Lk = np.linalg.cholesky(phi)
            except np.linalg.LinAlgError:
                Lk = None
            if Lk is None or not np.all(np.isfinite(Lk)) or np.any(np.diag(Lk) <= 0.0):
                if status[c] == 0:
                    status[c] = ST_NOTPD
                Lk = np.eye(n)
            Ls[c, k] = Lk
            a[c, :, 2 * k] = Lk @ z[c, :, 2 * k]
            a[c, :, 2 * k + 1] = Lk @ z[c, :, 2 * k + 1]
    sq_kdm = np.sqrt(kdm)                                  # (C, n, Kdm)
    adm = np.repeat(sq_kdm, 2, axis=2) * zdm               # (C, n, 2Kdm)
    b = prep.sigma_b * u                                   # (C, n, 3)

    # ---- TOA pass --------------------------------------------------
    logL = np.zeros(C)
    abar = np.zeros((C, n, 2 * K))
    abar_dm = np.zeros((C, n, 2 * Kdm))
    ubar = np.zeros((C, n, 3))
    cwbar = np.zeros((C, 8))
    # magnitude companions
    s_abar = np.zeros((C, n, 2 * K))
    s_abar_dm = np.zeros((C, n, 2 * Kdm))
    s_ubar = np.zeros((C, n, 3))
    s_cw = np.zeros((C, 8))
    s_logp = np.zeros(C)
    for I, P in enumerate(prep.psr):
        F, Fdm, M, N, w = P["F"], P["Fdm"], P["M"], P["N"], P["w"]
        tm = M @ b[:, I, :].T                               # (nI, C)
        R = F @ a[:, I, :].T
        Rdm = w[:, None] * (Fdm @ adm[:, I, :].T)
        h = np.zeros_like(R)
        dh = None
        if prep.has_cw:
            dh = []
            for c in range(C):
                hc, gc = cwmod.delay(P["t"], P["pos"], cwp[c], want_grad=True)
                h[:, c] = hc
                dh.append(gc)
        r = P["dt"][:, None] - tm - R - Rdm - h
        g = r / N[:, None]
        logL += -0.5 * np.sum(r * g + np.log(N)[:, None] + LN2PI, axis=0)
        abar[:, I, :] = (F.T @ g).T
        abar_dm[:, I, :] = (Fdm.T @ (w[:, None] * g)).T
        ubar[:, I, :] = prep.sigma_b * (M.T @ g).T
        if with_scale:
            sr = (np.abs(P["dt"])[:, None] + np.abs(M) @ np.abs(b[:, I, :]).T
                  + np.abs(F) @ np.abs(a[:, I, :]).T
                  + w[:, None] * (np.abs(Fdm) @ np.abs(adm[:, I, :]).T) + np.abs(h))
            sg = sr / N[:, None]
            s_abar[:, I, :] = (np.abs(F).T @ sg).T
            s_abar_dm[:, I, :] = (np.abs(Fdm).T @ (w[:, None] * sg)).T
            s_ubar[:, I, :] = prep.sigma_b * (np.abs(M).T @ sg).T
            s_logp += 0.5 * np.sum(np.abs(r * g) + np.abs(np.log(N))[:, None] + LN2PI, axis=0)
        if prep.has_cw:
            for c in range(C):
                cwbar[c] += g[:, c] @ dh[c]
                if with_scale:
                    s_cw[c] += sg[:, c] @ np.abs(dh[c])

    # ---- prior terms -----------------------------------------------
    dz = n * 2 * K + n * 2 * Kdm + 3 * n
    prior_const = -np.sum(np.log(prep.hi - prep.lo))
    zz = np.sum(z.reshape(C, -1) ** 2, 1) + np.sum(zdm.reshape(C, -1) ** 2, 1) + np.sum(u.reshape(C, -1) ** 2, 1)
    logp = logL - 0.5 * zz - 0.5 * dz * LN2PI + prior_const
    s_logp += 0.5 * zz + 0.5 * dz * LN2PI + abs(prior_const)

    # ---- gradient --------------------------------------------------
    grad = np.zeros((C, d))
    scale = np.zeros((C, d))
    gz = np.zeros((C, n, 2 * K))
    sz = np.zeros((C, n, 2 * K))
    drho = np.zeros((C, K))
    dkap = np.zeros((C, n, K))
    s_drho = np.zeros((C, K))
    s_dkap = np.zeros((C, n, K))
    for c in range(C):
        for k in range(K):
            Lk = Ls[c, k]
            A2 = abar[c, :, 2 * k:2 * k + 2]               # (n, 2): sin, cos
            Z2 = z[c, :, 2 * k:2 * k + 2]
            gz[c, :, 2 * k:2 * k + 2] = Lk.T @ A2 - Z2
            Lbar = A2 @ Z2.T
            phibar = chol_backward(Lk, Lbar)
            drho[c, k] = np.sum(phibar * Gam)
            dkap[c, :, k] = np.diag(phibar)
            if with_scale:
                SA2 = s_abar[c, :, 2 * k:2 * k + 2]
                sz[c, :, 2 * k:2 * k + 2] = np.abs(Lk).T @ SA2 + np.abs(Z2)
                Linv = solve_triangular(Lk, np.eye(n), lower=True)
                Pm = _tril_half(np.abs(Lk).T @ (SA2 @ np.abs(Z2).T))
                Sm = np.abs(Linv).T @ Pm @ np.abs(Linv)
                Sm = 0.5 * (Sm + Sm.T)
                s_drho[c, k] = np.sum(Sm * np.abs(Gam))
                s_dkap[c, :, k] = np.diag(Sm)
    lnfy = np.log(prep.freqs * YR)                        # ln(f_k yr)
    if prep.nf_gw > 0:
        kg = prep.nf_gw
        grad[:, lay.gw + 0] = np.sum(drho[:, :kg] * rho[:, :kg], 1) * 2.0 * LN10
        grad[:, lay.gw + 1] = np.sum(drho[:, :kg] * rho[:, :kg] * (-lnfy[None, :kg]), 1)
        scale[:, lay.gw + 0] = np.sum(s_drho[:, :kg] * rho[:, :kg], 1) * 2.0 * LN10
        scale[:, lay.gw + 1] = np.sum(s_drho[:, :kg] * rho[:, :kg] * np.abs(lnfy[None, :kg]), 1)
    if prep.nf_rn > 0:
        kr = prep.nf_rn
        t0 = np.sum(dkap[:, :, :kr] * kap[:, :, :kr], 2) * 2.0 * LN10
        t1 = np.sum(dkap[:, :, :kr] * kap[:, :, :kr] * (-lnfy[None, None, :kr]), 2)
        grad[:, lay.rn:lay.rn + 2 * n] = np.stack([t0, t1], 2).reshape(C, -1)
        s0 = np.sum(s_dkap[:, :, :kr] * kap[:, :, :kr], 2) * 2.0 * LN10
        s1 = np.sum(s_dkap[:, :, :kr] * kap[:, :, :kr] * np.abs(lnfy[None, None, :kr]), 2)
        scale[:, lay.rn:lay.rn + 2 * n] = np.stack([s0, s1], 2).reshape(C, -1)
    if prep.nf_dm > 0:
        # a_dm = sqrt(kdm) z_dm: d sqrt(kdm)/d log10A = ln10 sqrt(kdm),
        # d sqrt(kdm)/d gamma = -1/2 ln(f yr) sqrt(kdm)
        az = (abar_dm * zdm).reshape(C, n, Kdm, 2).sum(3) * sq_kdm      # (C, n, Kdm)
        saz = (s_abar_dm * np.abs(zdm)).reshape(C, n, Kdm, 2).sum(3) * sq_kdm
        t0 = np.sum(az, 2) * LN10
        t1 = np.sum(az * (-0.5 * lnfy[None, None, :Kdm]), 2)
        grad[:, lay.dm:lay.dm + 2 * n] = np.stack([t0, t1], 2).reshape(C, -1)
        s0 = np.sum(saz, 2) * LN10
        s1 = np.sum(saz * np.abs(0.5 * lnfy[None, None, :Kdm]), 2)
        scale[:, lay.dm:lay.dm + 2 * n] = np.stack([s0, s1], 2).reshape(C, -1)
    if prep.has_cw:
        grad[:, lay.cw:lay.cw + 8] = cwbar
        scale[:, lay.cw:lay.cw + 8] = s_cw
    grad[:, lay.u:lay.u + 3 * n] = (ubar - u).reshape(C, -1)
    scale[:, lay.u:lay.u + 3 * n] = (s_ubar + np.abs(u)).reshape(C, -1)
    grad[:, lay.z:lay.z + n * 2 * K] = gz.reshape(C, -1)
    scale[:, lay.z:lay.z + n * 2 * K] = sz.reshape(C, -1)
    gzdm = np.repeat(sq_kdm, 2, axis=2) * abar_dm - zdm
    szdm = np.repeat(sq_kdm, 2, axis=2) * s_abar_dm + np.abs(zdm)
    grad[:, lay.zdm:lay.zdm + n * 2 * Kdm] = gzdm.reshape(C, -1)
    scale[:, lay.zdm:lay.zdm + n * 2 * Kdm] = szdm.reshape(C, -1)

    # ---- per-chain conditions --------------------------------------
    fin = np.isfinite(logp) & np.all(np.isfinite(grad), axis=1)
    status[(status == 0) & ~fin] = ST_NONFINITE
    bad = status != 0
    logp[bad] = -np.inf
    grad[bad] = 0.0
    scale[bad] = 0.0
    s_logp[bad] = 0.0
    return dict(logp=logp, grad=grad, status=status, scale=scale, logp_scale=s_logp)
