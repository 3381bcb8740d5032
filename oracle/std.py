"""Oracle: the paper's standardized posterior (CURN standardizing transform)
with the timing model marginalised (FP64, PyTorch on the CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed, per parameter vector x = [theta | z] (Sec. IV.B):

  timing model  N~^-1 = G (G^T N G)^-1 G^T with G an orthonormal basis of the
                complement of the timing-model columns (Eq. Gmatrix_proj; G
                from the QR decomposition of M, the paper's alternative).
                M is the stored design matrix of the pulsar, or [1, tau, tau^2];
                linearly dependent columns are dropped by a column-pivoted QR.
  likelihood    log L(a) = -1/2 (dt - T a)^T N~^-1 (dt - T a)
                           - 1/2 ln det(2 pi G^T N G)
                per pulsar, T = [F, w F_dm] (Eqs. likelihood, raw_posterior,
                with every constant kept), written in the Gram form of
                Eq. posterior_implemented:
                -1/2 c + a^T d - 1/2 a^T S0 a - 1/2 ln det(2 pi G^T N G),
                S0 = T^T N~^-1 T, d = T^T N~^-1 dt, c = dt^T N~^-1 dt.
  prior         a ~ N(0, phi), phi per frequency rho_k Gamma + diag kappa_.k
                (Eqs. prior_cov, HD, power_law), DM diagonal kappa_dm.
  CURN factor   phi_CURN,I = diag(rho_k + kappa_Ik, ..., kappa_dm,Ik, ...)
                Sigma_I = (beta S0_I + phi_CURN,I^-1)^-1, L_I = chol(Sigma_I)
                (lower Cholesky factor), a_hat_I = beta Sigma_I d_I
                (Eqs. PTA_standard_transform_curn, and mv_normal_post_temp of
                App. B for the tempered likelihood p(dt|a)^beta).
  transform     a_I = a_hat_I + L_I z_I
  density       log p~ = beta log L(a) + log N(a; 0, phi) + sum_I ln det L_I
                         + log pi(theta)
                (Eq. standardized_stochastic_posterior with the Jacobian and
                the constants the paper drops put back).

Deterministic signal (Sec. IV.C, Eqs. det_F_basis, stoch_det_posterior,
det_mean, decenter_det_PTA, standardized_det_posterior), when the data set
has a CW: h = F_D a_D(theta_cw) per pulsar, F_D the sin/cos basis of
frequencies k / T_D, k = 1..K_D, on an extended span T_D, and a_D the
discrete Fourier transform of the time-domain CW delay (the Earth-term
waveform of cw.py) sampled at M = 2 K_D + 1 equally spaced times
t_j = j T_D / M: a_(k,sin) = (2/M) sum_j h_j sin(2 pi k j / M),
a_(k,cos) = (2/M) sum_j h_j cos(2 pi k j / M) (the mean of the samples, the
constant the timing model absorbs, is dropped).  With the stored products
S_D = T^T N~^-1 F_D, e_D = F_D^T N~^-1 dt, Q_D = F_D^T N~^-1 F_D the data
enter through
  d_bar = d - S_D a_D = T^T N~^-1 (dt - h),
  c_bar = c - 2 e_D^T a_D + a_D^T Q_D a_D = (dt - h)^T N~^-1 (dt - h),
so the transform centres on a_bar = beta Sigma d_bar (the shifted MAP of
Eq. det_mean) and the likelihood is the one of dt - h.  Status 3 when the CW
coalesces within [0, T_D) (evolution variable y >= 1 at a sample time).

Split coefficients (App. C, Eqs. separated_post, split_map_a,
split_standardizing_transform), when the data set asks for them: the common
process and the pulsar's own noise get separate coefficient sets on the same
basis, a_G (k = 1..K_gw) and a_R (k = 1..K_rn, then the DM block), with
a = E_G a_G + E_R a_R in the likelihood, priors a_G,k ~ N(0, rho_k Gamma) per
frequency and a_R ~ N(0, diag kappa), and
  Sigma_G = (beta S0_GG + diag rho^-1)^-1 = L_G L_G^T   (CURN: Gamma = I)
  Sigma_R = (beta S0_RR + diag phi_R^-1)^-1 = L_R L_R^T
  a_G = a_hat_G + L_G z_G,  a_R = a_hat_R + L_R z_R,
with (a_hat_G, a_hat_R) the MAP of the joint system of Eq. split_map_a under
the CURN prior.  Both sets share the basis, so that system is solved by the
CURN MAP of the combined coefficients a_hat = (beta S0 + D^-1)^-1 beta d,
D = rho + kappa, split in proportion to the prior variances:
a_hat_G = rho / D a_hat, a_hat_R = phi_R / D a_hat (the pins check this
against a direct solve of the joint system).  z per pulsar is [z_G | z_R].

Spectra are the power law of Eq. power_law (theta = log10 A, gamma per
process) or the free spectrum of Sec. IV.A (theta = log10 rho_k per
frequency, rho_k = 10^theta_k in s^2).  Uniform hyper-priors.

The gradient is PyTorch autograd of this plain definition (library
Cholesky, inverse and triangular solves), so it needs no hand derivation.
Per-chain conditions: 1 outside the prior box or non-finite theta,
2 a factorisation fails or a CURN variance is not positive and finite (a
prior covariance that is not positive definite), 3 the CW coalesces within
the extended span, 4 non-finite z or result (precedence 1, 4 for inputs, 3,
2, 4 for results).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import torch

from . import cw as cwmod
from .model import YR, hd_matrix

LN2PI = float(np.log(2.0 * np.pi))
ST_OK, ST_PRIOR, ST_NOTPD, ST_CW, ST_NONFINITE = 0, 1, 2, 3, 4


class NotPositiveDefinite(Exception):
    """A prior covariance of the transform is not positive definite."""


class StdLayout:
    """[theta | z]: theta = [gw | rn per pulsar | dm per pulsar | cw (8)],
    each process 2 entries (power law: log10 A, gamma) or one per frequency
    (free spectrum: log10 rho_k), the CW parameters in the order of cw.py;
    z per pulsar: 2 Ka entries (k = 1 sin, k = 1 cos, ...) for the
    red/common block, then 2 Kdm for DM."""

    def __init__(self, n_psr, nf_rn, nf_gw, nf_dm, free, has_cw=False, split=False):
        self.n_psr, self.nf_rn, self.nf_gw, self.nf_dm, self.free = n_psr, nf_rn, nf_gw, nf_dm, free
        self.has_cw = bool(has_cw)
        self.split = bool(split)
        if self.split and (nf_gw < 1 or nf_rn < 1):
            raise ValueError("split coefficients need a common process and pulsar red noise")
        self.Ka = max(nf_rn, nf_gw)
        self.Kdm = nf_dm
        self.P = 2 * self.Ka + 2 * self.Kdm     # combined coefficients (the likelihood's)
        # z per pulsar: the combined set, or [z_G (2 K_gw) | z_R (2 K_rn + 2 K_dm)]
        self.PG = 2 * nf_gw if self.split else 0
        self.PR = 2 * nf_rn + 2 * nf_dm if self.split else 0
        self.Pz = self.PG + self.PR if self.split else self.P
        w = (lambda k: k) if free else (lambda k: 2)
        o = 0
        self.gw = o; o += w(nf_gw) if nf_gw > 0 else 0
        self.rn = o; o += n_psr * w(nf_rn) if nf_rn > 0 else 0
        self.dm = o; o += n_psr * w(nf_dm) if nf_dm > 0 else 0
        self.cw = o; o += 8 if has_cw else 0
        self.n_theta = o
        self.z = o; o += n_psr * self.Pz
        self.d = o
        self.w_gw = w(nf_gw) if nf_gw > 0 else 0
        self.w_rn = w(nf_rn) if nf_rn > 0 else 0
        self.w_dm = w(nf_dm) if nf_dm > 0 else 0


def _rank_columns(M, tol=1e-12):
    """Indices of a linearly independent subset of M's columns (column-pivoted
    QR of the column-normalised matrix, pivots above tol of the largest)."""
    if M.shape[1] == 0:
        return np.zeros(0, np.int64)
    nrm = np.linalg.norm(M, axis=0)
    keep = np.nonzero(nrm > 0)[0]
    if keep.size == 0:
        return keep
    Ms = M[:, keep] / nrm[keep]
    _, R, piv = sla.qr(Ms, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    r = int(np.sum(d > tol * d[0]))
    return np.sort(keep[piv[:r]])


def projection(M, N, explicit):
    """N~^-1 as a function X -> N~^-1 X, and ln det(G^T N G), n - r.

    explicit=True builds G from the complete QR of the independent columns of
    M (Eq. Gmatrix_proj with Q_2); otherwise the same operator through
    N^-1 - N^-1 M (M^T N^-1 M)^-1 M^T N^-1 and
    ln det(G^T N G) = ln det N + ln det(M^T N^-1 M) - ln det(M^T M)
    (equal when G is orthonormal and the columns independent; tests pin the
    two against each other)."""
    cols = _rank_columns(M)
    Mr = M[:, cols]
    n, r = M.shape[0], cols.size
    if explicit:
        if r:
            Q, _ = np.linalg.qr(Mr, mode="complete")
            G = Q[:, r:]
        else:
            G = np.eye(n)
        GNG = G.T @ (N[:, None] * G)
        Lg = np.linalg.cholesky(GNG)
        logdet = 2.0 * np.sum(np.log(np.diag(Lg)))

        def apply(X):
            Y = sla.cho_solve((Lg, True), G.T @ X)
            return G @ Y
        return apply, logdet, n - r
    Ni = 1.0 / N
    if r:
        MNM = Mr.T @ (Ni[:, None] * Mr)
        Lm = np.linalg.cholesky(MNM)
        Lmm = np.linalg.cholesky(Mr.T @ Mr)
    logdet = float(np.sum(np.log(N)))
    if r:
        logdet += 2.0 * np.sum(np.log(np.diag(Lm))) - 2.0 * np.sum(np.log(np.diag(Lmm)))

    def apply(X):
        Y = Ni.reshape((-1,) + (1,) * (X.ndim - 1)) * X
        if r:
            Y = Y - Ni.reshape((-1,) + (1,) * (X.ndim - 1)) * (Mr @ sla.cho_solve((Lm, True), Mr.T @ Y))
        return Y
    return apply, logdet, n - r


class StdPrepared:
    """Per-pulsar Gram quantities of one data set (computed once, as the
    paper stores them), the HD matrix and the prior box."""

    def __init__(self, ds, explicit=None):
        self.ds = ds
        n = self.n_psr = int(ds["n_psr"])
        self.free = ds.get("spectrum", "powerlaw") == "free"
        self.has_cw = bool(ds.get("has_cw", 0))
        self.split = bool(ds.get("split", 0))
        self.lay = StdLayout(n, int(ds["nf_rn"]), int(ds["nf_gw"]), int(ds["nf_dm"]), self.free, self.has_cw,
                             self.split)
        lay = self.lay
        self.T = float(ds["tspan"])
        self.pos = np.asarray(ds["psr_pos"], np.float64).reshape(n, 3)
        if self.has_cw:
            self.Kd = int(ds.get("cw_nf", 60))
            self.Td = float(ds.get("cw_tspan", 2.0 * self.T))
            self.Md = 2 * self.Kd + 1
            self.ts_d = np.arange(self.Md) * self.Td / self.Md
            jk = 2.0 * np.pi * np.outer(np.arange(1, self.Kd + 1), np.arange(self.Md)) / self.Md
            self.dft = np.empty((2 * self.Kd, self.Md))
            self.dft[0::2] = (2.0 / self.Md) * np.sin(jk)
            self.dft[1::2] = (2.0 / self.Md) * np.cos(jk)
            self.SD, self.eD, self.QD, self.GabsD = [], [], [], []
        self.freqs = np.arange(1, max(lay.Ka, lay.Kdm, 1) + 1) / self.T
        self.Gamma = hd_matrix(np.asarray(ds["psr_pos"], np.float64))
        self.lo = np.asarray(ds["prior_lo"], np.float64)
        self.hi = np.asarray(ds["prior_hi"], np.float64)
        off = np.asarray(ds["toa_offsets"], np.int64)
        t_all = np.asarray(ds["t"], np.float64)
        tm = ds.get("tm")
        self.S0, self.dvec, self.cval, self.const = [], [], [], []
        self.Gabs, self.dabs = [], []            # per-TOA absolute sums (tolerance companions)
        self.ntoa = []
        kk = np.arange(1, max(lay.Ka, lay.Kdm, 1) + 1)
        for I in range(n):
            s, e = int(off[I]), int(off[I + 1])
            tt = t_all[s:e]
            if tm is None:
                c = 0.5 * (tt.min() + tt.max())
                hs = 0.5 * (tt.max() - tt.min())
                hs = hs if hs > 0 else 1.0
                tau = (tt - c) / hs
                M = np.stack([np.ones_like(tau), tau, tau * tau], axis=1)
            else:
                M = np.asarray(tm, np.float64)[s:e]
            arg = 2.0 * np.pi * np.outer(tt, kk) / self.T
            F = np.empty((tt.size, 2 * kk.size))
            F[:, 0::2] = np.sin(arg)
            F[:, 1::2] = np.cos(arg)
            w = float(ds["dm_scale"]) / np.asarray(ds["nu"][s:e], np.float64) ** 2
            Tm = np.concatenate([F[:, : 2 * lay.Ka], w[:, None] * F[:, : 2 * lay.Kdm]], axis=1)
            be = np.asarray(ds["backend"][s:e], np.int64)
            N = (np.asarray(ds["efac"])[be] * np.asarray(ds["sigma"][s:e])) ** 2 + np.asarray(ds["equad"])[be] ** 2
            dt = np.asarray(ds["dt"][s:e], np.float64)
            ex = (e - s) <= 1500 if explicit is None else explicit
            apply, logdet, nprime = projection(M, N, ex)
            NT = apply(Tm)
            self.ntoa.append(e - s)
            At = np.abs(Tm) / N[:, None]
            self.Gabs.append(At.T @ np.abs(Tm))
            self.dabs.append(At.T @ np.abs(dt))
            self.S0.append(Tm.T @ NT)
            self.dvec.append(NT.T @ dt)
            self.cval.append(float(dt @ apply(dt)))
            self.const.append(-0.5 * (nprime * LN2PI + logdet))
            if self.has_cw:
                argd = 2.0 * np.pi * np.outer(tt, np.arange(1, self.Kd + 1)) / self.Td
                FD = np.empty((tt.size, 2 * self.Kd))
                FD[:, 0::2] = np.sin(argd)
                FD[:, 1::2] = np.cos(argd)
                NFD = apply(FD)
                self.SD.append(Tm.T @ NFD)
                self.eD.append(NFD.T @ dt)
                self.QD.append(FD.T @ NFD)
                self.GabsD.append(At.T @ np.abs(FD))

    def spectra(self, th):
        """rho (Ka), kappa (Np, Ka), kappa_dm (Np, Kdm) as torch tensors."""
        lay, n = self.lay, self.n_psr
        f = torch.tensor(self.freqs, dtype=torch.float64)
        lnfy = torch.log(f * YR)

        def pl(l10a, gam, K):
            return 10.0 ** (2.0 * l10a) / (12.0 * np.pi ** 2) * YR ** 3 * torch.exp(-gam * lnfy[:K]) / self.T

        zero = torch.zeros((), dtype=torch.float64)
        rho = torch.zeros(lay.Ka, dtype=torch.float64)
        if lay.nf_gw > 0:
            seg = th[lay.gw:lay.gw + lay.w_gw]
            r = 10.0 ** seg if self.free else pl(seg[0], seg[1], lay.nf_gw)
            rho = torch.cat([r, zero.repeat(lay.Ka - lay.nf_gw)])
        kap = torch.zeros((n, lay.Ka), dtype=torch.float64)
        if lay.nf_rn > 0:
            rows = []
            for I in range(n):
                seg = th[lay.rn + I * lay.w_rn: lay.rn + (I + 1) * lay.w_rn]
                r = 10.0 ** seg if self.free else pl(seg[0], seg[1], lay.nf_rn)
                rows.append(torch.cat([r, zero.repeat(lay.Ka - lay.nf_rn)]))
            kap = torch.stack(rows)
        kdm = torch.zeros((n, lay.Kdm), dtype=torch.float64)
        if lay.nf_dm > 0:
            rows = []
            for I in range(n):
                seg = th[lay.dm + I * lay.w_dm: lay.dm + (I + 1) * lay.w_dm]
                rows.append(10.0 ** seg if self.free else pl(seg[0], seg[1], lay.nf_dm))
            kdm = torch.stack(rows)
        return rho, kap, kdm

    def cw_coefficients(self, th):
        """a_D (Np, 2 K_D) of the CW at theta (torch, differentiable): the DFT
        of the delay sampled at t_j = j T_D / M (Eq. det_F_basis)."""
        H = _CWSamples.apply(th[self.lay.cw:self.lay.cw + 8], self)
        return H @ torch.tensor(self.dft.T)

    def data_terms(self, th):
        """d_bar_I and c_bar_I (the data minus the deterministic signal), or d, c."""
        n = self.n_psr
        if not self.has_cw:
            return [torch.tensor(self.dvec[I]) for I in range(n)], [self.cval[I] for I in range(n)]
        aD = self.cw_coefficients(th)
        dbar, cbar = [], []
        for I in range(n):
            v = aD[I]
            dbar.append(torch.tensor(self.dvec[I]) - torch.tensor(self.SD[I]) @ v)
            cbar.append(self.cval[I] - 2.0 * (torch.tensor(self.eD[I]) @ v) + v @ (torch.tensor(self.QD[I]) @ v))
        return dbar, cbar

    def transform(self, th, z, beta):
        """a (Np, P), sum_I ln det L_I, beta sum_I log L(a_I) for one point."""
        lay, n = self.lay, self.n_psr
        rho, kap, kdm = self.spectra(th)
        dbar, cbar = self.data_terms(th)
        a_all, jac, lik = [], 0.0, 0.0
        for I in range(n):
            D = torch.cat([(rho + kap[I]).repeat_interleave(2), kdm[I].repeat_interleave(2)])
            if not bool(torch.all(torch.isfinite(D) & (D > 0))):
                # a CURN variance of 0 or inf (a spectrum that underflows or
                # overflows): phi_CURN is not positive definite
                raise NotPositiveDefinite("CURN prior variance not positive and finite")
            S0 = torch.tensor(self.S0[I])
            d = dbar[I]
            A = beta * S0 + torch.diag(1.0 / D)
            Sig = torch.linalg.inv(A)
            Sig = 0.5 * (Sig + Sig.T)
            L = torch.linalg.cholesky(Sig)
            ahat = Sig @ (beta * d)
            a = ahat + L @ z[I]
            a_all.append(a)
            jac = jac + torch.sum(torch.log(torch.diagonal(L)))
            lik = lik + beta * (-0.5 * cbar[I] + a @ d - 0.5 * a @ (S0 @ a) + self.const[I])
        return torch.stack(a_all), jac, lik, (rho, kap, kdm)

    def split_rows(self):
        """Combined-row indices of the G set (k <= K_gw, sin/cos) and of the R
        set (k <= K_rn, then the DM block)."""
        lay = self.lay
        g = np.arange(2 * lay.nf_gw)
        r = np.concatenate([np.arange(2 * lay.nf_rn), 2 * lay.Ka + np.arange(2 * lay.Kdm)])
        return g, r

    def split_variances(self, I, spec):
        """D (combined rows), rho on the G rows, phi_R on the R rows of pulsar I."""
        lay = self.lay
        rho, kap, kdm = spec
        D = torch.cat([(rho + kap[I]).repeat_interleave(2), kdm[I].repeat_interleave(2)])
        g, r = self.split_rows()
        vg = rho[: lay.nf_gw].repeat_interleave(2)
        vr = torch.cat([kap[I, : lay.nf_rn].repeat_interleave(2), kdm[I].repeat_interleave(2)])
        for v in (D, vg, vr):
            if not bool(torch.all(torch.isfinite(v) & (v > 0))):
                raise NotPositiveDefinite("prior variance not positive and finite")
        return D, vg, vr

    def split_map(self, th, beta):
        """(a_hat_G, a_hat_R) per pulsar: the CURN MAP of the combined
        coefficients split in proportion to the prior variances."""
        spec = self.spectra(th)
        dbar, _ = self.data_terms(th)
        g, r = self.split_rows()
        out = []
        for I in range(self.n_psr):
            D, vg, vr = self.split_variances(I, spec)
            A = beta * torch.tensor(self.S0[I]) + torch.diag(1.0 / D)
            ah = torch.linalg.solve(A, beta * dbar[I])
            out.append((vg / D[g] * ah[g], vr / D[r] * ah[r]))
        return out

    def transform_split(self, th, z, beta):
        """Split sets: a (Np, P) combined, a_G (Np, PG), a_R (Np, PR), sum of
        ln det L_G + ln det L_R, beta sum_I log L(a_I)."""
        lay, n = self.lay, self.n_psr
        spec = self.spectra(th)
        dbar, cbar = self.data_terms(th)
        g, r = self.split_rows()
        gt, rt = torch.tensor(g), torch.tensor(r)
        a_all, ag_all, ar_all, jac, lik = [], [], [], 0.0, 0.0
        for I in range(n):
            D, vg, vr = self.split_variances(I, spec)
            S0 = torch.tensor(self.S0[I])
            d = dbar[I]
            ah = torch.linalg.solve(beta * S0 + torch.diag(1.0 / D), beta * d)
            SG = torch.linalg.inv(beta * S0[gt][:, gt] + torch.diag(1.0 / vg))
            SR = torch.linalg.inv(beta * S0[rt][:, rt] + torch.diag(1.0 / vr))
            LG = torch.linalg.cholesky(0.5 * (SG + SG.T))
            LR = torch.linalg.cholesky(0.5 * (SR + SR.T))
            ag = vg / D[gt] * ah[gt] + LG @ z[I, : lay.PG]
            ar = vr / D[rt] * ah[rt] + LR @ z[I, lay.PG:]
            a = torch.zeros(lay.P, dtype=torch.float64)
            a = a.index_add(0, gt, ag).index_add(0, rt, ar)
            a_all.append(a)
            ag_all.append(ag)
            ar_all.append(ar)
            jac = jac + torch.sum(torch.log(torch.diagonal(LG))) + torch.sum(torch.log(torch.diagonal(LR)))
            lik = lik + beta * (-0.5 * cbar[I] + a @ d - 0.5 * a @ (S0 @ a) + self.const[I])
        return torch.stack(a_all), torch.stack(ag_all), torch.stack(ar_all), jac, lik, spec

    def log_prior_split(self, ag, ar, spec):
        """log N(a_G; 0, rho_k Gamma per frequency) + log N(a_R; 0, diag kappa)."""
        lay, n = self.lay, self.n_psr
        rho, kap, kdm = spec
        Lg = torch.linalg.cholesky(torch.tensor(self.Gamma))
        ldg = 2.0 * torch.sum(torch.log(torch.diagonal(Lg)))
        out = 0.0
        for k in range(lay.nf_gw):
            for c in range(2):
                y = torch.linalg.solve_triangular(Lg, ag[:, 2 * k + c].unsqueeze(1), upper=False)
                out = out - 0.5 * torch.sum(y * y) / rho[k] - 0.5 * (n * LN2PI + n * torch.log(rho[k]) + ldg)
        vr = torch.cat([kap[:, : lay.nf_rn].repeat_interleave(2, dim=1), kdm.repeat_interleave(2, dim=1)], dim=1)
        out = out - 0.5 * torch.sum(ar * ar / vr) - 0.5 * torch.sum(torch.log(2 * np.pi * vr))
        return out

    def log_prior_a(self, a, spec):
        """log N(a; 0, phi): per frequency rho_k Gamma + diag kappa_.k for the
        red/common block (sin and cos share it), diagonal for DM."""
        lay, n = self.lay, self.n_psr
        rho, kap, kdm = spec
        G = torch.tensor(self.Gamma)
        out = 0.0
        for k in range(lay.Ka):
            phi = rho[k] * G + torch.diag(kap[:, k])
            Lk = torch.linalg.cholesky(phi)
            ld = 2.0 * torch.sum(torch.log(torch.diagonal(Lk)))
            for c in range(2):
                y = torch.linalg.solve_triangular(Lk, a[:, 2 * k + c].unsqueeze(1), upper=False)
                out = out - 0.5 * torch.sum(y * y) - 0.5 * (n * LN2PI + ld)
        for k in range(lay.Kdm):
            for c in range(2):
                v = a[:, 2 * lay.Ka + 2 * k + c]
                out = out - 0.5 * torch.sum(v * v / kdm[:, k]) - 0.5 * torch.sum(torch.log(2 * np.pi * kdm[:, k]))
        return out

    def logp_one(self, x, beta):
        lay = self.lay
        th = x[: lay.n_theta]
        z = x[lay.z:].reshape(self.n_psr, lay.Pz)
        box = float(np.sum(np.log(self.hi - self.lo)))
        if self.split:
            _, ag, ar, jac, lik, spec = self.transform_split(th, z, beta)
            return lik + jac + self.log_prior_split(ag, ar, spec) - box
        a, jac, lik, spec = self.transform(th, z, beta)
        return lik + jac + self.log_prior_a(a, spec) - box


class _CWSamples(torch.autograd.Function):
    """The CW delay h_I(t_j) (Np, M) at the sample times of the deterministic
    basis, with the waveform's own derivative dh/dtheta (cw.py) as backward."""

    @staticmethod
    def forward(ctx, th_cw, prep):
        t = th_cw.detach().numpy()
        H, G = [], []
        for I in range(prep.n_psr):
            h, g = cwmod.delay(prep.ts_d, prep.pos[I], t, want_grad=True)
            H.append(h)
            G.append(g)
        ctx.save_for_backward(torch.tensor(np.stack(G)))
        return torch.tensor(np.stack(H))

    @staticmethod
    def backward(ctx, gH):
        (G,) = ctx.saved_tensors
        return torch.einsum("ij,ijk->k", gH, G), None


def logp_grad(prep: StdPrepared, X, beta=None):
    """log p~, its gradient (autograd) and a status per chain; X (C, d)."""
    X = np.atleast_2d(np.asarray(X, np.float64))
    C, d = X.shape
    lay = prep.lay
    assert d == lay.d
    beta = np.ones(C) if beta is None else np.broadcast_to(np.asarray(beta, np.float64), (C,))
    logp = np.full(C, -np.inf)
    grad = np.zeros((C, d))
    status = np.zeros(C, np.int32)
    for c in range(C):
        th = X[c, : lay.n_theta]
        if not (np.all(np.isfinite(th)) and np.all(th >= prep.lo) and np.all(th <= prep.hi)):
            status[c] = ST_PRIOR
            continue
        if not np.all(np.isfinite(X[c])):
            status[c] = ST_NONFINITE
            continue
        if prep.has_cw and cwmod.max_y(th[lay.cw:lay.cw + 8], prep.ts_d[-1]) >= 1.0:
            status[c] = ST_CW
            continue
        x = torch.tensor(X[c], requires_grad=True)
        try:
            lp = prep.logp_one(x, float(beta[c]))
            (g,) = torch.autograd.grad(lp, x)
        except (torch.linalg.LinAlgError, NotPositiveDefinite):
            status[c] = ST_NOTPD
            continue
        lpv, gv = float(lp.detach()), g.numpy()
        if not (np.isfinite(lpv) and np.all(np.isfinite(gv))):
            status[c] = ST_NONFINITE
            continue
        logp[c], grad[c] = lpv, gv
    return dict(logp=logp, grad=grad, status=status)


def z_scale(prep: StdPrepared, x, beta=1.0):
    """Magnitude companion of dlog p~/dz (the tolerance floor of the parity
    tests): the adjoint dz_I = L_I^T v_I, v_I = beta (d_I - S0_I a_I) - (phi^-1 a)_I,
    evaluated with the absolute value of every term down to the per-TOA sums
    that d and S0 hold (the timing-model projection cancels against them),
    S_I = |L_I|^T [beta (sum_i |T_i| |dt_i| / N_i + (sum_i |T_i| |T_i|^T / N_i) |a_I|)
                   + (|phi^-1| |a|)_I]   (Np, P)."""
    if prep.split:
        return _z_scale_split(prep, x, beta)
    lay, n = prep.lay, prep.n_psr
    xt = torch.tensor(np.asarray(x, np.float64))
    th, z = xt[: lay.n_theta], xt[lay.z:].reshape(n, lay.P)
    a, _, _, (rho, kap, kdm) = prep.transform(th, z, beta)
    a = a.detach().numpy()
    aD = prep.cw_coefficients(th).detach().numpy() if prep.has_cw else None
    rho, kap, kdm = rho.detach().numpy(), kap.detach().numpy(), kdm.detach().numpy()
    pa = np.zeros_like(a)                      # |phi^-1| |a|
    for k in range(lay.Ka):
        phinv = np.abs(np.linalg.inv(rho[k] * prep.Gamma + np.diag(kap[:, k])))
        for c in range(2):
            pa[:, 2 * k + c] = phinv @ np.abs(a[:, 2 * k + c])
    for k in range(lay.Kdm):
        for c in range(2):
            j = 2 * lay.Ka + 2 * k + c
            pa[:, j] = np.abs(a[:, j]) / kdm[:, k]
    out = np.zeros((n, lay.P))
    for I in range(n):
        D = np.concatenate([np.repeat(rho + kap[I], 2), np.repeat(kdm[I], 2)])
        Sig = np.linalg.inv(beta * prep.S0[I] + np.diag(1.0 / D))
        L = np.linalg.cholesky(0.5 * (Sig + Sig.T))
        dab = prep.dabs[I] if not prep.has_cw else prep.dabs[I] + prep.GabsD[I] @ np.abs(aD[I])
        V = beta * (dab + prep.Gabs[I] @ np.abs(a[I])) + pa[I]
        out[I] = np.abs(L).T @ V
    return out


def _z_scale_split(prep: StdPrepared, x, beta):
    """z_scale with split sets: dz_b = L_b^T g_b, g_b the likelihood's
    beta (d - S0 a) on the set's rows plus the set's prior term, bounded the
    same way term by term (Np, PG + PR)."""
    lay, n = prep.lay, prep.n_psr
    xt = torch.tensor(np.asarray(x, np.float64))
    th, z = xt[: lay.n_theta], xt[lay.z:].reshape(n, lay.Pz)
    a, ag, ar, _, _, spec = prep.transform_split(th, z, beta)
    a, ag, ar = a.detach().numpy(), ag.detach().numpy(), ar.detach().numpy()
    aD = prep.cw_coefficients(th).detach().numpy() if prep.has_cw else None
    rho = spec[0].detach().numpy()
    g, r = prep.split_rows()
    Ginv = np.abs(np.linalg.inv(prep.Gamma))
    pg = np.zeros_like(ag)                     # |phi_GWB^-1| |a_G|
    for k in range(lay.nf_gw):
        for c in range(2):
            pg[:, 2 * k + c] = Ginv @ np.abs(ag[:, 2 * k + c]) / rho[k]
    out = np.zeros((n, lay.Pz))
    for I in range(n):
        _, vg, vr = (v.detach().numpy() for v in prep.split_variances(I, spec))
        S0 = prep.S0[I]
        SG = np.linalg.inv(beta * S0[np.ix_(g, g)] + np.diag(1.0 / vg))
        SR = np.linalg.inv(beta * S0[np.ix_(r, r)] + np.diag(1.0 / vr))
        LG = np.linalg.cholesky(0.5 * (SG + SG.T))
        LR = np.linalg.cholesky(0.5 * (SR + SR.T))
        dab = prep.dabs[I] if not prep.has_cw else prep.dabs[I] + prep.GabsD[I] @ np.abs(aD[I])
        V = beta * (dab + prep.Gabs[I] @ np.abs(a[I]))
        out[I, : lay.PG] = np.abs(LG).T @ (V[g] + pg[I])
        out[I, lay.PG:] = np.abs(LR).T @ (V[r] + np.abs(ar[I]) / vr)
    return out


def rounding_sensitivity(prep: StdPrepared, X, beta=None, seed=0, draws=1):
    """The largest shift of the gradient over ``draws`` independent draws of
    _rounding_shift (below)."""
    out = None
    for k in range(draws):
        d = _rounding_shift(prep, X, beta, seed + k)
        out = d if out is None else np.maximum(out, d)
    return out


def _rounding_shift(prep: StdPrepared, X, beta=None, seed=0):
    """How far the oracle's own gradient moves when its stored Gram quantities
    carry rounding of the size a floating-point sum of n_I per-TOA terms has
    (eps_mach sqrt(n_I) relative to the sum of the absolute values of the
    terms), under two models: independent rounding of every entry of S0 and
    d, and rounding shared by all the sums a TOA enters (its weight 1/N_i
    perturbed, everything recomputed).  Returns the larger |grad' - grad|
    (C, d): two FP64 evaluations of the same per-TOA sums cannot be asked to
    agree more closely than this."""
    import copy
    rng = np.random.default_rng(seed)
    eps = np.finfo(np.float64).eps
    # (a) independent rounding of every stored entry
    p2 = copy.copy(prep)
    p2.S0, p2.dvec = list(prep.S0), list(prep.dvec)
    if prep.has_cw:
        p2.SD = list(prep.SD)
    for I in range(prep.n_psr):
        e = eps * np.sqrt(max(prep.ntoa[I], 1))
        xi = rng.uniform(-1.0, 1.0, prep.S0[I].shape)
        p2.S0[I] = prep.S0[I] + e * prep.Gabs[I] * 0.5 * (xi + xi.T)
        p2.dvec[I] = prep.dvec[I] + e * prep.dabs[I] * rng.uniform(-1.0, 1.0, prep.dvec[I].shape)
        if prep.has_cw:
            p2.SD[I] = prep.SD[I] + e * prep.GabsD[I] * rng.uniform(-1.0, 1.0, prep.SD[I].shape)
    # (b) rounding shared by every sum a TOA enters (and so by the
    # timing-model projection): each per-TOA weight 1/N_i scaled by
    # 1 + eps sqrt(n_I) u_i, the Gram quantities recomputed
    ds3 = dict(prep.ds)
    off = np.asarray(ds3["toa_offsets"], np.int64)
    scale = np.ones(np.asarray(ds3["t"]).size)
    for I in range(prep.n_psr):
        n = int(off[I + 1] - off[I])
        scale[off[I]:off[I + 1]] += eps * np.sqrt(max(n, 1)) * rng.uniform(-1.0, 1.0, n)
    # N_i -> N_i scale_i, carried by sigma_i (EQUAD is per backend, not per TOA)
    be = np.asarray(ds3["backend"], np.int64)
    ef = np.asarray(ds3["efac"], np.float64)[be]
    eq = np.asarray(ds3["equad"], np.float64)[be]
    N = (ef * np.asarray(prep.ds["sigma"], np.float64)) ** 2 + eq ** 2
    ds3["sigma"] = np.sqrt(np.maximum(N * scale - eq ** 2, 0.0)) / ef
    p3 = StdPrepared(ds3)
    p3.Gamma = prep.Gamma
    a = logp_grad(prep, X, beta)
    out = np.zeros_like(a["grad"])
    for pp in (p2, p3):
        b = logp_grad(pp, X, beta)
        d = np.abs(a["grad"] - b["grad"])
        d[(a["status"] != 0) | (b["status"] != 0)] = 0.0
        out = np.maximum(out, d)
    return out


def coefficients(prep: StdPrepared, x, beta=1.0):
    """The Fourier coefficients a (Np, P) that a point maps to; with split
    sets [a_G | a_R] (Np, PG + PR)."""
    lay = prep.lay
    xt = torch.tensor(np.asarray(x, np.float64))
    z = xt[lay.z:].reshape(prep.n_psr, lay.Pz)
    if prep.split:
        _, ag, ar, _, _, _ = prep.transform_split(xt[: lay.n_theta], z, beta)
        return torch.cat([ag, ar], dim=1).detach().numpy()
    a, _, _, _ = prep.transform(xt[: lay.n_theta], z, beta)
    return a.detach().numpy()
