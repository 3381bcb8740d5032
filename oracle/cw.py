"""Continuous-wave (single circular SMBHB, Earth term) timing delay.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names the CW model (Sec. III.D) and prints only its frequency and
phase evolution (Sec. V.A, Eqs. phase_evolve and CW_evolve).  The waveform
below is the reading this project fixed for the rest of the delay; it is
"parity unpinned" beyond the invariants the tests check (non-evolving limit,
the frequency ODE, amplitude scaling and the polarisation/phase symmetries).

Parameters, in order: cos(theta_s), phi_s, log10 Mc [Msun], log10 f_gw [Hz],
Phi0, cos(iota), psi, log10 h.

    M      = 10^log10Mc * T_sun                  (chirp mass in seconds)
    w0     = pi * f_gw                           (orbital angular frequency)
    y(t)   = 256/5 * M^(5/3) * w0^(8/3) * t      (must stay < 1)
    w(t)   = w0 * (1 - y)^(-3/8)                 Eq. CW_evolve
    Phi(t) = Phi0 + (1 - (1 - y)^(5/8)) / (32 (M w0)^(5/3))
                                                 Eq. phase_evolve, rewritten
    s_hat  = (sin th cos ph, sin th sin ph, cos th);  Omega = -s_hat
    m_hat  = (sin ph, -cos ph, 0);  n_hat = (-cos th cos ph, -cos th sin ph, sin th)
    F+     = ((m.p)^2 - (n.p)^2) / (2 (1 + Omega.p));  Fx = (m.p)(n.p) / (1 + Omega.p)
    alpha  = h / (2 w0^(2/3) w(t)^(1/3))
    P      = -sin(2 Phi) (1 + cos^2 iota);  Q = 2 cos(2 Phi) cos iota
    s+     = alpha (P cos 2psi - Q sin 2psi);  sx = alpha (P sin 2psi + Q cos 2psi)
    h(t)   = -(F+ s+ + Fx sx)
"""
from __future__ import annotations

import numpy as np

T_SUN = 4.925490947641e-6   # G Msun / c^3 in seconds (IAU nominal GM_sun)
LN10 = np.log(10.0)


def antenna(pos, cth, phi):
    """F+, Fx and their derivatives with respect to (cos theta, phi)."""
    sth = np.sqrt(1.0 - cth * cth)
    cph, sph = np.cos(phi), np.sin(phi)
    m = np.array([sph, -cph, 0.0])
    n = np.array([-cth * cph, -cth * sph, sth])
    om = -np.array([sth * cph, sth * sph, cth])
    dm_dc = np.zeros(3)
    dm_dp = np.array([cph, sph, 0.0])
    dn_dc = np.array([-cph, -sph, -cth / sth])
    dn_dp = np.array([cth * sph, -cth * cph, 0.0])
    dom_dc = -np.array([-cth / sth * cph, -cth / sth * sph, 1.0])
    dom_dp = -np.array([-sth * sph, sth * cph, 0.0])
    mp, np_, op = m @ pos, n @ pos, om @ pos
    den = 1.0 + op
    fp = 0.5 * (mp * mp - np_ * np_) / den
    fx = mp * np_ / den
    out = []
    for dm, dn, do in ((dm_dc, dn_dc, dom_dc), (dm_dp, dn_dp, dom_dp)):
        dmp, dnp, dop = dm @ pos, dn @ pos, do @ pos
        dfp = (mp * dmp - np_ * dnp) / den - fp * dop / den
        dfx = (dmp * np_ + mp * dnp) / den - fx * dop / den
        out.append((dfp, dfx))
    return fp, fx, out


def max_y(theta, tmax):
    """Largest evolution variable y over [0, tmax]; the model needs y < 1."""
    M = 10.0 ** theta[2] * T_SUN
    w0 = np.pi * 10.0 ** theta[3]
    return 256.0 / 5.0 * M ** (5.0 / 3.0) * w0 ** (8.0 / 3.0) * tmax


def delay(t, pos, theta, want_grad=True):
    """h(t) for one pulsar at unit vector ``pos``; optionally dh/dtheta (n, 8)."""
    cth, phi, lmc, lf, phi0, ci, psi, lh = theta
    M = 10.0 ** lmc * T_SUN
    w0 = np.pi * 10.0 ** lf
    amp = 10.0 ** lh
    y = 256.0 / 5.0 * M ** (5.0 / 3.0) * w0 ** (8.0 / 3.0) * t
    one_m_y = 1.0 - y
    w = w0 * one_m_y ** (-3.0 / 8.0)
    X = (M * w0) ** (5.0 / 3.0)
    E = -np.expm1(5.0 / 8.0 * np.log1p(-y))           # 1 - (1-y)^(5/8)
    Phi = phi0 + E / (32.0 * X)
    alpha = amp / (2.0 * w0 ** (2.0 / 3.0) * w ** (1.0 / 3.0))
    s2P, c2P = np.sin(2.0 * Phi), np.cos(2.0 * Phi)
    s2s, c2s = np.sin(2.0 * psi), np.cos(2.0 * psi)
    P = -s2P * (1.0 + ci * ci)
    Q = 2.0 * c2P * ci
    fp, fx, dF = antenna(pos, cth, phi)
    U = fp * c2s + fx * s2s
    V = fx * c2s - fp * s2s
    h = -alpha * (P * U + Q * V)
    if not want_grad:
        return h, None
    g = np.zeros((t.size, 8))
    splus = alpha * (P * c2s - Q * s2s)
    scross = alpha * (P * s2s + Q * c2s)
    # sky position enters through F+ and Fx only
    for j in range(2):
        dfp, dfx = dF[j]
        g[:, j] = -(dfp * splus + dfx * scross)
    # phase dependence
    dP_dPhi = -2.0 * c2P * (1.0 + ci * ci)
    dQ_dPhi = -4.0 * s2P * ci
    dh_dPhi = -alpha * (dP_dPhi * U + dQ_dPhi * V)
    # d/d ln M and d/d ln w0 through y, w (amplitude) and Phi
    dE_dy = 5.0 / 8.0 * one_m_y ** (-3.0 / 8.0)
    dPhi_dlnM = (dE_dy * (5.0 / 3.0) * y - (5.0 / 3.0) * E) / (32.0 * X)
    dPhi_dlnw0 = (dE_dy * (8.0 / 3.0) * y - (5.0 / 3.0) * E) / (32.0 * X)
    dlnw_dlnM = 5.0 / 8.0 * y / one_m_y
    dlnw_dlnw0 = 1.0 / one_m_y
    dlna_dlnM = -dlnw_dlnM / 3.0
    dlna_dlnw0 = -2.0 / 3.0 - dlnw_dlnw0 / 3.0
    g[:, 2] = LN10 * (h * dlna_dlnM + dh_dPhi * dPhi_dlnM)
    g[:, 3] = LN10 * (h * dlna_dlnw0 + dh_dPhi * dPhi_dlnw0)
    g[:, 4] = dh_dPhi
    dP_dci = -s2P * 2.0 * ci
    dQ_dci = 2.0 * c2P
    g[:, 5] = -alpha * (dP_dci * U + dQ_dci * V)
    g[:, 6] = -alpha * (2.0 * P * V - 2.0 * Q * U)
    g[:, 7] = LN10 * h
    return h, g
