// Continuous wave from one circular supermassive black-hole binary, Earth
// term only (Sec. III.D), with the frequency and phase evolution of Sec. V.A
// (Eqs. CW_evolve and phase_evolve).  Parameters of a chain, in order:
// cos(theta_s), phi_s, log10 Mc [Msun], log10 f_gw [Hz], Phi0, cos(iota),
// psi, log10 h.
//
// With M = Mc G/c^3 and w0 = pi f_gw (orbital angular frequency at t = 0):
//   y(t)    = 256/5 M^(5/3) w0^(8/3) t             (the binary merges at y = 1)
//   w(t)    = w0 (1 - y)^(-3/8)
//   Phi(t)  = Phi0 + (1 - (1 - y)^(5/8)) / (32 (M w0)^(5/3))
//   alpha   = h / (2 w0^(2/3) w^(1/3)) = h/(2 w0) (1 - y)^(1/8)
//   P = -sin 2Phi (1 + cos^2 iota),  Q = 2 cos 2Phi cos iota
//   delay   = -alpha (P U + Q V),  U = F+ cos 2psi + Fx sin 2psi,
//                                  V = Fx cos 2psi - F+ sin 2psi
// F+, Fx are the antenna patterns of the pulsar for a source at
// s = (sin th cos ph, sin th sin ph, cos th), propagation Omega = -s, with
// polarisation basis m = (sin ph, -cos ph, 0), n = (-cos th cos ph,
// -cos th sin ph, sin th):
//   F+ = ((m.p)^2 - (n.p)^2) / (2 (1 + Omega.p)),  Fx = (m.p)(n.p) / (1 + Omega.p)
#pragma once

#include "common.h"

namespace pt {

// Per (chain, pulsar) constants, stored as kCwConst rows of c_pad values.
enum CwRow {
  kCwK1 = 0,      // y = K1 t
  kCwInv32X,      // 1 / (32 (M w0)^(5/3))
  kCwPhi0,
  kCwA0,          // h / (2 w0)
  kCwCi,          // cos iota
  kCwU,
  kCwV,
  kCwC2s,         // cos 2 psi
  kCwS2s,         // sin 2 psi
  kCwDfpC,        // dF+/dcos(theta)
  kCwDfxC,
  kCwDfpP,        // dF+/dphi
  kCwDfxP,
  kCwRows
};
static_assert(kCwRows <= kCwConst, "CW constant table too small");

// Fill the constants of one chain for pulsar unit vector p.  th = the 8 CW
// parameters; a null th (padding chain or rejected chain) gives zero delay.
__device__ inline void cw_constants(const double *th, const double *p, double out[kCwRows]) {
  for (int i = 0; i < kCwRows; ++i) out[i] = 0.0;
  if (!th) return;
  const double cth = th[0], phi = th[1];
  const double M = exp(kLn10 * th[2]) * kTsun;
  const double w0 = kPi * exp(kLn10 * th[3]);
  const double X = exp((5.0 / 3.0) * log(M * w0));
  out[kCwK1] = 256.0 / 5.0 * X * w0;
  out[kCwInv32X] = 1.0 / (32.0 * X);
  out[kCwPhi0] = th[4];
  out[kCwA0] = exp(kLn10 * th[7]) / (2.0 * w0);
  out[kCwCi] = th[5];
  double s2s, c2s;
  sincos(2.0 * th[6], &s2s, &c2s);
  out[kCwC2s] = c2s;
  out[kCwS2s] = s2s;
  // antenna pattern and its derivatives in (cos theta, phi)
  const double sth = sqrt(1.0 - cth * cth);
  double sph, cph;
  sincos(phi, &sph, &cph);
  const double mp = sph * p[0] - cph * p[1];
  const double np = -cth * cph * p[0] - cth * sph * p[1] + sth * p[2];
  const double op = -(sth * cph * p[0] + sth * sph * p[1] + cth * p[2]);
  const double den = 1.0 + op;
  const double fp = 0.5 * (mp * mp - np * np) / den;
  const double fx = mp * np / den;
  out[kCwU] = fp * c2s + fx * s2s;
  out[kCwV] = fx * c2s - fp * s2s;
  // d/dcos(theta): dm = 0, dn = (-cph, -sph, -cth/sth), dOmega = (cth/sth cph, cth/sth sph, -1)
  const double r = cth / sth;
  {
    const double dmp = 0.0;
    const double dnp = -cph * p[0] - sph * p[1] - r * p[2];
    const double dop = r * cph * p[0] + r * sph * p[1] - p[2];
    out[kCwDfpC] = (mp * dmp - np * dnp) / den - fp * dop / den;
    out[kCwDfxC] = (dmp * np + mp * dnp) / den - fx * dop / den;
  }
  // d/dphi: dm = (cph, sph, 0), dn = (cth sph, -cth cph, 0), dOmega = (sth sph, -sth cph, 0)
  {
    const double dmp = cph * p[0] + sph * p[1];
    const double dnp = cth * sph * p[0] - cth * cph * p[1];
    const double dop = sth * sph * p[0] - sth * cph * p[1];
    out[kCwDfpP] = (mp * dmp - np * dnp) / den - fp * dop / den;
    out[kCwDfxP] = (dmp * np + mp * dnp) / den - fx * dop / den;
  }
}

// Per-TOA state kept between the delay and its adjoint.
struct CwToa {
  double y, L1, E, alpha, s2P, c2P, h;
};

// Constants of one (chain, pulsar) held in registers by a TOA-pass lane.
struct CwLane {
  double K1, inv32X, phi0, a0, ci, U, V, c2s, s2s;

  __device__ inline void load(const double *cwc, size_t cp, int p, int chain) {
    const double *b = cwc + (size_t)p * kCwConst * cp + chain;
    K1 = b[kCwK1 * cp];
    inv32X = b[kCwInv32X * cp];
    phi0 = b[kCwPhi0 * cp];
    a0 = b[kCwA0 * cp];
    ci = b[kCwCi * cp];
    U = b[kCwU * cp];
    V = b[kCwV * cp];
    c2s = b[kCwC2s * cp];
    s2s = b[kCwS2s * cp];
  }

  __device__ inline CwToa delay(double t) const {
    CwToa s;
    s.y = K1 * t;
    s.L1 = log1p(-s.y);                       // ln(1 - y)
    s.E = -expm1(0.625 * s.L1);               // 1 - (1 - y)^(5/8)
    const double Phi = phi0 + s.E * inv32X;
    s.alpha = a0 * exp(0.125 * s.L1);
    sincos(2.0 * Phi, &s.s2P, &s.c2P);
    const double P = -s.s2P * (1.0 + ci * ci);
    const double Q = 2.0 * s.c2P * ci;
    s.h = -s.alpha * (P * U + Q * V);
    return s;
  }

  // acc[j] += g * (partial of the delay with respect to parameter j), with
  // the sky-position pair held as sums against s+ and sx (mapped through the
  // antenna derivatives by cw_finish) and the ln 10 factors left to cw_finish.
  __device__ inline void adjoint(const CwToa &s, double g, double acc[8]) const {
    const double opc = 1.0 + ci * ci;
    const double P = -s.s2P * opc, Q = 2.0 * s.c2P * ci;
    const double dP = -2.0 * s.c2P * opc, dQ = -4.0 * s.s2P * ci;     // d/dPhi
    const double dhPhi = -s.alpha * (dP * U + dQ * V);
    const double omy = 1.0 - s.y;
    const double dEdy = 0.625 * exp(-0.375 * s.L1);                  // 5/8 (1-y)^(-3/8)
    const double t53 = (5.0 / 3.0) * s.E;
    const double dPhiM = (dEdy * (5.0 / 3.0) * s.y - t53) * inv32X;    // dPhi/dln M
    const double dPhiW = (dEdy * (8.0 / 3.0) * s.y - t53) * inv32X;    // dPhi/dln w0
    const double dlaM = -(0.625 * s.y / omy) / 3.0;                   // dln alpha/dln M
    const double dlaW = -2.0 / 3.0 - (1.0 / omy) / 3.0;               // dln alpha/dln w0
    const double sp = s.alpha * (P * c2s - Q * s2s);
    const double sx = s.alpha * (P * s2s + Q * c2s);
    acc[0] += g * sp;
    acc[1] += g * sx;
    acc[2] += g * (s.h * dlaM + dhPhi * dPhiM);
    acc[3] += g * (s.h * dlaW + dhPhi * dPhiW);
    acc[4] += g * dhPhi;
    acc[5] += g * (-s.alpha * (-2.0 * s.s2P * ci * U + 2.0 * s.c2P * V));
    acc[6] += g * (-s.alpha * (2.0 * P * V - 2.0 * Q * U));
    acc[7] += g * s.h;
  }
};

// Map lane sums to d log L / d(CW parameters) for one (chain, pulsar).
__device__ inline void cw_finish(const double *cwc, size_t cp, int p, int chain,
                                 const double acc[8], double out[8]) {
  const double *b = cwc + (size_t)p * kCwConst * cp + chain;
  out[0] = -(b[kCwDfpC * cp] * acc[0] + b[kCwDfxC * cp] * acc[1]);
  out[1] = -(b[kCwDfpP * cp] * acc[0] + b[kCwDfxP * cp] * acc[1]);
  out[2] = kLn10 * acc[2];
  out[3] = kLn10 * acc[3];
  out[4] = acc[4];
  out[5] = acc[5];
  out[6] = acc[6];
  out[7] = kLn10 * acc[7];
}

}  // namespace pt
