// Per-frequency kernels: power-law spectra, prior covariance, Cholesky
// factor and whitening transform (forward), and the Cholesky adjoint
// (backward).  One 64-lane wavefront per (chain, frequency).
//
// Forward (Sec. IV.A, Eqs. power_law, HD, prior_cov; Sec. II.B, Eq.
// standardizing_transform with mu = 0):
//   rho_k = A^2/(12 pi^2) yr^3 (f_k yr)^-gamma / T,  kappa_Ik likewise
//   phi_k = rho_k Gamma + diag(kappa_.k),  L_k = chol(phi_k)
//   a_.k,sin = L_k z_.k,sin,  a_.k,cos = L_k z_.k,cos,  a_dm = sqrt(kdm) z_dm
// Backward, with abar = d log L / d a from the TOA pass:
//   dz = L^T abar - z,  phibar = sym(L^-T Phi(L^T Lbar) L^-1),
//   Lbar = sum_c abar_c z_c^T, Phi = lower triangle with halved diagonal,
//   d/drho_k = <phibar, Gamma>,  d/dkappa_Ik = phibar_II.
#include "common.h"

namespace {

using pt::Dev;

__device__ inline double powerlaw(double f, double log10A, double gamma, double tspan) {
  // A^2/(12 pi^2) yr^3 (f yr)^-gamma / T, evaluated in logarithms.
  const double c = 3.0 * log(pt::kYear) - log(12.0 * pt::kPi * pt::kPi) - log(tspan);
  return exp(2.0 * pt::kLn10 * log10A - gamma * log(f * pt::kYear) + c);
}

// Packed lower-triangular storage, column-major: column m holds rows m..n-1.
__device__ inline int colstart(int m, int n) { return m * n - (m * (m - 1)) / 2; }

__device__ inline double wave_sum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline bool theta_in_box(const Dev &D, const double *xc) {
  bool ok = true;
  for (int i = threadIdx.x; i < D.n_theta; i += 64) {
    const double v = xc[i];
    if (!(v >= D.prior_lo[i] && v <= D.prior_hi[i])) ok = false;
  }
  return __all(ok);
}

constexpr int kMaxPsr = PTAFS_MAX_PSR;
constexpr int kRows = (kMaxPsr + 63) / 64;   // rows of a matrix per lane

// ---------------------------------------------------------------------------
// Forward: grid (kmax, c_pad), block 64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_spec_fwd(Dev D, const double *__restrict__ x) {
  extern __shared__ double lds[];
  const int k0 = blockIdx.x;           // frequency index, harmonic k = k0 + 1
  const int c = blockIdx.y;            // chain (padded)
  const int lane = threadIdx.x;
  const int n = D.n_psr;
  const int kmax = max(D.ka, D.nf_dm);
  const double f = (k0 + 1) / D.tspan;
  const bool real = c < D.n_chains;
  const double *xc = x + (size_t)(real ? c : 0) * D.d;
  const size_t cp = D.c_pad;

  bool bad = !real;
  if (real) bad = !theta_in_box(D, xc);

  if (k0 == 0) {
    // Per-chain status from the inputs, and the rows no frequency owns.
    int st = 0;
    if (real) {
      if (bad) {
        st = PTAFS_ST_PRIOR;
      } else {
        bool fin = true;
        for (int i = lane; i < D.d; i += 64) fin = fin && isfinite(xc[i]);
        if (!__all(fin)) st = PTAFS_ST_NONFINITE;
        if (st == 0 && D.has_cw) {
          const double *cw = xc + D.off_cw;
          const double M = exp(pt::kLn10 * cw[2]) * pt::kTsun;
          const double w0 = pt::kPi * exp(pt::kLn10 * cw[3]);
          const double y = 256.0 / 5.0 * exp(5.0 / 3.0 * log(M) + 8.0 / 3.0 * log(w0)) * D.tmax;
          if (!(y < 1.0)) st = PTAFS_ST_CW;
        }
      }
      if (lane == 0) D.st_pre[c] = st;
    } else if (lane == 0 && c < D.c_pad) {
      D.st_pre[c] = 0;
    }
    const bool zero = !real || st != 0;
    // timing-model rows and padding rows of both blocks
    for (int idx = lane; idx < n * D.rows_rn; idx += 64) {
      const int I = idx / D.rows_rn, row = idx % D.rows_rn;
      const pt::Slot sl = pt::rn_slot(row, D.kb);
      double v;
      if (sl.kind == 1) v = zero ? 0.0 : D.sigma_b * xc[D.off_u + 3 * I + sl.tm];
      else if (sl.kind == 0 && sl.harm <= D.ka) continue;     // owned by frequency harm
      else v = 0.0;
      D.coef_rn[((size_t)I * D.rows_rn + row) * cp + c] = v;
    }
    for (int idx = lane; idx < n * D.rows_dm; idx += 64) {
      const int I = idx / D.rows_dm, row = idx % D.rows_dm;
      const pt::Slot sl = pt::dm_slot(row, D.nf_dm);
      if (sl.kind == 0) continue;
      D.coef_dm[((size_t)I * D.rows_dm + row) * cp + c] = 0.0;
    }
  }

  // ---- red-noise / common block, harmonic k0 + 1 ---------------------------
  if (k0 < D.ka) {
    const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
    const double *zc = xc + D.off_z;
    const int K2 = 2 * D.ka;
    const bool dense = (k0 < D.nf_gw) && n > 0;
    int flag = 0;
    if (bad) {
      for (int I = lane; I < n; I += 64) {
        D.coef_rn[((size_t)I * D.rows_rn + rs) * cp + c] = 0.0;
        D.coef_rn[((size_t)I * D.rows_rn + rc) * cp + c] = 0.0;
      }
    } else if (!dense) {
      // phi_k = diag(kappa): L = diag(sqrt(kappa))
      for (int I = lane; I < n; I += 64) {
        const double *th = xc + D.off_rn + 2 * I;
        const double kap = (k0 < D.nf_rn) ? powerlaw(f, th[0], th[1], D.tspan) : 0.0;
        if (!(kap > 0.0) || !isfinite(kap)) flag = PTAFS_ST_NOTPD;
        const double sq = sqrt(kap);
        D.coef_rn[((size_t)I * D.rows_rn + rs) * cp + c] = sq * zc[I * K2 + 2 * k0];
        D.coef_rn[((size_t)I * D.rows_rn + rc) * cp + c] = sq * zc[I * K2 + 2 * k0 + 1];
      }
    } else {
      // dense: left-looking Cholesky, lane owns rows lane + 64 r
      double *LT = lds;                              // packed, n(n+1)/2
      double *zs = lds + (n * (n + 1)) / 2;          // [n][2]
      const double rho = powerlaw(f, xc[D.off_gw], xc[D.off_gw + 1], D.tspan);
      double kap[kRows];
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        const int I = lane + 64 * r;
        kap[r] = 0.0;
        if (I < n) {
          if (k0 < D.nf_rn) {
            const double *th = xc + D.off_rn + 2 * I;
            kap[r] = powerlaw(f, th[0], th[1], D.tspan);
          }
          zs[2 * I] = zc[I * K2 + 2 * k0];
          zs[2 * I + 1] = zc[I * K2 + 2 * k0 + 1];
        }
      }
      for (int j = 0; j < n; ++j) {
        double acc[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          const int I = lane + 64 * r;
          acc[r] = 0.0;
          if (I >= j && I < n) {
            double s = rho * D.gamma[(size_t)I * n + j] + (I == j ? kap[r] : 0.0);
            double s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int m = 0;
            for (; m + 3 < j; m += 4) {
              s -= LT[colstart(m, n) + I - m] * LT[colstart(m, n) + j - m];
              s1 -= LT[colstart(m + 1, n) + I - m - 1] * LT[colstart(m + 1, n) + j - m - 1];
              s2 -= LT[colstart(m + 2, n) + I - m - 2] * LT[colstart(m + 2, n) + j - m - 2];
              s3 -= LT[colstart(m + 3, n) + I - m - 3] * LT[colstart(m + 3, n) + j - m - 3];
            }
            for (; m < j; ++m) s -= LT[colstart(m, n) + I - m] * LT[colstart(m, n) + j - m];
            acc[r] = (s + s1) + (s2 + s3);
          }
        }
        // the owner of row j publishes the pivot
        const int owner = j & 63, ro = j >> 6;
        double piv = 0.0;
#pragma unroll
        for (int r = 0; r < kRows; ++r)
          if (r == ro) piv = __shfl(acc[r], owner, 64);
        if (!(piv > 0.0) || !isfinite(piv)) {
          flag = PTAFS_ST_NOTPD;
          piv = 1.0;
        }
        const double ljj = sqrt(piv);
        const double inv = 1.0 / ljj;
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          const int I = lane + 64 * r;
          if (I == j) LT[colstart(j, n)] = ljj;
          else if (I > j && I < n) LT[colstart(j, n) + I - j] = acc[r] * inv;
        }
        __syncthreads();
      }
      // a = L z for sin and cos
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        const int I = lane + 64 * r;
        if (I < n) {
          double as = 0.0, ac = 0.0;
          for (int m = 0; m <= I; ++m) {
            const double l = LT[colstart(m, n) + I - m];
            as += l * zs[2 * m];
            ac += l * zs[2 * m + 1];
          }
          D.coef_rn[((size_t)I * D.rows_rn + rs) * cp + c] = as;
          D.coef_rn[((size_t)I * D.rows_rn + rc) * cp + c] = ac;
        }
      }
      // keep L for the adjoint
      const int np = (n * (n + 1)) / 2;
      double *dst = D.lstore + ((size_t)c * D.nf_gw + k0) * np;
      for (int i = lane; i < np; i += 64) dst[i] = LT[i];
    }
    flag = __any(flag != 0) ? PTAFS_ST_NOTPD : 0;
    if (lane == 0) D.flag_k[(size_t)c * kmax + k0] = bad ? 0 : flag;
  } else if (lane == 0) {
    D.flag_k[(size_t)c * kmax + k0] = 0;
  }

  // ---- DM block -------------------------------------------------------------
  if (k0 < D.nf_dm) {
    const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
    const double *zd = xc + D.off_zdm;
    const int K2 = 2 * D.nf_dm;
    for (int I = lane; I < n; I += 64) {
      double vs = 0.0, vc = 0.0;
      if (!bad) {
        const double *th = xc + D.off_dm + 2 * I;
        const double sq = sqrt(powerlaw(f, th[0], th[1], D.tspan));
        vs = sq * zd[I * K2 + 2 * k0];
        vc = sq * zd[I * K2 + 2 * k0 + 1];
      }
      D.coef_dm[((size_t)I * D.rows_dm + rs) * cp + c] = vs;
      D.coef_dm[((size_t)I * D.rows_dm + rc) * cp + c] = vc;
    }
  }
}

// ---------------------------------------------------------------------------
// Backward: grid (kmax, n_chains), block 64.
// LDS: X [n][n+1] when the frequency carries the common process.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_spec_bwd(Dev D, const double *__restrict__ x,
                                                 double *__restrict__ grad) {
  extern __shared__ double lds[];
  const int k0 = blockIdx.x;
  const int c = blockIdx.y;
  const int lane = threadIdx.x;
  const int n = D.n_psr;
  const int kmax = max(D.ka, D.nf_dm);
  const double f = (k0 + 1) / D.tspan;
  const double lnfy = log(f * pt::kYear);
  const double *xc = x + (size_t)c * D.d;
  double *gc = grad + (size_t)c * D.d;
  const size_t cp = D.c_pad;
  const bool skip = D.st_pre[c] != 0 || D.flag_k[(size_t)c * kmax + k0] != 0;

  if (k0 < D.ka) {
    const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
    const double *zc = xc + D.off_z;
    const int K2 = 2 * D.ka;
    const bool dense = (k0 < D.nf_gw);
    double *dth = D.dth_k + ((size_t)c * D.ka + k0) * 2;
    double *drn = D.drn_k + ((size_t)c * D.ka + k0) * n * 2;
    if (skip) {
      for (int I = lane; I < n; I += 64) {
        gc[D.off_z + I * K2 + 2 * k0] = 0.0;
        gc[D.off_z + I * K2 + 2 * k0 + 1] = 0.0;
        drn[2 * I] = 0.0;
        drn[2 * I + 1] = 0.0;
      }
      if (lane == 0) { dth[0] = 0.0; dth[1] = 0.0; }
    } else if (!dense) {
      for (int I = lane; I < n; I += 64) {
        const double *th = xc + D.off_rn + 2 * I;
        const double sq = sqrt(powerlaw(f, th[0], th[1], D.tspan));
        const double ab_s = D.bar_rn[((size_t)I * D.rows_rn + rs) * cp + c];
        const double ab_c = D.bar_rn[((size_t)I * D.rows_rn + rc) * cp + c];
        const double z_s = zc[I * K2 + 2 * k0], z_c = zc[I * K2 + 2 * k0 + 1];
        gc[D.off_z + I * K2 + 2 * k0] = sq * ab_s - z_s;
        gc[D.off_z + I * K2 + 2 * k0 + 1] = sq * ab_c - z_c;
        // d sqrt(kappa)/d log10A = ln10 sqrt(kappa); d/dgamma = -1/2 ln(f yr) sqrt(kappa)
        const double az = (ab_s * z_s + ab_c * z_c) * sq;
        drn[2 * I] = (k0 < D.nf_rn) ? az * pt::kLn10 : 0.0;
        drn[2 * I + 1] = (k0 < D.nf_rn) ? az * (-0.5 * lnfy) : 0.0;
      }
      if (lane == 0) { dth[0] = 0.0; dth[1] = 0.0; }
    } else {
      const int np = (n * (n + 1)) / 2;
      const double *LT = D.lstore + ((size_t)c * D.nf_gw + k0) * np;   // global, uniform reads
      const int xs = n | 1;                                            // odd row stride
      double *X = lds;                                                 // [n][xs]
      double *vz = lds + (size_t)n * xs;                               // v_s, v_c, z_s, z_c [4][n]
      // v = L^T abar (lane owns I); dz = v - z
      for (int I = lane; I < n; I += 64) {
        double vs = 0.0, vc = 0.0;
        for (int m = I; m < n; ++m) {
          const double l = LT[colstart(I, n) + m - I];
          vs += l * D.bar_rn[((size_t)m * D.rows_rn + rs) * cp + c];
          vc += l * D.bar_rn[((size_t)m * D.rows_rn + rc) * cp + c];
        }
        const double z_s = zc[I * K2 + 2 * k0], z_c = zc[I * K2 + 2 * k0 + 1];
        gc[D.off_z + I * K2 + 2 * k0] = vs - z_s;
        gc[D.off_z + I * K2 + 2 * k0 + 1] = vc - z_c;
        vz[I] = vs;
        vz[n + I] = vc;
        vz[2 * n + I] = z_s;
        vz[3 * n + I] = z_c;
      }
      __syncthreads();
      // X = L^-T P, P = Phi(v_s z_s^T + v_c z_c^T); lane b owns column b.
      for (int b = lane; b < n; b += 64) {
        const double zsb = vz[2 * n + b], zcb = vz[3 * n + b];
        for (int a = n - 1; a >= 0; --a) {
          double pab = 0.0;
          if (a > b) pab = vz[a] * zsb + vz[n + a] * zcb;
          else if (a == b) pab = 0.5 * (vz[a] * zsb + vz[n + a] * zcb);
          double s = pab;
          const double *col = LT + colstart(a, n) - a;   // col[m] = L_ma
          for (int m = a + 1; m < n; ++m) s -= col[m] * X[(size_t)m * xs + b];
          X[(size_t)a * xs + b] = s / col[a];
        }
      }
      __syncthreads();
      // S = X L^-1 in place (row b: L^T s_b = x_b); accumulate <S, Gamma> and S_bb.
      double dr = 0.0;
      for (int b = lane; b < n; b += 64) {
        double *row = X + (size_t)b * xs;
        double acc = 0.0;
        for (int a = n - 1; a >= 0; --a) {
          const double *col = LT + colstart(a, n) - a;
          double s = row[a];
          for (int m = a + 1; m < n; ++m) s -= col[m] * row[m];
          s /= col[a];
          row[a] = s;
          acc += s * D.gamma[(size_t)b * n + a];
        }
        dr += acc;
        const double dk = row[b];
        const double kap = (k0 < D.nf_rn)
                               ? powerlaw(f, xc[D.off_rn + 2 * b], xc[D.off_rn + 2 * b + 1], D.tspan)
                               : 0.0;
        drn[2 * b] = dk * kap * 2.0 * pt::kLn10;
        drn[2 * b + 1] = dk * kap * (-lnfy);
      }
      dr = wave_sum(dr);
      if (lane == 0) {
        const double rho = powerlaw(f, xc[D.off_gw], xc[D.off_gw + 1], D.tspan);
        dth[0] = dr * rho * 2.0 * pt::kLn10;
        dth[1] = dr * rho * (-lnfy);
      }
    }
  }

  if (k0 < D.nf_dm) {
    const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
    const double *zd = xc + D.off_zdm;
    const int K2 = 2 * D.nf_dm;
    double *ddm = D.ddm_k + ((size_t)c * D.nf_dm + k0) * n * 2;
    for (int I = lane; I < n; I += 64) {
      if (skip) {
        gc[D.off_zdm + I * K2 + 2 * k0] = 0.0;
        gc[D.off_zdm + I * K2 + 2 * k0 + 1] = 0.0;
        ddm[2 * I] = 0.0;
        ddm[2 * I + 1] = 0.0;
        continue;
      }
      const double *th = xc + D.off_dm + 2 * I;
      const double sq = sqrt(powerlaw(f, th[0], th[1], D.tspan));
      const double ab_s = D.bar_dm[((size_t)I * D.rows_dm + rs) * cp + c];
      const double ab_c = D.bar_dm[((size_t)I * D.rows_dm + rc) * cp + c];
      const double z_s = zd[I * K2 + 2 * k0], z_c = zd[I * K2 + 2 * k0 + 1];
      gc[D.off_zdm + I * K2 + 2 * k0] = sq * ab_s - z_s;
      gc[D.off_zdm + I * K2 + 2 * k0 + 1] = sq * ab_c - z_c;
      const double az = (ab_s * z_s + ab_c * z_c) * sq;
      ddm[2 * I] = az * pt::kLn10;
      ddm[2 * I + 1] = az * (-0.5 * lnfy);
    }
  }
}

}  // namespace

namespace ptk {

hipError_t launch_spec_fwd(const pt::Dev &D, const double *x, hipStream_t s) {
  const int kmax = max(D.ka, D.nf_dm);
  if (kmax == 0 || D.c_pad == 0) return hipSuccess;
  const size_t lds = ((size_t)D.n_psr * (D.n_psr + 1) / 2 + 2 * D.n_psr) * sizeof(double);
  hipLaunchKernelGGL(k_spec_fwd, dim3(kmax, D.c_pad), dim3(64), lds, s, D, x);
  return hipGetLastError();
}

hipError_t set_spec_lds_limits(size_t fwd_bytes, size_t bwd_bytes) {
  hipError_t e = hipFuncSetAttribute((const void *)k_spec_fwd,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)fwd_bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)k_spec_bwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bwd_bytes);
}

hipError_t launch_spec_bwd(const pt::Dev &D, const double *x, double *grad, hipStream_t s) {
  const int kmax = max(D.ka, D.nf_dm);
  if (kmax == 0 || D.n_chains == 0) return hipSuccess;
  const int n = D.n_psr;
  const size_t lds = (D.nf_gw > 0) ? ((size_t)n * (n | 1) + 4 * n) * sizeof(double) : 0;
  hipLaunchKernelGGL(k_spec_bwd, dim3(kmax, D.n_chains), dim3(64), lds, s, D, x, grad);
  return hipGetLastError();
}

}  // namespace ptk
