// Per-frequency kernels: power-law spectra, prior covariance, Cholesky
// factor and whitening transform (forward), and the Cholesky adjoint
// (backward).  One 256-thread workgroup per (frequency, chain).
//
// Forward (Sec. IV.A, Eqs. power_law, HD, prior_cov; Sec. II.B, Eq.
// standardizing_transform with mu = 0):
//   rho_k = A^2/(12 pi^2) yr^3 (f_k yr)^-gamma / T,  kappa_Ik likewise
//   phi_k = rho_k Gamma + diag(kappa_.k),  L_k = chol(phi_k)
//   a_.k,sin = L_k z_.k,sin,  a_.k,cos = L_k z_.k,cos,  a_dm = sqrt(kdm) z_dm
//
// Backward, with abar = d log L / d a from the TOA pass and v_c = L^T abar_c:
//   dz_c = v_c - z_c
//   phibar = sym(W^T P W),  W = L^-1,  P = Phi(sum_c v_c z_c^T)
//   (Phi = lower triangle with halved diagonal; the adjoint of phi = L L^T)
//   d/dkappa_I = phibar_II = w_I^T P w_I        (w_I = column I of W)
//   d/drho     = <phibar, Gamma> = <P, M M^T>,  M = W G,  G = chol(Gamma)
// Both reductions are O(n^2) with prefix / suffix sums over the lower
// triangle of P; W and M are formed with blocked triangular products.
#include "common.h"
#include "cw_dev.h"

namespace {

using pt::Dev;

__device__ inline double powerlaw(double f, double log10A, double gamma, double tspan) {
  // A^2/(12 pi^2) yr^3 (f yr)^-gamma / T, evaluated in logarithms.
  const double c = 3.0 * log(pt::kYear) - log(12.0 * pt::kPi * pt::kPi) - log(tspan);
  return exp(2.0 * pt::kLn10 * log10A - gamma * log(f * pt::kYear) + c);
}

// Packed lower-triangular storage, row-major: row i holds columns 0..i.
__device__ inline int pk(int i, int j) { return (i * (i + 1)) / 2 + j; }

template <typename T>
__device__ T block_sum(T v, T *red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] = red[t] + red[t + o];
    __syncthreads();
  }
  const T r = red[0];
  __syncthreads();
  return r;
}

__device__ inline bool block_all(bool v, int *ired) { return block_sum<int>(v ? 0 : 1, ired) == 0; }

// ---------------------------------------------------------------------------
// Forward: 1-D grid of kmax * c_pad (frequency, chain) blocks followed by
// n_prep white-noise preparation blocks, block 256.
// LDS (dense frequencies): A [n][ns] row-major (ns = n | 1), z [2][n], diag [n].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_spec_fwd(Dev D, const double *__restrict__ x) {
  extern __shared__ double lds[];
  __shared__ double red[256];
  __shared__ int ired[256];
  const int tid = threadIdx.x;
  const int n = D.n_psr;
  const int kmax = max(D.ka, D.nf_dm);
  const int nspec = kmax * D.c_pad;
  if ((int)blockIdx.x >= nspec) {
    // Heteroscedastic white noise (Eq. WN_cov): N_i = (EFAC sigma_i)^2 + EQUAD^2,
    // its reciprocal per TOA and a fixed-partition partial sum of ln N_i.
    const int pb = blockIdx.x - nspec;
    const int i0 = pb * pt::kPrepToas, i1 = min(D.n_toa, i0 + pt::kPrepToas);
    double s = 0.0;
    for (int i = i0 + tid; i < i1; i += 256) {
      const int be = D.backend[i];
      const double es = D.efac[be] * D.sigma[i], eq = D.equad[be];
      const double N = es * es + eq * eq;
      D.invn[i] = 1.0 / N;
      s += log(N);
    }
    s = block_sum(s, red);
    if (tid == 0) D.lnn_blk[pb] = s;
    return;
  }
  const int k0 = blockIdx.x % kmax;    // frequency index, harmonic k = k0 + 1
  const int c = blockIdx.x / kmax;     // chain (padded)
  const double f = (k0 + 1) / D.tspan;
  const bool real = c < D.n_chains;
  const double *xc = x + (size_t)(real ? c : 0) * D.d;
  const size_t cp = D.c_pad;

  bool inbox = real;
  if (real) {
    bool ok = true;
    for (int i = tid; i < D.n_theta; i += 256) {
      const double v = xc[i];
      if (!(v >= D.prior_lo[i] && v <= D.prior_hi[i])) ok = false;
    }
    inbox = block_all(ok, ired);
  }
  const bool bad = !inbox;

  // finiteness and squared norm of the coordinates this frequency owns
  double zz = 0.0;
  bool fin = true;
  if (!bad) {
    if (k0 < D.ka) {
      const double *zc = xc + D.off_z;
      for (int e = tid; e < 2 * n; e += 256) {
        const double v = zc[(e >> 1) * 2 * D.ka + 2 * k0 + (e & 1)];
        fin = fin && isfinite(v);
        zz += v * v;
      }
    }
    if (k0 < D.nf_dm) {
      const double *zd = xc + D.off_zdm;
      for (int e = tid; e < 2 * n; e += 256) {
        const double v = zd[(e >> 1) * 2 * D.nf_dm + 2 * k0 + (e & 1)];
        fin = fin && isfinite(v);
        zz += v * v;
      }
    }
    if (k0 == 0) {
      for (int e = tid; e < 3 * n; e += 256) {
        const double v = xc[D.off_u + e];
        fin = fin && isfinite(v);
        zz += v * v;
      }
    }
  }
  zz = block_sum(zz, red);
  fin = block_all(fin, ired);
  int flag = fin ? 0 : pt::kFlagInNonfinite;

  if (k0 == 0) {
    // per-chain status from the hyper-parameters, and the rows no frequency owns
    int st = 0;
    if (real && bad) st = PTAFS_ST_PRIOR;
    if (real && !bad && D.has_cw) {
      const double *cw = xc + D.off_cw;
      const double M = exp(pt::kLn10 * cw[2]) * pt::kTsun;
      const double w0 = pt::kPi * exp(pt::kLn10 * cw[3]);
      const double y = 256.0 / 5.0 * exp(5.0 / 3.0 * log(M) + 8.0 / 3.0 * log(w0)) * D.tmax;
      if (!(y < 1.0)) st = PTAFS_ST_CW;
    }
    if (tid == 0) D.st_pre[c] = st;
    const bool zero = bad || st != 0;
    if (D.has_cw) {
      // CW constants per pulsar (zero delay for padding and rejected chains)
      const double *th = (real && !zero) ? xc + D.off_cw : nullptr;
      for (int I = tid; I < n; I += 256) {
        double v[pt::kCwRows];
        pt::cw_constants(th, D.pos + 3 * I, v);
        double *dst = D.cwc + (size_t)I * pt::kCwConst * cp + c;
#pragma unroll
        for (int j = 0; j < pt::kCwRows; ++j) dst[(size_t)j * cp] = v[j];
      }
    }
    for (int idx = tid; idx < n * D.rows_rn; idx += 256) {
      const int I = idx / D.rows_rn, row = idx % D.rows_rn;
      const pt::Slot sl = pt::rn_slot(row, D.kb);
      double v;
      if (sl.kind == 1) v = zero ? 0.0 : D.sigma_b * xc[D.off_u + 3 * I + sl.tm];
      else if (sl.kind == 0 && sl.harm <= D.ka) continue;     // owned by frequency harm
      else v = 0.0;
      D.coef_rn[((size_t)I * D.rows_rn + row) * cp + c] = v;
    }
    for (int idx = tid; idx < n * D.rows_dm; idx += 256) {
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
    const bool dense = k0 < D.nf_gw;
    if (bad) {
      for (int I = tid; I < n; I += 256) {
        D.coef_rn[((size_t)I * D.rows_rn + rs) * cp + c] = 0.0;
        D.coef_rn[((size_t)I * D.rows_rn + rc) * cp + c] = 0.0;
      }
    } else if (!dense) {
      // phi_k = diag(kappa): L = diag(sqrt(kappa))
      bool pd = true;
      for (int I = tid; I < n; I += 256) {
        const double *th = xc + D.off_rn + 2 * I;
        const double kap = (k0 < D.nf_rn) ? powerlaw(f, th[0], th[1], D.tspan) : 0.0;
        if (!(kap > 0.0) || !isfinite(kap)) pd = false;
        const double sq = sqrt(kap);
        D.coef_rn[((size_t)I * D.rows_rn + rs) * cp + c] = sq * zc[I * K2 + 2 * k0];
        D.coef_rn[((size_t)I * D.rows_rn + rc) * cp + c] = sq * zc[I * K2 + 2 * k0 + 1];
      }
      if (!block_all(pd, ired)) flag |= pt::kFlagNotPD;
    } else {
      // Right-looking Cholesky on the unscaled lower triangle: at column j,
      // A_ik -= A_ij A_kj / A_jj for j < k <= i; afterwards L_jj = sqrt(A_jj),
      // L_ij = A_ij / L_jj.  One barrier per column.
      const int ns = n | 1;
      double *A = lds;                      // [n][ns]
      double *zs = A + (size_t)n * ns;      // [2][n]
      double *dg = zs + 2 * n;              // [n]
      const double rho = powerlaw(f, xc[D.off_gw], xc[D.off_gw + 1], D.tspan);
      for (int I = tid; I < n; I += 256) {
        double kap = 0.0;
        if (k0 < D.nf_rn) kap = powerlaw(f, xc[D.off_rn + 2 * I], xc[D.off_rn + 2 * I + 1], D.tspan);
        dg[I] = kap;
        zs[I] = zc[I * K2 + 2 * k0];
        zs[n + I] = zc[I * K2 + 2 * k0 + 1];
      }
      __syncthreads();
      for (int e = tid; e < n * n; e += 256) {
        const int i = e / n, j = e - (e / n) * n;
        if (j <= i) A[i * ns + j] = rho * D.gamma[e] + (i == j ? dg[i] : 0.0);
      }
      __syncthreads();
      const int tx = tid & 15, ty = tid >> 4;
      bool pd = true;
      for (int j = 0; j < n; ++j) {
        const double ajj = A[j * ns + j];
        if (!(ajj > 0.0) || !isfinite(ajj)) {   // same value in every thread
          pd = false;
          break;
        }
        const double inv = 1.0 / ajj;
        for (int i = j + 1 + ty; i < n; i += 16) {
          const double aij = A[i * ns + j] * inv;
          for (int k = j + 1 + tx; k <= i; k += 16) A[i * ns + k] -= aij * A[k * ns + j];
        }
        __syncthreads();
      }
      if (!pd) {
        flag |= pt::kFlagNotPD;
        for (int I = tid; I < n; I += 256) {
          D.coef_rn[((size_t)I * D.rows_rn + rs) * cp + c] = 0.0;
          D.coef_rn[((size_t)I * D.rows_rn + rc) * cp + c] = 0.0;
        }
      } else {
        for (int j = tid; j < n; j += 256) dg[j] = sqrt(A[j * ns + j]);
        __syncthreads();
        for (int e = tid; e < n * n; e += 256) {
          const int i = e / n, j = e - (e / n) * n;
          if (j < i) A[i * ns + j] /= dg[j];
          else if (j == i) A[i * ns + j] = dg[j];
        }
        __syncthreads();
        // a = L z for sin and cos
        for (int e = tid; e < 2 * n; e += 256) {
          const int I = e >> 1, sc = e & 1;
          const double *zv = zs + sc * n;
          double s0 = 0.0, s1 = 0.0;
          int m = 0;
          for (; m + 1 <= I; m += 2) {
            s0 += A[I * ns + m] * zv[m];
            s1 += A[I * ns + m + 1] * zv[m + 1];
          }
          if (m <= I) s0 += A[I * ns + m] * zv[m];
          D.coef_rn[((size_t)I * D.rows_rn + (sc ? rc : rs)) * cp + c] = s0 + s1;
        }
        // keep L (packed row-major) for the adjoint
        const int np = (n * (n + 1)) / 2;
        double *dst = D.lstore + ((size_t)c * D.nf_gw + k0) * np;
        for (int e = tid; e < n * n; e += 256) {
          const int i = e / n, j = e - (e / n) * n;
          if (j <= i) dst[pk(i, j)] = A[i * ns + j];
        }
      }
    }
  }

  // ---- DM block -------------------------------------------------------------
  if (k0 < D.nf_dm) {
    const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
    const double *zd = xc + D.off_zdm;
    const int K2 = 2 * D.nf_dm;
    for (int I = tid; I < n; I += 256) {
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
  if (tid == 0) {
    D.flag_k[(size_t)c * kmax + k0] = bad ? 0 : flag;
    D.zsq_k[(size_t)c * kmax + k0] = bad ? 0.0 : zz;
  }
}

// ---------------------------------------------------------------------------
// Backward: grid (kmax, n_chains), block 256.
// LDS (dense frequencies): Lp, Wp packed over nb*16 rows, vectors.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_spec_bwd(Dev D, const double *__restrict__ x,
                                                  double *__restrict__ grad) {
  extern __shared__ double lds[];
  __shared__ double red[256];
  __shared__ int ired[256];
  const int k0 = blockIdx.x;
  const int c = blockIdx.y;
  const int tid = threadIdx.x;
  const int n = D.n_psr;
  const int kmax = max(D.ka, D.nf_dm);
  const double f = (k0 + 1) / D.tspan;
  const double lnfy = log(f * pt::kYear);
  const double *xc = x + (size_t)c * D.d;
  double *gc = grad + (size_t)c * D.d;
  const size_t cp = D.c_pad;
  const int fl0 = D.flag_k[(size_t)c * kmax + k0];
  const bool skip = D.st_pre[c] != 0 || fl0 != 0;
  bool fin = true;

  if (k0 < D.ka) {
    const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
    const double *zc = xc + D.off_z;
    const int K2 = 2 * D.ka;
    const bool dense = k0 < D.nf_gw;
    double *dth = D.dth_k + ((size_t)c * D.ka + k0) * 2;
    double *drn = D.drn_k + ((size_t)c * D.ka + k0) * n * 2;
    if (skip) {
      for (int I = tid; I < n; I += 256) {
        gc[D.off_z + I * K2 + 2 * k0] = 0.0;
        gc[D.off_z + I * K2 + 2 * k0 + 1] = 0.0;
        drn[2 * I] = 0.0;
        drn[2 * I + 1] = 0.0;
      }
      if (tid == 0) { dth[0] = 0.0; dth[1] = 0.0; }
    } else if (!dense) {
      for (int I = tid; I < n; I += 256) {
        const double *th = xc + D.off_rn + 2 * I;
        const double sq = sqrt(powerlaw(f, th[0], th[1], D.tspan));
        const double ab_s = D.bar_rn[((size_t)I * D.rows_rn + rs) * cp + c];
        const double ab_c = D.bar_rn[((size_t)I * D.rows_rn + rc) * cp + c];
        const double z_s = zc[I * K2 + 2 * k0], z_c = zc[I * K2 + 2 * k0 + 1];
        const double g_s = sq * ab_s - z_s, g_c = sq * ab_c - z_c;
        gc[D.off_z + I * K2 + 2 * k0] = g_s;
        gc[D.off_z + I * K2 + 2 * k0 + 1] = g_c;
        // d sqrt(kappa)/d log10A = ln10 sqrt(kappa); d/dgamma = -1/2 ln(f yr) sqrt(kappa)
        const double az = (ab_s * z_s + ab_c * z_c) * sq;
        const double d0 = (k0 < D.nf_rn) ? az * pt::kLn10 : 0.0;
        const double d1 = (k0 < D.nf_rn) ? az * (-0.5 * lnfy) : 0.0;
        drn[2 * I] = d0;
        drn[2 * I + 1] = d1;
        fin = fin && isfinite(g_s) && isfinite(g_c) && isfinite(d0) && isfinite(d1);
      }
      if (tid == 0) { dth[0] = 0.0; dth[1] = 0.0; }
    } else {
      const int nb = (n + 15) >> 4, np = 16 * nb;        // padded size
      const int npk = (np * (np + 1)) / 2;
      double *Lp = lds;                                  // packed [np], later M
      double *Wp = Lp + npk;                             // packed [np]
      double *v = Wp + npk;                              // [2][np]
      double *zv = v + 2 * np;                           // [2][np]
      double *ab = zv + 2 * np;                          // [2][np]
      const int nl = (n * (n + 1)) / 2;
      const double *src = D.lstore + ((size_t)c * D.nf_gw + k0) * nl;
      for (int e = tid; e < npk; e += 256) Lp[e] = 0.0;
      __syncthreads();
      for (int e = tid; e < nl; e += 256) Lp[e] = src[e];   // same packing for rows < n
      for (int i = n + tid; i < np; i += 256) Lp[pk(i, i)] = 1.0;   // identity padding
      for (int e = tid; e < 2 * np; e += 256) {
        const int I = e % np, sc = e / np;
        double zz = 0.0, aa = 0.0;
        if (I < n) {
          zz = zc[I * K2 + 2 * k0 + sc];
          aa = D.bar_rn[((size_t)I * D.rows_rn + (sc ? rc : rs)) * cp + c];
        }
        zv[e] = zz;
        ab[e] = aa;
      }
      __syncthreads();
      // v_c = L^T abar_c ; dz = v - z
      for (int e = tid; e < 2 * np; e += 256) {
        const int I = e % np, sc = e / np;
        double s = 0.0;
        if (I < n)
          for (int m = I; m < n; ++m) s += Lp[pk(m, I)] * ab[sc * np + m];
        v[e] = s;
        if (I < n) {
          const double g = s - zv[e];
          gc[D.off_z + I * K2 + 2 * k0 + sc] = g;
          fin = fin && isfinite(g);
        }
      }
      // W = L^-1, blocked 16x16: diagonal blocks first, then block rows.
      for (int e = tid; e < 16 * nb; e += 256) {
        const int B = e >> 4, col = e & 15, b0 = 16 * B;
        // column col of the inverse of the diagonal block B
        for (int a = col; a < 16; ++a) {
          double s = (a == col) ? 1.0 : 0.0;
          for (int m = col; m < a; ++m) s -= Lp[pk(b0 + a, b0 + m)] * Wp[pk(b0 + m, b0 + col)];
          Wp[pk(b0 + a, b0 + col)] = s / Lp[pk(b0 + a, b0 + a)];
        }
      }
      __syncthreads();
      {
        const int r = tid >> 4, cc = tid & 15;           // 256 threads = one 16x16 block
        for (int I = 1; I < nb; ++I) {
          // T_J = sum_{K=J}^{I-1} L_IK W_KJ for all J < I, stored in the (I, J)
          // blocks of W, then W_IJ = -W_II T_J.
          const int gi = 16 * I + r;
#pragma unroll
          for (int J = 0; J < 8; ++J) {
            if (J < I) {
              const int gj = 16 * J + cc;
              double s = 0.0;
              for (int m = gj; m < 16 * I; ++m) s += Lp[pk(gi, m)] * Wp[pk(m, gj)];
              Wp[pk(gi, gj)] = s;
            }
          }
          __syncthreads();
          double tv[8];
#pragma unroll
          for (int J = 0; J < 8; ++J) {
            tv[J] = 0.0;
            if (J < I) {
              const int gj = 16 * J + cc;
              double s = 0.0;
              for (int m = 0; m <= r; ++m) s += Wp[pk(gi, 16 * I + m)] * Wp[pk(16 * I + m, gj)];
              tv[J] = -s;
            }
          }
          __syncthreads();
#pragma unroll
          for (int J = 0; J < 8; ++J)
            if (J < I) Wp[pk(gi, 16 * J + cc)] = tv[J];
          __syncthreads();
        }
      }
      // d/dkappa_I = sum_c sum_{a>=I} W_aI v_a (sum_{I<=b<a} z_b W_bI + z_a W_aI / 2)
      for (int I = tid; I < n; I += 256) {
        double acc = 0.0;
        for (int sc = 0; sc < 2; ++sc) {
          double pre = 0.0;
          for (int a = I; a < n; ++a) {
            const double w = Wp[pk(a, I)];
            const double zw = zv[sc * np + a] * w;
            acc += w * v[sc * np + a] * (pre + 0.5 * zw);
            pre += zw;
          }
        }
        const double kap = (k0 < D.nf_rn)
                               ? powerlaw(f, xc[D.off_rn + 2 * I], xc[D.off_rn + 2 * I + 1], D.tspan)
                               : 0.0;
        const double d0 = acc * kap * 2.0 * pt::kLn10, d1 = acc * kap * (-lnfy);
        drn[2 * I] = d0;
        drn[2 * I + 1] = d1;
        fin = fin && isfinite(d0) && isfinite(d1);
      }
      __syncthreads();
      // M = W G (lower x lower) into Lp
      for (int e = tid; e < nl; e += 256) {
        // decode packed (a, I)
        int a = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (pk(a, 0) > e) --a;
        while (pk(a + 1, 0) <= e) ++a;
        const int I = e - pk(a, 0);
        double s = 0.0;
        for (int m = I; m <= a; ++m) s += Wp[pk(a, m)] * D.gchol[pk(m, I)];
        Lp[e] = s;
      }
      __syncthreads();
      // d/drho = sum_c sum_m sum_{b>=m} z_b M_bm (sum_{a>b} v_a M_am + v_b M_bm / 2)
      double dr = 0.0;
      for (int m = tid; m < n; m += 256) {
        for (int sc = 0; sc < 2; ++sc) {
          double suf = 0.0;
          for (int b = n - 1; b >= m; --b) {
            const double Mb = Lp[pk(b, m)];
            const double vm = v[sc * np + b] * Mb;
            dr += zv[sc * np + b] * Mb * (suf + 0.5 * vm);
            suf += vm;
          }
        }
      }
      dr = block_sum(dr, red);
      if (tid == 0) {
        const double rho = powerlaw(f, xc[D.off_gw], xc[D.off_gw + 1], D.tspan);
        dth[0] = dr * rho * 2.0 * pt::kLn10;
        dth[1] = dr * rho * (-lnfy);
        fin = fin && isfinite(dth[0]) && isfinite(dth[1]);
      }
    }
  }

  if (k0 < D.nf_dm) {
    const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
    const double *zd = xc + D.off_zdm;
    const int K2 = 2 * D.nf_dm;
    double *ddm = D.ddm_k + ((size_t)c * D.nf_dm + k0) * n * 2;
    for (int I = tid; I < n; I += 256) {
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
      const double g_s = sq * ab_s - z_s, g_c = sq * ab_c - z_c;
      gc[D.off_zdm + I * K2 + 2 * k0] = g_s;
      gc[D.off_zdm + I * K2 + 2 * k0 + 1] = g_c;
      const double az = (ab_s * z_s + ab_c * z_c) * sq;
      const double d0 = az * pt::kLn10, d1 = az * (-0.5 * lnfy);
      ddm[2 * I] = d0;
      ddm[2 * I + 1] = d1;
      fin = fin && isfinite(g_s) && isfinite(g_c) && isfinite(d0) && isfinite(d1);
    }
  }
  fin = block_all(fin, ired);
  if (tid == 0 && !fin) D.flag_k[(size_t)c * kmax + k0] = fl0 | pt::kFlagOutNonfinite;
}

}  // namespace

namespace ptk {

size_t spec_fwd_lds(int n) { return ((size_t)n * (n | 1) + 3 * (size_t)n) * sizeof(double); }

size_t spec_bwd_lds(int n) {
  const size_t np = 16 * (size_t)((n + 15) / 16);
  return (np * (np + 1) + 6 * np) * sizeof(double);
}

hipError_t set_spec_lds_limits(size_t fwd_bytes, size_t bwd_bytes) {
  hipError_t e = hipFuncSetAttribute((const void *)k_spec_fwd,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)fwd_bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)k_spec_bwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bwd_bytes);
}

hipError_t launch_spec_fwd(const pt::Dev &D, const double *x, hipStream_t s) {
  const int kmax = max(D.ka, D.nf_dm);
  const int nblk = kmax * D.c_pad + D.n_prep;
  if (nblk == 0) return hipSuccess;
  const size_t lds = D.nf_gw > 0 ? spec_fwd_lds(D.n_psr) : 0;
  hipLaunchKernelGGL(k_spec_fwd, dim3(nblk), dim3(256), lds, s, D, x);
  return hipGetLastError();
}

hipError_t launch_spec_bwd(const pt::Dev &D, const double *x, double *grad, hipStream_t s) {
  const int kmax = max(D.ka, D.nf_dm);
  if (kmax == 0 || D.n_chains == 0) return hipSuccess;
  const size_t lds = D.nf_gw > 0 ? spec_bwd_lds(D.n_psr) : 0;
  hipLaunchKernelGGL(k_spec_bwd, dim3(kmax, D.n_chains), dim3(256), lds, s, D, x, grad);
  return hipGetLastError();
}

}  // namespace ptk
