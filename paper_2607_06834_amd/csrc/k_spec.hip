// Per-frequency kernels that need no dense factorisation: power-law spectra
// (Sec. IV.A, Eq. power_law), the diagonal prior of the frequencies without
// the common process and the DM prior, with their whitening transforms
// (Sec. II.B, Eq. standardizing_transform, mu = 0) and adjoints; the input
// checks, the timing-model rows of the coefficient panels, the CW constants
// and the per-TOA white-noise preparation (Eq. WN_cov).  One 256-thread
// workgroup per (frequency, chain).  The frequencies that carry the common
// process (dense phi_k = rho_k Gamma + diag kappa) are factorised in k_chol.
//
//   diagonal frequencies:  a_Ik = sqrt(kappa_Ik) z_Ik,  dz = sqrt(kappa) abar - z,
//     d/dlog10A_I = ln10 sqrt(kappa) abar.z,  d/dgamma_I = -1/2 ln(f yr) sqrt(kappa) abar.z
//   DM: the same with kappa^DM and abar^DM.
#include "common.h"
#include "cw_dev.h"

namespace {

using pt::Dev;

using pt::pk;
using pt::powerlaw;

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
    }
    // dense frequencies: factorisation and transform in k_chol_fwd
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
    if (dense) {
      // dense frequencies: adjoint in k_chol_bwd
    } else if (skip) {
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

hipError_t launch_spec_fwd(const pt::Dev &D, const double *x, hipStream_t s) {
  const int kmax = max(D.ka, D.nf_dm);
  const int nblk = kmax * D.c_pad + D.n_prep;
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spec_fwd, dim3(nblk), dim3(256), 0, s, D, x);
  return hipGetLastError();
}

hipError_t launch_spec_bwd(const pt::Dev &D, const double *x, double *grad, hipStream_t s) {
  const int kmax = max(D.ka, D.nf_dm);
  if (kmax == 0 || D.n_chains == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spec_bwd, dim3(kmax, D.n_chains), dim3(256), 0, s, D, x, grad);
  return hipGetLastError();
}

}  // namespace ptk
