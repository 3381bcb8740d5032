// Per-chain kernels of the spectral side that need no dense factorisation:
// power-law spectra (Sec. IV.A, Eq. power_law), the diagonal prior of the
// frequencies without the common process and the DM prior with their
// whitening transforms (Sec. II.B, Eq. standardizing_transform, mu = 0) and
// adjoints; the input checks, the timing-model rows of the coefficient
// panels and the CW constants.  The frequencies that carry the common process (dense
// phi_k = rho_k Gamma + diag kappa) are factorised in k_cholt / k_chol.
//
//   diagonal frequencies:  a_Ik = sqrt(kappa_Ik) z_Ik,  dz = sqrt(kappa) abar - z,
//     d/dlog10A_I = ln10 sqrt(kappa) abar.z,  d/dgamma_I = -1/2 ln(f yr) sqrt(kappa) abar.z
//   DM: the same with kappa^DM and abar^DM.
#include "common.h"
#include "cw_dev.h"

namespace {

using pt::Dev;
using pt::powerlaw;

// ---------------------------------------------------------------------------
// Forward: grid (c_pad, segments), block 256.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_spec_fwd(Dev D, const double *__restrict__ x) {
  __shared__ double red[4];
  __shared__ int kflag[PTAFS_MAX_HARM];
  const int tid = threadIdx.x;
  const int n = D.n_psr;
  const int kmax = max(D.ka, D.nf_dm);
  const int c = blockIdx.x;                  // chain (padded)
  const int seg = blockIdx.y;                // frequency segment: k = seg, seg + kSpecSeg, ...
  const bool real = c < D.n_chains;
  const double *xc = x + (size_t)(real ? c : 0) * D.d;
  const size_t cp = D.c_pad;

  // ---- prior box (every segment needs it)
  bool ok = real;
  if (real)
    for (int i = tid; i < D.n_theta; i += 256) {
      const double v = xc[i];
      if (!(v >= D.prior_lo[i] && v <= D.prior_hi[i])) ok = false;
    }
  const bool bad = !__syncthreads_and(ok);
  if (tid < PTAFS_MAX_HARM) kflag[tid] = 0;
  // finiteness and squared norm of this segment's slice of (u, z, z_dm)
  {
    const int nseg = gridDim.y, len = D.d - D.off_u;
    const int e0 = D.off_u + (int)(((long long)len * seg) / nseg);
    const int e1 = D.off_u + (int)(((long long)len * (seg + 1)) / nseg);
    double zz = 0.0;
    bool fin = true;
    if (real)
      for (int e = e0 + tid; e < e1; e += 256) {
        const double v = xc[e];
        fin = fin && isfinite(v);
        zz += v * v;
      }
    zz = pt::block_sum256(zz, red);
    fin = __syncthreads_and(fin);
    if (tid == 0) {
      D.zz_seg[(size_t)c * pt::kSpecSeg + seg] = zz;
      D.fin_seg[(size_t)c * pt::kSpecSeg + seg] = fin ? 1 : 0;
    }
  }

  if (seg == 0) {
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
    // coefficient rows no frequency owns: timing model b = sigma_b u, zeros
    for (int idx = tid; idx < n * D.n_free_rn; idx += 256) {
      const int I = idx / D.n_free_rn, row = D.free_rn[idx - I * D.n_free_rn];
      const pt::Slot sl = pt::rn_slot(row, D.kb);
      const double v = (sl.kind == 1 && !zero) ? D.sigma_b * xc[D.off_u + 3 * I + sl.tm] : 0.0;
      D.coef_rn[((size_t)I * D.rows_rn + row) * cp + c] = v;
    }
    for (int idx = tid; idx < n * D.n_free_dm; idx += 256) {
      const int I = idx / D.n_free_dm, row = D.free_dm[idx - I * D.n_free_dm];
      D.coef_dm[((size_t)I * D.rows_dm + row) * cp + c] = 0.0;
    }
  }
  __syncthreads();

  // ---- this segment's frequencies: diagonal prior (no common process),
  //      L = diag(sqrt(kappa)), and the DM prior; thread = (frequency, pulsar)
  const int nks = (kmax - seg + pt::kSpecSeg - 1) / pt::kSpecSeg;
  const int K2 = 2 * D.ka, K2d = 2 * D.nf_dm;
  for (int idx = tid; idx < nks * n; idx += 256) {
    const int j = idx / n, I = idx - j * n;
    const int k0 = seg + pt::kSpecSeg * j;
    const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
    const double f = (k0 + 1) / D.tspan;
    if (k0 >= D.nf_gw && k0 < D.ka) {
      double vs = 0.0, vc = 0.0;
      if (!bad) {
        const double kap =
            (k0 < D.nf_rn) ? powerlaw(f, xc[D.off_rn + 2 * I], xc[D.off_rn + 2 * I + 1], D.tspan) : 0.0;
        if (!(kap > 0.0) || !isfinite(kap)) atomicOr(&kflag[k0], pt::kFlagNotPD);
        const double sq = sqrt(kap);
        vs = sq * xc[D.off_z + I * K2 + 2 * k0];
        vc = sq * xc[D.off_z + I * K2 + 2 * k0 + 1];
      }
      D.coef_rn[((size_t)I * D.rows_rn + rs) * cp + c] = vs;
      D.coef_rn[((size_t)I * D.rows_rn + rc) * cp + c] = vc;
    }
    if (k0 < D.nf_dm) {
      double vs = 0.0, vc = 0.0;
      if (!bad) {
        const double sq = sqrt(powerlaw(f, xc[D.off_dm + 2 * I], xc[D.off_dm + 2 * I + 1], D.tspan));
        vs = sq * xc[D.off_zdm + I * K2d + 2 * k0];
        vc = sq * xc[D.off_zdm + I * K2d + 2 * k0 + 1];
      }
      D.coef_dm[((size_t)I * D.rows_dm + rs) * cp + c] = vs;
      D.coef_dm[((size_t)I * D.rows_dm + rc) * cp + c] = vc;
    }
  }
  __syncthreads();
  // owned flags (the dense frequencies flag themselves in flag_dense)
  for (int j = tid; j < nks; j += 256) {
    const int k0 = seg + pt::kSpecSeg * j;
    D.flag_k[(size_t)c * kmax + k0] = bad ? 0 : kflag[k0];
  }
}

// ---------------------------------------------------------------------------
// Backward: grid (n_chains, segments), block 256 (the diagonal and DM
// frequencies; the dense ones are in k_cholt / k_chol).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_spec_bwd(Dev D, const double *__restrict__ x,
                                                  double *__restrict__ grad) {
  const int c = blockIdx.x, seg = blockIdx.y;
  const int tid = threadIdx.x;
  const int n = D.n_psr;
  const int kmax = max(D.ka, D.nf_dm);
  const double *xc = x + (size_t)c * D.d;
  double *gc = grad + (size_t)c * D.d;
  const size_t cp = D.c_pad;
  int fl = 0;
  for (int k = tid; k < kmax; k += 256) fl |= D.flag_k[(size_t)c * kmax + k];
  for (int k = tid; k < D.nf_gw; k += 256) fl |= D.flag_dense[(size_t)c * D.nf_gw + k];
  const bool skip = __syncthreads_or(fl != 0 || D.st_pre[c] != 0);
  bool fin = true;

  const int nks = (kmax - seg + pt::kSpecSeg - 1) / pt::kSpecSeg;
  const int K2 = 2 * D.ka, K2d = 2 * D.nf_dm;
  for (int idx = tid; idx < nks * n; idx += 256) {
    const int j = idx / n, I = idx - j * n;
    const int k0 = seg + pt::kSpecSeg * j;
    const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
    const double f = (k0 + 1) / D.tspan;
    const double lnfy = log(f * pt::kYear);
    if (k0 >= D.nf_gw && k0 < D.ka) {
      double *drn = D.drn_k + ((size_t)c * D.ka + k0) * n * 2;
      double g_s = 0.0, g_c = 0.0, d0 = 0.0, d1 = 0.0;
      if (!skip) {
        const double sq = sqrt(powerlaw(f, xc[D.off_rn + 2 * I], xc[D.off_rn + 2 * I + 1], D.tspan));
        const double ab_s = D.bar_rn[((size_t)I * D.rows_rn + rs) * cp + c];
        const double ab_c = D.bar_rn[((size_t)I * D.rows_rn + rc) * cp + c];
        const double z_s = xc[D.off_z + I * K2 + 2 * k0], z_c = xc[D.off_z + I * K2 + 2 * k0 + 1];
        g_s = sq * ab_s - z_s;
        g_c = sq * ab_c - z_c;
        // d sqrt(kappa)/d log10A = ln10 sqrt(kappa); d/dgamma = -1/2 ln(f yr) sqrt(kappa)
        const double az = (ab_s * z_s + ab_c * z_c) * sq;
        d0 = (k0 < D.nf_rn) ? az * pt::kLn10 : 0.0;
        d1 = (k0 < D.nf_rn) ? az * (-0.5 * lnfy) : 0.0;
        fin = fin && isfinite(g_s) && isfinite(g_c) && isfinite(d0) && isfinite(d1);
      }
      gc[D.off_z + I * K2 + 2 * k0] = g_s;
      gc[D.off_z + I * K2 + 2 * k0 + 1] = g_c;
      drn[2 * I] = d0;
      drn[2 * I + 1] = d1;
      if (I == 0) {
        double *dth = D.dth_k + ((size_t)c * D.ka + k0) * 2;
        dth[0] = 0.0;
        dth[1] = 0.0;
      }
    }
    if (k0 < D.nf_dm) {
      double *ddm = D.ddm_k + ((size_t)c * D.nf_dm + k0) * n * 2;
      double g_s = 0.0, g_c = 0.0, d0 = 0.0, d1 = 0.0;
      if (!skip) {
        const double sq = sqrt(powerlaw(f, xc[D.off_dm + 2 * I], xc[D.off_dm + 2 * I + 1], D.tspan));
        const double ab_s = D.bar_dm[((size_t)I * D.rows_dm + rs) * cp + c];
        const double ab_c = D.bar_dm[((size_t)I * D.rows_dm + rc) * cp + c];
        const double z_s = xc[D.off_zdm + I * K2d + 2 * k0], z_c = xc[D.off_zdm + I * K2d + 2 * k0 + 1];
        g_s = sq * ab_s - z_s;
        g_c = sq * ab_c - z_c;
        const double az = (ab_s * z_s + ab_c * z_c) * sq;
        d0 = az * pt::kLn10;
        d1 = az * (-0.5 * lnfy);
        fin = fin && isfinite(g_s) && isfinite(g_c) && isfinite(d0) && isfinite(d1);
      }
      gc[D.off_zdm + I * K2d + 2 * k0] = g_s;
      gc[D.off_zdm + I * K2d + 2 * k0 + 1] = g_c;
      ddm[2 * I] = d0;
      ddm[2 * I + 1] = d1;
    }
  }
  fin = __syncthreads_and(fin);
  if (tid == 0) D.flag_out[(size_t)c * (kmax + pt::kSpecSeg) + kmax + seg] = fin ? 0 : pt::kFlagOutNonfinite;
}

}  // namespace

namespace ptk {

hipError_t launch_spec_fwd(const pt::Dev &D, const double *x, hipStream_t s) {
  const int kmax = max(D.ka, D.nf_dm);
  const int nseg = max(1, min(pt::kSpecSeg, kmax));
  if (D.c_pad == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spec_fwd, dim3(D.c_pad, nseg), dim3(256), 0, s, D, x);
  return hipGetLastError();
}

hipError_t launch_spec_bwd(const pt::Dev &D, const double *x, double *grad, hipStream_t s) {
  if (D.n_chains == 0) return hipSuccess;
  const int kmax = max(D.ka, D.nf_dm);
  const int nseg = max(1, min(pt::kSpecSeg, kmax));
  hipLaunchKernelGGL(k_spec_bwd, dim3(D.n_chains, nseg), dim3(256), 0, s, D, x, grad);
  return hipGetLastError();
}

}  // namespace ptk
