// Assembly of log p and the hyper-parameter / timing-model gradient per chain
// (Sec. IV: Eqs. likelihood and a_prior under the whitening a = L z, with the
// uniform hyper-priors of Sec. IV.A):
//
//   log p = sum_I (-1/2 chi2_I) - 1/2 sum_i ln N_i - n/2 ln 2pi
//           - 1/2 (|u|^2 + |z|^2 + |z_dm|^2) - d_z/2 ln 2pi - sum ln(hi - lo)
//
// Per-frequency contributions to the hyper-parameter gradient are summed in
// frequency order; chains flagged by any stage get log p = -inf, gradient 0.
// Inside a leapfrog trajectory the same workgroup then applies the kick and
// drift to its chain (App. A, Eq. Hamilton's_eq), saving a launch.
#include "common.h"

namespace {

using pt::Dev;

// a gradient entry computed by this thread: stored (overwritten with zero
// below if the chain's status turns out nonzero) and tested for finiteness
__device__ inline void gtheta_or_u(double *gc, int i, double g, bool &fin) {
  gc[i] = g;
  fin = fin && isfinite(g);
}

// one workgroup of kFinT threads per chain
constexpr int kFinT = 1024;
constexpr int kFinW = kFinT / 64;

__global__ __launch_bounds__(kFinT) void k_finalize(Dev D, const double *x, double *__restrict__ logp,
                                                  double *grad, int32_t *__restrict__ status,
                                                  pt::Kick kick, int has_kick) {
  __shared__ double red[kFinW], red2[kFinW];
  __shared__ int ired[kFinW];
  // this kernel's gradient entries (theta, then the timing model), for the kick
  __shared__ double g_s[4 * PTAFS_MAX_PSR + 10 + 3 * PTAFS_MAX_PSR];
  const int c = blockIdx.x;
  const int t = threadIdx.x;
  const double *xc = x + (size_t)c * D.d;
  double *gc = grad + (size_t)c * D.d;
  const size_t cp = D.c_pad;
  const int n = D.n_psr;
  const int kmax = max(D.ka, D.nf_dm);

  // Every input of the assembly (condition flags, the norm of the whitened
  // inputs, the chi^2 partials, the per-frequency gradient parts) is loaded
  // before the first reduction waits on it.  A thread computes the theta
  // gradient entry t and the timing-model entry t whatever the status, and
  // writes them (or zeros) once the status is known.
  const int nseg = max(1, min(pt::kSpecSeg, kmax));
  const int32_t *fo = D.flag_out + (size_t)c * (kmax + pt::kSpecSeg);
  const int pre = D.st_pre[c];
  // every frequency, segment, theta entry, timing-model entry and pulsar has
  // one thread
  static_assert(4 * PTAFS_MAX_PSR + 10 <= kFinT && 3 * PTAFS_MAX_PSR <= kFinT, "one entry per thread");
  static_assert(PTAFS_MAX_HARM <= kFinT && pt::kSpecSeg <= kFinT, "one frequency per thread");
  // the condition flags: clamped indices under uniform conditions, selected
  // when combined, so that no load waits for another
  int f1 = 0, f2 = 0, f3 = 0, f4 = 0;
  if (kmax > 0) f1 = D.flag_k[(size_t)c * kmax + min(t, kmax - 1)];
  if (D.nf_gw > 0) {
    const int k = min(t, D.nf_gw - 1);
    f2 = D.flag_dense[(size_t)c * D.nf_gw + k];
    f3 = fo[k];
  }
  f4 = fo[kmax + min(t, nseg - 1)];
  // the timing-model gradient's inputs and the chi^2 partial first (their
  // loads overlap those below)
  double ub = 0.0, ux = 0.0;
  if (t < 3 * n) {
    const int I = t / 3, row = pt::tm_row(t % 3, D.kb);
    ub = D.bar_rn[((size_t)I * D.rows_rn + row) * cp + c];
    ux = xc[D.off_u + t];
  }
  double ch = (t < n) ? D.chi_p[(size_t)t * cp + c] : 0.0;
  // the per-frequency parts of this thread's power-law entry (the common
  // process's two, then red noise and DM per pulsar and component; the CW's
  // follow below), loaded here, summed in frequency order after the norm
  const int n_pl = D.has_cw ? D.off_cw : D.n_theta;
  int K = 0;
  double tv[32];
  if (t < n_pl) {
    const double *src;
    if (t < D.off_rn) {
      src = D.dth_k + (size_t)c * D.ka * 2 + (t - D.off_gw);
      K = D.ka;
    } else if (t < D.off_dm) {
      src = pt::drn_at(D, c, (t - D.off_rn) >> 1, 0) + ((t - D.off_rn) & 1);
      K = D.ka;
    } else {
      src = pt::ddm_at(D, c, (t - D.off_dm) >> 1, 0) + ((t - D.off_dm) & 1);
      K = D.nf_dm;
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) tv[k] = src[2 * min(k, K - 1)];
  }
  // finiteness and squared norm of (u, z, z_dm): twelve elements per thread
  // with their loads issued together (one pass up to 12288 of them)
  double zz = 0.0;
  bool fin_in = true;
  {
    constexpr int B = 12;
    for (int i0 = D.off_u + t; i0 < D.d; i0 += kFinT * B) {
      double v[B];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int i = i0 + kFinT * b;
        v[b] = i < D.d ? xc[i] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        fin_in = fin_in && isfinite(v[b]);
        zz += v[b] * v[b];
      }
    }
  }
  // hyper-parameter gradient entries (frequency sums in order) and the
  // timing model, d/du = sigma_b M^T g - u
  int fl = (t < kmax ? f1 : 0) | (t < D.nf_gw ? f2 | f3 : 0) | (t < nseg ? f4 : 0);
  bool fin = true;
  if (t < n_pl) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 32; ++k) s += (k < K) ? tv[k] : 0.0;
    gtheta_or_u(gc, t, s, fin);
    g_s[t] = s;
  } else if (D.has_cw && t < D.n_theta) {
    // the CW parameters' entries, over the pulsars in order, eight loads at a time
    const double *q = D.cw_p + (size_t)(t - D.off_cw) * cp + c;
    double s = 0.0;
#pragma unroll 1
    for (int p0 = 0; p0 < n; p0 += 8) {
      double v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = (p0 + k < n) ? q[(size_t)(p0 + k) * 8 * cp] : 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) s += v[k];
    }
    gtheta_or_u(gc, t, s, fin);
    g_s[t] = s;
  }
  if (t < 3 * n) {
    const double gu = D.sigma_b * ub - ux;
    gtheta_or_u(gc, D.off_u + t, gu, fin);
    g_s[D.off_u + t] = gu;
  }
  // Inside a trajectory, the kick's operands for the first BK elements per
  // thread (all of them up to BK kFinT = 9216 coordinates): p, x, M^-1 and
  // the gradient entries the earlier kernels wrote (from off_z on; this
  // kernel's own come from g_s).  Issued here, with clamped in-range
  // addresses and no branch between them, they arrive while the reductions
  // below wait.
  constexpr int BK = 9;
  double kp[BK], kg[BK], kx[BK], km[BK];
  if (has_kick) {
    const double *pw = kick.p + (size_t)c * D.d, *xw = kick.x + (size_t)c * D.d;
    const int last = D.d - 1;
#pragma unroll
    for (int b = 0; b < BK; ++b) {
      const int ic = min(t + kFinT * b, last);
      kp[b] = pw[ic];
      kx[b] = xw[ic];
      kg[b] = gc[max(ic, D.off_z)];
      km[b] = kick.inv_mass ? kick.inv_mass[ic] : 1.0;
    }
  }
  // ---- the reductions: one OR (flags, and the two finiteness tests as
  //      bits), two fixed-order sums
  constexpr int kBitInput = 1 << 28, kBitOutput = 1 << 29;
  {
    // all three in one pass: wave reductions, one barrier, then in every
    // wave lane i takes wave i's values and a second wave reduction combines
    // them (a fixed order, in three registers)
    const int f = pt::wave_or(fl | (fin_in ? 0 : kBitInput) | (fin ? 0 : kBitOutput));
    const double z = pt::wave_sum(zz), h = pt::wave_sum(ch);
    const int w = t >> 6, ln = t & 63;
    if (ln == 0) {
      ired[w] = f;
      red[w] = z;
      red2[w] = h;
    }
    __syncthreads();
    fl = pt::wave_or(ln < kFinW ? ired[ln] : 0);
    zz = pt::wave_sum(ln < kFinW ? red[ln] : 0.0);
    ch = pt::wave_sum(ln < kFinW ? red2[ln] : 0.0);
  }

  // ---- per-chain condition, in the order: prior box, non-finite input,
  //      CW coalescence, phi not positive definite, non-finite output
  int st = 0;
  if (pre == PTAFS_ST_PRIOR) st = PTAFS_ST_PRIOR;
  else if (fl & kBitInput) st = PTAFS_ST_NONFINITE;
  else if (pre == PTAFS_ST_CW) st = PTAFS_ST_CW;
  else if (fl & pt::kFlagNotPD) st = PTAFS_ST_NOTPD;
  else if (fl & pt::kFlagOutNonfinite) st = PTAFS_ST_NONFINITE;

  // ---- log p
  const double dz = (double)(D.d - D.off_u);
  double lp = -0.5 * ch - 0.5 * D.lnn_total - 0.5 * (double)D.n_toa * pt::kLn2Pi -
              0.5 * zz - 0.5 * dz * pt::kLn2Pi + D.prior_const;
  if (st == 0 && ((fl & kBitOutput) || !isfinite(lp))) st = PTAFS_ST_NONFINITE;
  if (st != 0) {
    // the theta and u entries this thread computed, then the rest
    for (int e = t; e < D.n_theta; e += kFinT) gc[e] = 0.0;
    for (int e = t; e < 3 * n; e += kFinT) gc[D.off_u + e] = 0.0;
    for (int i = D.off_z + t; i < D.d; i += kFinT) gc[i] = 0.0;
    lp = -INFINITY;
  }
  if (t == 0) {
    logp[c] = lp;
    status[c] = st;
  }
  if (has_kick) {
    if (t == 0 && kick.n_invalid && st != 0) kick.n_invalid[c] += 1;
    double *xw = kick.x + (size_t)c * D.d, *pw = kick.p + (size_t)c * D.d;
#pragma unroll
    for (int b = 0; b < BK; ++b) {
      const int i = t + kFinT * b;
      if (i >= D.d) continue;
      // (the gradient is zero when the status is nonzero)
      const double g = st != 0 ? 0.0 : (i < D.off_z ? g_s[i] : kg[b]);
      const double pi = kp[b] + kick.eps * g;
      pw[i] = pi;
      xw[i] = kx[b] + kick.eps * km[b] * pi;
    }
    if (D.d <= BK * kFinT) return;
    // the rest, beyond off_z: the gradient as stored (zeros when the status
    // is nonzero)
    __syncthreads();   // the workgroup's gradient stores are visible to all its threads
    constexpr int B = 12;  // elements per thread whose loads are issued together
    for (int i0 = BK * kFinT + t; i0 < D.d; i0 += kFinT * B) {
      double pv[B], gv[B], xv[B], iv[B];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int i = i0 + kFinT * b;
        const bool in = i < D.d;
        pv[b] = in ? pw[i] : 0.0;
        gv[b] = in ? gc[i] : 0.0;
        xv[b] = in ? xw[i] : 0.0;
        iv[b] = (in && kick.inv_mass) ? kick.inv_mass[i] : 1.0;
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int i = i0 + kFinT * b;
        if (i >= D.d) continue;
        const double pi = pv[b] + kick.eps * gv[b];
        pw[i] = pi;
        xw[i] = xv[b] + kick.eps * iv[b] * pi;
      }
    }
  }
}

}  // namespace

namespace ptk {

hipError_t launch_finalize(const pt::Dev &D, const double *x, double *logp, double *grad,
                           int32_t *status, hipStream_t s, const pt::Kick *kick) {
  if (D.n_chains == 0) return hipSuccess;
  const pt::Kick k = kick ? *kick : pt::Kick{};
  hipLaunchKernelGGL(k_finalize, dim3(D.n_chains), dim3(kFinT), 0, s, D, x, logp, grad, status, k,
                     kick ? 1 : 0);
  return hipGetLastError();
}

}  // namespace ptk
