// Work of the spectral side that needs no dense factorisation, as device
// bodies: k_spec's kernels call the per-chain forms (spec_fwd_block,
// spec_bwd_block), and the dense-frequency launches carry the 16-chain-block
// forms (spec_fwd_cb, spec_bwd_cb) in extra workgroups.  It covers the
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
#pragma once
#include "common.h"
#include "cw_dev.h"

namespace pt {

// Items per thread whose loads are issued together: up to 10 loads an item,
// within the 63 loads a wave can have in flight.
constexpr int kSpecBatch = 6;

// sqrt of a power-law spectrum (powerlaw_sqrt_k) given ln(f_k yr) already loaded
__device__ inline double powerlaw_sqrt_l(const Dev &D, double lnfy_k, double log10A, double gamma) {
  return exp(kLn10 * log10A - 0.5 * gamma * lnfy_k + 0.5 * D.pl_c);
}

// Forward of chain c (< c_pad) over the diagonal and DM frequencies
// k = k_first, k_first + k_step, ...; segment 0 also does the per-chain work
// (status of the prior box and the CW check, CW constants, timing-model
// rows).  One block of 256 threads; every thread of the block calls it.  The
// norm and finiteness of (u, z, z_dm) are taken in k_finalize.
// ---------------------------------------------------------------------------
__device__ inline void spec_fwd_block(const Dev &D, const double *__restrict__ x, int c, int seg,
                                      int k_first, int k_step) {
  __shared__ int kflag[PTAFS_MAX_HARM];
  const int tid = threadIdx.x;
  const int n = D.n_psr;
  const int kmax = max(D.ka, D.nf_dm);
  const bool real = c < D.n_chains;
  const double *xc = x + (size_t)(real ? c : 0) * D.d;
  const size_t cp = D.c_pad;

  // ---- prior box (every segment needs it): four parameters per thread per
  //      batch, loads issued together, indexes clamped to the last parameter
  bool ok = real;
  if (real) {
    constexpr int kB = 4;
    const int last = D.n_theta - 1;
    for (int i0 = 0; i0 < D.n_theta; i0 += 256 * kB) {
      double v[kB], lo[kB], hi[kB];
#pragma unroll
      for (int j = 0; j < kB; ++j) {
        const int i = min(i0 + tid + 256 * j, last);
        v[j] = xc[i];
        lo[j] = D.prior_lo[i];
        hi[j] = D.prior_hi[i];
      }
#pragma unroll
      for (int j = 0; j < kB; ++j)
        if (!(v[j] >= lo[j] && v[j] <= hi[j])) ok = false;
    }
  }
  const bool bad = !__syncthreads_and(ok);
  if (tid < PTAFS_MAX_HARM) kflag[tid] = 0;

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

  // ---- the frequencies: diagonal prior (no common process),
  //      L = diag(sqrt(kappa)), and the DM prior; thread = (frequency, pulsar)
  const int nks = (kmax - k_first + k_step - 1) / k_step;
  const int K2 = 2 * D.ka, K2d = 2 * D.nf_dm;
  const int total = nks * n;
  for (int base = tid; base < total; base += 256 * kSpecBatch) {
    // the inputs of kSpecBatch items first (their loads overlap), then the items
    double ra[kSpecBatch], rg[kSpecBatch], zs[kSpecBatch], zc[kSpecBatch];
    double da[kSpecBatch], dg[kSpecBatch], ws[kSpecBatch], wc[kSpecBatch], lf[kSpecBatch];
#pragma unroll
    for (int b = 0; b < kSpecBatch; ++b) {
      const int idx = base + 256 * b;
      ra[b] = rg[b] = zs[b] = zc[b] = da[b] = dg[b] = ws[b] = wc[b] = 0.0;
      // the frequency's ln(f yr), with the other inputs
      lf[b] = D.lnfy[min(k_first + k_step * ((idx < total ? idx : 0) / n), kmax - 1)];
      if (idx < total && !bad) {
        const int j = idx / n, I = idx - j * n;
        const int k0 = k_first + k_step * j;
        if (k0 >= D.nf_gw && k0 < D.ka) {
          if (k0 < D.nf_rn) {
            ra[b] = xc[D.off_rn + 2 * I];
            rg[b] = xc[D.off_rn + 2 * I + 1];
          }
          zs[b] = xc[D.off_z + I * K2 + 2 * k0];
          zc[b] = xc[D.off_z + I * K2 + 2 * k0 + 1];
        }
        if (k0 < D.nf_dm) {
          da[b] = xc[D.off_dm + 2 * I];
          dg[b] = xc[D.off_dm + 2 * I + 1];
          ws[b] = xc[D.off_zdm + I * K2d + 2 * k0];
          wc[b] = xc[D.off_zdm + I * K2d + 2 * k0 + 1];
        }
      }
    }
#pragma unroll
    for (int b = 0; b < kSpecBatch; ++b) {
      const int idx = base + 256 * b;
      if (idx >= total) continue;
      const int j = idx / n, I = idx - j * n;
      const int k0 = k_first + k_step * j;
      const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
      if (k0 >= D.nf_gw && k0 < D.ka) {
        double vs = 0.0, vc = 0.0;
        if (!bad) {
          const double sq = (k0 < D.nf_rn) ? powerlaw_sqrt_l(D, lf[b], ra[b], rg[b]) : 0.0;
          const double kap = sq * sq;
          if (!(kap > 0.0) || !isfinite(kap)) atomicOr(&kflag[k0], pt::kFlagNotPD);
          vs = sq * zs[b];
          vc = sq * zc[b];
          D.sqk_rn[sqk_at(D, c, I, k0)] = sq;   // for the adjoint
        }
        D.coef_rn[((size_t)I * D.rows_rn + rs) * cp + c] = vs;
        D.coef_rn[((size_t)I * D.rows_rn + rc) * cp + c] = vc;
      }
      if (k0 < D.nf_dm) {
        double vs = 0.0, vc = 0.0;
        if (!bad) {
          const double sq = powerlaw_sqrt_l(D, lf[b], da[b], dg[b]);
          vs = sq * ws[b];
          vc = sq * wc[b];
          D.sqk_dm[sqk_at(D, c, I, k0)] = sq;
        }
        D.coef_dm[((size_t)I * D.rows_dm + rs) * cp + c] = vs;
        D.coef_dm[((size_t)I * D.rows_dm + rc) * cp + c] = vc;
      }
    }
  }
  __syncthreads();
  // owned flags (the dense frequencies flag themselves in flag_dense)
  for (int j = tid; j < nks; j += 256) {
    const int k0 = k_first + k_step * j;
    D.flag_k[(size_t)c * kmax + k0] = bad ? 0 : kflag[k0];
  }
}

// ---------------------------------------------------------------------------
// Backward of chain c (< n_chains) over the diagonal and DM frequencies
// k = k_first, k_first + k_step, ... (the dense ones are in k_cholt / k_chol);
// the non-finite flag goes to slot `slot` of the chain's segment flags.  One
// block of 256 threads; every thread of the block calls it.
// ---------------------------------------------------------------------------
__device__ inline void spec_bwd_block(const Dev &D, const double *__restrict__ x,
                                      double *__restrict__ grad, int c, int k_first, int k_step,
                                      int slot) {
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

  const int nks = (kmax - k_first + k_step - 1) / k_step;
  const int K2 = 2 * D.ka, K2d = 2 * D.nf_dm;
  const int total = nks * n;
  for (int base = tid; base < total; base += 256 * kSpecBatch) {
    // the inputs of kSpecBatch items first (their loads overlap), then the items
    // (sqrt(kappa) as the forward stored it)
    double sr[kSpecBatch], as_[kSpecBatch], ac_[kSpecBatch], zs[kSpecBatch], zc[kSpecBatch];
    double sd[kSpecBatch], bs_[kSpecBatch], bc_[kSpecBatch], ws[kSpecBatch], wc[kSpecBatch];
    double lf[kSpecBatch];
#pragma unroll
    for (int b = 0; b < kSpecBatch; ++b) {
      const int idx = base + 256 * b;
      sr[b] = as_[b] = ac_[b] = zs[b] = zc[b] = 0.0;
      sd[b] = bs_[b] = bc_[b] = ws[b] = wc[b] = 0.0;
      // the frequency's ln(f yr), with the other inputs
      lf[b] = D.lnfy[min(k_first + k_step * ((idx < total ? idx : 0) / n), kmax - 1)];
      if (idx < total && !skip) {
        const int j = idx / n, I = idx - j * n;
        const int k0 = k_first + k_step * j;
        const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
        if (k0 >= D.nf_gw && k0 < D.ka) {
          sr[b] = D.sqk_rn[sqk_at(D, c, I, k0)];
          as_[b] = D.bar_rn[((size_t)I * D.rows_rn + rs) * cp + c];
          ac_[b] = D.bar_rn[((size_t)I * D.rows_rn + rc) * cp + c];
          zs[b] = xc[D.off_z + I * K2 + 2 * k0];
          zc[b] = xc[D.off_z + I * K2 + 2 * k0 + 1];
        }
        if (k0 < D.nf_dm) {
          sd[b] = D.sqk_dm[sqk_at(D, c, I, k0)];
          bs_[b] = D.bar_dm[((size_t)I * D.rows_dm + rs) * cp + c];
          bc_[b] = D.bar_dm[((size_t)I * D.rows_dm + rc) * cp + c];
          ws[b] = xc[D.off_zdm + I * K2d + 2 * k0];
          wc[b] = xc[D.off_zdm + I * K2d + 2 * k0 + 1];
        }
      }
    }
#pragma unroll
    for (int b = 0; b < kSpecBatch; ++b) {
      const int idx = base + 256 * b;
      if (idx >= total) continue;
      const int j = idx / n, I = idx - j * n;
      const int k0 = k_first + k_step * j;
      const double lnfy = lf[b];
      if (k0 >= D.nf_gw && k0 < D.ka) {
        double *drn = drn_at(D, c, I, k0);
        double g_s = 0.0, g_c = 0.0, d0 = 0.0, d1 = 0.0;
        if (!skip) {
          const double sq = sr[b];
          g_s = sq * as_[b] - zs[b];
          g_c = sq * ac_[b] - zc[b];
          // d sqrt(kappa)/d log10A = ln10 sqrt(kappa); d/dgamma = -1/2 ln(f yr) sqrt(kappa)
          const double az = (as_[b] * zs[b] + ac_[b] * zc[b]) * sq;
          d0 = (k0 < D.nf_rn) ? az * pt::kLn10 : 0.0;
          d1 = (k0 < D.nf_rn) ? az * (-0.5 * lnfy) : 0.0;
          fin = fin && isfinite(g_s) && isfinite(g_c) && isfinite(d0) && isfinite(d1);
        }
        gc[D.off_z + I * K2 + 2 * k0] = g_s;
        gc[D.off_z + I * K2 + 2 * k0 + 1] = g_c;
        drn[0] = d0;
        drn[1] = d1;
        if (I == 0) {
          double *dth = D.dth_k + ((size_t)c * D.ka + k0) * 2;
          dth[0] = 0.0;
          dth[1] = 0.0;
        }
      }
      if (k0 < D.nf_dm) {
        double *ddm = ddm_at(D, c, I, k0);
        double g_s = 0.0, g_c = 0.0, d0 = 0.0, d1 = 0.0;
        if (!skip) {
          const double sq = sd[b];
          g_s = sq * bs_[b] - ws[b];
          g_c = sq * bc_[b] - wc[b];
          const double az = (bs_[b] * ws[b] + bc_[b] * wc[b]) * sq;
          d0 = az * pt::kLn10;
          d1 = az * (-0.5 * lnfy);
          fin = fin && isfinite(g_s) && isfinite(g_c) && isfinite(d0) && isfinite(d1);
        }
        gc[D.off_zdm + I * K2d + 2 * k0] = g_s;
        gc[D.off_zdm + I * K2d + 2 * k0 + 1] = g_c;
        ddm[0] = d0;
        ddm[1] = d1;
      }
    }
  }
  fin = __syncthreads_and(fin);
  if (tid == 0) D.flag_out[(size_t)c * (kmax + pt::kSpecSeg) + kmax + slot] = fin ? 0 : pt::kFlagOutNonfinite;
}

// ---------------------------------------------------------------------------
// Chain-blocked forms, for the extra workgroups of the dense launches: the
// 16 chains c0 .. c0 + 15 over the frequencies [k_lo, k_hi); in the forward,
// segment 0 also writes the chains' status, and segment seg of nseg the
// seg-th share of the per-pulsar rows (CW constants, timing-model rows, zero
// rows).  The chain runs fastest over the threads,
// and a chain's frequencies next, so the chain-minor coefficient panels,
// adjoint panels and sqrt(kappa) move 16 chains (128 bytes) per access, and a
// chain's whitened inputs and gradient several frequencies at a time.  The
// results are those of spec_fwd_block / spec_bwd_block element for element.
// One block of 256 threads; every thread of the block calls them.
// ---------------------------------------------------------------------------
constexpr int kCB = 16;

__device__ inline void spec_fwd_cb(const Dev &D, const double *__restrict__ x, int c0, int k_lo,
                                   int k_hi, int seg, int nseg) {
  __shared__ int ired[4];
  __shared__ int kflag[kCB][PTAFS_MAX_HARM];
  __shared__ int czero[kCB];
  const int tid = threadIdx.x;
  const int n = D.n_psr;
  const int kmax = max(D.ka, D.nf_dm);
  const size_t cp = D.c_pad;
  auto row = [&](int cc) { return x + (size_t)(c0 + cc < D.n_chains ? c0 + cc : 0) * D.d; };
  for (int i = tid; i < kCB * PTAFS_MAX_HARM; i += 256) (&kflag[0][0])[i] = 0;

  // ---- prior box of the 16 chains: a thread takes a parameter, with the
  //      16 chains' values and the bounds loaded together
  int m = 0;
  {
    const int last = D.n_theta - 1;
    for (int i0 = 0; i0 < D.n_theta; i0 += 256) {
      const int i = min(i0 + tid, last);
      const double lo = D.prior_lo[i], hi = D.prior_hi[i];
      double v[kCB];
#pragma unroll
      for (int cc = 0; cc < kCB; ++cc) v[cc] = row(cc)[i];
#pragma unroll
      for (int cc = 0; cc < kCB; ++cc)
        if (!(v[cc] >= lo && v[cc] <= hi)) m |= 1 << cc;
    }
  }
  int badm = block_or256(m, ired);
#pragma unroll
  for (int cc = 0; cc < kCB; ++cc)
    if (c0 + cc >= D.n_chains) badm |= 1 << cc;

  {
    if (tid < kCB) {
      const int c = c0 + tid;
      const bool real = c < D.n_chains, bad = (badm >> tid) & 1;
      int st = 0;
      if (real && bad) st = PTAFS_ST_PRIOR;
      if (real && !bad && D.has_cw) {
        const double *cw = row(tid) + D.off_cw;
        const double M = exp(kLn10 * cw[2]) * kTsun;
        const double w0 = kPi * exp(kLn10 * cw[3]);
        const double y = 256.0 / 5.0 * exp(5.0 / 3.0 * log(M) + 8.0 / 3.0 * log(w0)) * D.tmax;
        if (!(y < 1.0)) st = PTAFS_ST_CW;
      }
      if (seg == 0) D.st_pre[c] = st;
      czero[tid] = (bad || st != 0) ? 1 : 0;
    }
    __syncthreads();
    // the segments share the per-pulsar rows, as (pulsar, chain) pairs
    const int pr_lo = n * kCB * seg / nseg, pr_hi = n * kCB * (seg + 1) / nseg;
    if (D.has_cw)
      for (int idx = pr_lo + tid; idx < pr_hi; idx += 256) {
        const int cc = idx & (kCB - 1), I = idx / kCB;
        const double *th = czero[cc] ? nullptr : row(cc) + D.off_cw;
        double v[kCwRows];
        cw_constants(th, D.pos + 3 * I, v);
        double *dst = D.cwc + (size_t)I * kCwConst * cp + c0 + cc;
#pragma unroll
        for (int j = 0; j < kCwRows; ++j) dst[(size_t)j * cp] = v[j];
      }
    // rows no frequency owns (timing model, padding), as bit masks per
    // 16-row tile: the same for every thread, so no loads in the loops below
    uint32_t free_rn[kMaxRows / 16], free_dm[kMaxRows / 16];
#pragma unroll
    for (int t = 0; t < kMaxRows / 16; ++t) {
      uint32_t mr = 0, md = 0;
      for (int j = 0; j < 16; ++j) {
        const int rw = 16 * t + j;
        if (rw < D.rows_rn) {
          const Slot sl = rn_slot(rw, D.kb);
          if (sl.kind != 0 || sl.harm > D.ka) mr |= 1u << j;
        }
        if (rw < D.rows_dm && dm_slot(rw, D.nf_dm).kind != 0) md |= 1u << j;
      }
      free_rn[t] = mr;
      free_dm[t] = md;
    }
    // a thread takes (pulsar, chain) pairs, two at a time with their u
    // values loaded first
    for (int p0 = pr_lo + tid; p0 < pr_hi; p0 += 2 * 256) {
      double u[2][3];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int pr = p0 + 256 * h, cc = pr & (kCB - 1), I = pr / kCB;
        const bool use = pr < pr_hi && !czero[cc];
#pragma unroll
        for (int t = 0; t < 3; ++t) u[h][t] = use ? row(cc)[D.off_u + 3 * I + t] : 0.0;
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int pr = p0 + 256 * h, cc = pr & (kCB - 1), I = pr / kCB;
        if (pr >= pr_hi) continue;
        double *dst = D.coef_rn + (size_t)I * D.rows_rn * cp + c0 + cc;
        double *ddm = D.coef_dm + (size_t)I * D.rows_dm * cp + c0 + cc;
#pragma unroll
        for (int t = 0; t < kMaxRows / 16; ++t) {
          for (uint32_t m = free_rn[t]; m; m &= m - 1) {
            const int rw = 16 * t + __builtin_ctz(m);
            const Slot sl = rn_slot(rw, D.kb);
            const double t0 = sl.tm == 0 ? u[h][0] : (sl.tm == 1 ? u[h][1] : u[h][2]);
            dst[(size_t)rw * cp] = sl.kind == 1 ? D.sigma_b * t0 : 0.0;
          }
          for (uint32_t m = free_dm[t]; m; m &= m - 1) ddm[(size_t)(16 * t + __builtin_ctz(m)) * cp] = 0.0;
        }
      }
    }
  }
  __syncthreads();

  // ---- the frequencies: item (chain, frequency, pulsar), chain fastest,
  //      then frequency, kSpecBatch items per thread with their loads first
  {
    const int nk = k_hi - k_lo;
    const int K2 = 2 * D.ka, K2d = 2 * D.nf_dm;
    const int total = nk * n * kCB;
    // a thread's items are 256 apart: item it = idx / 16 steps by 16, i.e.
    // the pulsar by q16 and the frequency by r16 (with carry), so a batch
    // needs one division
    const int q16 = nk > 0 ? 16 / nk : 0, r16 = 16 - q16 * nk;
    const int cc = tid & (kCB - 1);   // the same chain for all of a thread's items
    const bool bad_c = (badm >> cc) & 1;
    const double *xc = row(cc);
    for (int base = tid; base < total; base += 256 * kSpecBatch) {
      double ra[kSpecBatch], rg[kSpecBatch], zs[kSpecBatch], zc[kSpecBatch];
      double da[kSpecBatch], dg[kSpecBatch], ws[kSpecBatch], wc[kSpecBatch], lf[kSpecBatch];
      int Ib[kSpecBatch], kb_[kSpecBatch];
      {
        const int it0 = base / kCB;
        int I = it0 / nk, kk = it0 - I * nk;
#pragma unroll
        for (int b = 0; b < kSpecBatch; ++b) {
          Ib[b] = I;
          kb_[b] = k_lo + kk;
          I += q16;
          kk += r16;
          if (kk >= nk) {
            kk -= nk;
            ++I;
          }
        }
      }
#pragma unroll
      for (int b = 0; b < kSpecBatch; ++b) {
        const int idx = base + 256 * b;
        ra[b] = rg[b] = zs[b] = zc[b] = da[b] = dg[b] = ws[b] = wc[b] = 0.0;
        lf[b] = D.lnfy[kb_[b]];   // the frequency's ln(f yr), with the other inputs
        if (idx < total && !bad_c) {
          const int I = Ib[b], k0 = kb_[b];
          if (k0 >= D.nf_gw && k0 < D.ka) {
            if (k0 < D.nf_rn) {
              ra[b] = xc[D.off_rn + 2 * I];
              rg[b] = xc[D.off_rn + 2 * I + 1];
            }
            zs[b] = xc[D.off_z + I * K2 + 2 * k0];
            zc[b] = xc[D.off_z + I * K2 + 2 * k0 + 1];
          }
          if (k0 < D.nf_dm) {
            da[b] = xc[D.off_dm + 2 * I];
            dg[b] = xc[D.off_dm + 2 * I + 1];
            ws[b] = xc[D.off_zdm + I * K2d + 2 * k0];
            wc[b] = xc[D.off_zdm + I * K2d + 2 * k0 + 1];
          }
        }
      }
#pragma unroll
      for (int b = 0; b < kSpecBatch; ++b) {
        const int idx = base + 256 * b;
        if (idx >= total) continue;
        const int c = c0 + cc, I = Ib[b], k0 = kb_[b];
        const bool bad = bad_c;
        const int rs = harm_row(k0 + 1, 0), rc = harm_row(k0 + 1, 1);
        if (k0 >= D.nf_gw && k0 < D.ka) {
          double vs = 0.0, vc = 0.0;
          if (!bad) {
            const double sq = (k0 < D.nf_rn) ? powerlaw_sqrt_l(D, lf[b], ra[b], rg[b]) : 0.0;
            const double kap = sq * sq;
            if (!(kap > 0.0) || !isfinite(kap)) atomicOr(&kflag[cc][k0], kFlagNotPD);
            vs = sq * zs[b];
            vc = sq * zc[b];
            D.sqk_rn[sqk_at(D, c, I, k0)] = sq;
          }
          D.coef_rn[((size_t)I * D.rows_rn + rs) * cp + c] = vs;
          D.coef_rn[((size_t)I * D.rows_rn + rc) * cp + c] = vc;
        }
        if (k0 < D.nf_dm) {
          double vs = 0.0, vc = 0.0;
          if (!bad) {
            const double sq = powerlaw_sqrt_l(D, lf[b], da[b], dg[b]);
            vs = sq * ws[b];
            vc = sq * wc[b];
            D.sqk_dm[sqk_at(D, c, I, k0)] = sq;
          }
          D.coef_dm[((size_t)I * D.rows_dm + rs) * cp + c] = vs;
          D.coef_dm[((size_t)I * D.rows_dm + rc) * cp + c] = vc;
        }
      }
    }
  }
  __syncthreads();
  const int nk = k_hi - k_lo;
  for (int idx = tid; idx < nk * kCB; idx += 256) {
    const int cc = idx & (kCB - 1), k0 = k_lo + idx / kCB;
    D.flag_k[(size_t)(c0 + cc) * kmax + k0] = ((badm >> cc) & 1) ? 0 : kflag[cc][k0];
  }
}

// Adjoint of the chain block c0 .. c0 + 15 (chains below n_chains) over the
// frequencies [k_lo, k_hi); the non-finite flags go to slot `slot` of each
// chain's segment flags, and segment 0 sets the slots nslot .. kSpecSeg - 1 to
// zero.
__device__ inline void spec_bwd_cb(const Dev &D, const double *__restrict__ x,
                                   double *__restrict__ grad, int c0, int k_lo, int k_hi, int slot,
                                   int nslot) {
  __shared__ int ired[4];
  const int tid = threadIdx.x;
  const int n = D.n_psr;
  const int kmax = max(D.ka, D.nf_dm);
  const size_t cp = D.c_pad;
  // ---- chains to skip: flagged by a forward stage (or padding)
  int sm = 0;
  {
    const int per = kmax + D.nf_gw + 1;   // flag_k, flag_dense, st_pre of a chain
    constexpr int kB = 4;
    for (int i0 = tid; i0 < kCB * per; i0 += 256 * kB) {
      int f[kB];
#pragma unroll
      for (int b = 0; b < kB; ++b) {
        const int idx = i0 + 256 * b;
        const int cc = idx % kCB, e = idx / kCB, c = c0 + cc;
        f[b] = 0;
        if (idx < kCB * per && c < D.n_chains) {
          if (e < kmax) f[b] = D.flag_k[(size_t)c * kmax + e];
          else if (e < kmax + D.nf_gw) f[b] = D.flag_dense[(size_t)c * D.nf_gw + e - kmax];
          else f[b] = D.st_pre[c];
        }
      }
#pragma unroll
      for (int b = 0; b < kB; ++b)
        if (f[b]) sm |= 1 << ((i0 + 256 * b) % kCB);
    }
  }
  const int skipm = block_or256(sm, ired);
  int nfin = 0;   // chains with a non-finite result

  const int nk = k_hi - k_lo;
  const int K2 = 2 * D.ka, K2d = 2 * D.nf_dm;
  const int total = nk * n * kCB;
  // a thread keeps one chain; its items step by 16 (pulsar by q16, frequency
  // by r16 with carry), so a batch needs one division
  const int cc = tid & (kCB - 1), c = c0 + cc;
  const bool skip_c = (skipm >> cc) & 1;
  const int q16 = nk > 0 ? 16 / nk : 0, r16 = 16 - q16 * nk;
  for (int base = tid; base < total; base += 256 * kSpecBatch) {
    double sr[kSpecBatch], as_[kSpecBatch], ac_[kSpecBatch], zs[kSpecBatch], zc[kSpecBatch];
    double sd[kSpecBatch], bs_[kSpecBatch], bc_[kSpecBatch], ws[kSpecBatch], wc[kSpecBatch];
    double lf[kSpecBatch];
    int Ib[kSpecBatch], kb_[kSpecBatch];
    {
      const int it0 = base / kCB;
      int I = it0 / nk, kk = it0 - I * nk;
#pragma unroll
      for (int b = 0; b < kSpecBatch; ++b) {
        Ib[b] = I;
        kb_[b] = k_lo + kk;
        I += q16;
        kk += r16;
        if (kk >= nk) {
          kk -= nk;
          ++I;
        }
      }
    }
#pragma unroll
    for (int b = 0; b < kSpecBatch; ++b) {
      const int idx = base + 256 * b;
      sr[b] = as_[b] = ac_[b] = zs[b] = zc[b] = 0.0;
      sd[b] = bs_[b] = bc_[b] = ws[b] = wc[b] = 0.0;
      lf[b] = D.lnfy[kb_[b]];   // the frequency's ln(f yr), with the other inputs
      if (idx < total && c < D.n_chains && !skip_c) {
        const int I = Ib[b], k0 = kb_[b];
        const int rs = harm_row(k0 + 1, 0), rc = harm_row(k0 + 1, 1);
        const double *xc = x + (size_t)c * D.d;
        if (k0 >= D.nf_gw && k0 < D.ka) {
          sr[b] = D.sqk_rn[sqk_at(D, c, I, k0)];
          as_[b] = D.bar_rn[((size_t)I * D.rows_rn + rs) * cp + c];
          ac_[b] = D.bar_rn[((size_t)I * D.rows_rn + rc) * cp + c];
          zs[b] = xc[D.off_z + I * K2 + 2 * k0];
          zc[b] = xc[D.off_z + I * K2 + 2 * k0 + 1];
        }
        if (k0 < D.nf_dm) {
          sd[b] = D.sqk_dm[sqk_at(D, c, I, k0)];
          bs_[b] = D.bar_dm[((size_t)I * D.rows_dm + rs) * cp + c];
          bc_[b] = D.bar_dm[((size_t)I * D.rows_dm + rc) * cp + c];
          ws[b] = xc[D.off_zdm + I * K2d + 2 * k0];
          wc[b] = xc[D.off_zdm + I * K2d + 2 * k0 + 1];
        }
      }
    }
#pragma unroll
    for (int b = 0; b < kSpecBatch; ++b) {
      const int idx = base + 256 * b;
      if (idx >= total || c >= D.n_chains) continue;
      const bool skip = skip_c;
      const int I = Ib[b], k0 = kb_[b];
      const double lnfy = lf[b];
      double *gc = grad + (size_t)c * D.d;
      bool fin = true;
      if (k0 >= D.nf_gw && k0 < D.ka) {
        double g_s = 0.0, g_c = 0.0, d0 = 0.0, d1 = 0.0;
        if (!skip) {
          const double sq = sr[b];
          g_s = sq * as_[b] - zs[b];
          g_c = sq * ac_[b] - zc[b];
          const double az = (as_[b] * zs[b] + ac_[b] * zc[b]) * sq;
          d0 = (k0 < D.nf_rn) ? az * kLn10 : 0.0;
          d1 = (k0 < D.nf_rn) ? az * (-0.5 * lnfy) : 0.0;
          fin = isfinite(g_s) && isfinite(g_c) && isfinite(d0) && isfinite(d1);
        }
        gc[D.off_z + I * K2 + 2 * k0] = g_s;
        gc[D.off_z + I * K2 + 2 * k0 + 1] = g_c;
        double *drn = drn_at(D, c, I, k0);
        drn[0] = d0;
        drn[1] = d1;
        if (I == 0) {
          double *dth = D.dth_k + ((size_t)c * D.ka + k0) * 2;
          dth[0] = 0.0;
          dth[1] = 0.0;
        }
      }
      if (k0 < D.nf_dm) {
        double g_s = 0.0, g_c = 0.0, d0 = 0.0, d1 = 0.0;
        if (!skip) {
          const double sq = sd[b];
          g_s = sq * bs_[b] - ws[b];
          g_c = sq * bc_[b] - wc[b];
          const double az = (bs_[b] * ws[b] + bc_[b] * wc[b]) * sq;
          d0 = az * kLn10;
          d1 = az * (-0.5 * lnfy);
          fin = fin && isfinite(g_s) && isfinite(g_c) && isfinite(d0) && isfinite(d1);
        }
        gc[D.off_zdm + I * K2d + 2 * k0] = g_s;
        gc[D.off_zdm + I * K2d + 2 * k0 + 1] = g_c;
        double *ddm = ddm_at(D, c, I, k0);
        ddm[0] = d0;
        ddm[1] = d1;
      }
      if (!fin) nfin |= 1 << cc;
    }
  }
  nfin = block_or256(nfin, ired);
  if (tid < kCB && c0 + tid < D.n_chains) {
    int32_t *fo = D.flag_out + (size_t)(c0 + tid) * (kmax + kSpecSeg) + kmax;
    fo[slot] = ((nfin >> tid) & 1) ? kFlagOutNonfinite : 0;
    if (k_lo == 0)
      for (int s2 = nslot; s2 < kSpecSeg; ++s2) fo[s2] = 0;
  }
}

}  // namespace pt
