// Host side of the standardized form: data-set preparation (per-pulsar Gram
// quantities with the timing model marginalised), workspace, the evaluation
// pipeline and the HMC driver.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "common.h"
#include "pool.h"
#include "std.h"

struct ptafs_std {
  int device = 0;
  ps::StdDev base{};
  int64_t n_toa = 0;
  hipMemPool_t pool = nullptr;
  hipStream_t aux = nullptr;
  hipEvent_t done = nullptr;
  std::vector<void *> allocs;
  size_t ds_bytes = 0;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  void *hmc = nullptr;
  size_t hmc_bytes = 0;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap = nullptr;
  struct GraphKey {
    int n_chains, n_leapfrog;
    double eps;
    const void *inv_mass, *beta, *x, *logp, *grad, *acc, *samples, *invalid;
    uint64_t seed;
    void *ws, *hmc;
    bool operator==(const GraphKey &o) const { return std::memcmp(this, &o, sizeof(*this)) == 0; }
  } gkey{};
};

namespace {

#define PS_TRY(expr)                                  \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return PTAFS_E_HIP;         \
  } while (0)
#define PS_RC(expr)                                   \
  do {                                                \
    const int r_ = (expr);                            \
    if (r_) return r_;                                \
  } while (0)

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

int dalloc(ptafs_std *ds, void **p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  if (hipMallocFromPoolAsync(p, std::max<size_t>(bytes, 8), ds->pool, s) != hipSuccess) {
    *p = nullptr;
    return PTAFS_E_NOMEM;
  }
  return PTAFS_OK;
}
void dfree(void *p, hipStream_t s) {
  if (p) (void)hipFreeAsync(p, s);
}
int begin_call(ptafs_std *ds, hipStream_t s) {
  PS_TRY(hipStreamWaitEvent(s, ds->done, 0));
  return PTAFS_OK;
}
int end_call(ptafs_std *ds, hipStream_t s) {
  PS_TRY(hipEventRecord(ds->done, s));
  return PTAFS_OK;
}
int drop_graph(ptafs_std *ds) {
  if (!ds->gexec && !ds->graph) return PTAFS_OK;
  PS_TRY(hipEventSynchronize(ds->done));
  if (ds->gexec) (void)hipGraphExecDestroy(ds->gexec);
  if (ds->graph) (void)hipGraphDestroy(ds->graph);
  ds->gexec = nullptr;
  ds->graph = nullptr;
  return PTAFS_OK;
}

std::once_flag g_attr_once;
hipError_t g_attr_err = hipSuccess;

// ---------------------------------------------------------------- layout ---
int plan(const ptafs_std_desc *d, ps::StdDev &B, int64_t &ntoa) {
  B = ps::StdDev{};
  if (!d) return PTAFS_E_ARG;
  const int n = d->n_psr;
  if (n < 1 || !d->toa_offsets) return PTAFS_E_ARG;
  if (n > PTAFS_MAX_PSR) return PTAFS_E_LIMIT;
  if (d->nf_rn < 0 || d->nf_gw < 0 || d->nf_dm < 0) return PTAFS_E_ARG;
  if (std::max({d->nf_rn, d->nf_gw, d->nf_dm}) > PTAFS_MAX_HARM) return PTAFS_E_LIMIT;
  if (d->nf_rn + d->nf_gw + d->nf_dm == 0) return PTAFS_E_ARG;
  if (d->spectrum != PTAFS_SPEC_POWERLAW && d->spectrum != PTAFS_SPEC_FREE) return PTAFS_E_ARG;
  if (d->n_tm < 0 || (d->n_tm > 0) != (d->tm != nullptr)) return PTAFS_E_ARG;
  if (d->n_tm > PTAFS_MAX_TM) return PTAFS_E_LIMIT;
  if (!(d->tspan > 0.0) || d->n_backend < 1 || !d->efac || !d->equad || !d->psr_pos) return PTAFS_E_ARG;
  if (d->toa_offsets[0] != 0) return PTAFS_E_ARG;
  for (int p = 0; p < n; ++p)
    if (d->toa_offsets[p + 1] <= d->toa_offsets[p]) return PTAFS_E_ARG;
  ntoa = d->toa_offsets[n];
  if (!d->t || !d->dt || !d->sigma || !d->nu || !d->backend) return PTAFS_E_ARG;
  for (int64_t i = 0; i < ntoa; ++i) {
    if (d->backend[i] < 0 || d->backend[i] >= d->n_backend) return PTAFS_E_ARG;
    if (!(d->sigma[i] > 0.0) || !(d->nu[i] > 0.0) || !std::isfinite(d->t[i]) || !std::isfinite(d->dt[i]))
      return PTAFS_E_ARG;
  }
  for (int64_t i = 0; i < ntoa * (int64_t)d->n_tm; ++i)
    if (!std::isfinite(d->tm[i])) return PTAFS_E_ARG;
  B.n_psr = n;
  B.nf_rn = d->nf_rn;
  B.nf_gw = d->nf_gw;
  B.nf_dm = d->nf_dm;
  B.ka = std::max(d->nf_rn, d->nf_gw);
  B.kdm = d->nf_dm;
  B.P = 2 * B.ka + 2 * B.kdm;
  B.tp = ps::tiles_for(B.P);
  B.pp = 16 * B.tp;
  B.tg = ps::tiles_for(n);
  B.free_spec = d->spectrum == PTAFS_SPEC_FREE ? 1 : 0;
  B.w_gw = d->nf_gw > 0 ? (B.free_spec ? d->nf_gw : 2) : 0;
  B.w_rn = d->nf_rn > 0 ? (B.free_spec ? d->nf_rn : 2) : 0;
  B.w_dm = d->nf_dm > 0 ? (B.free_spec ? d->nf_dm : 2) : 0;
  int o = 0;
  B.off_gw = o; o += B.w_gw;
  B.off_rn = o; o += n * B.w_rn;
  B.off_dm = o; o += n * B.w_dm;
  B.has_cw = d->has_cw ? 1 : 0;
  B.off_cw = B.has_cw ? o : -1;
  if (B.has_cw) {
    if (d->cw_nf < 1 || !(d->cw_tspan > 0.0) || !std::isfinite(d->cw_tspan)) return PTAFS_E_ARG;
    if (d->cw_nf > PTAFS_MAX_CW_HARM) return PTAFS_E_LIMIT;
    B.kd = d->cw_nf;
    B.md = 2 * B.kd + 1;
    B.td = d->cw_tspan;
    o += 8;
  }
  B.n_theta = o;
  B.split = d->split ? 1 : 0;
  B.pz = B.P;
  if (B.split) {
    // separate common-process and pulsar-noise sets need both processes
    if (d->nf_gw < 1 || d->nf_rn < 1) return PTAFS_E_ARG;
    B.PG = 2 * d->nf_gw;
    B.PR = 2 * d->nf_rn + 2 * d->nf_dm;
    B.tpg = ps::tiles_for(B.PG);
    B.tpr = ps::tiles_for(B.PR);
    B.ppg = 16 * B.tpg;
    B.ppr = 16 * B.tpr;
    B.pz = B.PG + B.PR;
  }
  B.off_z = o; o += n * B.pz;
  B.d = o;
  if (B.n_theta > 0 && (!d->prior_lo || !d->prior_hi)) return PTAFS_E_ARG;
  double pc = 0.0;
  for (int i = 0; i < B.n_theta; ++i) {
    if (!(d->prior_hi[i] > d->prior_lo[i])) return PTAFS_E_ARG;
    pc -= std::log(d->prior_hi[i] - d->prior_lo[i]);
  }
  B.prior_const = pc;
  return PTAFS_OK;
}

size_t dataset_bytes_of(const ps::StdDev &B) {
  const size_t n = B.n_psr, pp = B.pp, nt = ps::ntiles(B.tg) * 256;
  size_t cw = 0;
  if (B.has_cw) {
    const size_t k2 = 2 * (size_t)B.kd;
    cw = n * B.P * k2 + n * k2 + n * k2 * k2 + k2 * B.md + 3 * n;
  }
  const size_t sp = B.split ? n * ((size_t)B.ppg * B.ppg + (size_t)B.ppr * B.ppr) + n * n : 0;
  return (n * pp * pp + n * pp + 2 * n + 2 * nt + n * n + 2 * std::max(B.n_theta, 1) + PTAFS_MAX_HARM + cw +
          sp) * sizeof(double) + 24 * 256;
}

struct WsLayout {
  size_t xinv, avec, ahat, v1, v2, lik, quad_k, drho_e, dkap_e, ddm_e, diag_q, dD_rn, dD_dm, flag1,
      flag2, flag3, cw_ad, dbar, cbar, gdbar, dcw, xg, xr, lzg, lzr, ag, ar, v2r, gag, gar, ddg, ddr,
      jac_s, flag_s, drho_p, total;
};
WsLayout ws_layout(const ps::StdDev &B, int C) {
  WsLayout L{};
  const size_t n = B.n_psr, pp = B.pp, c = C, ka = B.ka, kd = B.kdm;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o += al256(std::max<size_t>(bytes, 8));
    return r;
  };
  const size_t D8 = sizeof(double), I4 = sizeof(int32_t);
  L.xinv = take(c * n * ps::ntiles(B.tp) * 256 * D8);
  L.avec = take(c * n * pp * D8);
  L.ahat = take(c * n * pp * D8);
  L.v1 = take(c * n * pp * D8);
  L.v2 = take(c * n * pp * D8);
  L.lik = take(c * n * 2 * D8);
  L.quad_k = take(c * ka * 2 * D8);
  L.drho_e = take(c * ka * D8);
  L.dkap_e = take(c * n * ka * D8);
  L.ddm_e = take(c * n * kd * D8);
  L.diag_q = take(c * n * (ka + kd) * 2 * D8);
  L.dD_rn = take(c * n * ka * D8);
  L.dD_dm = take(c * n * kd * D8);
  L.flag1 = take(c * n * I4);
  L.flag2 = take(c * ka * I4);
  L.flag3 = take(c * n * (ka + kd) * I4);
  if (B.has_cw) {
    L.cw_ad = take(c * n * 2 * (size_t)B.kd * D8);
    L.dbar = take(c * n * pp * D8);
    L.cbar = take(c * n * D8);
    L.gdbar = take(c * n * (size_t)B.P * D8);
    L.dcw = take(c * n * 8 * D8);
  }
  if (B.split) {
    const size_t pg = B.ppg, pr = B.ppr;
    L.xg = take(c * n * ps::ntiles(B.tpg) * 256 * D8);
    L.xr = take(c * n * ps::ntiles(B.tpr) * 256 * D8);
    L.lzg = take(c * n * pg * D8);
    L.lzr = take(c * n * pr * D8);
    L.ag = take(c * n * pg * D8);
    L.ar = take(c * n * pr * D8);
    L.v2r = take(c * n * pr * D8);
    L.gag = take(c * n * pg * D8);
    L.gar = take(c * n * pr * D8);
    L.ddg = take(c * n * pg * D8);
    L.ddr = take(c * n * pr * D8);
    L.jac_s = take(c * n * 2 * D8);
    L.flag_s = take(c * n * 2 * I4);
    L.drho_p = take(c * n * ka * D8);
  }
  L.total = o;
  return L;
}

size_t hmc_bytes_of(const ps::StdDev &B, int C) {
  const size_t cd = (size_t)C * B.d;
  return al256(3 * cd * sizeof(double)) + al256((1 + pt::kHmcBeginG) * (size_t)C * sizeof(double)) +
         al256((size_t)C * sizeof(int32_t)) + 256;
}

int ensure_ws(ptafs_std *ds, int C, hipStream_t s) {
  const WsLayout L = ws_layout(ds->base, C);
  if (L.total <= ds->ws_bytes) return PTAFS_OK;
  PS_RC(drop_graph(ds));
  dfree(ds->ws, s);
  ds->ws = nullptr;
  ds->ws_bytes = 0;
  PS_RC(dalloc(ds, &ds->ws, L.total, s));
  ds->ws_bytes = L.total;
  return PTAFS_OK;
}

ps::StdDev make_dev(const ptafs_std *ds, int C, const double *beta) {
  ps::StdDev S = ds->base;
  S.n_chains = C;
  S.beta = beta;
  const WsLayout L = ws_layout(ds->base, C);
  char *w = static_cast<char *>(ds->ws);
  S.xinv = reinterpret_cast<double *>(w + L.xinv);
  S.avec = reinterpret_cast<double *>(w + L.avec);
  S.ahat = reinterpret_cast<double *>(w + L.ahat);
  S.v1 = reinterpret_cast<double *>(w + L.v1);
  S.v2 = reinterpret_cast<double *>(w + L.v2);
  S.lik = reinterpret_cast<double *>(w + L.lik);
  S.quad_k = reinterpret_cast<double *>(w + L.quad_k);
  S.drho_e = reinterpret_cast<double *>(w + L.drho_e);
  S.dkap_e = reinterpret_cast<double *>(w + L.dkap_e);
  S.ddm_e = reinterpret_cast<double *>(w + L.ddm_e);
  S.diag_q = reinterpret_cast<double *>(w + L.diag_q);
  S.dD_rn = reinterpret_cast<double *>(w + L.dD_rn);
  S.dD_dm = reinterpret_cast<double *>(w + L.dD_dm);
  S.flag1 = reinterpret_cast<int32_t *>(w + L.flag1);
  S.flag2 = reinterpret_cast<int32_t *>(w + L.flag2);
  S.flag3 = reinterpret_cast<int32_t *>(w + L.flag3);
  if (S.has_cw) {
    S.cw_ad = reinterpret_cast<double *>(w + L.cw_ad);
    S.dbar = reinterpret_cast<double *>(w + L.dbar);
    S.cbar = reinterpret_cast<double *>(w + L.cbar);
    S.gdbar = reinterpret_cast<double *>(w + L.gdbar);
    S.dcw = reinterpret_cast<double *>(w + L.dcw);
  }
  if (S.split) {
    S.xg = reinterpret_cast<double *>(w + L.xg);
    S.xr = reinterpret_cast<double *>(w + L.xr);
    S.lzg = reinterpret_cast<double *>(w + L.lzg);
    S.lzr = reinterpret_cast<double *>(w + L.lzr);
    S.ag = reinterpret_cast<double *>(w + L.ag);
    S.ar = reinterpret_cast<double *>(w + L.ar);
    S.v2r = reinterpret_cast<double *>(w + L.v2r);
    S.gag = reinterpret_cast<double *>(w + L.gag);
    S.gar = reinterpret_cast<double *>(w + L.gar);
    S.ddg = reinterpret_cast<double *>(w + L.ddg);
    S.ddr = reinterpret_cast<double *>(w + L.ddr);
    S.jac_s = reinterpret_cast<double *>(w + L.jac_s);
    S.flag_s = reinterpret_cast<int32_t *>(w + L.flag_s);
    S.drho_p = reinterpret_cast<double *>(w + L.drho_p);
  }
  return S;
}

int enqueue_eval(ptafs_std *ds, int C, const double *x, const double *beta, double *logp, double *grad,
                 int32_t *status, hipStream_t s, const ps::StdKick *kick = nullptr) {
  const ps::StdDev S = make_dev(ds, C, beta);
  PS_TRY(psk::launch_std_cw_fwd(S, x, s));
  PS_TRY(psk::launch_std_fwd(S, x, s));
  PS_TRY(psk::launch_split_fwd(S, x, s));
  PS_TRY(psk::launch_std_prior(S, x, s));
  PS_TRY(S.split ? psk::launch_split_bwd(S, x, grad, s) : psk::launch_std_bwd(S, x, grad, s));
  PS_TRY(psk::launch_std_cw_bwd(S, x, s));
  PS_TRY(psk::launch_std_finalize(S, x, logp, grad, status, s, kick));
  return PTAFS_OK;
}

// ------------------------------------------------------ Gram precompute ---
//
// Per pulsar: the weighted Gram matrix of B = [F~ | F_D | M | dt] with weights
// 1/N (F_D, the basis of the deterministic signal, only with a CW), then the
// timing model is marginalised.  With the columns of M scaled to
// unit weighted norm, a column-pivoted Cholesky factorisation of M^T N^-1 M
// (the same R factor as a column-pivoted QR of N^-1/2 M) selects r
// independent columns S (pivots below 1e-10 of the first end the
// factorisation) and gives Y = Lm^-1 M_S^T N^-1 [F~ | dt]; then
//   F~^T N~^-1 F~ = F~^T N^-1 F~ - Y_F^T Y_F, and the same for F~^T N~^-1 dt,
//   dt^T N~^-1 dt, since N~^-1 = N^-1 - N^-1 M_S (M_S^T N^-1 M_S)^-1 M_S^T N^-1
//   is the projection of Eq. Gmatrix_proj, and
//   ln det(G^T N G) = ln det N + ln det(M_S^T N^-1 M_S) - ln det(M_S^T M_S).
struct PsrGram {
  std::vector<double> s0, dv;   // P x P, P (original order)
  std::vector<double> sd, ed, qd;   // with a CW: P x 2K_D, 2K_D, 2K_D x 2K_D
  double c = 0.0, cst = 0.0;
  int rank = 0;
};

void gram_pulsar(const ptafs_std_desc *d, const ps::StdDev &B, int I, PsrGram &out) {
  const int64_t b = d->toa_offsets[I], e = d->toa_offsets[I + 1];
  const int ka = B.ka, kdm = B.kdm, kmax = std::max(ka, kdm);
  const int PS = B.P, K2 = B.has_cw ? 2 * B.kd : 0;
  const int P = PS + K2;   // the projected basis columns: F~, then F_D
  const int m = d->n_tm > 0 ? d->n_tm : 3;
  const int Q = P + m + 1;
  std::vector<double> G((size_t)Q * Q, 0.0), MMu((size_t)m * m, 0.0), row(Q), sn(kmax), cs(kmax);
  double lo = d->t[b], hi = lo;
  for (int64_t i = b; i < e; ++i) {
    lo = std::min(lo, d->t[i]);
    hi = std::max(hi, d->t[i]);
  }
  const double tc = 0.5 * (lo + hi), hs = 0.5 * (hi - lo) > 0.0 ? 0.5 * (hi - lo) : 1.0;
  double lnN = 0.0;
  for (int64_t i = b; i < e; ++i) {
    const double ph = 2.0 * M_PI * d->t[i] / d->tspan;
    for (int k = 0; k < kmax; ++k) {
      sn[k] = std::sin((k + 1) * ph);
      cs[k] = std::cos((k + 1) * ph);
    }
    const double w = d->dm_scale / (d->nu[i] * d->nu[i]);
    int o = 0;
    for (int k = 0; k < ka; ++k) {
      row[o++] = sn[k];
      row[o++] = cs[k];
    }
    for (int k = 0; k < kdm; ++k) {
      row[o++] = w * sn[k];
      row[o++] = w * cs[k];
    }
    if (K2) {
      const double phd = 2.0 * M_PI * d->t[i] / B.td;
      for (int k = 0; k < B.kd; ++k) {
        double sv, cv;
        sincos((k + 1) * phd, &sv, &cv);
        row[o++] = sv;
        row[o++] = cv;
      }
    }
    if (d->n_tm > 0) {
      for (int j = 0; j < m; ++j) row[o++] = d->tm[(size_t)i * d->n_tm + j];
    } else {
      const double tau = (d->t[i] - tc) / hs;
      row[o++] = 1.0;
      row[o++] = tau;
      row[o++] = tau * tau;
    }
    row[o++] = d->dt[i];
    const int be = d->backend[i];
    const double es = d->efac[be] * d->sigma[i], eq = d->equad[be];
    const double N = es * es + eq * eq;
    const double wn = 1.0 / N;
    lnN += std::log(N);
    for (int a = 0; a < Q; ++a) {
      const double wa = wn * row[a];
      double *g = &G[(size_t)a * Q];
      for (int c = 0; c <= a; ++c) g[c] += wa * row[c];
    }
    for (int a = 0; a < m; ++a)
      for (int c = 0; c <= a; ++c) MMu[(size_t)a * m + c] += row[P + a] * row[P + c];
  }
  for (int a = 0; a < Q; ++a)
    for (int c = a + 1; c < Q; ++c) G[(size_t)a * Q + c] = G[(size_t)c * Q + a];
  for (int a = 0; a < m; ++a)
    for (int c = a + 1; c < m; ++c) MMu[(size_t)a * m + c] = MMu[(size_t)c * m + a];
  auto g = [&](int a, int c) { return G[(size_t)a * Q + c]; };
  // column-pivoted Cholesky of the scaled M^T N^-1 M
  std::vector<double> sc(m, 0.0), W((size_t)m * m), Lm((size_t)m * m, 0.0);
  std::vector<int> perm(m);
  for (int j = 0; j < m; ++j) {
    const double v = g(P + j, P + j);
    sc[j] = v > 0.0 ? 1.0 / std::sqrt(v) : 0.0;
    perm[j] = j;
  }
  for (int a = 0; a < m; ++a)
    for (int c = 0; c < m; ++c) W[(size_t)a * m + c] = sc[a] * sc[c] * g(P + a, P + c);
  int r = 0;
  double first = 0.0;
  for (; r < m; ++r) {
    int best = r;
    for (int j = r + 1; j < m; ++j)
      if (W[(size_t)j * m + j] > W[(size_t)best * m + best]) best = j;
    const double pv = W[(size_t)best * m + best];
    if (r == 0) first = pv;
    if (!(pv > 1e-10 * first) || !(pv > 0.0)) break;
    if (best != r) {
      std::swap(perm[r], perm[best]);
      for (int c = 0; c < m; ++c) std::swap(W[(size_t)r * m + c], W[(size_t)best * m + c]);
      for (int a = 0; a < m; ++a) std::swap(W[(size_t)a * m + r], W[(size_t)a * m + best]);
      for (int c = 0; c < r; ++c) std::swap(Lm[(size_t)r * m + c], Lm[(size_t)best * m + c]);
    }
    const double l = std::sqrt(pv);
    Lm[(size_t)r * m + r] = l;
    for (int a = r + 1; a < m; ++a) Lm[(size_t)a * m + r] = W[(size_t)a * m + r] / l;
    for (int a = r + 1; a < m; ++a)
      for (int c = r + 1; c <= a; ++c) {
        W[(size_t)a * m + c] -= Lm[(size_t)a * m + r] * Lm[(size_t)c * m + r];
        W[(size_t)c * m + a] = W[(size_t)a * m + c];
      }
  }
  // Y = Lm^-1 (scaled rows M_S^T N^-1 [F~ | dt]) by forward substitution
  const int NC = P + 1;
  std::vector<double> Y((size_t)std::max(r, 1) * NC, 0.0);
  for (int i = 0; i < r; ++i) {
    const int col = perm[i];
    for (int j = 0; j < NC; ++j) {
      const int src = j < P ? j : P + m;
      double v = sc[col] * g(P + col, src);
      for (int k = 0; k < i; ++k) v -= Lm[(size_t)i * m + k] * Y[(size_t)k * NC + j];
      Y[(size_t)i * NC + j] = v / Lm[(size_t)i * m + i];
    }
  }
  // the projected Gram matrix of the basis columns and their products with dt
  std::vector<double> sg((size_t)P * P), dg(P);
  for (int a = 0; a < P; ++a) {
    for (int c = 0; c < P; ++c) {
      double v = g(a, c);
      for (int k = 0; k < r; ++k) v -= Y[(size_t)k * NC + a] * Y[(size_t)k * NC + c];
      sg[(size_t)a * P + c] = v;
    }
    double v = g(a, P + m);
    for (int k = 0; k < r; ++k) v -= Y[(size_t)k * NC + a] * Y[(size_t)k * NC + P];
    dg[a] = v;
  }
  out.s0.assign((size_t)PS * PS, 0.0);
  out.dv.assign(PS, 0.0);
  for (int a = 0; a < PS; ++a) {
    for (int c = 0; c < PS; ++c) out.s0[(size_t)a * PS + c] = sg[(size_t)a * P + c];
    out.dv[a] = dg[a];
  }
  if (K2) {
    out.sd.assign((size_t)PS * K2, 0.0);
    out.ed.assign(K2, 0.0);
    out.qd.assign((size_t)K2 * K2, 0.0);
    for (int a = 0; a < PS; ++a)
      for (int j = 0; j < K2; ++j) out.sd[(size_t)a * K2 + j] = sg[(size_t)a * P + PS + j];
    for (int j = 0; j < K2; ++j) {
      out.ed[j] = dg[PS + j];
      for (int k = 0; k < K2; ++k) out.qd[(size_t)j * K2 + k] = sg[(size_t)(PS + j) * P + PS + k];
    }
  }
  double cc = g(P + m, P + m);
  for (int k = 0; k < r; ++k) cc -= Y[(size_t)k * NC + P] * Y[(size_t)k * NC + P];
  out.c = cc;
  double ld_mnm = 0.0;
  for (int i = 0; i < r; ++i) ld_mnm += 2.0 * std::log(Lm[(size_t)i * m + i]) - 2.0 * std::log(sc[perm[i]]);
  // ln det(M_S^T M_S) of the selected columns
  double ld_mm = 0.0;
  {
    std::vector<double> U((size_t)std::max(r, 1) * std::max(r, 1), 0.0);
    for (int a = 0; a < r; ++a)
      for (int c = 0; c < r; ++c) U[(size_t)a * r + c] = MMu[(size_t)perm[a] * m + perm[c]];
    for (int j = 0; j < r; ++j) {
      double s = U[(size_t)j * r + j];
      for (int k = 0; k < j; ++k) s -= U[(size_t)j * r + k] * U[(size_t)j * r + k];
      const double l = std::sqrt(s);
      U[(size_t)j * r + j] = l;
      ld_mm += 2.0 * std::log(l);
      for (int a = j + 1; a < r; ++a) {
        double t = U[(size_t)a * r + j];
        for (int k = 0; k < j; ++k) t -= U[(size_t)a * r + k] * U[(size_t)j * r + k];
        U[(size_t)a * r + j] = t / l;
      }
    }
  }
  const int64_t n = e - b;
  out.cst = -0.5 * ((double)(n - r) * ps::kLn2Pi + lnN + ld_mnm - ld_mm);
  out.rank = r;
}

template <typename T>
int upload(ptafs_std *ds, const T *src, size_t count, const T **dst, hipStream_t s) {
  void *p = nullptr;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  PS_RC(dalloc(ds, &p, bytes, s));
  ds->allocs.push_back(p);
  ds->ds_bytes += bytes;
  if (count) PS_TRY(hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyHostToDevice, s));
  *dst = static_cast<const T *>(p);
  return PTAFS_OK;
}

void free_all(ptafs_std *ds) {
  if (!ds) return;
  (void)hipSetDevice(ds->device);
  if (ds->done) (void)hipEventSynchronize(ds->done);
  if (ds->gexec) (void)hipGraphExecDestroy(ds->gexec);
  if (ds->graph) (void)hipGraphDestroy(ds->graph);
  if (ds->cap) (void)hipStreamDestroy(ds->cap);
  if (ds->aux) {
    for (void *p : ds->allocs) dfree(p, ds->aux);
    dfree(ds->ws, ds->aux);
    dfree(ds->hmc, ds->aux);
  }
  if (ds->done) (void)hipEventDestroy(ds->done);
  delete ds;
}

void fill_layout(const ps::StdDev &B, int64_t ntoa, int C, ptafs_std_layout_info *out) {
  out->d = B.d;
  out->n_theta = B.n_theta;
  out->off_gw = B.off_gw;
  out->off_rn = B.off_rn;
  out->off_dm = B.off_dm;
  out->off_z = B.off_z;
  out->n_psr = B.n_psr;
  out->n_toa = ntoa;
  out->k_coef = B.ka;
  out->k_dm = B.kdm;
  out->p = B.P;
  out->dataset_bytes = dataset_bytes_of(B);
  out->workspace_bytes = ws_layout(B, C).total;
  out->hmc_bytes = hmc_bytes_of(B, C);
  out->off_cw = B.has_cw ? B.off_cw : -1;
  out->pz = B.pz;
}

}  // namespace

extern "C" {

int ptafs_std_create(const ptafs_std_desc *d, void *stream, ptafs_std **out) {
  if (!d || !out) return PTAFS_E_ARG;
  *out = nullptr;
  ps::StdDev B;
  int64_t ntoa = 0;
  PS_RC(plan(d, B, ntoa));
  const int n = d->n_psr;
  // HD matrix (Eq. HD) and its Cholesky factor
  std::vector<double> gam((size_t)n * n), gch((size_t)n * n, 0.0);
  for (int I = 0; I < n; ++I)
    for (int J = 0; J < n; ++J) {
      if (I == J) {
        gam[(size_t)I * n + J] = 1.0;
        continue;
      }
      const double *a = d->psr_pos + 3 * I, *b = d->psr_pos + 3 * J;
      const double beta = 0.5 * (1.0 - (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]));
      const double blb = beta > 0.0 ? beta * std::log(beta) : 0.0;
      gam[(size_t)I * n + J] = 1.5 * blb - 0.25 * beta + 0.5;
    }
  for (int j = 0; j < n; ++j) {
    double s = gam[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= gch[(size_t)j * n + k] * gch[(size_t)j * n + k];
    if (!(s > 0.0)) return PTAFS_E_ARG;
    const double l = std::sqrt(s);
    gch[(size_t)j * n + j] = l;
    for (int i = j + 1; i < n; ++i) {
      double t = gam[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= gch[(size_t)i * n + k] * gch[(size_t)j * n + k];
      gch[(size_t)i * n + j] = t / l;
    }
  }
  // per-pulsar Gram quantities, pulsars spread over the host threads
  std::vector<PsrGram> gr(n);
  {
    const int nt = std::max(1, std::min<int>(n, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int w = 0; w < nt; ++w)
      th.emplace_back([&, w]() {
        for (int I = w; I < n; I += nt) gram_pulsar(d, B, I, gr[I]);
      });
    for (auto &t : th) t.join();
  }
  ptafs_std *ds = new (std::nothrow) ptafs_std();
  if (!ds) return PTAFS_E_NOMEM;
  if (hipGetDevice(&ds->device) != hipSuccess) {
    delete ds;
    return PTAFS_E_HIP;
  }
  std::call_once(g_attr_once, [] { g_attr_err = psk::init_attributes(); });
  if (g_attr_err != hipSuccess || ptr::device_pool(ds->device, &ds->pool, &ds->aux) ||
      hipEventCreateWithFlags(&ds->done, hipEventDisableTiming) != hipSuccess) {
    free_all(ds);
    return PTAFS_E_HIP;
  }
  hipStream_t s = (hipStream_t)stream;
  ds->base = B;
  ds->n_toa = ntoa;
  ps::StdDev &D = ds->base;
  const int P = B.P, pp = B.pp;
  // host sources of the asynchronous uploads: alive until the stream is synchronised
  std::vector<double> s0r((size_t)n * pp * pp, 0.0), dr((size_t)n * pp, 0.0), cc((size_t)n * 2);
  for (int I = 0; I < n; ++I) {
    for (int r = 0; r < P; ++r) {
      for (int c = 0; c < P; ++c) s0r[((size_t)I * pp + r) * pp + c] = gr[I].s0[(size_t)(P - 1 - r) * P + (P - 1 - c)];
      dr[(size_t)I * pp + r] = gr[I].dv[P - 1 - r];
    }
    cc[2 * I] = gr[I].c;
    cc[2 * I + 1] = gr[I].cst;
  }
  const int tg = B.tg, ntl = ps::ntiles(tg) * 256;
  std::vector<double> gt(ntl, 0.0), ct(ntl, 0.0);
  for (int TI = 0; TI < tg; ++TI)
    for (int TJ = 0; TJ <= TI; ++TJ)
      for (int rr = 0; rr < 16; ++rr)
        for (int c2 = 0; c2 < 16; ++c2) {
          const int r = 16 * TI + rr, c = 16 * TJ + c2;
          const size_t e = (size_t)ps::tix(TI, TJ) * 256 + rr * 16 + c2;
          if (r < n && c < n) {
            gt[e] = gam[(size_t)r * n + c];
            ct[e] = (c <= r) ? gch[(size_t)r * n + c] : 0.0;
          }
        }
  std::vector<double> lf(PTAFS_MAX_HARM);
  for (int k = 0; k < PTAFS_MAX_HARM; ++k) lf[k] = std::log((k + 1) / d->tspan * pt::kYear);
  D.pl_c = 3.0 * std::log(pt::kYear) - std::log(12.0 * pt::kPi * pt::kPi) - std::log(d->tspan);
  int rc = PTAFS_OK;
  auto chk = [&](int r) { if (r && !rc) rc = r; };
  chk(upload(ds, s0r.data(), s0r.size(), &D.s0, s));
  chk(upload(ds, dr.data(), dr.size(), &D.dvec, s));
  chk(upload(ds, cc.data(), cc.size(), &D.cconst, s));
  chk(upload(ds, gt.data(), gt.size(), &D.gam_tiles, s));
  chk(upload(ds, ct.data(), ct.size(), &D.gch_tiles, s));
  chk(upload(ds, gam.data(), gam.size(), &D.gamma, s));
  // split coefficients: S0 on each set's rows (reversed order, zero-padded),
  // Gamma^-1 = chol(Gamma)^-T chol(Gamma)^-1 and ln det Gamma
  std::vector<double> s0g, s0rr, ginv;
  if (B.split) {
    const int PG = B.PG, PR = B.PR, pg = B.ppg, pr = B.ppr;
    auto rrow = [&](int j) { return j < 2 * B.nf_rn ? j : 2 * B.ka + (j - 2 * B.nf_rn); };
    s0g.assign((size_t)n * pg * pg, 0.0);
    s0rr.assign((size_t)n * pr * pr, 0.0);
    for (int I = 0; I < n; ++I) {
      for (int r = 0; r < PG; ++r)
        for (int c = 0; c < PG; ++c)
          s0g[((size_t)I * pg + r) * pg + c] = gr[I].s0[(size_t)(PG - 1 - r) * P + (PG - 1 - c)];
      for (int r = 0; r < PR; ++r)
        for (int c = 0; c < PR; ++c)
          s0rr[((size_t)I * pr + r) * pr + c] = gr[I].s0[(size_t)rrow(PR - 1 - r) * P + rrow(PR - 1 - c)];
    }
    std::vector<double> li((size_t)n * n, 0.0);   // chol(Gamma)^-1, lower
    double ldg = 0.0;
    for (int j = 0; j < n; ++j) {
      ldg += 2.0 * std::log(gch[(size_t)j * n + j]);
      for (int i = j; i < n; ++i) {
        double t = (i == j) ? 1.0 : 0.0;
        for (int k = j; k < i; ++k) t -= gch[(size_t)i * n + k] * li[(size_t)k * n + j];
        li[(size_t)i * n + j] = t / gch[(size_t)i * n + i];
      }
    }
    ginv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double t = 0.0;
        for (int k = std::max(i, j); k < n; ++k) t += li[(size_t)k * n + i] * li[(size_t)k * n + j];
        ginv[(size_t)i * n + j] = t;
      }
    D.ldet_gamma = ldg;
    chk(upload(ds, s0g.data(), s0g.size(), &D.s0g, s));
    chk(upload(ds, s0rr.data(), s0rr.size(), &D.s0r, s));
    chk(upload(ds, ginv.data(), ginv.size(), &D.gam_inv, s));
  }
  chk(upload(ds, lf.data(), lf.size(), &D.lnfy, s));
  chk(upload(ds, d->prior_lo, (size_t)B.n_theta, &D.prior_lo, s));
  chk(upload(ds, d->prior_hi, (size_t)B.n_theta, &D.prior_hi, s));
  std::vector<double> sd, ed, qd, dft;
  if (B.has_cw) {
    const int K2 = 2 * B.kd, M = B.md;
    sd.resize((size_t)n * P * K2);
    ed.resize((size_t)n * K2);
    qd.resize((size_t)n * K2 * K2);
    for (int I = 0; I < n; ++I) {
      std::memcpy(&sd[(size_t)I * P * K2], gr[I].sd.data(), (size_t)P * K2 * sizeof(double));
      std::memcpy(&ed[(size_t)I * K2], gr[I].ed.data(), (size_t)K2 * sizeof(double));
      std::memcpy(&qd[(size_t)I * K2 * K2], gr[I].qd.data(), (size_t)K2 * K2 * sizeof(double));
    }
    // a_(k,sin) = 2/M sum_j h_j sin(2 pi k j / M), a_(k,cos) likewise; the
    // angle reduced to k j mod M first, so that it is exact in the argument
    dft.resize((size_t)K2 * M);
    for (int k = 1; k <= B.kd; ++k)
      for (int j = 0; j < M; ++j) {
        const double ang = 2.0 * M_PI * (double)(((int64_t)k * j) % M) / M;
        dft[(size_t)(2 * k - 2) * M + j] = 2.0 / M * std::sin(ang);
        dft[(size_t)(2 * k - 1) * M + j] = 2.0 / M * std::cos(ang);
      }
    chk(upload(ds, sd.data(), sd.size(), &D.cw_sd, s));
    chk(upload(ds, ed.data(), ed.size(), &D.cw_ed, s));
    chk(upload(ds, qd.data(), qd.size(), &D.cw_qd, s));
    chk(upload(ds, dft.data(), dft.size(), &D.cw_dft, s));
    chk(upload(ds, d->psr_pos, (size_t)3 * n, &D.cw_pos, s));
  }
  if (!rc) rc = end_call(ds, s);
  if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = PTAFS_E_HIP;
  if (rc) {
    free_all(ds);
    return rc;
  }
  *out = ds;
  return PTAFS_OK;
}

void ptafs_std_destroy(ptafs_std *ds) { free_all(ds); }

int ptafs_std_precompute(const ptafs_std_desc *desc, int32_t pulsar, double *s0, double *dvec,
                         double *scal) {
  ps::StdDev B;
  int64_t ntoa = 0;
  PS_RC(plan(desc, B, ntoa));
  if (pulsar < 0 || pulsar >= B.n_psr || !s0 || !dvec || !scal) return PTAFS_E_ARG;
  PsrGram g;
  gram_pulsar(desc, B, pulsar, g);
  std::memcpy(s0, g.s0.data(), g.s0.size() * sizeof(double));
  std::memcpy(dvec, g.dv.data(), g.dv.size() * sizeof(double));
  scal[0] = g.c;
  scal[1] = g.cst;
  scal[2] = g.rank;
  return PTAFS_OK;
}

int ptafs_std_precompute_cw(const ptafs_std_desc *desc, int32_t pulsar, double *sd, double *ed,
                            double *qd) {
  ps::StdDev B;
  int64_t ntoa = 0;
  PS_RC(plan(desc, B, ntoa));
  if (!B.has_cw || pulsar < 0 || pulsar >= B.n_psr || !sd || !ed || !qd) return PTAFS_E_ARG;
  PsrGram g;
  gram_pulsar(desc, B, pulsar, g);
  std::memcpy(sd, g.sd.data(), g.sd.size() * sizeof(double));
  std::memcpy(ed, g.ed.data(), g.ed.size() * sizeof(double));
  std::memcpy(qd, g.qd.data(), g.qd.size() * sizeof(double));
  return PTAFS_OK;
}

int ptafs_std_layout(const ptafs_std *ds, int32_t n_chains, ptafs_std_layout_info *out) {
  if (!ds || !out || n_chains < 0) return PTAFS_E_ARG;
  fill_layout(ds->base, ds->n_toa, n_chains, out);
  return PTAFS_OK;
}

int ptafs_std_logp_grad(ptafs_std *ds, int32_t n_chains, const double *x, const double *beta,
                        double *logp, double *grad, int32_t *status, void *stream) {
  if (!ds || n_chains < 0) return PTAFS_E_ARG;
  if (n_chains == 0) return PTAFS_OK;
  if (!x || !logp || !grad || !status) return PTAFS_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  PS_TRY(hipSetDevice(ds->device));
  PS_RC(begin_call(ds, s));
  PS_RC(ensure_ws(ds, n_chains, s));
  PS_RC(enqueue_eval(ds, n_chains, x, beta, logp, grad, status, s));
  return end_call(ds, s);
}

int ptafs_std_profile_stages(ptafs_std *ds, int32_t n_chains, const double *x, const double *beta,
                             double *logp, double *grad, int32_t *status, int32_t reps,
                             double *ms_out, void *stream) {
  if (!ds || n_chains < 1 || reps < 1 || !ms_out || !x || !logp || !grad || !status) return PTAFS_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  PS_TRY(hipSetDevice(ds->device));
  PS_RC(begin_call(ds, s));
  PS_RC(ensure_ws(ds, n_chains, s));
  const ps::StdDev S = make_dev(ds, n_chains, beta);
  constexpr int kStages = 4;
  hipEvent_t ev[kStages + 1];
  for (auto &e : ev) PS_TRY(hipEventCreate(&e));
  double acc[kStages] = {0, 0, 0, 0};
  int err = PTAFS_OK;
  for (int r = 0; r < reps && !err; ++r) {
    auto step = [&](int i, hipError_t e) {
      if (e != hipSuccess && !err) err = PTAFS_E_HIP;
      (void)hipEventRecord(ev[i + 1], s);
    };
    (void)hipEventRecord(ev[0], s);
    hipError_t e0 = psk::launch_std_cw_fwd(S, x, s);
    if (e0 == hipSuccess) e0 = psk::launch_std_fwd(S, x, s);
    step(0, e0 != hipSuccess ? e0 : psk::launch_split_fwd(S, x, s));
    step(1, psk::launch_std_prior(S, x, s));
    const hipError_t e2 = S.split ? psk::launch_split_bwd(S, x, grad, s) : psk::launch_std_bwd(S, x, grad, s);
    step(2, e2 != hipSuccess ? e2 : psk::launch_std_cw_bwd(S, x, s));
    step(3, psk::launch_std_finalize(S, x, logp, grad, status, s));
    if (hipEventSynchronize(ev[kStages]) != hipSuccess) err = PTAFS_E_HIP;
    for (int i = 0; i < kStages && !err; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) err = PTAFS_E_HIP;
      acc[i] += ms;
    }
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  for (int i = 0; i < kStages; ++i) ms_out[i] = acc[i] / reps;
  if (!err) err = end_call(ds, s);
  return err;
}

int ptafs_std_coefficients(ptafs_std *ds, int32_t n_chains, const double *x, const double *beta,
                           double *a, void *stream) {
  if (!ds || n_chains < 0) return PTAFS_E_ARG;
  if (n_chains == 0) return PTAFS_OK;
  if (!x || !a) return PTAFS_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  PS_TRY(hipSetDevice(ds->device));
  PS_RC(begin_call(ds, s));
  PS_RC(ensure_ws(ds, n_chains, s));
  const ps::StdDev S = make_dev(ds, n_chains, beta);
  PS_TRY(psk::launch_std_cw_fwd(S, x, s));
  PS_TRY(psk::launch_std_fwd(S, x, s));
  const size_t rows = (size_t)n_chains * S.n_psr, D8 = sizeof(double);
  if (S.split) {
    PS_TRY(psk::launch_split_fwd(S, x, s));
    PS_TRY(hipMemcpy2DAsync(a, S.pz * D8, S.ag, S.ppg * D8, S.PG * D8, rows, hipMemcpyDeviceToDevice, s));
    PS_TRY(hipMemcpy2DAsync(a + S.PG, S.pz * D8, S.ar, S.ppr * D8, S.PR * D8, rows, hipMemcpyDeviceToDevice,
                            s));
  } else {
    PS_TRY(hipMemcpy2DAsync(a, S.P * D8, S.avec, S.pp * D8, S.P * D8, rows, hipMemcpyDeviceToDevice, s));
  }
  return end_call(ds, s);
}

int ptafs_std_hmc_run(ptafs_std *ds, int32_t n_chains, int32_t n_traj, int32_t n_leapfrog, double eps,
                      const double *inv_mass, uint64_t seed, uint64_t traj0, const double *beta, double *x,
                      double *logp, double *grad, int64_t *n_accept, double *samples, int64_t *n_invalid,
                      int32_t use_graph, void *stream) {
  if (!ds || n_chains < 0 || n_traj < 0 || n_leapfrog < 1 || !(eps > 0.0)) return PTAFS_E_ARG;
  if (n_chains == 0 || n_traj == 0) return PTAFS_OK;
  if (!x || !logp || !grad || !n_accept) return PTAFS_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  PS_TRY(hipSetDevice(ds->device));
  PS_RC(begin_call(ds, s));
  PS_RC(ensure_ws(ds, n_chains, s));
  const int d = ds->base.d;
  const size_t cd = (size_t)n_chains * d;
  const size_t need = hmc_bytes_of(ds->base, n_chains);
  if (need > ds->hmc_bytes) {
    PS_RC(drop_graph(ds));
    dfree(ds->hmc, s);
    ds->hmc = nullptr;
    ds->hmc_bytes = 0;
    PS_RC(dalloc(ds, &ds->hmc, need, s));
    ds->hmc_bytes = need;
  }
  char *h = static_cast<char *>(ds->hmc);
  double *p = reinterpret_cast<double *>(h);
  double *x0 = p + cd;
  double *g0 = x0 + cd;
  char *h2 = h + al256(3 * cd * sizeof(double));
  double *lp0 = reinterpret_cast<double *>(h2);
  double *h0 = lp0 + n_chains;
  char *h3 = h2 + al256((1 + pt::kHmcBeginG) * (size_t)n_chains * sizeof(double));
  int32_t *st = reinterpret_cast<int32_t *>(h3);
  uint64_t *traj = reinterpret_cast<uint64_t *>(h3 + al256((size_t)n_chains * sizeof(int32_t)));
  PS_TRY(ptk::launch_traj_set(traj, traj0, s));
  pt::Dev hd{};   // the HMC kernels read only the chain count
  hd.n_chains = n_chains;
  auto one_traj = [&](hipStream_t q) -> int {
    PS_TRY(ptk::launch_hmc_begin(hd, d, eps, inv_mass, seed, traj, x, logp, grad, p, x0, lp0, g0, h0, q));
    const ps::StdKick kick{eps, inv_mass, x, p, n_invalid};
    for (int l = 0; l < n_leapfrog; ++l)
      PS_RC(enqueue_eval(ds, n_chains, x, beta, logp, grad, st, q, l + 1 < n_leapfrog ? &kick : nullptr));
    PS_TRY(ptk::launch_hmc_end(n_chains, d, eps, inv_mass, seed, traj, x, logp, grad, p, x0, lp0, g0, h0,
                               n_accept, samples, st, n_invalid, q));
    PS_TRY(ptk::launch_traj_inc(traj, q));
    return PTAFS_OK;
  };
  if (!use_graph) {
    for (int j = 0; j < n_traj; ++j) PS_RC(one_traj(s));
    return end_call(ds, s);
  }
  ptafs_std::GraphKey key{};
  std::memset(&key, 0, sizeof(key));
  key.n_chains = n_chains;
  key.n_leapfrog = n_leapfrog;
  key.eps = eps;
  key.inv_mass = inv_mass;
  key.beta = beta;
  key.x = x;
  key.logp = logp;
  key.grad = grad;
  key.acc = n_accept;
  key.samples = samples;
  key.invalid = n_invalid;
  key.seed = seed;
  key.ws = ds->ws;
  key.hmc = ds->hmc;
  if (!ds->gexec || !(key == ds->gkey)) {
    PS_RC(drop_graph(ds));
    if (!ds->cap) PS_TRY(hipStreamCreateWithFlags(&ds->cap, hipStreamNonBlocking));
    PS_TRY(hipStreamBeginCapture(ds->cap, hipStreamCaptureModeRelaxed));
    const int rc = one_traj(ds->cap);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(ds->cap, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return PTAFS_E_HIP;
    if (hipGraphInstantiate(&ds->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return PTAFS_E_HIP;
    }
    ds->graph = g;
    ds->gkey = key;
  }
  for (int j = 0; j < n_traj; ++j) PS_TRY(hipGraphLaunch(ds->gexec, s));
  return end_call(ds, s);
}

}  // extern "C"
