// Internal definitions of the standardized form (Sec. IV.B: the CURN
// standardizing transform on the Gram form of the likelihood, timing model
// marginalised) shared by its host code and kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ptafs.h"

namespace ps {

constexpr double kLn10 = 2.30258509299404568401799145468;
constexpr double kLn2Pi = 1.83787706640934548356065947281;
constexpr int kThreads = 256;                    // threads per problem workgroup
constexpr int kMaxTiles = 8;                     // 16-wide tiles per dimension (128)
constexpr int kMaxRhoK = 32;                     // frequencies of the common process (>= PTAFS_MAX_HARM)
constexpr int kMaxCw2 = 2 * PTAFS_MAX_CW_HARM;   // coefficients of the deterministic basis
constexpr int kMaxCwM = kMaxCw2 + 1;             // its sample times

// Lower tiles of a 16T x 16T matrix: tile (I, J), J <= I, at I (I + 1) / 2 + J,
// row-major inside (element (r, c) of the tile at 16 r + c).
__host__ __device__ constexpr int tix(int I, int J) { return I * (I + 1) / 2 + J; }
__host__ __device__ constexpr int ntiles(int T) { return T * (T + 1) / 2; }
__host__ __device__ inline int tiles_for(int n) { return (n + 15) / 16; }

// Device view of a standardized-form data set and the workspace of one call.
//
// Per pulsar I the coefficient vector has P = 2 ka + 2 kdm entries: k = 1 sin,
// k = 1 cos, ... for the red/common block, then the DM block.  The per-pulsar
// factorisation runs in reversed index order r = P - 1 - j (the lower Cholesky
// factor of the reversed precision gives the lower Cholesky factor of the
// covariance, see k_std.hip), padded to pp = 16 tp with an identity block.
struct StdDev {
  int n_psr, nf_rn, nf_gw, nf_dm, ka, kdm, P, tp, pp;
  int free_spec;                 // 0 power law, 1 free spectrum
  int n_theta, d, off_gw, off_rn, off_dm, off_z;
  int w_gw, w_rn, w_dm;          // theta entries per process (2 or one per frequency)
  int tg;                        // tiles of the per-frequency N_p x N_p problems
  double prior_const;
  // data set (device)
  const double *s0;              // [n_psr][pp][pp] beta-free Gram F~^T N~^-1 F~, reversed order, zero-padded
  const double *dvec;            // [n_psr][pp] F~^T N~^-1 dt, reversed order, zero-padded
  const double *cconst;          // [n_psr][2]: dt^T N~^-1 dt, -1/2 ln det(2 pi G^T N G)
  const double *gam_tiles;       // Gamma: lower tiles (diagonal tiles full), zero-padded
  const double *gch_tiles;       // chol(Gamma): lower tiles, zero-padded
  const double *gamma;           // Gamma, n_psr x n_psr
  const double *prior_lo, *prior_hi;
  const double *lnfy;            // ln(f_k yr), k < PTAFS_MAX_HARM
  double pl_c;                   // ln(yr^3 / (12 pi^2 T))
  // deterministic CW in its own basis (has_cw): K_D = kd frequencies k / td,
  // md = 2 kd + 1 sample times j td / md
  int has_cw, kd, md, off_cw;
  double td;
  const double *cw_sd;           // [n_psr][P][2 kd] F~^T N~^-1 F_D (original coefficient order)
  const double *cw_ed;           // [n_psr][2 kd] F_D^T N~^-1 dt
  const double *cw_qd;           // [n_psr][2 kd][2 kd] F_D^T N~^-1 F_D
  const double *cw_dft;          // [2 kd][md] the transform of the samples to a_D
  const double *cw_pos;          // [n_psr][3] pulsar unit vectors
  // split coefficients (App. C): a common-process set a_G over the rows
  // k < nf_gw (PG = 2 nf_gw) and a pulsar-noise set a_R over the rows k < nf_rn
  // then the DM block (PR = 2 nf_rn + 2 nf_dm), each with its own factorisation
  // (tpg, tpr tiles); z per pulsar holds pz = PG + PR entries (P without split)
  int split, PG, PR, tpg, tpr, ppg, ppr, pz;
  const double *s0g;             // [n_psr][ppg][ppg] S0 on the common rows, reversed order, zero-padded
  const double *s0r;             // [n_psr][ppr][ppr] S0 on the pulsar-noise rows, likewise
  const double *gam_inv;         // Gamma^-1, n_psr x n_psr
  double ldet_gamma;             // ln det Gamma
  // call
  int n_chains;
  const double *beta;            // [n_chains] or nullptr (1)
  // workspace
  double *xinv;                  // [n_chains][n_psr][ntiles(tp)][256] inverse of the reversed precision's factor
  double *avec;                  // [n_chains][n_psr][pp] a, original order
  double *ahat;                  // [n_chains][n_psr][pp] a_hat, reversed order
  double *v1;                    // [n_chains][n_psr][pp] beta (d - S0 a), reversed order
  double *v2;                    // [n_chains][n_psr][pp] -phi^-1 a, original order
  double *lik;                   // [n_chains][n_psr][2]: beta log L(a_I), ln det L_I
  double *quad_k;                // [n_chains][ka][2]: a^T phi_k^-1 a (sin + cos), ln det phi_k (dense k < nf_gw)
  double *drho_e;                // [n_chains][ka] explicit d/drho_k of the prior
  double *dkap_e;                // [n_chains][n_psr][ka] explicit d/dkappa_Ik of the prior
  double *ddm_e;                 // [n_chains][n_psr][kdm]
  double *diag_q;                // [n_chains][n_psr][ka + kdm][2]: quadratic term, ln kappa (diagonal items)
  double *dD_rn;                 // [n_chains][n_psr][ka] d/dD through the transform
  double *dD_dm;                 // [n_chains][n_psr][kdm]
  int32_t *flag1;                // [n_chains][n_psr] factorisation failures of the transform
  int32_t *flag2;                // [n_chains][ka] dense prior factorisations
  int32_t *flag3;                // [n_chains][n_psr][ka + kdm] diagonal items
  double *cw_ad;                 // [n_chains][n_psr][2 kd] a_D of each chain
  double *dbar;                  // [n_chains][n_psr][pp] d of dt - h, reversed order, zero-padded
  double *cbar;                  // [n_chains][n_psr] dt~^T N~^-1 dt~ of dt~ = dt - h
  double *gdbar;                 // [n_chains][n_psr][P] dlog p / d d_bar (original order)
  double *dcw;                   // [n_chains][n_psr][8] the pulsar's part of dlog p / d theta_cw
  // split coefficients (set b: 0 common, 1 pulsar noise; vectors in the set's
  // original row order, strides ppg / ppr)
  double *xg, *xr;               // [n_chains][n_psr][ntiles(tpg|tpr)][256] X of each set's reversed precision
  double *lzg, *lzr;             // L_b z_b
  double *ag, *ar;               // a_G, a_R
  double *v2r;                   // -phi_R^-1 a_R (the common set's prior term goes to v2)
  double *gag, *gar;             // dlog p / d a_b
  double *ddg, *ddr;             // the set's transform part of dlog p / d(prior variance) per row
  double *jac_s;                 // [n_chains][n_psr][2] ln det L_G, ln det L_R
  int32_t *flag_s;               // [n_chains][n_psr][2] failures of the two factorisations
  double *drho_p;                // [n_chains][n_psr][ka] the pulsar's part of dlog p / d rho_k
};

// Spectrum of process proc (0 common, 1 red noise of pulsar I, 2 DM of pulsar
// I) at frequency k (0-based): power law (Eq. power_law, yr^3 reading) or free
// spectrum rho = 10^theta_k (s^2).
__device__ inline double spec_value(const StdDev &S, const double *x, int proc, int I, int k) {
  int off, w;
  if (proc == 0) { off = S.off_gw; w = S.w_gw; }
  else if (proc == 1) { off = S.off_rn + I * S.w_rn; w = S.w_rn; }
  else { off = S.off_dm + I * S.w_dm; w = S.w_dm; }
  (void)w;
  if (S.free_spec) return exp(kLn10 * x[off + k]);
  return exp(2.0 * kLn10 * x[off] - x[off + 1] * S.lnfy[k] + S.pl_c);
}

// Coefficient variance D_j of column j (original order) of pulsar I under the
// CURN prior: rho_k + kappa_Ik on the red/common block, kappa_dm,Ik on DM.
__device__ inline double curn_var(const StdDev &S, const double *x, int I, int j) {
  if (j < 2 * S.ka) {
    const int k = j >> 1;
    double v = 0.0;
    if (k < S.nf_gw) v += spec_value(S, x, 0, I, k);
    if (k < S.nf_rn) v += spec_value(S, x, 1, I, k);
    return v;
  }
  return spec_value(S, x, 2, I, (j - 2 * S.ka) >> 1);
}

// Split coefficients: combined row of row j of set b, and the set's own prior
// variance there (rho_k for the common set; kappa_Ik, then kappa_dm,Ik).
__device__ inline int split_row(const StdDev &S, int b, int j) {
  return (b == 0 || j < 2 * S.nf_rn) ? j : 2 * S.ka + (j - 2 * S.nf_rn);
}
__device__ inline double split_var(const StdDev &S, const double *x, int I, int b, int j) {
  if (b == 0) return spec_value(S, x, 0, I, j >> 1);
  if (j < 2 * S.nf_rn) return spec_value(S, x, 1, I, j >> 1);
  return spec_value(S, x, 2, I, (j - 2 * S.nf_rn) >> 1);
}

constexpr int kFlagNotPD = 1;

// Leapfrog kick and drift applied by k_std_finalize to its chain right after
// the gradient (inside an HMC trajectory): p += eps grad, x += eps M^-1 p, and
// one invalid evaluation counted when the status is nonzero.
struct StdKick {
  double eps;
  const double *inv_mass;   // [d] or null (identity)
  double *x, *p;            // [n_chains][d]
  int64_t *n_invalid;       // [n_chains] or null
};

}  // namespace ps

namespace psk {
hipError_t init_attributes();
hipError_t launch_std_fwd(const ps::StdDev &S, const double *x, hipStream_t s);
hipError_t launch_std_prior(const ps::StdDev &S, const double *x, hipStream_t s);
hipError_t launch_std_bwd(const ps::StdDev &S, const double *x, double *grad, hipStream_t s);
hipError_t launch_std_finalize(const ps::StdDev &S, const double *x, double *logp, double *grad,
                               int32_t *status, hipStream_t s, const ps::StdKick *kick = nullptr);
hipError_t launch_std_cw_fwd(const ps::StdDev &S, const double *x, hipStream_t s);
hipError_t launch_std_cw_bwd(const ps::StdDev &S, const double *x, hipStream_t s);
hipError_t launch_split_fwd(const ps::StdDev &S, const double *x, hipStream_t s);
hipError_t launch_split_bwd(const ps::StdDev &S, const double *x, double *grad, hipStream_t s);
}  // namespace psk
