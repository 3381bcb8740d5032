/*
 * ptafs.h -- C ABI of the Fourier-space PTA log-posterior library (gfx950).
 *
 * The library evaluates, for many parameter vectors ("chains") at once, the
 * whitened Fourier-space log-posterior of a pulsar timing array and its full
 * gradient, and runs fixed-step HMC on it.  The density is the one of the
 * paper's Sec. IV (Eqs. likelihood, WN_cov, Fourier_series, RN=Fa, prior_cov,
 * HD, power_law, a_prior, raw_det_posterior) with the Fourier coefficients
 * reparameterised as a = L(eta) z per frequency, L the Cholesky factor of the
 * per-frequency prior covariance (Sec. II.B, Eqs. standardizing_transform and
 * standardized_density with mu = 0, Sigma = phi):
 *
 *   r      = dt - M b - F a - w F a_dm - h(theta_cw)      per TOA
 *   log p  = -1/2 sum_i (r_i^2/N_i + ln N_i + ln 2pi)
 *            - 1/2 (|z|^2 + |z_dm|^2 + |u|^2) - d_z/2 ln 2pi + log pi(theta)
 *   N_i    = (EFAC_mu sigma_i)^2 + EQUAD_mu^2
 *   rho_k  = A^2/(12 pi^2) yr^3 (f_k yr)^-gamma / T      (power law; yr^3 reading)
 *   phi_k  = rho_k Gamma_HD + diag(kappa_.k),  L_k = chol(phi_k)
 *   a_.k,sin = L_k z_.k,sin,  a_.k,cos = L_k z_.k,cos,  a_dm = sqrt(kappa_dm) z_dm,
 *   b = sigma_b u on M = [1, tau, tau^2], tau = (t - mid_I)/halfspan_I.
 *
 * Units: seconds and Hz; every floating-point value is IEEE binary64.
 *
 * Conventions
 *   - Return codes: 0 = success, negative = call-level error (ptafs_strerror).
 *   - Per-chain conditions are not call errors: such a chain gets
 *     logp = -INFINITY, an all-zero gradient and a nonzero status:
 *       1 hyper-parameter outside its prior box (or not finite),
 *       2 phi_k not positive definite,
 *       3 CW evolution variable y >= 1 within the data span (coalescence),
 *       4 non-finite input coordinate or non-finite result.
 *     Other chains are unaffected.
 *   - "device" pointers are HIP device pointers on the dataset's device and are
 *     owned by the caller; all device work is enqueued on the given stream
 *     (hipStream_t passed as void*, NULL = default stream) and the calls return
 *     without synchronising, except where stated.
 *   - Threading: a dataset may be used by one stream at a time (its workspace
 *     is shared by all its calls).  Each call is ordered after the data set's
 *     previous call even when that one ran on another stream (an event the
 *     library records at the end of every call).  No call synchronises the
 *     whole device.
 */
#ifndef PTAFS_H
#define PTAFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PTAFS_OK 0
#define PTAFS_E_ARG (-1)       /* invalid argument or unsupported shape */
#define PTAFS_E_HIP (-2)       /* a HIP runtime call failed */
#define PTAFS_E_NOMEM (-3)     /* device allocation failed */
#define PTAFS_E_LIMIT (-4)     /* a size exceeds a documented limit */

/* Status values written per chain. */
#define PTAFS_ST_OK 0
#define PTAFS_ST_PRIOR 1
#define PTAFS_ST_NOTPD 2
#define PTAFS_ST_CW 3
#define PTAFS_ST_NONFINITE 4

/* Limits of this implementation (PTAFS_E_LIMIT beyond them). */
#define PTAFS_MAX_PSR 128      /* pulsars per data set */
#define PTAFS_MAX_HARM 30      /* max(nf_rn, nf_gw, nf_dm) */

typedef struct ptafs_dataset ptafs_dataset;   /* opaque */

/*
 * Description of one data set (Sec. III: TOAs, uncertainties, backends and
 * their white-noise parameters, radio frequencies, sky positions; Sec. IV.A:
 * basis sizes and hyper-prior box).  All pointers are HOST pointers; the
 * library copies everything during ptafs_dataset_create, so the caller may
 * free them afterwards.
 */
typedef struct {
  int32_t n_psr;                 /* number of pulsars, 1..PTAFS_MAX_PSR */
  const int64_t *toa_offsets;    /* n_psr+1 ascending offsets into the TOA arrays
                                    (CSR over the concatenated pulsars); every
                                    pulsar needs at least one TOA */
  const double *t;               /* TOA times from the array epoch, s, in [0, tspan] */
  const double *dt;              /* timing residuals, s */
  const double *sigma;           /* TOA uncertainties, s (> 0) */
  const double *nu;              /* radio frequency per TOA, Hz (> 0) */
  const int32_t *backend;        /* backend index per TOA, 0..n_backend-1 */
  int32_t n_backend;
  const double *efac;            /* per backend, Eq. WN_cov */
  const double *equad;           /* per backend, s */
  const double *psr_pos;         /* 3*n_psr unit vectors (x, y, z per pulsar) */
  double tspan;                  /* T of Eq. Fourier_series, s (> 0) */
  int32_t nf_rn;                 /* intrinsic red-noise frequencies k = 1..nf_rn (0 = off) */
  int32_t nf_gw;                 /* common HD-correlated frequencies (0 = off) */
  int32_t nf_dm;                 /* DM-noise frequencies (0 = off) */
  double dm_scale;               /* DM basis weight w_i = dm_scale / nu_i^2 */
  double sigma_b;                /* scale of the timing-model coefficients, b = sigma_b u */
  int32_t has_cw;                /* 1: eight CW parameters in theta (Earth term) */
  const double *prior_lo;        /* n_theta lower box edges, theta order below */
  const double *prior_hi;        /* n_theta upper box edges */
} ptafs_dataset_desc;

/*
 * Flat parameter vector of one chain (length d), in this order:
 *   theta: [gw (log10A, gamma) if nf_gw>0 | rn (log10A_I, gamma_I) x n_psr if nf_rn>0 |
 *           dm (log10A_I, gamma_I) x n_psr if nf_dm>0 |
 *           cw (cos theta, phi, log10 Mc, log10 f_gw, Phi0, cos iota, psi, log10 h) if has_cw]
 *   u    : 3 x n_psr (pulsar-major)
 *   z    : n_psr x 2K, K = max(nf_rn, nf_gw), per pulsar k=1 sin, k=1 cos, k=2 sin, ...
 *   z_dm : n_psr x 2 nf_dm, same ordering
 * Offsets below are in elements.
 */
typedef struct {
  int64_t d, n_theta;
  int64_t off_gw, off_rn, off_dm, off_cw, off_u, off_z, off_zdm;
  int64_t n_psr, n_toa, k_coef, k_dm;
  size_t dataset_bytes;          /* device memory held by the data set itself */
  size_t workspace_bytes;        /* workspace needed for the requested n_chains */
  size_t hmc_bytes;              /* scratch of ptafs_hmc_run for the requested n_chains */
} ptafs_layout_info;

/* Copy a data set to the current HIP device and prepare it (per-pulsar tau
 * centring, HD matrix of Eq. HD, backend table).  Synchronises `stream` (and
 * only it).  On success *out owns device memory until ptafs_dataset_destroy.
 * Device memory of data sets comes from a stream-ordered pool the library
 * keeps per device: blocks released by destroyed data sets are reused. */
int ptafs_dataset_create(const ptafs_dataset_desc *desc, void *stream, ptafs_dataset **out);

/* Release a data set and its workspace.  Waits on the host for the data set's
 * own last enqueued work (not for other streams) and returns the memory to the
 * library's pool in stream order.  NULL is a no-op. */
void ptafs_dataset_destroy(ptafs_dataset *ds);

/* Layout of the parameter vector and memory needs for n_chains (>= 0). */
int ptafs_layout(const ptafs_dataset *ds, int32_t n_chains, ptafs_layout_info *out);

/* The same layout and device footprint for a data set that has not been
 * created: validates the descriptor (same checks and error codes as
 * ptafs_dataset_create) and makes no GPU call, so a scheduler can admit work
 * by memory footprint.  Chunking assumes the default tuning. */
int ptafs_estimate(const ptafs_dataset_desc *desc, int32_t n_chains, ptafs_layout_info *out);

/* Grow the data set's workspace to serve up to n_chains per call, on the
 * library's stream after the data set's previous work (no synchronisation).
 * Calls with more chains than reserved grow it themselves, on their stream. */
int ptafs_reserve(ptafs_dataset *ds, int32_t n_chains);

/*
 * Batched log-posterior and gradient (the fused form): one launch of the
 * per-frequency Cholesky + transform, one ragged launch of the TOA pass over
 * all pulsars (FP64 MFMA over 16-chain blocks), a fixed-order reduction, the
 * per-frequency Cholesky adjoint and the assembly.
 *   x      device, [n_chains][d]  input
 *   logp   device, [n_chains]     output
 *   grad   device, [n_chains][d]  output, d log p / d x
 *   status device, [n_chains]     output (values above)
 * n_chains == 0 is a no-op.  Results are bit-identical for identical inputs
 * and the same tuning (fixed reduction order, no floating-point atomics).
 */
int ptafs_logp_grad(ptafs_dataset *ds, int32_t n_chains, const double *x, double *logp,
                    double *grad, int32_t *status, void *stream);

/*
 * ptafs_logp_grad without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, kernels and results (bit-identical to
 * ptafs_logp_grad at the same tuning); the workspace is a static array of the
 * library of PTAFS_NOALLOC_SCRATCH_BYTES per device instead of the data set's
 * own.  Returns PTAFS_E_LIMIT when the workspace for n_chains (the
 * workspace_bytes of ptafs_layout) exceeds that size.  Every call on a device
 * shares that device's array, and no region of it needs to start at zero
 * (each call writes every part it reads), so calls that overlap in time on one
 * device race: serialise them (one stream, or events).  Makes no hipMalloc,
 * hipFree or other allocating call and never synchronises.
 */
#define PTAFS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int ptafs_logp_grad_noalloc(ptafs_dataset *ds, int32_t n_chains, const double *x, double *logp,
                            double *grad, int32_t *status, void *stream);

/*
 * Same result through the plain form: one TOA-pass launch per pulsar with a
 * vector-ALU kernel (no matrix cores), everything else as above.  A
 * reference point for the batched form; same arguments and outputs.
 */
int ptafs_logp_grad_plain(ptafs_dataset *ds, int32_t n_chains, const double *x, double *logp,
                          double *grad, int32_t *status, void *stream);

/*
 * Tuning of the batched TOA pass.  tiles_per_chunk: 16-TOA tiles a workgroup
 * covers (ragged pulsars are cut into chunks of this many tiles);
 * waves_per_block: 1, 2 or 4 waves splitting a chunk; xcd_map: 0 leaves the
 * work items in launch order, 1 places the chain blocks of one chunk on the
 * same XCD, 2 (balanced) also gives every compute unit chunks of near-equal
 * total TOA count when the launch is one full round of resident workgroups
 * (chunks x chain blocks a multiple of the compute units, at most 8 per unit,
 * up to 256 chains; other launches fall back to 1); any other value is
 * PTAFS_E_ARG.  The placement moves no arithmetic: results are bit-identical
 * across xcd_map values at a given chunk length and waves per workgroup.
 * Takes effect on the next call; a new chunk length waits on the host for the
 * data set's own previous work and rebuilds the chunk table on the library's
 * stream.
 */
int ptafs_set_tuning(ptafs_dataset *ds, int32_t tiles_per_chunk, int32_t waves_per_block,
                     int32_t xcd_map);
int ptafs_get_tuning(const ptafs_dataset *ds, int32_t *tiles_per_chunk, int32_t *waves_per_block,
                     int32_t *xcd_map);

/*
 * Fixed-step HMC (App. A: Eqs. Hamiltonian, Gaussian_momentum, HMC_acceptance)
 * with a diagonal inverse mass.  For each trajectory j = traj0 .. traj0+n_traj-1
 * and chain c: momenta p_i = n_i / sqrt(m_i) (n standard normal, Philox4x32-10
 * with key (seed lo, seed hi) and counter (i>>1, c, j, 0), Box-Muller; p_i = 0
 * where the inverse mass m_i is 0), a half kick, n_leapfrog drift/kick steps
 * (the last kick a half kick), and acceptance when ln u < H0 - H1 with u from
 * counter (0, c, j, 1).  Rejected chains keep their state.
 *   inv_mass     device [d] or NULL (identity)
 *   x, logp, grad device, in/out: the chains' state; logp and grad must be the
 *                values at x on entry (e.g. from ptafs_logp_grad)
 *   n_accept     device [n_chains] int64, incremented per accepted trajectory
 *   samples      device [n_traj][n_chains][d] or NULL: state after each trajectory
 *   n_invalid    device [n_chains] int64 or NULL: incremented for every leapfrog
 *                evaluation of the chain that returned a nonzero status
 * use_graph: 1 captures one trajectory as a HIP graph and replays it.  The
 *   graph is kept for later calls with the same arguments (chain count, leapfrog
 *   count, eps, seed, buffers, tuning) and dropped whenever the data set frees
 *   memory it reads (a tuning change, workspace or HMC-buffer growth).
 */
int ptafs_hmc_run(ptafs_dataset *ds, int32_t n_chains, int32_t n_traj, int32_t n_leapfrog,
                  double eps, const double *inv_mass, uint64_t seed, uint64_t traj0, double *x,
                  double *logp, double *grad, int64_t *n_accept, double *samples,
                  int64_t *n_invalid, int32_t use_graph, void *stream);

/*
 * Stage timing of the evaluation pipeline: runs `reps` evaluations (batched,
 * or plain when plain != 0) with a HIP event between consecutive stages on
 * `stream` and writes the mean duration in ms of each stage to the HOST
 * array ms_out[5]: per-frequency forward, TOA pass, chunk reduction,
 * per-frequency adjoint, assembly.  Synchronises the stream.
 */
int ptafs_profile_stages(ptafs_dataset *ds, int32_t n_chains, const double *x, double *logp,
                         double *grad, int32_t *status, int32_t reps, int32_t plain,
                         double *ms_out, void *stream);

/* ======================================================================
 * Standardized form (Sec. IV.B): the paper's own evaluation.
 *
 * The timing model is marginalised analytically (Eq. Gmatrix_proj: N^-1 is
 * replaced by N~^-1 = G (G^T N G)^-1 G^T, G an orthonormal basis of the
 * complement of the timing-model columns), the per-pulsar Gram quantities
 * F~^T N~^-1 F~, F~^T N~^-1 dt, dt^T N~^-1 dt (F~ = [F, w F_dm]) are computed
 * once per data set, and the Fourier coefficients are sampled through the CURN
 * standardizing transform (Eqs. PTA_standard_transform_curn,
 * standardized_stochastic_posterior):
 *
 *   Sigma_I = (beta F~^T N~^-1 F~ + phi_CURN,I^-1)^-1 = L_I L_I^T  (L_I lower Cholesky)
 *   a_I     = beta Sigma_I F~^T N~^-1 dt + L_I z_I
 *   log p~  = beta log L(a) + log N(a; 0, phi) + sum_I ln det L_I + log pi(theta)
 *   log L(a)= sum_I [-1/2 dt^T N~^-1 dt + a_I^T F~^T N~^-1 dt
 *                    - 1/2 a_I^T F~^T N~^-1 F~ a_I - 1/2 ln det(2 pi G^T N G)]
 *
 * phi keeps the HD correlations per frequency (Eq. prior_cov); phi_CURN is its
 * diagonal with Gamma = I (rho_k + kappa_Ik, kappa_dm,Ik).  beta is a per-chain
 * likelihood temperature (App. B, Eqs. tempered_post, mv_normal_post_temp; 1
 * is the untempered posterior).  Every constant is kept (normalised density).
 *
 * Deterministic signal (Sec. IV.C, Eqs. det_F_basis, stoch_det_posterior,
 * det_mean, decenter_det_PTA, standardized_det_posterior), optional: a CW
 * (the Earth-term waveform of the per-TOA form) represented per pulsar as
 * h = F_D a_D(theta_cw) in its own basis F_D of frequencies k / T_D,
 * k = 1..K_D, on an extended span T_D.  a_D is the discrete Fourier transform
 * of the delay sampled at M = 2 K_D + 1 times t_j = j T_D / M:
 * a_(k,sin) = 2/M sum_j h_j sin(2 pi k j / M), a_(k,cos) likewise with cos
 * (the samples' mean, which the timing model absorbs, is dropped).  The data
 * set stores F~^T N~^-1 F_D, F_D^T N~^-1 dt and F_D^T N~^-1 F_D per pulsar;
 * per evaluation d and dt^T N~^-1 dt above become those of dt - h, so the
 * transform centres on the shifted MAP a_bar_CURN (Eq. det_mean) and the
 * likelihood is that of dt - h.
 *
 * Split coefficients (App. C, Eqs. separated_post, split_map_a,
 * split_standardizing_transform), optional: the common process and the
 * pulsar noise get coefficient sets of their own on the same basis, a_G over
 * k = 1..nf_gw and a_R over k = 1..nf_rn then the DM block, with
 * a = a_G + a_R in the likelihood (each on its rows), priors
 * a_G,k ~ N(0, rho_k Gamma) per frequency (HD) and a_R ~ N(0, diag kappa), and
 *   Sigma_G = (beta F~^T N~^-1 F~|_GG + diag rho^-1)^-1 = L_G L_G^T,
 *   Sigma_R = (beta F~^T N~^-1 F~|_RR + diag phi_R^-1)^-1 = L_R L_R^T,
 *   a_G = a_hat_G + L_G z_G,  a_R = a_hat_R + L_R z_R,
 *   log p~ = beta log L(a) + log N(a_G; 0, phi_GWB) + log N(a_R; 0, phi_RN)
 *            + sum_I (ln det L_G,I + ln det L_R,I) + log pi(theta).
 * (a_hat_G, a_hat_R) is the MAP of the joint linear system (Eq. split_map_a)
 * under the CURN prior (Gamma = I, as for the transform above).  Since both
 * sets share the basis it equals the CURN MAP a_hat of the combined
 * coefficients split in proportion to the prior variances:
 * a_hat_G = rho / (rho + phi_R) a_hat, a_hat_R = phi_R / (rho + phi_R) a_hat.
 * Per (pulsar, chain) this takes the combined factorisation and one of each
 * set; Gamma^-1 is formed once per data set.  Needs nf_gw >= 1 and nf_rn >= 1.
 *
 * Parameter vector: [theta | z], theta = [gw | rn per pulsar | dm per pulsar |
 * cw (8, with a CW)] with 2 entries per process for the power law (log10 A,
 * gamma) or one per frequency for the free spectrum (log10 rho_k,
 * rho_k = 10^theta in s^2, Sec. IV.A), the CW parameters in the order of the
 * per-TOA form; z per pulsar: P = 2 ka + 2 nf_dm entries (k = 1 sin, k = 1 cos,
 * ... of the red/common block, ka = max(nf_rn, nf_gw), then the DM block);
 * with split coefficients pz = 2 nf_gw + 2 nf_rn + 2 nf_dm entries per pulsar,
 * z_G (k = 1 sin, k = 1 cos, ... up to nf_gw) then z_R (up to nf_rn, then DM).
 * Per-chain statuses as above (1 box, 2 a factorisation fails, 3 the CW
 * coalesces at a sample time of [0, T_D), 4 non-finite).
 * ====================================================================== */

#define PTAFS_SPEC_POWERLAW 0
#define PTAFS_SPEC_FREE 1
#define PTAFS_MAX_TM 64        /* timing-model columns per TOA */
#define PTAFS_MAX_CW_HARM 64   /* K_D of the deterministic basis */

typedef struct ptafs_std ptafs_std;   /* opaque */

typedef struct {
  int32_t n_psr;                 /* 1..PTAFS_MAX_PSR */
  const int64_t *toa_offsets;    /* n_psr+1 ascending offsets (CSR), >= 1 TOA per pulsar */
  const double *t, *dt, *sigma, *nu;   /* per TOA: s from the array epoch, s, s, Hz */
  const int32_t *backend;        /* per TOA, 0..n_backend-1 */
  int32_t n_backend;
  const double *efac, *equad;    /* per backend (EQUAD in s) */
  const double *psr_pos;         /* 3*n_psr unit vectors */
  double tspan;                  /* T of Eq. Fourier_series, s */
  int32_t nf_rn, nf_gw, nf_dm;   /* frequencies k = 1..nf (0 = process off); not all zero */
  double dm_scale;               /* DM weight w_i = dm_scale / nu_i^2 */
  int32_t n_tm;                  /* timing-model columns per TOA, 0..PTAFS_MAX_TM */
  const double *tm;              /* [n_toa][n_tm] row-major design matrix, or NULL with
                                    n_tm = 0 for M = [1, tau, tau^2] per pulsar.  Columns
                                    that are zero or linearly dependent within a pulsar
                                    are dropped (column-pivoted factorisation). */
  int32_t spectrum;              /* PTAFS_SPEC_POWERLAW or PTAFS_SPEC_FREE (all processes) */
  const double *prior_lo, *prior_hi;   /* n_theta box edges */
  int32_t has_cw;                /* 1: a CW in the deterministic basis (8 more theta entries) */
  int32_t cw_nf;                 /* K_D, 1..PTAFS_MAX_CW_HARM (ignored without a CW) */
  double cw_tspan;               /* T_D > 0, s (ignored without a CW) */
  int32_t split;                 /* 1: split common-process / pulsar-noise coefficients */
} ptafs_std_desc;

typedef struct {
  int64_t d, n_theta, off_gw, off_rn, off_dm, off_z;
  int64_t n_psr, n_toa, k_coef, k_dm, p;   /* p = 2 k_coef + 2 k_dm coefficients per pulsar */
  size_t dataset_bytes, workspace_bytes, hmc_bytes;
  int64_t off_cw;                /* first CW entry of theta, -1 without a CW */
  int64_t pz;                    /* z entries per pulsar: p, or 2 (nf_gw + nf_rn + nf_dm) when split */
} ptafs_std_layout_info;

/* Copy a data set, marginalise its timing model and store the per-pulsar Gram
 * quantities (host, once).  Synchronises `stream` only. */
int ptafs_std_create(const ptafs_std_desc *desc, void *stream, ptafs_std **out);
/* Release (waits for the data set's own last work only).  NULL is a no-op. */
void ptafs_std_destroy(ptafs_std *ds);

/* The per-pulsar quantities ptafs_std_create stores, computed on the host
 * with no GPU call (for checks and for sizing): for pulsar `pulsar`,
 * s0 [p][p] = F~^T N~^-1 F~, dvec [p] = F~^T N~^-1 dt and
 * scal[0] = dt^T N~^-1 dt, scal[1] = -1/2 ln det(2 pi G^T N G), scal[2] = the
 * number of timing-model columns kept (host pointers, original order).
 * ptafs_std_precompute_cw gives the CW products of a data set with a CW:
 * sd [p][2 K_D] = F~^T N~^-1 F_D, ed [2 K_D] = F_D^T N~^-1 dt,
 * qd [2 K_D][2 K_D] = F_D^T N~^-1 F_D (basis order k = 1 sin, k = 1 cos, ...). */
int ptafs_std_precompute(const ptafs_std_desc *desc, int32_t pulsar, double *s0, double *dvec,
                         double *scal);
int ptafs_std_precompute_cw(const ptafs_std_desc *desc, int32_t pulsar, double *sd, double *ed,
                            double *qd);
int ptafs_std_layout(const ptafs_std *ds, int32_t n_chains, ptafs_std_layout_info *out);

/*
 * log p~ and its gradient for n_chains points.
 *   x      device [n_chains][d]     beta  device [n_chains] or NULL (all 1)
 *   logp   device [n_chains]        grad  device [n_chains][d]
 *   status device [n_chains]
 * Per (pulsar, chain) one factorisation of the P x P CURN precision and its
 * inverse (with split coefficients also one of each set's precision), per
 * (frequency, chain) one N_p x N_p factorisation of phi_k (with split
 * coefficients none: Gamma^-1 is formed once), on FP64 matrix cores; results
 * are bit-identical for identical inputs.
 */
int ptafs_std_logp_grad(ptafs_std *ds, int32_t n_chains, const double *x, const double *beta,
                        double *logp, double *grad, int32_t *status, void *stream);

/* The Fourier coefficients a = a_hat + L z of each point (the map back from
 * z, Eq. PTA_standard_transform_curn): a device [n_chains][n_psr][p]; with
 * split coefficients [a_G | a_R] (Eq. split_standardizing_transform),
 * a device [n_chains][n_psr][pz]. */
int ptafs_std_coefficients(ptafs_std *ds, int32_t n_chains, const double *x, const double *beta,
                           double *a, void *stream);

/* Stage timing of ptafs_std_logp_grad: `reps` evaluations with a HIP event
 * between the stages on `stream`; mean ms per stage to the HOST array
 * ms_out[4]: per-pulsar transform (k_std_fwd; with a CW its k_std_cw_fwd,
 * with split coefficients the sets' factorisations and k_split_comb), prior
 * per frequency (k_std_prior_* or k_split_prior_g), per-pulsar adjoint
 * (k_std_bwd or the k_split_bwd kernels; with a CW k_std_cw_bwd), assembly.
 * Synchronises the stream. */
int ptafs_std_profile_stages(ptafs_std *ds, int32_t n_chains, const double *x, const double *beta,
                             double *logp, double *grad, int32_t *status, int32_t reps,
                             double *ms_out, void *stream);

/* Fixed-step HMC on log p~ with the conventions of ptafs_hmc_run (same
 * momenta, accept test, graph capture and buffers); beta as above. */
int ptafs_std_hmc_run(ptafs_std *ds, int32_t n_chains, int32_t n_traj, int32_t n_leapfrog,
                      double eps, const double *inv_mass, uint64_t seed, uint64_t traj0,
                      const double *beta, double *x, double *logp, double *grad,
                      int64_t *n_accept, double *samples, int64_t *n_invalid, int32_t use_graph,
                      void *stream);

/* Human-readable text for a return code (static storage). */
const char *ptafs_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* PTAFS_H */
