// Internal definitions shared by the HIP translation units of libptafs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ptafs.h"

namespace pt {

constexpr double kYear = 365.25 * 86400.0;      // Julian year, s
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.14159265358979323846264338328;
constexpr double kLn10 = 2.30258509299404568401799145468;
constexpr double kLn2Pi = 1.83787706640934548356065947281;
constexpr double kTsun = 4.925490947641e-6;      // G Msun / c^3, s

constexpr int kChainBlock = 16;                  // chains per MFMA column block
constexpr int kToaPad = 128;                     // zero padding of per-TOA arrays
constexpr int kSpecSeg = 16;                     // frequency segments per chain (spectral kernels)
constexpr int kTile = 16;                        // TOAs per MFMA row tile

// ---------------------------------------------------------------------------
// Basis slots of the TOA pass.
//
// The TOA pass contracts over basis "rows" j.  Row j sits at MFMA K-step
// s = j / 4 and lane group q = j % 4 of the forward F-operand; pairs of steps
// (2m, 2m+1) give lane group q the sin and cos of harmonic h + 1, h = 4m + q,
// so every lane walks the harmonics q+1, q+5, q+9, ... with one angle-addition
// step per pair.  In the red-noise block, slots with h >= kb carry the timing
// model columns (1, tau, tau^2) and then zeros; in the DM block slots with
// h >= kdm are zero.
// ---------------------------------------------------------------------------
struct Slot {
  int kind;   // 0 Fourier harmonic, 1 timing-model column, 2 padding
  int harm;   // harmonic k (1-based) for kind 0
  int sc;     // 0 sin, 1 cos (kind 0)
  int tm;     // 0,1,2 -> 1, tau, tau^2 (kind 1)
};

__host__ __device__ inline Slot rn_slot(int row, int kb) {
  const int s = row >> 2, q = row & 3, m = s >> 1, h = 4 * m + q, sc = s & 1;
  Slot r{2, 0, 0, 0};
  if (h < kb) {
    r.kind = 0; r.harm = h + 1; r.sc = sc;
  } else {
    const int ti = 2 * (h - kb) + sc;
    if (ti < 3) { r.kind = 1; r.tm = ti; }
  }
  return r;
}

__host__ __device__ inline Slot dm_slot(int row, int kdm) {
  const int s = row >> 2, q = row & 3, m = s >> 1, h = 4 * m + q, sc = s & 1;
  Slot r{2, 0, 0, 0};
  if (h < kdm) { r.kind = 0; r.harm = h + 1; r.sc = sc; }
  return r;
}

// Row of harmonic k (1-based) / sin-cos sc in either block.
__host__ __device__ inline int harm_row(int k, int sc) {
  const int h = k - 1, m = h >> 2, q = h & 3;
  return 4 * (2 * m + sc) + q;
}
// Row of timing-model column ti in the red-noise block.
__host__ __device__ inline int tm_row(int ti, int kb) {
  const int h = kb + (ti >> 1), m = h >> 2, q = h & 3;
  return 4 * (2 * m + (ti & 1)) + q;
}

// 16-row tiles of a block holding `nslots_pairs` harmonic/TM pair slots.
__host__ __device__ inline int tiles_for_pairs(int pairs) {
  const int steps = 2 * ((pairs + 3) / 4);
  return (steps + 3) / 4;
}
// rows of a coefficient block: at most PTAFS_MAX_HARM + 2 pairs, four tiles
constexpr int kMaxRows = 64;
// workgroups per chain of the HMC momentum draw (its kinetic energy in as
// many partial sums, added in order by the accept step)
constexpr int kHmcBeginG = 4;


// Packed lower-triangular storage, row-major: row i holds columns 0..i.
__host__ __device__ inline int pk(int i, int j) { return (i * (i + 1)) / 2 + j; }

// Dense per-frequency factors: up to kTileMaxNT 16-row tiles they are kept
// tile-major (the lower tiles of the padded matrix, 256 doubles each, row-major
// inside a tile); beyond that packed row-major.
// The tiled factorisation (k_cholt_fwd) holds up to kTileFwdMaxNT tiles in
// registers; the tiled adjoint (k_cholt_bwd) all of C^-1 up to kTileMaxNT
// tiles, one block column of it (the rest in LDS) up to kTileFwdMaxNT.
constexpr int kTileMaxNT = 5;
constexpr int kTileFwdMaxNT = 7;
__host__ __device__ inline int chol_tiles(int n) { return (n + 15) / 16; }
__host__ __device__ inline size_t chol_store_doubles(int n) {
  const int nt = chol_tiles(n);
  return nt <= kTileFwdMaxNT ? (size_t)(nt * (nt + 1) / 2) * 256 : (size_t)n * (n + 1) / 2;
}

// ---------------------------------------------------------------------------
// Device view of a data set plus the workspace of one call.
// ---------------------------------------------------------------------------
struct Dev {
  // sizes
  int n_psr, n_toa, n_backend;
  int nf_rn, nf_gw, nf_dm, has_cw;
  int ka;        // coefficient frequencies max(nf_rn, nf_gw)
  int kb;        // basis harmonics of the TOA pass max(ka, nf_dm)
  int jt_rn, jt_dm, rows_rn, rows_dm;
  // coefficient rows no frequency owns (timing model, padding), per block
  int n_free_rn, n_free_dm;
  int16_t free_rn[kMaxRows], free_dm[kMaxRows];
  int n_theta, d;
  int off_gw, off_rn, off_dm, off_cw, off_u, off_z, off_zdm;
  double tspan, dm_scale, sigma_b, tmax, prior_const;
  // data-set arrays (device)
  const double *t, *dt, *sigma, *nu;
  const int32_t *backend;
  const double *efac, *equad;
  const int64_t *toa_off;
  const double *tau_c, *tau_sinv;
  // per-TOA basis phases, padded by kToaPad zeros: sin, cos of 2 pi t / T,
  // tau = (t - mid_I) / halfspan_I, DM weight w = dm_scale / nu^2
  const double *sth, *cth, *tau, *wdm;
  // white noise (Eq. WN_cov; EFAC, EQUAD fixed per backend): 1/N per TOA
  // (zeros in the padding) and sum_i ln N_i
  const double *invn;
  double lnn_total;
  const double *pos, *gamma;
  const double *gchol;         // chol(Gamma), packed row-major lower
  const double *gtile;         // chol(Gamma) zero-padded, lower 16x16 tiles (up to kTileFwdMaxNT)
  const double *gam_tile;      // Gamma zero-padded, lower 16x16 tiles stored column-major, diagonal tiles full (up to kTileFwdMaxNT)
  const double *prior_lo, *prior_hi;
  // power-law spectra: ln(f_k yr) for f_k = (k + 1) / T, k < PTAFS_MAX_HARM, and ln(yr^3 / (12 pi^2 T))
  const double *lnfy;
  double pl_c;
  // chunk table of the batched TOA pass
  int n_chunks, tiles_per_chunk;
  const int32_t *chunk_psr, *chunk_begin, *chunk_end, *psr_chunk0;
  // work item (chunk * n_cb + chain block) of each TOA-pass workgroup under
  // the balanced placement, or null (then the XCD-grouped order, or none)
  const int32_t *wg_map;
  int n_cu;                    // compute units of the device
  int n_xcd;                   // their XCDs (workgroups are dealt to them round-robin)
  // call
  int n_chains, c_pad, n_cb;
  // workspace
  double *coef_rn, *coef_dm;   // [n_psr][rows][c_pad]
  double *lstore;              // [c_pad][nf_gw][n_psr*(n_psr+1)/2]
  double *sqk_rn, *sqk_dm;     // [ka | nf_dm][n_psr][c_pad] sqrt(kappa) of the diagonal frequencies
  double *cwc;                 // [n_psr][kCwConst][c_pad] per chain/pulsar CW constants
  double *part_rn, *part_dm;   // [n_wg][rows][16]
  double *part_chi, *part_cw;  // [n_wg][16], [n_wg][8][16]
  double *bar_rn, *bar_dm;     // [n_psr][rows][c_pad]
  double *chi_p, *cw_p;        // [n_psr][c_pad], [n_psr][8][c_pad]
  double *dth_k;               // [c_pad][K][2] gw parts per frequency
  double *drn_k;               // [c_pad][n_psr][ka][2]
  double *ddm_k;               // [c_pad][n_psr][nf_dm][2]

  int32_t *flag_k;             // [c_pad][kmax] kFlagNotPD of the diagonal frequencies (k_spec_fwd)
  int32_t *flag_dense;         // [c_pad][nf_gw] kFlagNotPD of the dense frequencies (k_cholt/k_chol)
  int32_t *flag_out;           // [c_pad][kmax + kSpecSeg] kFlagOutNonfinite of the adjoints:
                               //   [k] dense frequency k (k < nf_gw), [kmax + seg] k_spec_bwd segment
  int32_t *st_pre;             // [c_pad] status from the input checks
};

// Power-law spectrum A^2/(12 pi^2) yr^3 (f yr)^-gamma / T at f_k = (k + 1) / T
// (Sec. IV.A, Eq. power_law with yr^3), evaluated in logarithms.
// Per-frequency parts of the red-noise and DM hyper-parameter gradient,
// [c][I][k][2] with the frequency innermost (k_finalize sums them over k from
// consecutive words), and sqrt(kappa) of the diagonal frequencies kept by the
// forward for the adjoint, [k][I][c] (chain-minor like the coefficient
// panels, so 16 consecutive chains fill 128 bytes).
__device__ inline double *drn_at(const Dev &D, int c, int I, int k) {
  return D.drn_k + (((size_t)c * D.n_psr + I) * D.ka + k) * 2;
}
__device__ inline double *ddm_at(const Dev &D, int c, int I, int k) {
  return D.ddm_k + (((size_t)c * D.n_psr + I) * D.nf_dm + k) * 2;
}
__device__ inline size_t sqk_at(const Dev &D, int c, int I, int k) {
  return ((size_t)k * D.n_psr + I) * D.c_pad + c;
}

__device__ inline double powerlaw_k(const Dev &D, int k, double log10A, double gamma) {
  return exp(2.0 * kLn10 * log10A - gamma * D.lnfy[k] + D.pl_c);
}
// sqrt of the same, as one exponential of half the exponent
__device__ inline double powerlaw_sqrt_k(const Dev &D, int k, double log10A, double gamma) {
  return exp(kLn10 * log10A - 0.5 * gamma * D.lnfy[k] + 0.5 * D.pl_c);
}

constexpr int kFlagNotPD = 1;          // phi_k not positive definite
constexpr int kFlagOutNonfinite = 4;   // a non-finite gradient entry

constexpr int kCwConst = 16;   // rows of the per (chain, pulsar) CW constant table

}  // namespace pt

namespace pt {

// Prior box of a chain's hyper-parameters, checked by one wave.
__device__ inline bool theta_in_box_wave(const Dev &D, const double *xc) {
  // eight parameters per lane per batch, all loads issued together (indexes
  // clamped to the last parameter, so no lane branches around a load)
  constexpr int kB = 8;
  bool ok = true;
  const int l = (int)(threadIdx.x & 63), last = D.n_theta - 1;
  for (int i0 = 0; i0 < D.n_theta; i0 += 64 * kB) {
    double v[kB], lo[kB], hi[kB];
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const int i = min(i0 + l + 64 * j, last);
      v[j] = xc[i];
      lo[j] = D.prior_lo[i];
      hi[j] = D.prior_hi[i];
    }
#pragma unroll
    for (int j = 0; j < kB; ++j)
      if (!(v[j] >= lo[j] && v[j] <= hi[j])) ok = false;
  }
  return __all(ok);
}

// Wave64 / workgroup reductions in a fixed order (deterministic).
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline int wave_or(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}
// Sum over a 256-thread workgroup; every thread gets the result.
__device__ inline double block_sum256(double v, double *red4) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red4[w] = v;
  __syncthreads();
  return (red4[0] + red4[1]) + (red4[2] + red4[3]);
}
__device__ inline int block_or256(int v, int *red4) {
  v = wave_or(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red4[w] = v;
  __syncthreads();
  return red4[0] | red4[1] | red4[2] | red4[3];
}
// The same over a workgroup of NW waves (wave sums added in wave order).
template <int NW>
__device__ inline double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) s += red[i];
  return s;
}
template <int NW>
__device__ inline int block_or(int v, int *red) {
  v = wave_or(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  int s = red[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) s |= red[i];
  return s;
}

// A leapfrog kick and drift that k_finalize applies to a chain right after
// its gradient: p += eps grad, x += eps M^-1 p, and one more invalid
// evaluation counted when the status is nonzero.
struct Kick {
  double eps;
  const double *inv_mass;   // [d], or null for the identity
  double *x;                // [n_chains][d], the evaluated points
  double *p;                // [n_chains][d]
  int64_t *n_invalid;       // [n_chains], or null
};

}  // namespace pt

// Launch helpers implemented in the kernel translation units.
namespace ptk {
hipError_t launch_spectral_fwd(const pt::Dev &D, const double *x, hipStream_t s);
hipError_t launch_spectral_bwd(const pt::Dev &D, const double *x, double *grad, hipStream_t s);
hipError_t launch_spec_fwd(const pt::Dev &D, const double *x, hipStream_t s);
hipError_t launch_toa_mfma(const pt::Dev &D, int waves_per_block, int xcd_map, hipStream_t s);
hipError_t launch_toa_plain_psr(const pt::Dev &D, int p, int n_chunks_p, hipStream_t s);
hipError_t set_plain_lds_limit(size_t bytes);
hipError_t launch_chol_fwd(const pt::Dev &D, const double *x, hipStream_t s);
hipError_t launch_chol_bwd(const pt::Dev &D, const double *x, double *grad, hipStream_t s);
hipError_t launch_cholt_fwd(const pt::Dev &D, const double *x, hipStream_t s);
hipError_t launch_cholt_bwd(const pt::Dev &D, const double *x, double *grad, hipStream_t s);
hipError_t launch_reduce_chunks(const pt::Dev &D, hipStream_t s);
hipError_t launch_spec_bwd(const pt::Dev &D, const double *x, double *grad, hipStream_t s);
hipError_t launch_finalize(const pt::Dev &D, const double *x, double *logp, double *grad,
                           int32_t *status, hipStream_t s, const pt::Kick *kick = nullptr);
// HMC pieces
hipError_t launch_hmc_begin(const pt::Dev &D, int d, double eps, const double *inv_mass,
                            uint64_t seed, const uint64_t *traj, double *x, const double *logp,
                            const double *grad, double *p, double *x0, double *lp0, double *g0,
                            double *h0, hipStream_t s);
hipError_t launch_hmc_end(int n_chains, int d, double eps, const double *inv_mass, uint64_t seed,
                          const uint64_t *traj, double *x, double *logp,
                          double *grad, double *p, const double *x0, const double *lp0,
                          const double *g0, const double *h0, int64_t *n_accept, double *samples,
                          const int32_t *status, int64_t *n_invalid, hipStream_t s);
hipError_t launch_traj_inc(uint64_t *traj, hipStream_t s);
hipError_t launch_traj_set(uint64_t *traj, uint64_t traj0, hipStream_t s);
}  // namespace ptk
