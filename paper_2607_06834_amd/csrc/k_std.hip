// Kernels of the standardized form (Sec. IV.B; Eqs. PTA_standard_transform_curn,
// standardized_stochastic_posterior in the Gram form of Eq. posterior_implemented;
// App. B for a tempered likelihood).
//
// Per pulsar I and chain c (one 256-thread workgroup each):
//   A = beta S0_I + diag(1 / D),  D = CURN variances of the chain (rho_k + kappa_Ik,
//   kappa_dm,Ik);  Sigma = A^-1 = L L^T with L the lower Cholesky factor.
// In the reversed index order r = P - 1 - j the matrix A~ = J A J has a lower
// Cholesky factor L~, and L = J L~^-T J: the lower Cholesky factor of the
// covariance comes from the ordinary factorisation of the reversed precision.
// With X = L~^-1 (lower):
//   a~ = X^T (X beta d~ + z~)      (a = a_hat + L z)
//   ln det L = sum_r ln X_rr
// The adjoint (k_std_bwd) takes v = dF/da = beta (d - S0 a) - phi^-1 a:
//   dlogp/dz~ = X v~
//   dlogp/dD_j = [a_hat_j (Sigma v)_j + T_j + Sigma_jj / 2] / D_j^2
// with (Sigma v)~ = X^T X v~, Sigma~_rr = |X e_r|^2 and T_r a suffix sum down
// column r of X (the diagonal of L Phi(L^T v z^T) L^T).
//
// Per frequency k and chain (k_std_prior): phi_k = rho_k Gamma + diag kappa_.k
// (Eq. prior_cov) factorised the same way, y = X_k a, u = X_k^T y = phi_k^-1 a,
// and the explicit prior derivatives 1/2 u^T Gamma u - tr(phi_k^-1 Gamma) (rho)
// and 1/2 u_I^2 - (phi_k^-1)_II (kappa), with tr(phi^-1 Gamma) = |X_k chol Gamma|_F^2.
//
// With a deterministic CW in its own basis (Sec. IV.C), k_std_cw_fwd replaces
// d and dt^T N~^-1 dt of each (pulsar, chain) by those of dt - F_D a_D before
// the transform, and k_std_cw_bwd takes dlog p / d d_bar = beta (a + Sigma v)
// (the likelihood's explicit term plus the shift of a_hat) back to the CW
// parameters through S_D, Q_D, e_D, the transform of the samples and the
// waveform's derivative.
//
// Matrices live in LDS as lower 16x16 tiles (row-major inside).  The
// factorisation is right-looking by block columns: a diagonal tile is factorised
// and inverted by one wave (lane r holds row r, operands by readlane), the
// panel and the trailing tiles are updated on FP64 matrix cores
// (v_mfma_f64_16x16x4f64), and X = L^-1 follows by block forward substitution,
// also on matrix cores.  MFMA operand convention (lane l = c + 16 q): slice s of
// a 16x16x16 product takes A[c][q + 4s] and B[q + 4s][c] (reduction index
// q + 4s); the result holds R[q + 4v][c] in register v (the row of the A
// operand's lane q + 4v), which is directly the B operand of a next product.
#include <cmath>

#include "cw_dev.h"
#include "std.h"

namespace {

using ps::StdDev;
using v4d = double __attribute__((ext_vector_type(4)));

__device__ inline double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/sqrt(a) and 1/a: hardware estimates refined by two Newton steps
__device__ inline double rsqrt_nr(double a) {
  double y = __builtin_amdgcn_rsq(a);
  y = y * (1.5 - 0.5 * a * y * y);
  y = y * (1.5 - 0.5 * a * y * y);
  return y;
}
__device__ inline double rcp_nr(double a) {
  double y = __builtin_amdgcn_rcp(a);
  y = fma(y, fma(-a, y, 1.0), y);
  y = fma(y, fma(-a, y, 1.0), y);
  return y;
}

// LDS tiles are row-major with the column index XOR-ed with the row index,
// element (r, c) at 16 r + (c ^ r): the 16 lanes that read one column (a row
// each), or one row (a column each), or an MFMA operand, hit 16 different
// banks.
__device__ inline int sw(int r, int c) { return (r << 4) + (c ^ r); }

// Tile loads for the MFMA operands (see the convention above).
__device__ inline v4d ld_rm(const double *t, int c, int q) {   // Y[c][q+4s]: A of Y, B of Y^T
  return v4d{t[sw(c, q)], t[sw(c, q + 4)], t[sw(c, q + 8)], t[sw(c, q + 12)]};
}
__device__ inline v4d ld_cm(const double *t, int c, int q) {   // Y[q+4s][c]: B of Y, result of Y
  return v4d{t[sw(q, c)], t[sw(q + 4, c)], t[sw(q + 8, c)], t[sw(q + 12, c)]};
}
__device__ inline void st_cm(double *t, int c, int q, v4d v) {
  t[sw(q, c)] = v[0];
  t[sw(q + 4, c)] = v[1];
  t[sw(q + 8, c)] = v[2];
  t[sw(q + 12, c)] = v[3];
}
// the same from a plain row-major tile in global memory
__device__ inline v4d ldg_cm(const double *t, int c, int q) {
  const double *p = t + 16 * q + c;
  return v4d{p[0], p[64], p[128], p[192]};
}
__device__ inline v4d mma(v4d a, v4d b, v4d acc) {
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], b[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], b[3], acc, 0, 0, 0);
  return acc;
}

// Keeps a register row computed here: the updates before it happen before the
// loads after it (no load is hoisted above, no update sunk below).
__device__ inline void pin_row(double (&v)[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) asm volatile("" : "+v"(v[k]));
  asm volatile("" ::: "memory");
}

// A pointer into LDS that stays one (DS instructions, not flat ones).
using lds_dp = __attribute__((address_space(3))) double *;

__device__ inline void wave_sync() {   // LDS writes of the wave visible to its later reads
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cholesky factor of the symmetric 16x16 tile t (both triangles present), in
// place in the lower triangle (the upper one is left undefined).  Executed by
// one wave; lane r holds row r.  Right-looking: pivot j's multipliers reach
// rows j + 1 and j + 2 at once by readlane, the other rows through an LDS copy
// of column j (bc, three buffers of 16) read two pivots later, when the store
// has long completed (a wave's LDS accesses are executed in order).  idg
// receives 1 / L_jj.  With LZ, lzJ[r] += sum_c L_rc zJ[c].  Returns false in
// every lane when a pivot is not positive and finite.
template <bool LZ>
__device__ __forceinline__ bool diag_factor(double *t, lds_dp bc, lds_dp idg, int lane, const double *zJ,
                                            double *lzJ) {
  const int r = lane & 15;
  double row[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) row[c] = t[sw(r, c)];
  bool ok = true;
  double l1 = 0.0, l2 = 0.0;   // this lane's multipliers of the two previous pivots
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const double piv = readlane_d(row[j], j);
    double bv[16];
    const bool def = (j >= 2) && (j <= 14);   // pivot j - 2 still owes rows j + 1 ...
    if (def) {
      const auto bp = bc + 16 * ((j - 2) % 3);
#pragma unroll
      for (int k = j + 1; k < 16; ++k) bv[k] = bp[k];
    }
    ok = ok && (piv > 0.0) && isfinite(piv);
    const double rs = rsqrt_nr(piv);
    const double l = row[j] * rs;       // L[r][j] (r >= j)
    row[j] = l;
    // the next pivot's column first (the path from pivot to pivot), then the rest
    if (j + 1 < 16) {
      if (def) row[j + 1] = fma(-l2, bv[j + 1], row[j + 1]);
      row[j + 1] = fma(-l, readlane_d(l, j + 1), row[j + 1]);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (def) {
#pragma unroll
      for (int k = j + 2; k < 16; ++k) row[k] = fma(-l2, bv[k], row[k]);
    }
    if (j + 2 < 16) row[j + 2] = fma(-l, readlane_d(l, j + 2), row[j + 2]);
    pin_row(row);   // the updates before the stores: a wait for the loads then
                    // does not also wait for the stores (LDS completes in order)
    if (j <= 12 && lane < 16) bc[16 * (j % 3) + r] = l;
    if (lane == 0) idg[j] = rs;
    l2 = l1;
    l1 = l;
    asm volatile("" ::: "memory");
  }
  if (lane < 16) {
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c <= r) t[sw(r, c)] = row[c];
    if (LZ) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < 16; ++c) s = fma((c <= r) ? row[c] : 0.0, zJ[c], s);
      lzJ[r] += s;
    }
  }
  return ok;
}

// The lower-triangular tile t (L, upper triangle undefined) replaced by
// X = L^-1 (zeros above); idg = 1 / L_jj.  Executed by one wave: lane c < 16
// solves L x = e_c for column c, x_m = (delta_mc - sum_{k<m} L_mk x_k) / L_mm,
// with L read from the tile at the same address in every lane.  Column m + 1
// of L is loaded while column m is applied; the solve and the stores sit in
// one branch so that the wave's loads all precede its stores.
__device__ __forceinline__ void diag_inverse(double *t, lds_dp idg, int lane) {
  const int r = lane & 15;
  if (lane < 16) {
    double acc[16], xc[16], lc[2][16], dg[2];
#pragma unroll
    for (int m = 0; m < 16; ++m) acc[m] = 0.0;
    dg[0] = idg[0];
#pragma unroll
    for (int k = 1; k < 16; ++k) lc[0][k] = t[sw(k, 0)];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int b = m & 1;
      if (m < 15) {
        dg[b ^ 1] = idg[m + 1];
#pragma unroll
        for (int k = m + 2; k < 16; ++k) lc[b ^ 1][k] = t[sw(k, m + 1)];
      }
      const double xm = (((m == r) ? 1.0 : 0.0) - acc[m]) * dg[b];
      xc[m] = xm;
#pragma unroll
      for (int k = m + 1; k < 16; ++k) acc[k] = fma(lc[b][k], xm, acc[k]);
      pin_row(acc);
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) t[sw(m, r)] = (m >= r) ? xc[m] : 0.0;
  }
}

// Row r of a panel tile: L_IJ = A_IJ L_JJ^-T by substitution,
// x_c = (a_c - sum_{k<c} x_k L_ck) / L_cc, one row per thread, L_JJ (lower)
// read at the same address by every lane.  With LZ, lzI[r] += sum_c x_c zJ[c].
template <bool LZ>
__device__ __forceinline__ void panel_row(double *t, const double *ljj, lds_dp idg, int r,
                                          const double *zJ, double *lzI) {
  double x[16], lc[2][16], dg[2];
#pragma unroll
  for (int c = 0; c < 16; ++c) x[c] = t[sw(r, c)];
  dg[0] = idg[0];
#pragma unroll
  for (int k = 1; k < 16; ++k) lc[0][k] = ljj[sw(k, 0)];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int b = c & 1;
    if (c < 15) {   // column c + 1 of L_JJ while column c is applied
      dg[b ^ 1] = idg[c + 1];
#pragma unroll
      for (int k = c + 2; k < 16; ++k) lc[b ^ 1][k] = ljj[sw(k, c + 1)];
    }
    x[c] *= dg[b];
#pragma unroll
    for (int k = c + 1; k < 16; ++k) x[k] = fma(-x[c], lc[b][k], x[k]);
    pin_row(x);
  }
#pragma unroll
  for (int c = 0; c < 16; ++c) t[sw(r, c)] = x[c];
  if (LZ) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) s = fma(x[c], zJ[c], s);
    lzI[r] += s;
  }
}

// Trailing update A_IK -= L_IJ L_KJ^T of two tiles at once (two independent
// MFMA chains); the second is computed but not stored when has1 is false.
__device__ inline void trail_pair(double *A, int J, int I0, int K0, int I1, int K1, bool has1, int c, int q) {
  double *t0 = A + ps::tix(I0, K0) * 256, *t1 = A + ps::tix(I1, K1) * 256;
  const v4d a0 = ld_rm(A + ps::tix(I0, J) * 256, c, q), b0 = ld_rm(A + ps::tix(K0, J) * 256, c, q);
  const v4d a1 = ld_rm(A + ps::tix(I1, J) * 256, c, q), b1 = ld_rm(A + ps::tix(K1, J) * 256, c, q);
  const v4d r0 = mma(-a0, b0, ld_cm(t0, c, q));
  const v4d r1 = mma(-a1, b1, ld_cm(t1, c, q));
  st_cm(t0, c, q, r0);
  if (has1) st_cm(t1, c, q, r1);
}

// (K, I) of trailing task n at step J: the pairs J < K <= I < T in order
template <int T>
__device__ inline void task_ki(int J, int n, int &K, int &I) {
  K = J + 1;
  while (n >= T - K) { n -= T - K; ++K; }
  I = K + n;
}

// In-place X = L^-1 of the symmetric positive-definite matrix held as lower
// tiles in A (diagonal tiles with both triangles).  All 256 threads call it.
// flag (LDS) is set to 0 when a pivot fails; the return value is the flag;
// flag[1] serves as a work counter.  ws: 48 + 16 T doubles of LDS scratch.  With LZ the product L z of the factor
// with the vector z (LDS, 16 T) is accumulated into lz (LDS, zero on entry).
//
// Factorisation: right-looking by block columns with a lookahead of one: at
// step J the panel is solved against L_JJ (a row per thread), then one wave
// updates the next diagonal tile and factorises it while the other waves take
// the rest of the trailing update and the inverse of tile J from a shared
// counter (the factorising wave joins when done).  Inverse: X_CA = -X_CC (L_CA X_AA) for
// neighbouring diagonal blocks A and C of s tiles, s = 1, 2, 4, ... (rows of
// L_CA X_AA, then columns of X_CA dealt to the waves).
template <int T, bool LZ>
__device__ __forceinline__ bool factor_invert(double *A, int tid, int *flag, double *ws,
                                              const double *z, double *lz) {
  int *ctr = flag + 1;   // work counter of the trailing phases
  const int w = tid >> 6, lane = tid & 63, c = lane & 15, q = lane >> 4;
  const int wd = 0;   // the wave that factorises the diagonal tiles
  // The scratch sits past 64 KB of LDS in the larger kernels, beyond a DS
  // instruction's immediate offset: held in a register (the asm hides its
  // constant value), its accesses take the offsets as immediates instead of
  // forming each address anew.
  lds_dp bc = (lds_dp)ws;
  asm volatile("" : "+v"(bc));
  lds_dp idg = bc + 48;   // idg: 16 per diagonal tile
  if (w == wd) {
    const bool ok = diag_factor<LZ>(A, bc, idg, lane, z, lz);
    if (lane == 0 && !ok) *flag = 0;
  }
  __syncthreads();
#pragma unroll 1
  for (int J = 0; J < T; ++J) {
    {
      const int I = J + 1 + (tid >> 4);
      if (I < T)
        panel_row<LZ>(A + ps::tix(I, J) * 256, A + ps::tix(J, J) * 256, idg + 16 * J, tid & 15,
                      LZ ? z + 16 * J : nullptr, LZ ? lz + 16 * I : nullptr);
    }
    if (tid == 0) *ctr = 0;
    __syncthreads();
    if (J + 1 == T) break;
    if (w == wd) {
      // lookahead: tile (J+1, J+1), then its factorisation
      double *t = A + ps::tix(J + 1, J + 1) * 256;
      const v4d l = ld_rm(A + ps::tix(J + 1, J) * 256, c, q);
      st_cm(t, c, q, mma(-l, l, ld_cm(t, c, q)));
      wave_sync();
      const bool ok = diag_factor<LZ>(t, bc, idg + 16 * (J + 1), lane, LZ ? z + 16 * (J + 1) : nullptr,
                                      LZ ? lz + 16 * (J + 1) : nullptr);
      if (lane == 0 && !ok) *flag = 0;
    }
    // the rest of the step's work, taken two items at a time from a counter:
    // item 0 inverts tile J (its panel is done), items 1..nt are the other
    // trailing tiles (trailing task 0 is the diagonal tile); the factorising
    // wave joins when done
    {
      const int m = T - 1 - J, nt = m * (m + 1) / 2 - 1;
      for (;;) {
        int n0 = 0;
        if (lane == 0) n0 = atomicAdd(ctr, 2);
        n0 = __builtin_amdgcn_readfirstlane(n0);
        if (n0 > nt) break;
        if (n0 == 0) {
          diag_inverse(A + ps::tix(J, J) * 256, idg + 16 * J, lane);
          if (nt < 1) continue;
          n0 = 1;
        }
        const bool has1 = n0 > 1 && n0 + 1 <= nt;
        int K0, I0, K1, I1;
        task_ki<T>(J, n0, K0, I0);
        task_ki<T>(J, has1 ? n0 + 1 : n0, K1, I1);
        trail_pair(A, J, I0, K0, I1, K1, has1, c, q);
      }
    }
    __syncthreads();
  }
  // the last diagonal tile's inverse
  if (w == 0) diag_inverse(A + ps::tix(T - 1, T - 1) * 256, idg + 16 * (T - 1), lane);
  __syncthreads();
  // X from the diagonal inverses by doubling
#pragma unroll
  for (int sb = 1; sb < T; sb *= 2) {
    // rows i of Y = L_CA X_AA over L_CA: block b (A = [b, b+sb), C = [b+sb, min(b+2sb, T)))
    {
      int item = 0;
#pragma unroll
      for (int b = 0; b + sb < T; b += 2 * sb) {
#pragma unroll
        for (int i = b + sb; i < b + 2 * sb && i < T; ++i, ++item) {
          if ((item & 3) != w) continue;
          v4d yv[4];
#pragma unroll
          for (int j = b; j < b + sb; ++j) {
            v4d u{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = j; k < b + sb; ++k)
              u = mma(ld_rm(A + ps::tix(i, k) * 256, c, q), ld_cm(A + ps::tix(k, j) * 256, c, q), u);
            yv[j - b] = u;
          }
#pragma unroll
          for (int j = b; j < b + sb; ++j) st_cm(A + ps::tix(i, j) * 256, c, q, yv[j - b]);
        }
      }
    }
    __syncthreads();
    // columns j of X_CA = -X_CC Y over Y
    {
      int item = 0;
#pragma unroll
      for (int b = 0; b + sb < T; b += 2 * sb) {
        const int e = (b + 2 * sb < T) ? b + 2 * sb : T;
#pragma unroll
        for (int j = b; j < b + sb; ++j, ++item) {
          if ((item & 3) != w) continue;
          v4d xv[4];
#pragma unroll
          for (int i = b + sb; i < e; ++i) {
            v4d u{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = b + sb; k <= i; ++k)
              u = mma(ld_rm(A + ps::tix(i, k) * 256, c, q), ld_cm(A + ps::tix(k, j) * 256, c, q), u);
            xv[i - b - sb] = -u;
          }
#pragma unroll
          for (int i = b + sb; i < e; ++i) st_cm(A + ps::tix(i, j) * 256, c, q, xv[i - b - sb]);
        }
      }
    }
    __syncthreads();
  }
  return *flag != 0;
}

__device__ inline double mat_at(const double *A, int r, int c) {   // lower element (r >= c)
  return A[ps::tix(r >> 4, c >> 4) * 256 + sw(r & 15, c & 15)];
}

// Block sum of one value per thread (256 threads); every thread gets the sum.
__device__ inline double block_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int tid = threadIdx.x;
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Problem index of block b in a grid of n: consecutive blocks are dealt to
// the 8 XCDs in turn, so XCD x = b % 8 is given the x-th contiguous range of
// problem indices (with pulsar-major problems, a few pulsars' data per L2).
__device__ inline int xcd_index(int b, int n) {
  const int x = b & 7, k = b >> 3, q = n >> 3, rm = n & 7;
  return x * q + (x < rm ? x : rm) + k;
}

// Block sum of three values per thread (256 threads) in one pass; red: 12
// doubles of LDS.  Every thread gets the three sums.
__device__ inline void block_sum3(double &a, double &b, double &c, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  const int tid = threadIdx.x;
  __syncthreads();
  if ((tid & 63) == 0) {
    red[tid >> 6] = a;
    red[4 + (tid >> 6)] = b;
    red[8 + (tid >> 6)] = c;
  }
  __syncthreads();
  a = (red[0] + red[1]) + (red[2] + red[3]);
  b = (red[4] + red[5]) + (red[6] + red[7]);
  c = (red[8] + red[9]) + (red[10] + red[11]);
}

template <int T>
constexpr size_t lds_bytes() {
  // tiles, six vectors of 16 T, 8 reduction slots, the flag (two doubles' room)
  // and 48 + 16 T doubles of scratch for the factorisation
  return (size_t)(ps::ntiles(T) * 256 + 6 * 16 * T + 8 + 2 + 48 + 16 * T) * sizeof(double);
}

// ---------------------------------------------------------------------------
// Forward per (pulsar, chain): transform, likelihood, Jacobian.
// ---------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(256, 2) void k_std_fwd(StdDev S, const double *__restrict__ x) {
  extern __shared__ double lds[];
  constexpr int pp = 16 * T, NE = ps::ntiles(T) * 256, NT = ps::ntiles(T);
  double *A = lds;
  double *vd = A + NE, *vz = vd + pp, *vt = vz + pp, *va = vt + pp, *vdi = va + pp, *lz = vdi + pp;
  double *red = lz + pp;
  int *flag = reinterpret_cast<int *>(red + 8);
  const int tid = threadIdx.x;
  const int pi = xcd_index(blockIdx.x, gridDim.x);
  const int I = pi / S.n_chains, c = pi - I * S.n_chains;
  const double *xc = x + (size_t)c * S.d;
  const double beta = S.beta ? S.beta[c] : 1.0;
  const int P = S.P;
  const double *s0 = S.s0 + (size_t)I * pp * pp;
  // A~ = beta S0~ + diag(1 / D~), lower tiles: thread tid holds element
  // (tid / 16, tid % 16) of every tile; all loads are issued before any use
  const int rr = tid >> 4, cc = tid & 15;
  double sv[NT];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    int TI = 0;
    while (ps::tix(TI + 1, 0) <= tt) ++TI;
    const int TJ = tt - ps::tix(TI, 0);
    sv[tt] = s0[(size_t)(16 * TI + rr) * pp + 16 * TJ + cc];
  }
  int bad = 0;
  double dr = 0.0;   // d~_r (unscaled) of this thread's row, kept for the likelihood
  // d of the data, or of the data minus the deterministic signal
  const double *dsrc = S.has_cw ? S.dbar + ((size_t)c * S.n_psr + I) * pp : S.dvec + (size_t)I * pp;
  for (int r = tid; r < pp; r += 256) {
    dr = (r < P) ? dsrc[r] : 0.0;
    vd[r] = beta * dr;
    // with split coefficients this is the combined MAP only (z = 0)
    vz[r] = (r < P && !S.split) ? xc[S.off_z + I * P + (P - 1 - r)] : 0.0;
    lz[r] = 0.0;
    // a CURN variance that is not positive and finite leaves phi_CURN not
    // positive definite
    double di = 1.0;
    if (r < P) {
      const double Dv = ps::curn_var(S, xc, I, P - 1 - r);
      if (!(Dv > 0.0 && isfinite(Dv))) bad = 1;
      di = 1.0 / Dv;
    }
    vdi[r] = di;
  }
  bad = __syncthreads_or(bad);
  if (tid == 0) *flag = bad ? 0 : 1;
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    int TI = 0;
    while (ps::tix(TI + 1, 0) <= tt) ++TI;
    const int TJ = tt - ps::tix(TI, 0);
    double v = beta * sv[tt];
    if (TI == TJ && rr == cc) v += vdi[16 * TI + rr];
    A[(tt << 8) + sw(rr, cc)] = v;
  }
  __syncthreads();
  // X = L~^-1 and L~ z~
  const bool ok = factor_invert<T, true>(A, tid, flag, red + 10, vz, lz);
  // t = X beta d~ by rows: row r of X over tiles K <= r / 16 (the diagonal
  // tiles hold zeros above), the tiles split by parity between threads r and
  // r + 128; va and vd hold the second thread's partial sums
  const int h = tid >> 7, r = tid & 127, R = r >> 4, r16 = r & 15;
  const bool live = r < pp;
  {
    double s = 0.0;
    if (live) {
#pragma unroll
      for (int K = 0; K < T; ++K) {
        if ((K & 1) != h || K > R) continue;
        const double *t = A + ps::tix(R, K) * 256;
#pragma unroll
        for (int k = 0; k < 16; ++k) s = fma(t[sw(r16, k)], vd[16 * K + k], s);
      }
      if (h == 1) va[r] = s;
    }
    __syncthreads();
    if (live && h == 0) vt[r] = s + va[r];
    __syncthreads();
  }
  // a~ = X^T (t + z~), a_hat~ = X^T t by columns: column r over tiles K >= r / 16
  const size_t vb = ((size_t)c * S.n_psr + I) * pp;
  double part_d = 0.0, part_v = 0.0, part_j = 0.0;
  {
    double sa = 0.0, sh = 0.0;
    if (live) {
#pragma unroll
      for (int K = 0; K < T; ++K) {
        if ((K & 1) != h || K < R) continue;
        const double *t = A + ps::tix(K, R) * 256;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const double xv = t[sw(k, r16)], tv = vt[16 * K + k];
          sa = fma(xv, tv + vz[16 * K + k], sa);
          sh = fma(xv, tv, sh);
        }
      }
      if (h == 1) {
        va[r] = sa;
        vd[r] = sh;
      }
    }
    __syncthreads();
    if (live && h == 0) {
      sa += va[r];
      sh += vd[r];
      S.ahat[vb + r] = sh;
      if (r < P) S.avec[vb + (P - 1 - r)] = sa;
      // beta (d - S0 a) in the reversed order: A~ a~ = L~ (t + z~) = beta d~ + L~ z~,
      // so beta S0~ a~ = beta d~ + L~ z~ - a~ / D~ and v1 = a~ / D~ - L~ z~
      const double v1 = sa * vdi[r] - lz[r];
      S.v1[vb + r] = v1;
      part_d = sa * dr;
      part_v = sa * v1;
      part_j = (r < P) ? log(A[ps::tix(R, R) * 256 + sw(r16, r16)]) : 0.0;
    }
  }
  block_sum3(part_d, part_v, part_j, red + 10);
  if (tid == 0) {
    // beta log L = beta (-dt N~^-1 dt / 2 + a.d - a.S0 a / 2 + c1), with
    // beta a.S0 a = beta a.d - a.v1
    const double *k2 = S.cconst + 2 * I;
    const double c0 = S.has_cw ? S.cbar[(size_t)c * S.n_psr + I] : k2[0];
    double *o = S.lik + ((size_t)c * S.n_psr + I) * 2;
    o[0] = beta * (k2[1] - 0.5 * c0) + 0.5 * beta * part_d + 0.5 * part_v;
    o[1] = part_j;
    S.flag1[(size_t)c * S.n_psr + I] = ok ? 0 : ps::kFlagNotPD;
  }
  // X for the adjoint (16-byte copies)
  double2 *xo = reinterpret_cast<double2 *>(S.xinv + ((size_t)c * S.n_psr + I) * NE);
  const double2 *xa = reinterpret_cast<const double2 *>(A);
  constexpr int N2 = NE / 2;
#pragma unroll
  for (int i = 0; i < (N2 + 255) / 256; ++i) {
    const int e = tid + 256 * i;
    if (e < N2) xo[e] = xa[e];
  }
}

// ---------------------------------------------------------------------------
// Prior per (frequency k < nf_gw, chain): phi_k = rho_k Gamma + diag kappa_.k.
// ---------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(256, 2) void k_std_prior_dense(StdDev S, const double *__restrict__ x) {
  extern __shared__ double lds[];
  constexpr int pp = 16 * T, NE = ps::ntiles(T) * 256, NT = ps::ntiles(T);
  double *A = lds;
  double *va = A + NE, *vb = va + 2 * pp, *vu = vb + 2 * pp, *red = vu + 2 * pp;
  int *flag = reinterpret_cast<int *>(red + 8);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, c16 = lane & 15, q = lane >> 4;
  const int c = blockIdx.x / S.nf_gw, k = blockIdx.x - c * S.nf_gw;
  const int n = S.n_psr;
  const double *xc = x + (size_t)c * S.d;
  // phi_k tiles: thread tid holds element (tid / 16, tid % 16) of every tile
  // and of every diagonal tile's diagonal; all loads are issued before any use
  const int rr = tid >> 4, cc = tid & 15;
  double gv[NT], dg[T];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) gv[tt] = S.gam_tiles[tt * 256 + rr * 16 + cc];
  const double rho = ps::spec_value(S, xc, 0, 0, k);
#pragma unroll
  for (int TI = 0; TI < T; ++TI) {
    const int r = 16 * TI + rr;
    dg[TI] = (rr != cc) ? 0.0 : (r < n) ? ((k < S.nf_rn) ? ps::spec_value(S, xc, 1, r, k) : 0.0) : 1.0;
  }
  for (int i = tid; i < pp; i += 256) {
    const double *av = S.avec + ((size_t)c * n + i) * S.pp;
    va[i] = (i < n) ? av[2 * k] : 0.0;
    va[pp + i] = (i < n) ? av[2 * k + 1] : 0.0;
  }
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    int TI = 0;
    while (ps::tix(TI + 1, 0) <= tt) ++TI;
    const int TJ = tt - ps::tix(TI, 0);
    A[(tt << 8) + sw(rr, cc)] = (TI == TJ) ? fma(rho, gv[tt], dg[TI]) : rho * gv[tt];
  }
  if (tid == 0) *flag = 1;
  __syncthreads();
  const bool ok = factor_invert<T, false>(A, tid, flag, red + 10, nullptr, nullptr);
  // y = X a (rows), then u = X^T y (columns), for sin and cos
  if (tid < 2 * pp) {
    const int i = tid % pp, h = tid / pp;
    double s = 0.0;
    for (int m = 0; m <= i; ++m) s = fma(mat_at(A, i, m), va[h * pp + m], s);
    vb[h * pp + i] = s;
  }
  __syncthreads();
  double part_q = 0.0, part_l = 0.0;
  if (tid < 2 * pp) {
    const int i = tid % pp, h = tid / pp;
    double s = 0.0, cn = 0.0;
    for (int m = i; m < pp; ++m) {
      const double xv = mat_at(A, m, i);
      s = fma(xv, vb[h * pp + m], s);
      cn = fma(xv, xv, cn);
    }
    vu[h * pp + i] = s;
    part_q = vb[h * pp + i] * vb[h * pp + i];
    if (h == 0 && i < n) {
      part_l = -2.0 * log(mat_at(A, i, i));
      va[i] = cn;                                // (phi^-1)_II; a (sin) is no longer read
    }
  }
  __syncthreads();
  // Gamma u (columns of the symmetric Gamma, coalesced) for the rho term,
  // eight loads in flight at a time
  double part_g = 0.0;
  if (tid < 2 * pp) {
    const int i = tid % pp, h = tid / pp;
    if (i < n) {
      double s = 0.0;
      int m = 0;
      for (; m + 8 <= n; m += 8) {
        double g[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) g[u] = S.gamma[(size_t)(m + u) * n + i];
#pragma unroll
        for (int u = 0; u < 8; ++u) s = fma(g[u], vu[h * pp + m + u], s);
      }
      for (; m < n; ++m) s = fma(S.gamma[(size_t)m * n + i], vu[h * pp + m], s);
      part_g = s * vu[h * pp + i];
    }
  }
  // tr(phi^-1 Gamma) = |X G|_F^2, G = chol(Gamma): tiles (X G)_IJ = sum_{K=J}^{I} X_IK G_KJ,
  // a task's G tiles loaded together before its products
  double part_t = 0.0;
  {
    int task = 0;
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
      for (int J = 0; J <= I; ++J, ++task) {
        if ((task & 3) != w) continue;
        v4d g[T];
#pragma unroll
        for (int K = J; K <= I; ++K) g[K - J] = ldg_cm(S.gch_tiles + ps::tix(K, J) * 256, c16, q);
        v4d r{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int K = J; K <= I; ++K) r = mma(ld_rm(A + ps::tix(I, K) * 256, c16, q), g[K - J], r);
        part_t += (r[0] * r[0] + r[1] * r[1]) + (r[2] * r[2] + r[3] * r[3]);
      }
  }
  const double quad = block_sum(part_q, red);
  const double ldet = block_sum(part_l, red);
  const double ugu = block_sum(part_g, red);
  const double tr = block_sum(part_t, red);
  if (tid < n) {
    const double u0 = vu[tid], u1 = vu[pp + tid];
    S.dkap_e[((size_t)c * n + tid) * S.ka + k] = 0.5 * (u0 * u0 + u1 * u1) - va[tid];
    double *v2 = S.v2 + ((size_t)c * n + tid) * S.pp;
    v2[2 * k] = -u0;
    v2[2 * k + 1] = -u1;
  }
  if (tid == 0) {
    double *o = S.quad_k + ((size_t)c * S.ka + k) * 2;
    o[0] = quad;
    o[1] = ldet;
    S.drho_e[(size_t)c * S.ka + k] = 0.5 * ugu - tr;
    S.flag2[(size_t)c * S.ka + k] = ok ? 0 : ps::kFlagNotPD;
  }
}

// ---------------------------------------------------------------------------
// Prior of the diagonal items: red-noise frequencies beyond the common process
// (phi_k = diag kappa_.k) and DM (diag kappa_dm): one thread per (chain, pulsar,
// item), items k in [nf_gw, ka) then the DM frequencies.  With split
// coefficients: the whole pulsar-noise set a_R, items k < nf_rn then DM.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_std_prior_diag(StdDev S, const double *__restrict__ x) {
  const int k0 = S.split ? 0 : S.nf_gw;
  const int nrn = S.split ? S.nf_rn : S.ka - S.nf_gw, per = nrn + S.kdm;
  const size_t total = (size_t)S.n_chains * S.n_psr * per;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int it = (int)(e % per);
  const size_t ci = e / per;
  const int I = (int)(ci % S.n_psr), c = (int)(ci / S.n_psr);
  const double *xc = x + (size_t)c * S.d;
  int k, col;
  double kap;
  if (it < nrn) {
    k = k0 + it;
    col = 2 * k;
    kap = ps::spec_value(S, xc, 1, I, k);
  } else {
    k = it - nrn;
    col = (S.split ? 2 * S.nf_rn : 2 * S.ka) + 2 * k;   // row in a_R, or in a
    kap = ps::spec_value(S, xc, 2, I, k);
  }
  const double *av = S.split ? S.ar + ci * S.ppr : S.avec + ci * S.pp;
  const double a0 = av[col], a1 = av[col + 1];
  const double ik = 1.0 / kap;
  const double u0 = a0 * ik, u1 = a1 * ik;
  double *v2 = S.split ? S.v2r + ci * S.ppr : S.v2 + ci * S.pp;
  v2[col] = -u0;
  v2[col + 1] = -u1;
  const double dk = 0.5 * (u0 * u0 + u1 * u1) - ik;
  if (it < nrn) S.dkap_e[((size_t)c * S.n_psr + I) * S.ka + k] = dk;
  else S.ddm_e[((size_t)c * S.n_psr + I) * S.kdm + k] = dk;
  double *o = S.diag_q + (((size_t)c * S.n_psr + I) * (S.ka + S.kdm) + (it < nrn ? k : S.ka + k)) * 2;
  o[0] = a0 * u0 + a1 * u1;
  o[1] = log(kap);
  S.flag3[((size_t)c * S.n_psr + I) * (S.ka + S.kdm) + (it < nrn ? k : S.ka + k)] =
      ((kap > 0.0) && isfinite(kap)) ? 0 : ps::kFlagNotPD;
}

// ---------------------------------------------------------------------------
// Adjoint per (pulsar, chain): dlogp/dz and dlogp/dD.
// ---------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(256) void k_std_bwd(StdDev S, const double *__restrict__ x,
                                                  double *__restrict__ grad) {
  extern __shared__ double lds[];
  constexpr int pp = 16 * T, NE = ps::ntiles(T) * 256;
  double *A = lds;
  double *vv = A + NE, *vz = vv + pp, *vw = vz + pp, *vh = vw + pp, *gd = vh + pp, *tmp = gd + pp;
  const int tid = threadIdx.x;
  const int pi = xcd_index(blockIdx.x, gridDim.x);
  const int I = pi / S.n_chains, c = pi - I * S.n_chains;
  const double *xc = x + (size_t)c * S.d;
  const int P = S.P;
  const size_t vb = ((size_t)c * S.n_psr + I) * pp;
  {
    const double2 *xi = reinterpret_cast<const double2 *>(S.xinv + ((size_t)c * S.n_psr + I) * NE);
    double2 *xa = reinterpret_cast<double2 *>(A);
    constexpr int N2 = NE / 2;
#pragma unroll
    for (int i = 0; i < (N2 + 255) / 256; ++i) {
      const int e = tid + 256 * i;
      if (e < N2) xa[e] = xi[e];
    }
  }
  for (int r = tid; r < pp; r += 256) {
    vv[r] = (r < P) ? S.v1[vb + r] + S.v2[vb + (P - 1 - r)] : 0.0;
    vz[r] = (r < P) ? xc[S.off_z + I * P + (P - 1 - r)] : 0.0;
    vh[r] = S.ahat[vb + r];
  }
  __syncthreads();
  const int h = tid >> 7, r = tid & 127, R = r >> 4, r16 = r & 15;
  // w~ = X v~ (dlogp/dz~) by rows, the tiles split by parity between threads r
  // and r + 128
  {
    double s = 0.0;
    if (r < pp) {
#pragma unroll
      for (int K = 0; K < T; ++K) {
        if ((K & 1) != h || K > R) continue;
        const double *t = A + ps::tix(R, K) * 256;
#pragma unroll
        for (int k = 0; k < 16; ++k) s = fma(t[sw(r16, k)], vv[16 * K + k], s);
      }
      if (h == 1) tmp[r] = s;
    }
    __syncthreads();
    if (r < pp && h == 0) {
      s += tmp[r];
      vw[r] = s;
      if (r < P) grad[(size_t)c * S.d + S.off_z + I * P + (P - 1 - r)] = s;
    }
    __syncthreads();
  }
  // per column r, over rows a >= r from the bottom: (Sigma v)~_r = sum_a X_ar w~_a,
  // Sigma~_rr = sum_a X_ar^2 and T_r = sum_a X_ar w~_a (sum_{b>a} X_br z~_b + X_ar z~_a / 2),
  // dlogp/dD~_r = (a_hat~_r (Sigma v)~_r + T_r + Sigma~_rr / 2) / D~_r^2.
  // Thread r + 128 takes the lower tiles K >= M, thread r the tiles R..M-1; the
  // upper part's suffix sums miss the lower part's s = sum_b X_br z~_b, which
  // adds s times the upper part's sum_a X_ar w~_a.  The lower part hands over
  // s and its own a_hat (Sigma v) + T + Sigma / 2.
  double sv = 0.0, ss = 0.0, tt = 0.0, suf = 0.0;
  if (r < P) {
    const int M = R + (T - R + 1) / 2;
#pragma unroll
    for (int K = T - 1; K >= 0; --K) {
      if (K < R || (h == 1) != (K >= M)) continue;
      const double *t = A + ps::tix(K, R) * 256;
#pragma unroll
      for (int k = 15; k >= 0; --k) {
        const double xv = t[sw(k, r16)], wv = vw[16 * K + k], zv = vz[16 * K + k];
        sv = fma(xv, wv, sv);
        ss = fma(xv, xv, ss);
        tt = fma(xv * wv, fma(0.5 * xv, zv, suf), tt);
        suf = fma(xv, zv, suf);
      }
    }
    if (h == 1) {
      tmp[r] = suf;
      tmp[pp + r] = fma(vh[r], sv, tt + 0.5 * ss);
      vv[r] = sv;   // v~ is no longer read
    }
  }
  __syncthreads();
  if (r < P && h == 0) {
    const double Dv = ps::curn_var(S, xc, I, P - 1 - r);
    gd[r] = (fma(sv, vh[r] + tmp[r], tt + 0.5 * ss) + tmp[pp + r]) / (Dv * Dv);
    if (S.has_cw) {
      // dlog p / d d_bar (original order): beta a (likelihood) + beta Sigma v (a_hat)
      const double beta = S.beta ? S.beta[c] : 1.0;
      const int j = P - 1 - r;
      S.gdbar[((size_t)c * S.n_psr + I) * P + j] = beta * (S.avec[vb + j] + (sv + vv[r]));
    }
  }
  __syncthreads();
  if (tid < S.ka) {
    const int r0 = P - 1 - 2 * tid, r1 = r0 - 1;
    S.dD_rn[((size_t)c * S.n_psr + I) * S.ka + tid] = gd[r0] + gd[r1];
  } else if (tid >= 64 && tid - 64 < S.kdm) {
    const int k = tid - 64, r0 = P - 1 - (2 * S.ka + 2 * k), r1 = r0 - 1;
    S.dD_dm[((size_t)c * S.n_psr + I) * S.kdm + k] = gd[r0] + gd[r1];
  }
}

// ---------------------------------------------------------------------------
// Deterministic CW in its own basis (Sec. IV.C), per (pulsar, chain).
// ---------------------------------------------------------------------------
__device__ inline pt::CwLane cw_lane(const double cst[pt::kCwRows]) {
  pt::CwLane L;
  L.K1 = cst[pt::kCwK1];
  L.inv32X = cst[pt::kCwInv32X];
  L.phi0 = cst[pt::kCwPhi0];
  L.a0 = cst[pt::kCwA0];
  L.ci = cst[pt::kCwCi];
  L.U = cst[pt::kCwU];
  L.V = cst[pt::kCwV];
  L.c2s = cst[pt::kCwC2s];
  L.s2s = cst[pt::kCwS2s];
  return L;
}

// The CW kernels take a pulsar and a block of kCwChains chains per workgroup,
// so that every table entry (the transform, S_D, Q_D) is loaded once for the
// block; thread t works on row t % 128 for the chains of half t / 128.
constexpr int kCwChains = 16;

// Constants of the block's chains for pulsar I (cst: kCwChains x kCwRows, LDS).
__device__ inline void cw_block_constants(const StdDev &S, const double *x, int I, int c0, int nc,
                                          double *cst) {
  const int tid = threadIdx.x;
  if (tid < nc) pt::cw_constants(x + (size_t)(c0 + tid) * S.d + S.off_cw, S.cw_pos + 3 * I,
                                 cst + tid * pt::kCwRows);
}

// Forward: the delay at the md sample times t_j = j T_D / md, its transform a_D
// (Eq. det_F_basis), then d_bar = d - S_D a_D (reversed order, zero-padded, as
// k_std_fwd reads it) and c_bar = c - 2 e_D^T a_D + a_D^T Q_D a_D.
__global__ __launch_bounds__(256) void k_std_cw_fwd(StdDev S, const double *__restrict__ x) {
  constexpr int H = kCwChains / 2;
  __shared__ double cst[kCwChains * pt::kCwRows];
  __shared__ double hs[kCwChains][ps::kMaxCwM];
  __shared__ double ad[kCwChains][ps::kMaxCw2];
  __shared__ double cpart[2][kCwChains][4];
  const int tid = threadIdx.x;
  const int nb = (S.n_chains + kCwChains - 1) / kCwChains;
  const int pi = xcd_index(blockIdx.x, gridDim.x);
  const int I = pi / nb, c0 = (pi - I * nb) * kCwChains;
  const int nc = min(kCwChains, S.n_chains - c0);
  const int K2 = 2 * S.kd, M = S.md, P = S.P, pp = S.pp;
  cw_block_constants(S, x, I, c0, nc, cst);
  __syncthreads();
  for (int e = tid; e < kCwChains * M; e += 256) {
    const int ch = e / M, j = e - ch * M;
    hs[ch][j] = ch < nc ? cw_lane(cst + ch * pt::kCwRows).delay((double)j * S.td / M).h : 0.0;
  }
  __syncthreads();
  const int row = tid & 127, h0 = (tid >> 7) * H;
  // a_D
  if (row < K2) {
    double acc[H];
#pragma unroll
    for (int u = 0; u < H; ++u) acc[u] = 0.0;
    const double *f = S.cw_dft + (size_t)row * M;
    for (int j = 0; j < M; ++j) {
      const double fv = f[j];
#pragma unroll
      for (int u = 0; u < H; ++u) acc[u] = fma(fv, hs[h0 + u][j], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < H; ++u) {
      ad[h0 + u][row] = acc[u];
      if (h0 + u < nc) S.cw_ad[((size_t)(c0 + h0 + u) * S.n_psr + I) * K2 + row] = acc[u];
    }
  }
  __syncthreads();
  // d_bar, row = the reversed index r
  if (row < pp) {
    double acc[H];
#pragma unroll
    for (int u = 0; u < H; ++u) acc[u] = 0.0;
    if (row < P) {
      const double *sd = S.cw_sd + ((size_t)I * P + (P - 1 - row)) * K2;
      for (int k = 0; k < K2; ++k) {
        const double sv = sd[k];
#pragma unroll
        for (int u = 0; u < H; ++u) acc[u] = fma(sv, ad[h0 + u][k], acc[u]);
      }
    }
    const double dv = row < P ? S.dvec[(size_t)I * pp + row] : 0.0;
#pragma unroll
    for (int u = 0; u < H; ++u)
      if (h0 + u < nc) S.dbar[((size_t)(c0 + h0 + u) * S.n_psr + I) * pp + row] = row < P ? dv - acc[u] : 0.0;
  }
  // c_bar: a_D^T (Q_D a_D - 2 e_D) per chain, summed over the rows of each wave
  {
    double part[H];
#pragma unroll
    for (int u = 0; u < H; ++u) part[u] = 0.0;
    if (row < K2) {
      double acc[H];
#pragma unroll
      for (int u = 0; u < H; ++u) acc[u] = 0.0;
      const double *qd = S.cw_qd + (size_t)I * K2 * K2 + row;   // Q_D is symmetric: column row
      for (int k = 0; k < K2; ++k) {
        const double qv = qd[(size_t)k * K2];
#pragma unroll
        for (int u = 0; u < H; ++u) acc[u] = fma(qv, ad[h0 + u][k], acc[u]);
      }
      const double ev = S.cw_ed[(size_t)I * K2 + row];
#pragma unroll
      for (int u = 0; u < H; ++u) part[u] = ad[h0 + u][row] * (acc[u] - 2.0 * ev);
    }
#pragma unroll
    for (int u = 0; u < H; ++u) {
      double v = part[u];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if ((tid & 63) == 0) cpart[tid >> 7][h0 + u][(tid >> 6) & 1] = v;
    }
    __syncthreads();
    if (tid < nc) {
      const int hh = tid / H;
      const double v = cpart[hh][tid][0] + cpart[hh][tid][1];
      S.cbar[(size_t)(c0 + tid) * S.n_psr + I] = S.cconst[2 * I] + v;
    }
  }
}

// dlog p / d a_D = -S_D^T g + beta (e_D - Q_D a_D) with g = dlog p / d d_bar
// (k_std_bwd), then g_h = (transform)^T dlog p / d a_D at the sample times and
// the pulsar's part of dlog p / d theta_cw = sum_j g_h,j dh_j / d theta.
__global__ __launch_bounds__(256) void k_std_cw_bwd(StdDev S, const double *__restrict__ x) {
  constexpr int H = kCwChains / 2;
  __shared__ double cst[kCwChains * pt::kCwRows];
  __shared__ double gb[kCwChains][ps::kMaxCwM];   // dlog p / d d_bar, later g_h
  __shared__ double ad[kCwChains][ps::kMaxCw2];
  __shared__ double ga[kCwChains][ps::kMaxCw2];
  const int tid = threadIdx.x;
  const int nb = (S.n_chains + kCwChains - 1) / kCwChains;
  const int pi = xcd_index(blockIdx.x, gridDim.x);
  const int I = pi / nb, c0 = (pi - I * nb) * kCwChains;
  const int nc = min(kCwChains, S.n_chains - c0);
  const int K2 = 2 * S.kd, M = S.md, P = S.P;
  cw_block_constants(S, x, I, c0, nc, cst);
  for (int e = tid; e < kCwChains * P; e += 256) {
    const int ch = e / P, j = e - ch * P;
    gb[ch][j] = ch < nc ? S.gdbar[((size_t)(c0 + ch) * S.n_psr + I) * P + j] : 0.0;
  }
  for (int e = tid; e < kCwChains * K2; e += 256) {
    const int ch = e / K2, k = e - ch * K2;
    ad[ch][k] = ch < nc ? S.cw_ad[((size_t)(c0 + ch) * S.n_psr + I) * K2 + k] : 0.0;
  }
  __syncthreads();
  const int row = tid & 127, h0 = (tid >> 7) * H;
  if (row < K2) {
    double s1[H], s2[H];
#pragma unroll
    for (int u = 0; u < H; ++u) s1[u] = s2[u] = 0.0;
    const double *sd = S.cw_sd + (size_t)I * P * K2 + row;
    for (int j = 0; j < P; ++j) {
      const double sv = sd[(size_t)j * K2];
#pragma unroll
      for (int u = 0; u < H; ++u) s1[u] = fma(sv, gb[h0 + u][j], s1[u]);
    }
    const double *qd = S.cw_qd + (size_t)I * K2 * K2 + row;   // Q_D is symmetric: column row
    for (int k = 0; k < K2; ++k) {
      const double qv = qd[(size_t)k * K2];
#pragma unroll
      for (int u = 0; u < H; ++u) s2[u] = fma(qv, ad[h0 + u][k], s2[u]);
    }
    const double ev = S.cw_ed[(size_t)I * K2 + row];
#pragma unroll
    for (int u = 0; u < H; ++u) {
      const int ch = h0 + u;
      const double beta = (ch < nc && S.beta) ? S.beta[c0 + ch] : 1.0;
      ga[ch][row] = beta * (ev - s2[u]) - s1[u];
    }
  }
  __syncthreads();
  // g_h at the sample times (up to 129 of them: rows 0..127, then 128)
  for (int j = row; j < M; j += 128) {
    double acc[H];
#pragma unroll
    for (int u = 0; u < H; ++u) acc[u] = 0.0;
    for (int k = 0; k < K2; ++k) {
      const double fv = S.cw_dft[(size_t)k * M + j];
#pragma unroll
      for (int u = 0; u < H; ++u) acc[u] = fma(fv, ga[h0 + u][k], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < H; ++u) gb[h0 + u][j] = acc[u];
  }
  __syncthreads();
  // the waveform's derivative: chain tid / 16, samples tid % 16 + 16 i, then
  // the 16 lanes of the chain summed in order
  {
    const int ch = tid >> 4, l16 = tid & 15;
    double out[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (ch < nc) {
      const double *cc = cst + ch * pt::kCwRows;
      const pt::CwLane L = cw_lane(cc);
      double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (int j = l16; j < M; j += 16) L.adjoint(L.delay((double)j * S.td / M), gb[ch][j], acc);
      // the sky pair through the antenna derivatives, ln 10 for the log10 parameters
      out[0] = -(cc[pt::kCwDfpC] * acc[0] + cc[pt::kCwDfxC] * acc[1]);
      out[1] = -(cc[pt::kCwDfpP] * acc[0] + cc[pt::kCwDfxP] * acc[1]);
      out[2] = ps::kLn10 * acc[2];
      out[3] = ps::kLn10 * acc[3];
      out[4] = acc[4];
      out[5] = acc[5];
      out[6] = acc[6];
      out[7] = ps::kLn10 * acc[7];
    }
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      double t = out[v];
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
      out[v] = t;
    }
    if (ch < nc && l16 == 0) {
      double *o = S.dcw + ((size_t)(c0 + ch) * S.n_psr + I) * 8;
#pragma unroll
      for (int v = 0; v < 8; ++v) o[v] = out[v];
    }
  }
}

// ---------------------------------------------------------------------------
// Assembly per chain: log p, the hyper-parameter gradient and the status.
// One workgroup of kFinT threads per chain.  Loops over the chain's entries
// issue their loads together; every sum is taken in a fixed order (per-lane
// strides, then fixed shuffle trees and wave partials in wave order).
// ---------------------------------------------------------------------------
constexpr int kFinT = 1024, kFinW = kFinT / 64;

// Sum over the 32 lanes of a half-wave (fixed tree).
__device__ inline double half_sum(double v) {
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(kFinT) void k_std_finalize(StdDev S, const double *x,
                                                         double *__restrict__ logp, double *__restrict__ grad,
                                                         int32_t *__restrict__ status, ps::StdKick kick,
                                                         int has_kick) {
  __shared__ double red[kFinW];
  __shared__ int sb[kFinW][1];
  __shared__ double drho_tot[ps::kMaxRhoK];
  __shared__ double cwp[kFinW][8];
  const int tid = threadIdx.x, c = blockIdx.x, wv = tid >> 6;
  const int n = S.n_psr;
  const double *xc = x + (size_t)c * S.d;
  double *gc = grad + (size_t)c * S.d;
  // Phase one: every load of the input checks, the flags and the log p parts
  // is issued before any is used (fixed batches per thread with clamped
  // in-range addresses, selected when consumed; a remainder loop beyond the
  // batch), then they are combined in the same per-thread order.
  int bad_box = 0, bad_in = 0;
  // the box on theta (two entries a thread per pass)
  constexpr int BB = 2;
  double bxv[BB], blo[BB], bhi[BB];
  {
    const int lt = max(S.n_theta - 1, 0);
#pragma unroll
    for (int u = 0; u < BB; ++u) {
      const int i = min(tid + u * kFinT, lt);
      bxv[u] = S.n_theta > 0 ? xc[i] : 0.0;
      blo[u] = S.n_theta > 0 ? S.prior_lo[i] : 0.0;
      bhi[u] = S.n_theta > 0 ? S.prior_hi[i] : 0.0;
    }
  }
  // finiteness of z (eight entries a thread per pass)
  constexpr int BZ = 8;
  double zv[BZ];
#pragma unroll
  for (int u = 0; u < BZ; ++u) zv[u] = xc[min(S.n_theta + tid + u * kFinT, S.d - 1)];
  // factorisation flags and the log p parts of the pulsars (one a thread)
  int fl = 0;
  double lp = 0.0;
  int f1 = 0, fs = 0, f2 = 0;
  double l0 = 0.0, l1 = 0.0, q0 = 0.0, q1 = 0.0;
  {
    const int i = min(tid, n - 1);
    f1 = S.flag1[(size_t)c * n + i];
    const double *o = S.lik + ((size_t)c * n + i) * 2;
    l0 = o[0];
    l1 = o[1];
  }
  // diagonal prior items: red-only frequencies and DM, or with split
  // coefficients the whole pulsar-noise set (eight a thread per pass; the
  // planner admits no data set without frequencies, so nd >= 1)
  const int kt = S.ka + S.kdm, nd = n * kt;
  constexpr int BD = 8;
  int f3[BD];
  double d0[BD], d1[BD];
#pragma unroll
  for (int u = 0; u < BD; ++u) {
    const int i = min(tid + u * kFinT, nd - 1);
    f3[u] = S.flag3[(size_t)c * nd + i];
    const double *o = S.diag_q + ((size_t)c * nd + i) * 2;
    d0[u] = o[0];
    d1[u] = o[1];
  }
  // the loads that exist only with split coefficients or a common process
  // come last (a wait their branches may take leaves the rest in flight)
  if (S.split) fs = S.flag_s[(size_t)c * 2 * n + min(tid, 2 * n - 1)];
  if (S.nf_gw > 0) {
    const int k = min(tid, S.nf_gw - 1);
    f2 = S.flag2[(size_t)c * S.ka + k];
    const double *oq = S.quad_k + ((size_t)c * S.ka + k) * 2;
    q0 = oq[0];
    q1 = oq[1];
  }
  // d/drho_k in total: the explicit prior part plus the transform's part
  // summed over the pulsars (with split coefficients the pulsars' rho parts
  // are drho_p, and dD_rn holds their kappa parts only), 32 lanes per
  // frequency, pulsars h, h + 32, ... in order
  const int kr = tid >> 5, hr = tid & 31;
  static_assert(4 * 32 >= PTAFS_MAX_PSR, "four passes of 32 lanes cover the pulsars");
  double rv[4], re = 0.0;
  if (S.nf_gw > 0) {
    const double *src = S.split ? S.drho_p : S.dD_rn;
    const int kc = min(kr, S.nf_gw - 1);
#pragma unroll
    for (int m = 0; m < 4; ++m) rv[m] = src[((size_t)c * n + min(hr + 32 * m, n - 1)) * S.ka + kc];
    re = S.drho_e[(size_t)c * S.ka + kc];
  }
  // the box and z checks
#pragma unroll
  for (int u = 0; u < BB; ++u)
    if (tid + u * kFinT < S.n_theta && !(bxv[u] >= blo[u] && bxv[u] <= bhi[u])) bad_box = 1;
  for (int i = tid + BB * kFinT; i < S.n_theta; i += kFinT) {
    const double v = xc[i];
    if (!(v >= S.prior_lo[i] && v <= S.prior_hi[i])) bad_box = 1;
  }
#pragma unroll
  for (int u = 0; u < BZ; ++u)
    if (S.n_theta + tid + u * kFinT < S.d && !isfinite(zv[u])) bad_in = 1;
  for (int i0 = S.n_theta + BZ * kFinT + tid; i0 < S.d; i0 += 4 * kFinT) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = (i0 + u * kFinT < S.d) ? xc[i0 + u * kFinT] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (!isfinite(v[u])) bad_in = 1;
  }
  // the CW must not coalesce before the last sample time of its basis
  int bad_cw = 0;
  if (S.has_cw && tid == 0) {
    const double *tc = xc + S.off_cw;
    const double M = exp(ps::kLn10 * tc[2]) * pt::kTsun, w0 = pt::kPi * exp(ps::kLn10 * tc[3]);
    const double K1 = 256.0 / 5.0 * exp((5.0 / 3.0) * log(M * w0)) * w0;
    const double y = K1 * ((double)(S.md - 1) * S.td / S.md);
    bad_cw = !(y < 1.0);
  }
  if (tid < n) {
    fl |= f1;
    lp += l0 + l1;
  }
  if (S.split && tid < 2 * n) fl |= fs;
  if (tid < S.nf_gw) {
    fl |= f2;
    lp += -0.5 * q0 - (n * ps::kLn2Pi + q1);
  }
#pragma unroll
  for (int u = 0; u < BD; ++u) {
    const int i = tid + u * kFinT;
    const int kk = i % kt;
    if (i < nd && (S.split ? (kk < S.nf_rn || kk >= S.ka) : kk >= S.nf_gw)) {
      fl |= f3[u];
      lp += -0.5 * d0[u] - (ps::kLn2Pi + d1[u]);
    }
  }
  for (int i = tid + BD * kFinT; i < nd; i += kFinT) {
    const int kk = i % kt;
    if (S.split ? (kk < S.nf_rn || kk >= S.ka) : kk >= S.nf_gw) {
      fl |= S.flag3[(size_t)c * nd + i];
      const double *o = S.diag_q + ((size_t)c * nd + i) * 2;
      lp += -0.5 * o[0] - (ps::kLn2Pi + o[1]);
    }
  }
  // (d/drho_k: the pulsars' parts summed per frequency)
  if (S.nf_gw > 0) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (kr < S.nf_gw && hr + 32 * m < n) s += rv[m];
    s = half_sum(s);
    if (hr == 0 && kr < S.nf_gw) drho_tot[kr] = re + s;
  }
  // the CW parameters' parts, pulsars in order: lane groups of 8 per wave,
  // then the waves in order
  if (S.has_cw) {
    const int v = tid & 7, I0 = tid >> 3;
    double s = 0.0;
    for (int I = I0; I < n; I += kFinT / 8) s += S.dcw[((size_t)c * n + I) * 8 + v];
#pragma unroll
    for (int o = 8; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
    if ((tid & 63) < 8) cwp[wv][v] = s;
  }
  __syncthreads();
  // hyper-parameter gradient, 32 lanes per process instance (the common
  // process, then red noise and DM per pulsar), lane k taking frequency k;
  // a lane group's instances it = g, g + 32, ... take their loads together
  {
    constexpr int RB = (1 + 2 * PTAFS_MAX_PSR + kFinT / 32 - 1) / (kFinT / 32);
    const int k = tid & 31, g = tid >> 5, n_it = 1 + 2 * n;
    const int kl = min(k, PTAFS_MAX_HARM - 1);
    double dd[RB], sa[RB], sb2[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int it = g + (kFinT / 32) * r;
      int proc, I, off, K;
      if (it == 0) { proc = 0; I = 0; off = S.off_gw; K = S.nf_gw; }
      else if (it <= n) { proc = 1; I = it - 1; off = S.off_rn + I * S.w_rn; K = S.nf_rn; }
      else { proc = 2; I = min(it - 1 - n, n - 1); off = S.off_dm + I * S.w_dm; K = S.kdm; }
      const bool ok = it < n_it && k < K;
      const int kc = ok ? k : 0;
      dd[r] = 0.0;
      if (ok && proc == 0) dd[r] = drho_tot[kc];
      else if (ok && proc == 1)
        dd[r] = S.dkap_e[((size_t)c * n + I) * S.ka + kc] + S.dD_rn[((size_t)c * n + I) * S.ka + kc];
      else if (ok)
        dd[r] = S.ddm_e[((size_t)c * n + I) * S.kdm + kc] + S.dD_dm[((size_t)c * n + I) * S.kdm + kc];
      // the spectrum's inputs: theta_k (free spectrum) or (log10 A, gamma)
      const int o1 = min(ok ? off + (S.free_spec ? kc : 0) : 0, S.d - 1);
      sa[r] = xc[o1];
      sb2[r] = S.free_spec ? 0.0 : xc[min(o1 + 1, S.d - 1)];
    }
    const double lf = S.lnfy[kl];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int it = g + (kFinT / 32) * r;
      if (it >= n_it) break;
      int off, K;
      if (it == 0) { off = S.off_gw; K = S.nf_gw; }
      else if (it <= n) { off = S.off_rn + (it - 1) * S.w_rn; K = S.nf_rn; }
      else { off = S.off_dm + (it - 1 - n) * S.w_dm; K = S.kdm; }
      if (K == 0) continue;
      double v = 0.0;
      if (k < K) {
        // the spectrum as spec_value forms it
        const double sv = S.free_spec ? exp(ps::kLn10 * sa[r])
                                      : exp(2.0 * ps::kLn10 * sa[r] - sb2[r] * lf + S.pl_c);
        v = sv * dd[r];
      }
      if (S.free_spec) {
        if (k < K) gc[off + k] = ps::kLn10 * v;
      } else {
        const double ga = half_sum(2.0 * ps::kLn10 * v);
        const double gg = half_sum(k < K ? -lf * v : 0.0);
        if (k == 0) {
          gc[off] = ga;
          gc[off + 1] = gg;
        }
      }
    }
  }
  if (S.has_cw && tid < 8) {
    double g = 0.0;
    for (int w = 0; w < kFinW; ++w) g += cwp[w][tid];
    gc[S.off_cw + tid] = g;
  }
  // reduce the flags and log p
  {
    double v = lp;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int bb = __any(bad_box), bi = __any(bad_in), bf = __any(fl != 0), bc = __any(bad_cw);
    if ((tid & 63) == 0) {
      red[wv] = v;
      sb[wv][0] = bb | (bi << 1) | (bf << 2) | (bc << 3);
    }
    __syncthreads();
    // lane i of every wave takes wave i's values, then a second wave
    // reduction (a fixed tree; two registers instead of all waves' values)
    const int ln = tid & 63;
    double t = ln < kFinW ? red[ln] : 0.0;
    int f = ln < kFinW ? sb[ln][0] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      t += __shfl_xor(t, o, 64);
      f |= __shfl_xor(f, o, 64);
    }
    lp = t;
    bad_box = f & 1;
    bad_in = (f >> 1) & 1;
    fl = (f >> 2) & 1;
    bad_cw = (f >> 3) & 1;
  }
  lp += S.prior_const;
  // output finiteness (the theta entries written above by other threads)
  // and, inside a trajectory, the kick's operands: loaded together, nine
  // entries a thread (every coordinate up to 9216), the rest after
  constexpr int BK = 9;
  double gv[BK], pv[BK], xv[BK], mv[BK];
  double *xw = kick.x + (size_t)c * S.d, *pw = kick.p + (size_t)c * S.d;
#pragma unroll
  for (int u = 0; u < BK; ++u) {
    const int i = min(tid + u * kFinT, S.d - 1);
    gv[u] = gc[i];
    pv[u] = has_kick ? pw[i] : 0.0;
    xv[u] = has_kick ? xw[i] : 0.0;
    mv[u] = (has_kick && kick.inv_mass) ? kick.inv_mass[i] : 1.0;
  }
  int nonfin = !isfinite(lp);
#pragma unroll
  for (int u = 0; u < BK; ++u)
    if (tid + u * kFinT < S.d && !isfinite(gv[u])) nonfin = 1;
  for (int i0 = BK * kFinT + tid; i0 < S.d; i0 += 4 * kFinT) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = (i0 + u * kFinT < S.d) ? gc[i0 + u * kFinT] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (!isfinite(v[u])) nonfin = 1;
  }
  nonfin = __syncthreads_or(nonfin);
  int st = PTAFS_ST_OK;
  if (bad_box) st = PTAFS_ST_PRIOR;
  else if (bad_in) st = PTAFS_ST_NONFINITE;
  else if (bad_cw) st = PTAFS_ST_CW;
  else if (fl) st = PTAFS_ST_NOTPD;
  else if (nonfin) st = PTAFS_ST_NONFINITE;
  if (st != PTAFS_ST_OK)
    for (int i = tid; i < S.d; i += kFinT) gc[i] = 0.0;
  if (tid == 0) {
    logp[c] = (st == PTAFS_ST_OK) ? lp : -INFINITY;
    status[c] = st;
  }
  if (has_kick) {
    // inside a trajectory: kick and drift of this chain (the gradient is
    // zero when the status is nonzero)
    if (tid == 0 && kick.n_invalid && st != PTAFS_ST_OK) kick.n_invalid[c] += 1;
#pragma unroll
    for (int u = 0; u < BK; ++u) {
      const int i = tid + u * kFinT;
      if (i < S.d) {
        const double pi = pv[u] + kick.eps * (st != PTAFS_ST_OK ? 0.0 : gv[u]);
        pw[i] = pi;
        xw[i] = xv[u] + kick.eps * mv[u] * pi;
      }
    }
    if (S.d <= BK * kFinT) return;
    __syncthreads();   // every entry of the gradient row is final
    for (int i0 = BK * kFinT + tid; i0 < S.d; i0 += 2 * kFinT) {
      double rg[2], rp[2], rx[2], rm[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int i = i0 + u * kFinT;
        const bool in = i < S.d;
        rg[u] = in ? gc[i] : 0.0;
        rp[u] = in ? pw[i] : 0.0;
        rx[u] = in ? xw[i] : 0.0;
        rm[u] = (in && kick.inv_mass) ? kick.inv_mass[i] : 1.0;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int i = i0 + u * kFinT;
        if (i < S.d) {
          const double pi = rp[u] + kick.eps * rg[u];
          pw[i] = pi;
          xw[i] = rx[u] + kick.eps * rm[u] * pi;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Split coefficients (App. C, Eqs. separated_post, split_map_a,
// split_standardizing_transform).  The common process and the pulsar noise
// get coefficient sets of their own on the same basis, a = E_G a_G + E_R a_R,
//   a_G = a_hat_G + L_G z_G,  L_G L_G^T = (beta S0_GG + diag rho^-1)^-1,
//   a_R = a_hat_R + L_R z_R,  L_R L_R^T = (beta S0_RR + diag phi_R^-1)^-1,
// and the MAP pair of the joint system is the CURN MAP of the combined
// coefficients split in proportion to the prior variances:
// a_hat_G = rho / D a_hat, a_hat_R = phi_R / D a_hat, D = rho + phi_R (a
// shared row's likelihood sees only the sum, and for a fixed sum the two
// independent Gaussian priors are largest at that split).  k_std_fwd with
// z = 0 gives a_hat; k_split_fac factorises each set; k_split_comb forms
// a_G, a_R, a and the likelihood.  The prior keeps the HD correlations on
// a_G (rho_k Gamma per frequency, Gamma^-1 once per data set) and is
// diagonal on a_R.
// ---------------------------------------------------------------------------

// Set b of pulsar I, chain c: A~ = beta S0_b~ + diag(1 / v~) factorised and
// inverted as the CURN precision is; L_b z_b = X^T z~ and ln det L_b.
template <int T>
__global__ __launch_bounds__(256, 2) void k_split_fac(StdDev S, const double *__restrict__ x, int b) {
  extern __shared__ double lds[];
  constexpr int pp = 16 * T, NE = ps::ntiles(T) * 256, NT = ps::ntiles(T);
  double *A = lds;
  double *vz = A + NE, *va = vz + pp, *red = va + pp;
  int *flag = reinterpret_cast<int *>(red + 8);
  const int tid = threadIdx.x;
  const int pi = xcd_index(blockIdx.x, gridDim.x);
  const int I = pi / S.n_chains, c = pi - I * S.n_chains;
  const double *xc = x + (size_t)c * S.d;
  const double beta = S.beta ? S.beta[c] : 1.0;
  const int PB = b ? S.PR : S.PG;
  const double *s0 = (b ? S.s0r : S.s0g) + (size_t)I * pp * pp;
  const int rr = tid >> 4, cc = tid & 15;
  double sv[NT];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    int TI = 0;
    while (ps::tix(TI + 1, 0) <= tt) ++TI;
    const int TJ = tt - ps::tix(TI, 0);
    sv[tt] = s0[(size_t)(16 * TI + rr) * pp + 16 * TJ + cc];
  }
  int bad = 0;
  for (int r = tid; r < pp; r += 256) {
    vz[r] = (r < PB) ? xc[S.off_z + I * S.pz + (b ? S.PG : 0) + (PB - 1 - r)] : 0.0;
    double di = 1.0;
    if (r < PB) {
      const double v = ps::split_var(S, xc, I, b, PB - 1 - r);
      if (!(v > 0.0 && isfinite(v))) bad = 1;
      di = 1.0 / v;
    }
    va[r] = di;
  }
  bad = __syncthreads_or(bad);
  if (tid == 0) *flag = bad ? 0 : 1;
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    int TI = 0;
    while (ps::tix(TI + 1, 0) <= tt) ++TI;
    const int TJ = tt - ps::tix(TI, 0);
    double v = beta * sv[tt];
    if (TI == TJ && rr == cc) v += va[16 * TI + rr];
    A[(tt << 8) + sw(rr, cc)] = v;
  }
  __syncthreads();
  const bool ok = factor_invert<T, false>(A, tid, flag, red + 10, nullptr, nullptr);
  // X^T z~ by columns (column r over tiles K >= r / 16), the tiles split by
  // parity between threads r and r + 128
  const int h = tid >> 7, r = tid & 127, R = r >> 4, r16 = r & 15;
  const size_t ci = (size_t)c * S.n_psr + I;
  double part_j = 0.0;
  {
    double sa = 0.0;
    if (r < pp) {
#pragma unroll
      for (int K = 0; K < T; ++K) {
        if ((K & 1) != h || K < R) continue;
        const double *t = A + ps::tix(K, R) * 256;
#pragma unroll
        for (int k = 0; k < 16; ++k) sa = fma(t[sw(k, r16)], vz[16 * K + k], sa);
      }
      if (h == 1) va[r] = sa;
    }
    __syncthreads();
    if (r < PB && h == 0) {
      (b ? S.lzr : S.lzg)[ci * pp + (PB - 1 - r)] = sa + va[r];
      part_j = log(A[ps::tix(R, R) * 256 + sw(r16, r16)]);
    }
  }
  part_j = block_sum(part_j, red);
  if (tid == 0) {
    S.jac_s[ci * 2 + b] = part_j;
    S.flag_s[ci * 2 + b] = ok ? 0 : ps::kFlagNotPD;
  }
  double2 *xo = reinterpret_cast<double2 *>((b ? S.xr : S.xg) + ci * NE);
  const double2 *xa = reinterpret_cast<const double2 *>(A);
  constexpr int N2 = NE / 2;
#pragma unroll
  for (int i = 0; i < (N2 + 255) / 256; ++i) {
    const int e = tid + 256 * i;
    if (e < N2) xo[e] = xa[e];
  }
}

// Per (pulsar, chain): a_G, a_R and a from the combined MAP (avec, written by
// k_std_fwd with z = 0) and the sets' L_b z_b; v1 = beta (d - S0 a) and
// beta log L(a) with S0 a formed directly (a is no longer a_hat + L z of one
// factorisation); the Jacobian ln det L_G + ln det L_R.
__global__ __launch_bounds__(256) void k_split_comb(StdDev S, const double *__restrict__ x) {
  __shared__ double av[16 * ps::kMaxTiles];
  __shared__ double red[12];
  const int tid = threadIdx.x;
  const int pi = xcd_index(blockIdx.x, gridDim.x);
  const int I = pi / S.n_chains, c = pi - I * S.n_chains;
  const double *xc = x + (size_t)c * S.d;
  const double beta = S.beta ? S.beta[c] : 1.0;
  const int P = S.P, pp = S.pp, j = tid;
  const size_t ci = (size_t)c * S.n_psr + I, vb = ci * pp;
  double a = 0.0, d = 0.0;
  if (j < P) {
    const double ah = S.avec[vb + j];
    const double id = 1.0 / ps::curn_var(S, xc, I, j);
    if (j < S.PG) {
      const double g = ps::spec_value(S, xc, 0, I, j >> 1) * id * ah + S.lzg[ci * S.ppg + j];
      S.ag[ci * S.ppg + j] = g;
      a += g;
    }
    if (j < 2 * S.nf_rn || j >= 2 * S.ka) {
      const int jr = j < 2 * S.nf_rn ? j : j - 2 * S.ka + 2 * S.nf_rn;
      const double g = ps::split_var(S, xc, I, 1, jr) * id * ah + S.lzr[ci * S.ppr + jr];
      S.ar[ci * S.ppr + jr] = g;
      a += g;
    }
    av[j] = a;
    d = (S.has_cw ? S.dbar + vb : S.dvec + (size_t)I * pp)[P - 1 - j];
  }
  __syncthreads();
  double part_d = 0.0, part_q = 0.0, part_n = 0.0;
  if (j < P) {
    // (S0 a)_j down column P - 1 - j of the symmetric S0~ (coalesced over j)
    const double *s0 = S.s0 + (size_t)I * pp * pp + (P - 1 - j);
    double s = 0.0;
    for (int m = 0; m < P; ++m) s = fma(s0[(size_t)(P - 1 - m) * pp], av[m], s);
    S.avec[vb + j] = a;
    S.v1[vb + (P - 1 - j)] = beta * (d - s);
    part_d = a * d;
    part_q = a * s;
  }
  block_sum3(part_d, part_q, part_n, red);
  if (tid == 0) {
    const double *k2 = S.cconst + 2 * I;
    const double c0 = S.has_cw ? S.cbar[ci] : k2[0];
    double *o = S.lik + ci * 2;
    o[0] = beta * ((k2[1] - 0.5 * c0) + (part_d - 0.5 * part_q));
    o[1] = S.jac_s[ci * 2] + S.jac_s[ci * 2 + 1];
  }
}

// Prior of the common set per (frequency k < nf_gw, chain): a_G,k ~ N(0,
// rho_k Gamma) for sin and cos; u = Gamma^-1 a, the quadratic form a^T u /
// rho_k, ln det = N_p ln rho_k + ln det Gamma, -u / rho_k into v2 and the
// explicit derivative (a_s^T u_s + a_c^T u_c) / (2 rho_k^2) - N_p / rho_k.
__global__ __launch_bounds__(256) void k_split_prior_g(StdDev S, const double *__restrict__ x) {
  __shared__ double as[2][16 * ps::kMaxTiles];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int c = blockIdx.x / S.nf_gw, k = blockIdx.x - c * S.nf_gw;
  const int n = S.n_psr;
  const double *xc = x + (size_t)c * S.d;
  const double rho = ps::spec_value(S, xc, 0, 0, k);
  const int i = tid & 127, h = tid >> 7;
  if (i < n) as[h][i] = S.ag[((size_t)c * n + i) * S.ppg + 2 * k + h];
  __syncthreads();
  double part = 0.0;
  if (i < n) {
    double u = 0.0;
    for (int m = 0; m < n; ++m) u = fma(S.gam_inv[(size_t)m * n + i], as[h][m], u);
    part = as[h][i] * u;
    S.v2[((size_t)c * n + i) * S.pp + 2 * k + h] = -u / rho;
  }
  const double q = block_sum(part, red);
  if (tid == 0) {
    double *o = S.quad_k + ((size_t)c * S.ka + k) * 2;
    o[0] = q / rho;
    o[1] = n * log(rho) + S.ldet_gamma;
    S.drho_e[(size_t)c * S.ka + k] = 0.5 * q / (rho * rho) - n / rho;
    S.flag2[(size_t)c * S.ka + k] = (rho > 0.0 && isfinite(rho)) ? 0 : ps::kFlagNotPD;
  }
}

// Adjoint of set b per (pulsar, chain): g = dlog p / d a_b (the likelihood's
// beta (d - S0 a) on the set's rows plus its prior term), dlog p / dz~ = X g~,
// and the set's transform part of dlog p / dv_r, (T_r + Sigma~_rr / 2) / v_r^2
// with T_r and Sigma~_rr as in k_std_bwd (no MAP term: the sets' MAP comes
// from the combined problem).
template <int T>
__global__ __launch_bounds__(256) void k_split_bwd(StdDev S, const double *__restrict__ x,
                                                    double *__restrict__ grad, int b) {
  extern __shared__ double lds[];
  constexpr int pp = 16 * T, NE = ps::ntiles(T) * 256;
  double *A = lds;
  double *vv = A + NE, *vz = vv + pp, *vw = vz + pp, *tmp = vw + pp;
  const int tid = threadIdx.x;
  const int pi = xcd_index(blockIdx.x, gridDim.x);
  const int I = pi / S.n_chains, c = pi - I * S.n_chains;
  const double *xc = x + (size_t)c * S.d;
  const int PB = b ? S.PR : S.PG, P = S.P;
  const size_t ci = (size_t)c * S.n_psr + I;
  {
    const double2 *xi = reinterpret_cast<const double2 *>((b ? S.xr : S.xg) + ci * NE);
    double2 *xa = reinterpret_cast<double2 *>(A);
    constexpr int N2 = NE / 2;
#pragma unroll
    for (int i = 0; i < (N2 + 255) / 256; ++i) {
      const int e = tid + 256 * i;
      if (e < N2) xa[e] = xi[e];
    }
  }
  const int zo = S.off_z + I * S.pz + (b ? S.PG : 0);
  for (int r = tid; r < pp; r += 256) {
    double g = 0.0, z = 0.0;
    if (r < PB) {
      const int j = PB - 1 - r, jc = ps::split_row(S, b, j);
      g = S.v1[ci * S.pp + (P - 1 - jc)] + (b ? S.v2r[ci * pp + j] : S.v2[ci * S.pp + j]);
      (b ? S.gar : S.gag)[ci * pp + j] = g;
      z = xc[zo + j];
    }
    vv[r] = g;
    vz[r] = z;
  }
  __syncthreads();
  const int h = tid >> 7, r = tid & 127, R = r >> 4, r16 = r & 15;
  {
    double s = 0.0;
    if (r < pp) {
#pragma unroll
      for (int K = 0; K < T; ++K) {
        if ((K & 1) != h || K > R) continue;
        const double *t = A + ps::tix(R, K) * 256;
#pragma unroll
        for (int k = 0; k < 16; ++k) s = fma(t[sw(r16, k)], vv[16 * K + k], s);
      }
      if (h == 1) tmp[r] = s;
    }
    __syncthreads();
    if (r < pp && h == 0) {
      s += tmp[r];
      vw[r] = s;
      if (r < PB) grad[(size_t)c * S.d + zo + (PB - 1 - r)] = s;
    }
    __syncthreads();
  }
  // column r from the bottom: Sigma~_rr = sum_a X_ar^2 and
  // T_r = sum_a X_ar w~_a (sum_{b>a} X_br z~_b + X_ar z~_a / 2)
  if (tid < PB) {
    double ss = 0.0, tt = 0.0, suf = 0.0;
    for (int K = T - 1; K >= R; --K) {
      const double *t = A + ps::tix(K, R) * 256;
#pragma unroll
      for (int k = 15; k >= 0; --k) {
        const double xv = t[sw(k, r16)], wv = vw[16 * K + k], zv = vz[16 * K + k];
        ss = fma(xv, xv, ss);
        tt = fma(xv * wv, fma(0.5 * xv, zv, suf), tt);
        suf = fma(xv, zv, suf);
      }
    }
    const int j = PB - 1 - r;
    const double v = ps::split_var(S, xc, I, b, j);
    (b ? S.ddr : S.ddg)[ci * pp + j] = (tt + 0.5 * ss) / (v * v);
  }
}

// Adjoint of the combined MAP per (pulsar, chain) and the chain rule to the
// prior variances.  Upstream of a_hat: g_j = (rho_j g_G,j + phi_j g_R,j) / D_j
// (rho_j = 0 off the common rows, phi_j = 0 off the pulsar-noise rows);
// dlog p / dD_j = a_hat_j (Sigma g)_j / D_j^2 through a_hat, and with
// q_j = a_hat_j / D_j^2 the proportional split adds
//   d/drho_j: phi_j q_j (g_G,j - g_R,j),   d/dphi_j: rho_j q_j (g_R,j - g_G,j);
// each set adds its own transform part.  Rows summed in sin/cos pairs: the
// pulsar's part of dlog p / drho_k (drho_p) and dlog p / dkappa (dD_rn, dD_dm).
// With a CW, dlog p / d d_bar = beta (a + Sigma g).
template <int T>
__global__ __launch_bounds__(256) void k_split_bwd_c(StdDev S, const double *__restrict__ x) {
  extern __shared__ double lds[];
  constexpr int pp = 16 * T, NE = ps::ntiles(T) * 256;
  double *A = lds;
  double *vv = A + NE, *vw = vv + pp, *tmp = vw + pp, *prt = tmp + pp, *pkt = prt + pp;
  const int tid = threadIdx.x;
  const int pi = xcd_index(blockIdx.x, gridDim.x);
  const int I = pi / S.n_chains, c = pi - I * S.n_chains;
  const double *xc = x + (size_t)c * S.d;
  const int P = S.P;
  const size_t ci = (size_t)c * S.n_psr + I, vb = ci * pp;
  {
    const double2 *xi = reinterpret_cast<const double2 *>(S.xinv + ci * NE);
    double2 *xa = reinterpret_cast<double2 *>(A);
    constexpr int N2 = NE / 2;
#pragma unroll
    for (int i = 0; i < (N2 + 255) / 256; ++i) {
      const int e = tid + 256 * i;
      if (e < N2) xa[e] = xi[e];
    }
  }
  // this thread's row j (original order), kept for the chain rule
  double rho = 0.0, phi = 0.0, gG = 0.0, gR = 0.0, D = 1.0;
  int jr = -1;
  if (tid < P) {
    const int j = tid;
    D = ps::curn_var(S, xc, I, j);
    if (j < S.PG) {
      rho = ps::spec_value(S, xc, 0, I, j >> 1);
      gG = S.gag[ci * S.ppg + j];
    }
    if (j < 2 * S.nf_rn || j >= 2 * S.ka) {
      jr = j < 2 * S.nf_rn ? j : j - 2 * S.ka + 2 * S.nf_rn;
      phi = ps::split_var(S, xc, I, 1, jr);
      gR = S.gar[ci * S.ppr + jr];
    }
  }
  for (int r = tid; r < pp; r += 256) vv[r] = 0.0;
  __syncthreads();
  if (tid < P) vv[P - 1 - tid] = (rho * gG + phi * gR) / D;
  __syncthreads();
  const int h = tid >> 7, r = tid & 127, R = r >> 4, r16 = r & 15;
  {
    double s = 0.0;
    if (r < pp) {
#pragma unroll
      for (int K = 0; K < T; ++K) {
        if ((K & 1) != h || K > R) continue;
        const double *t = A + ps::tix(R, K) * 256;
#pragma unroll
        for (int k = 0; k < 16; ++k) s = fma(t[sw(r16, k)], vv[16 * K + k], s);
      }
      if (h == 1) tmp[r] = s;
    }
    __syncthreads();
    if (r < pp && h == 0) vw[r] = s + tmp[r];
    __syncthreads();
  }
  // (Sigma g)~_r = sum_{a >= r} X_ar w~_a, one thread per column
  if (tid < P) {
    const int rc = P - 1 - tid, Rc = rc >> 4, rc16 = rc & 15;
    double sg = 0.0;
    for (int K = Rc; K < T; ++K) {
      const double *t = A + ps::tix(K, Rc) * 256;
#pragma unroll
      for (int k = 0; k < 16; ++k) sg = fma(t[sw(k, rc16)], vw[16 * K + k], sg);
    }
    const int j = tid;
    const double ah = S.ahat[vb + rc];
    const double q = ah / (D * D);
    const double dD = sg * q;
    prt[j] = (j < S.PG) ? dD + phi * q * (gG - gR) + S.ddg[ci * S.ppg + j] : 0.0;
    pkt[j] = (jr >= 0) ? dD + rho * q * (gR - gG) + S.ddr[ci * S.ppr + jr] : 0.0;
    if (S.has_cw) {
      const double beta = S.beta ? S.beta[c] : 1.0;
      S.gdbar[ci * P + j] = beta * (S.avec[vb + j] + sg);
    }
  }
  __syncthreads();
  if (tid < S.nf_gw) {
    S.drho_p[ci * S.ka + tid] = prt[2 * tid] + prt[2 * tid + 1];
  } else if (tid >= 64 && tid - 64 < S.nf_rn) {
    const int k = tid - 64;
    S.dD_rn[ci * S.ka + k] = pkt[2 * k] + pkt[2 * k + 1];
  } else if (tid >= 128 && tid - 128 < S.kdm) {
    const int k = tid - 128;
    S.dD_dm[ci * S.kdm + k] = pkt[2 * S.ka + 2 * k] + pkt[2 * S.ka + 2 * k + 1];
  }
}

template <int T>
hipError_t set_attr_t() {
  hipError_t e = hipFuncSetAttribute((const void *)k_std_fwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds_bytes<T>());
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_std_prior_dense<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds_bytes<T>());
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_split_fac<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds_bytes<T>());
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_split_bwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds_bytes<T>());
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_split_bwd_c<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds_bytes<T>());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)k_std_bwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds_bytes<T>());
}

}  // namespace

namespace psk {

hipError_t init_attributes() {
  hipError_t e;
  if ((e = set_attr_t<1>()) != hipSuccess) return e;
  if ((e = set_attr_t<2>()) != hipSuccess) return e;
  if ((e = set_attr_t<3>()) != hipSuccess) return e;
  if ((e = set_attr_t<4>()) != hipSuccess) return e;
  if ((e = set_attr_t<5>()) != hipSuccess) return e;
  if ((e = set_attr_t<6>()) != hipSuccess) return e;
  if ((e = set_attr_t<7>()) != hipSuccess) return e;
  return set_attr_t<8>();
}

#define PS_DISPATCH(TT, KERNEL, GRID, ...)                                                          \
  switch (TT) {                                                                                     \
    case 1: hipLaunchKernelGGL(KERNEL<1>, dim3(GRID), dim3(256), lds_bytes<1>(), s, __VA_ARGS__); break; \
    case 2: hipLaunchKernelGGL(KERNEL<2>, dim3(GRID), dim3(256), lds_bytes<2>(), s, __VA_ARGS__); break; \
    case 3: hipLaunchKernelGGL(KERNEL<3>, dim3(GRID), dim3(256), lds_bytes<3>(), s, __VA_ARGS__); break; \
    case 4: hipLaunchKernelGGL(KERNEL<4>, dim3(GRID), dim3(256), lds_bytes<4>(), s, __VA_ARGS__); break; \
    case 5: hipLaunchKernelGGL(KERNEL<5>, dim3(GRID), dim3(256), lds_bytes<5>(), s, __VA_ARGS__); break; \
    case 6: hipLaunchKernelGGL(KERNEL<6>, dim3(GRID), dim3(256), lds_bytes<6>(), s, __VA_ARGS__); break; \
    case 7: hipLaunchKernelGGL(KERNEL<7>, dim3(GRID), dim3(256), lds_bytes<7>(), s, __VA_ARGS__); break; \
    case 8: hipLaunchKernelGGL(KERNEL<8>, dim3(GRID), dim3(256), lds_bytes<8>(), s, __VA_ARGS__); break; \
    default: return hipErrorInvalidValue;                                                           \
  }

hipError_t launch_std_cw_fwd(const StdDev &S, const double *x, hipStream_t s) {
  const int grid = ((S.n_chains + kCwChains - 1) / kCwChains) * S.n_psr;
  if (grid == 0 || !S.has_cw) return hipSuccess;
  hipLaunchKernelGGL(k_std_cw_fwd, dim3(grid), dim3(256), 0, s, S, x);
  return hipGetLastError();
}

hipError_t launch_std_cw_bwd(const StdDev &S, const double *x, hipStream_t s) {
  const int grid = ((S.n_chains + kCwChains - 1) / kCwChains) * S.n_psr;
  if (grid == 0 || !S.has_cw) return hipSuccess;
  hipLaunchKernelGGL(k_std_cw_bwd, dim3(grid), dim3(256), 0, s, S, x);
  return hipGetLastError();
}

hipError_t launch_std_fwd(const StdDev &S, const double *x, hipStream_t s) {
  const int grid = S.n_chains * S.n_psr;
  if (grid == 0) return hipSuccess;
  PS_DISPATCH(S.tp, k_std_fwd, grid, S, x);
  return hipGetLastError();
}

hipError_t launch_std_prior(const StdDev &S, const double *x, hipStream_t s) {
  if (S.nf_gw > 0) {
    const int grid = S.n_chains * S.nf_gw;
    if (S.split) hipLaunchKernelGGL(k_split_prior_g, dim3(grid), dim3(256), 0, s, S, x);
    else PS_DISPATCH(S.tg, k_std_prior_dense, grid, S, x);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const size_t items =
      (size_t)S.n_chains * S.n_psr * ((S.split ? S.nf_rn : S.ka - S.nf_gw) + S.kdm);
  if (items) hipLaunchKernelGGL(k_std_prior_diag, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, S, x);
  return hipGetLastError();
}

hipError_t launch_std_bwd(const StdDev &S, const double *x, double *grad, hipStream_t s) {
  const int grid = S.n_chains * S.n_psr;
  if (grid == 0) return hipSuccess;
  PS_DISPATCH(S.tp, k_std_bwd, grid, S, x, grad);
  return hipGetLastError();
}

// Split coefficients: the two sets' factorisations, then a_G, a_R, a and the
// likelihood (after launch_std_fwd, which gives the combined MAP).
hipError_t launch_split_fwd(const StdDev &S, const double *x, hipStream_t s) {
  const int grid = S.n_chains * S.n_psr;
  if (grid == 0 || !S.split) return hipSuccess;
  PS_DISPATCH(S.tpg, k_split_fac, grid, S, x, 0);
  PS_DISPATCH(S.tpr, k_split_fac, grid, S, x, 1);
  hipLaunchKernelGGL(k_split_comb, dim3(grid), dim3(256), 0, s, S, x);
  return hipGetLastError();
}

// Split coefficients: the sets' adjoints, then the combined MAP's and the
// chain rule (in place of launch_std_bwd).
hipError_t launch_split_bwd(const StdDev &S, const double *x, double *grad, hipStream_t s) {
  const int grid = S.n_chains * S.n_psr;
  if (grid == 0 || !S.split) return hipSuccess;
  PS_DISPATCH(S.tpg, k_split_bwd, grid, S, x, grad, 0);
  PS_DISPATCH(S.tpr, k_split_bwd, grid, S, x, grad, 1);
  PS_DISPATCH(S.tp, k_split_bwd_c, grid, S, x);
  return hipGetLastError();
}

hipError_t launch_std_finalize(const StdDev &S, const double *x, double *logp, double *grad,
                               int32_t *status, hipStream_t s, const ps::StdKick *kick) {
  if (S.n_chains == 0) return hipSuccess;
  const ps::StdKick k = kick ? *kick : ps::StdKick{};
  hipLaunchKernelGGL(k_std_finalize, dim3(S.n_chains), dim3(kFinT), 0, s, S, x, logp, grad, status, k,
                     kick ? 1 : 0);
  return hipGetLastError();
}

}  // namespace psk
