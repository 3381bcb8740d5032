// Dense per-frequency prior covariance for the frequencies that carry the
// common process (k <= nf_gw), for the arrays the matrix-core kernels of
// k_cholt do not take: the factorisation and whitening transform (forward)
// beyond 112 pulsars, the adjoint of both (backward) beyond 80.  Up to 112
// pulsars the adjoint reads k_cholt's tile-major factor; beyond, the packed
// factor of the forward here.
//
// Forward (Sec. IV.A, Eqs. HD, prior_cov; Sec. II.B, Eq.
// standardizing_transform with mu = 0):
//   phi_k = rho_k Gamma + diag(kappa_.k) = L D L^T (unit lower L),
//   C_k = L D^(1/2) (the Cholesky factor),  a_.k,{sin,cos} = C_k z_.k,{sin,cos}
// One workgroup of ceil(n/64) waves per (frequency, chain); thread i owns
// pulsar row i.  Left-looking: at step j every row forms its unscaled entry
//   Y_ij = phi_ij - sum_{m<j} Y_im L_jm      (Y_im = L_im D_m, Y_jj = D_j)
// from its own row (registers) and the scaled row j of L broadcast from LDS.
// Scaling by 1/D_j is deferred one step, so every step needs one barrier.
//
// Backward, with abar = d log L / d a from the TOA pass and v_c = C^T abar_c:
//   dz_c = v_c - z_c
//   dlogp/dkappa_I = w_I^T P w_I,     w_I = C^-1 e_I
//   dlogp/drho     = sum_I m_I^T P m_I,  m_I = C^-1 g_I  (g_I: column I of chol Gamma)
//   P = Phi(sum_c v_c z_c^T)  (strict lower triangle plus half the diagonal;
//   the adjoint of phi = C C^T)
// One wave per (frequency, chain): thread l solves the two triangular systems
// for columns l and l + 64 by forward substitution, reading the rows of C as
// uniform (scalar) loads; the quadratic forms with the semiseparable P are
// O(n) prefix sums.
#include "common.h"

namespace {

using pt::Dev;
using pt::pk;

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NW>
__device__ inline void group_sync() {
  if constexpr (NW == 1) wave_sync();
  else __syncthreads();
}

// ---------------------------------------------------------------------------
// Forward: grid (nf_gw, c_pad), block 64 * NW.
// ---------------------------------------------------------------------------
template <int NMAX>
__global__ __launch_bounds__(NMAX > 64 ? 128 : 64) void k_chol_fwd(Dev D, const double *__restrict__ x) {
  constexpr int NW = NMAX > 64 ? 2 : 1;
  constexpr int LS = NMAX + 2;                 // row stride of the broadcast copy of L
  __shared__ __align__(16) double Ls[NMAX * LS];
  __shared__ double colb[2][NMAX];             // unscaled column of the previous step
  __shared__ double piv[NMAX];                 // D_j
  __shared__ double rsd[NMAX];                 // 1 / sqrt(D_j)
  __shared__ double zr[2][NMAX];               // z_{sin,cos} / sqrt(D)
  __shared__ double pos[NMAX][3];              // pulsar unit vectors
  const int k0 = blockIdx.x, c = blockIdx.y;
  const int i = threadIdx.x;
  const int w = i >> 6;
  const int n = D.n_psr;
  const size_t cp = D.c_pad;
  const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
  const bool row = i < n;
  double *out_s = D.coef_rn + ((size_t)i * D.rows_rn + rs) * cp + c;
  double *out_c = D.coef_rn + ((size_t)i * D.rows_rn + rc) * cp + c;
  // padding chains and chains outside the prior box carry zero coefficients
  // (the prior box is checked here, so nothing is read from k_spec_fwd)
  int32_t *flag = D.flag_dense + (size_t)c * D.nf_gw + k0;
  const double *xc = x + (size_t)(c < D.n_chains ? c : 0) * D.d;
  bool ok = c < D.n_chains;
  if (ok)
    for (int t = i; t < D.n_theta; t += 64 * NW) {
      const double v = xc[t];
      if (!(v >= D.prior_lo[t] && v <= D.prior_hi[t])) ok = false;
    }
  if (!__syncthreads_and(ok)) {
    if (row) {
      *out_s = 0.0;
      *out_c = 0.0;
    }
    if (i == 0) *flag = 0;
    return;
  }
  const double rho = pt::powerlaw_k(D, k0, xc[D.off_gw], xc[D.off_gw + 1]);
  double kap = 0.0;
  if (row && k0 < D.nf_rn) kap = pt::powerlaw_k(D, k0, xc[D.off_rn + 2 * i], xc[D.off_rn + 2 * i + 1]);
  double pi0 = 0.0, pi1 = 0.0, pi2 = 0.0;
  if (row) {
    pi0 = D.pos[3 * i];
    pi1 = D.pos[3 * i + 1];
    pi2 = D.pos[3 * i + 2];
    pos[i][0] = pi0;
    pos[i][1] = pi1;
    pos[i][2] = pi2;
  }
  group_sync<NW>();

  double Y[NMAX];
  bool pd = true;
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    Y[j] = 0.0;
    if (j >= n || !pd) continue;                // same value in every thread
    double rp = 0.0, ljm1 = 0.0;
    if (j > 0) {
      const double p = piv[j - 1];
      pd = (p > 0.0) && isfinite(p);
      rp = 1.0 / p;
      ljm1 = colb[(j - 1) & 1][j] * rp;        // L_{j,j-1}
    }
    if (!pd) continue;
    // rows below 64 own no entry right of column 63
    const bool act = !(NW == 2 && j >= 64 && w == 0);
    if (act) {
      if (j > 0 && row) Ls[i * LS + (j - 1)] = (i > j - 1) ? Y[j - 1] * rp : 0.0;
      // phi_ij = rho Gamma_ij + delta_ij kappa_i, with the Hellings-Downs
      // Gamma (Eq. HD) formed from the pulsar directions
      double s = 0.0;
      if (row) {
        double g = 1.0;
        if (i != j) {
          const double beta = 0.5 * (1.0 - (pi0 * pos[j][0] + pi1 * pos[j][1] + pi2 * pos[j][2]));
          const double blb = beta > 0.0 ? beta * log(beta) : 0.0;
          g = 1.5 * blb - 0.25 * beta + 0.5;
        }
        s = rho * g + (i == j ? kap : 0.0);
      }
      const double *Lj = Ls + j * LS;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
      for (int m = 0; m + 1 < j; m += 4) {
        a0 += Y[m] * Lj[m];
        if (m + 1 < j - 1) a1 += Y[m + 1] * Lj[m + 1];
        if (m + 2 < j - 1) a2 += Y[m + 2] * Lj[m + 2];
        if (m + 3 < j - 1) a3 += Y[m + 3] * Lj[m + 3];
      }
      if (j > 0) a0 += Y[j - 1] * ljm1;
      s -= (a0 + a1) + (a2 + a3);
      Y[j] = (i >= j) ? s : 0.0;
      if (row) colb[j & 1][i] = s;             // threads past n (and NMAX) own no row
      if (i == j) piv[j] = s;
    }
    group_sync<NW>();
  }
  if (pd) {
    const double p = piv[n - 1];
    pd = (p > 0.0) && isfinite(p);
  }
  if (!pd) {
    if (row) {
      *out_s = 0.0;
      *out_c = 0.0;
    }
    if (i == 0) *flag = pt::kFlagNotPD;
    return;
  }
  if (i == 0) *flag = 0;
  if (row) {
    const double r = 1.0 / sqrt(piv[i]);
    const double *zc = xc + D.off_z + (size_t)i * 2 * D.ka + 2 * k0;
    rsd[i] = r;
    zr[0][i] = r * zc[0];
    zr[1][i] = r * zc[1];
  }
  group_sync<NW>();
  // a_i = sum_m C_im z_m with C_im = Y_im / sqrt(D_m)
  double as0 = 0.0, as1 = 0.0, ac0 = 0.0, ac1 = 0.0;
#pragma unroll
  for (int m = 0; m < NMAX; m += 2) {
    if (m < n) {
      as0 += Y[m] * zr[0][m];
      ac0 += Y[m] * zr[1][m];
    }
    if (m + 1 < n) {
      as1 += Y[m + 1] * zr[0][m + 1];
      ac1 += Y[m + 1] * zr[1][m + 1];
    }
  }
  if (row) {
    *out_s = as0 + as1;
    *out_c = ac0 + ac1;
  }
  // keep C (packed row-major) for the adjoint: rows through LDS, then coalesced
#pragma unroll
  for (int m = 0; m < NMAX; ++m)
    if (row && m < n && m <= i) Ls[i * LS + m] = Y[m] * rsd[m];
  group_sync<NW>();
  const int np = (n * (n + 1)) / 2;
  double *dst = D.lstore + ((size_t)c * D.nf_gw + k0) * np;
  for (int r = 0; r < n; ++r)
    for (int m = i; m <= r; m += 64 * NW) dst[pk(r, m)] = Ls[r * LS + m];
}

// ---------------------------------------------------------------------------
// Backward: grid (nf_gw, n_chains), one wave; thread l owns columns l and
// l + 64 (the second only has rows >= 64).
// ---------------------------------------------------------------------------
// sum_c sum_i x_i v_ci (sum_{j<i} z_cj x_j + z_ci x_i / 2) over rows R0..n-1
// Element (i, m), m <= i, of a stored factor: tile-major (lower 16x16 tiles,
// row-major inside) up to kTileFwdMaxNT tiles, packed row-major beyond.
template <int NMAX>
__device__ inline double cel(const double *__restrict__ Cp, int i, int m) {
  if constexpr (NMAX <= 16 * pt::kTileFwdMaxNT) {
    const int I = i >> 4, J = m >> 4;
    return Cp[(I * (I + 1) / 2 + J) * 256 + (i & 15) * 16 + (m & 15)];
  } else {
    return Cp[pk(i, m)];
  }
}

template <int NMAX, int R0>
__device__ inline double quad_form(const double (&X)[NMAX - R0], const double (*vz)[4], int n) {
  double ss = 0.0, sc = 0.0, q = 0.0;
#pragma unroll
  for (int i = R0; i < NMAX; ++i) {
    if (i < n) {
      const double xi = X[i - R0];
      const double vs = vz[i][0], vc = vz[i][1], zs = vz[i][2], zc = vz[i][3];
      q += xi * (vs * (ss + 0.5 * zs * xi) + vc * (sc + 0.5 * zc * xi));
      ss += zs * xi;
      sc += zc * xi;
    }
  }
  return q;
}

// X = C^-1 b for a column whose rows above R0 vanish, by forward
// substitution; the rows of C are uniform across the wave (scalar loads).
// b = e_I, or column I of chol(Gamma) when GCOL.
template <int NMAX, int R0, bool GCOL>
__device__ inline void forward_subst(double (&X)[NMAX - R0], const double *__restrict__ Cp,
                                     const double *__restrict__ gch, int I, int n) {
#pragma unroll
  for (int i = R0; i < NMAX; ++i) {
    if (i < n) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
      for (int m = R0; m < i; m += 4) {
        a0 += cel<NMAX>(Cp, i, m) * X[m - R0];
        if (m + 1 < i) a1 += cel<NMAX>(Cp, i, m + 1) * X[m + 1 - R0];
        if (m + 2 < i) a2 += cel<NMAX>(Cp, i, m + 2) * X[m + 2 - R0];
        if (m + 3 < i) a3 += cel<NMAX>(Cp, i, m + 3) * X[m + 3 - R0];
      }
      double b;
      if constexpr (GCOL) b = (I <= i && I < n) ? gch[pk(i, I)] : 0.0;
      else b = (i == I) ? 1.0 : 0.0;
      X[i - R0] = (b - ((a0 + a1) + (a2 + a3))) / cel<NMAX>(Cp, i, i);
    } else {
      X[i - R0] = 0.0;
    }
  }
}

template <int NMAX>
__global__ __launch_bounds__(64) void k_chol_bwd(Dev D, const double *__restrict__ x,
                                                 double *__restrict__ grad,
                                                 const double *__restrict__ lst,
                                                 const double *__restrict__ gch,
                                                 const double *__restrict__ bar) {
  constexpr bool TWO = NMAX > 64;
  constexpr int R1 = TWO ? 64 : NMAX - 1;      // first row of the second column set
  __shared__ double vz[NMAX][4];               // v_sin, v_cos, z_sin, z_cos
  const int k0 = blockIdx.x, c = blockIdx.y;
  const int l = threadIdx.x;
  const int n = D.n_psr;
  const int kmax = max(D.ka, D.nf_dm);
  const size_t cp = D.c_pad;
  const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
  const int K2 = 2 * D.ka;
  const int I1 = l, I2 = l + 64;
  const bool c1 = I1 < n, c2 = TWO && I2 < n;
  const double *xc = x + (size_t)c * D.d;
  double *gz = grad + (size_t)c * D.d + D.off_z + 2 * k0;
  double *drn = pt::drn_at(D, c, 0, k0);   // pulsar I at drn[2 ka I]
  const size_t dI = 2 * (size_t)D.ka;
  double *dth = D.dth_k + ((size_t)c * D.ka + k0) * 2;
  const int fl0 = D.flag_k[(size_t)c * kmax + k0] | D.flag_dense[(size_t)c * D.nf_gw + k0];
  int32_t *fout = D.flag_out + (size_t)c * (kmax + pt::kSpecSeg) + k0;
  if (D.st_pre[c] != 0 || fl0 != 0) {
    if (l == 0) *fout = 0;
    for (int I = l; I < n; I += 64) {
      gz[(size_t)I * K2] = 0.0;
      gz[(size_t)I * K2 + 1] = 0.0;
      drn[dI * I] = 0.0;
      drn[dI * I + 1] = 0.0;
    }
    if (l == 0) {
      dth[0] = 0.0;
      dth[1] = 0.0;
    }
    return;
  }
  const double *Cp = lst + ((size_t)c * D.nf_gw + k0) * pt::chol_store_doubles(n);

  // v_c = C^T abar_c for both owned columns
  double v1s = 0.0, v1c = 0.0, v2s = 0.0, v2c = 0.0;
#pragma unroll 4
  for (int m = 0; m < n; ++m) {
    const double as = bar[((size_t)m * D.rows_rn + rs) * cp + c];
    const double ac = bar[((size_t)m * D.rows_rn + rc) * cp + c];
    const double e1 = (c1 && I1 <= m) ? cel<NMAX>(Cp, m, I1) : 0.0;
    v1s += e1 * as;
    v1c += e1 * ac;
    if constexpr (TWO) {
      const double e2 = (c2 && I2 <= m) ? cel<NMAX>(Cp, m, I2) : 0.0;
      v2s += e2 * as;
      v2c += e2 * ac;
    }
  }
  double z1s = 0.0, z1c = 0.0, z2s = 0.0, z2c = 0.0;
  if (c1) {
    z1s = xc[D.off_z + (size_t)I1 * K2 + 2 * k0];
    z1c = xc[D.off_z + (size_t)I1 * K2 + 2 * k0 + 1];
  }
  if (c2) {
    z2s = xc[D.off_z + (size_t)I2 * K2 + 2 * k0];
    z2c = xc[D.off_z + (size_t)I2 * K2 + 2 * k0 + 1];
  }
  if (I1 < NMAX) {
    vz[I1][0] = v1s;
    vz[I1][1] = v1c;
    vz[I1][2] = z1s;
    vz[I1][3] = z1c;
  }
  if (TWO && I2 < NMAX) {
    vz[I2][0] = v2s;
    vz[I2][1] = v2c;
    vz[I2][2] = z2s;
    vz[I2][3] = z2c;
  }
  wave_sync();

  double X1[NMAX];
  double X2[NMAX - R1];
  forward_subst<NMAX, 0, false>(X1, Cp, gch, I1, n);
  const double dk1 = quad_form<NMAX, 0>(X1, vz, n);
  double dk2 = 0.0;
  if constexpr (TWO) {
    forward_subst<NMAX, R1, false>(X2, Cp, gch, I2, n);
    dk2 = quad_form<NMAX, R1>(X2, vz, n);
  }
  forward_subst<NMAX, 0, true>(X1, Cp, gch, I1, n);
  double dr = c1 ? quad_form<NMAX, 0>(X1, vz, n) : 0.0;
  if constexpr (TWO) {
    forward_subst<NMAX, R1, true>(X2, Cp, gch, I2, n);
    if (c2) dr += quad_form<NMAX, R1>(X2, vz, n);
  }

  // d/drho: sum over columns in a fixed order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dr += __shfl_xor(dr, o, 64);
  const double lnfy = D.lnfy[k0];
  bool fin = true;
  auto put = [&](int I, double vs, double vc, double zs, double zc, double dk) {
    const double g0 = vs - zs, g1 = vc - zc;
    gz[(size_t)I * K2] = g0;
    gz[(size_t)I * K2 + 1] = g1;
    const double kap = (k0 < D.nf_rn)
                           ? pt::powerlaw_k(D, k0, xc[D.off_rn + 2 * I], xc[D.off_rn + 2 * I + 1])
                           : 0.0;
    const double d0 = dk * kap * 2.0 * pt::kLn10, d1 = dk * kap * (-lnfy);
    drn[dI * I] = d0;
    drn[dI * I + 1] = d1;
    fin = fin && isfinite(g0) && isfinite(g1) && isfinite(d0) && isfinite(d1);
  };
  if (c1) put(I1, v1s, v1c, z1s, z1c, dk1);
  if (c2) put(I2, v2s, v2c, z2s, z2c, dk2);
  const int nbad = __popcll(__ballot(!fin));
  if (l == 0) {
    const double rho = pt::powerlaw_k(D, k0, xc[D.off_gw], xc[D.off_gw + 1]);
    dth[0] = dr * rho * 2.0 * pt::kLn10;
    dth[1] = dr * rho * (-lnfy);
    *fout = (nbad || !isfinite(dth[0]) || !isfinite(dth[1])) ? pt::kFlagOutNonfinite : 0;
  }
}

template <int NMAX>
hipError_t launch_fwd_t(const Dev &D, const double *x, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_fwd<NMAX>, dim3(D.nf_gw, D.c_pad), dim3(NMAX > 64 ? 128 : 64), 0, s, D, x);
  return hipGetLastError();
}

template <int NMAX>
hipError_t launch_bwd_t(const Dev &D, const double *x, double *grad, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_bwd<NMAX>, dim3(D.nf_gw, D.n_chains), dim3(64), 0, s, D, x, grad,
                     (const double *)D.lstore, D.gchol, (const double *)D.bar_rn);
  return hipGetLastError();
}

}  // namespace

namespace ptk {

// Forward and adjoint spectral stages: the diagonal-frequency work
// (k_spec) and the dense-frequency factorisation, in one launch where the
// tiled kernels take both.
hipError_t launch_spectral_fwd(const pt::Dev &D, const double *x, hipStream_t s) {
  if (D.c_pad == 0) return hipSuccess;
  if (D.nf_gw > 0 && pt::chol_tiles(D.n_psr) <= pt::kTileFwdMaxNT) return launch_cholt_fwd(D, x, s);
  const hipError_t e = launch_spec_fwd(D, x, s);
  return e == hipSuccess ? launch_chol_fwd(D, x, s) : e;
}

hipError_t launch_spectral_bwd(const pt::Dev &D, const double *x, double *grad, hipStream_t s) {
  if (D.n_chains == 0) return hipSuccess;
  const int nt = pt::chol_tiles(D.n_psr);
  if (D.nf_gw > 0 && nt <= pt::kTileMaxNT) return launch_cholt_bwd(D, x, grad, s);
  const hipError_t e = launch_spec_bwd(D, x, grad, s);
  if (e != hipSuccess || D.nf_gw == 0) return e;
  return nt <= pt::kTileFwdMaxNT ? launch_cholt_bwd(D, x, grad, s) : launch_chol_bwd(D, x, grad, s);
}

// dense frequencies of more than kTileMaxNT tiles (the row-per-thread kernels)
hipError_t launch_chol_fwd(const pt::Dev &D, const double *x, hipStream_t s) {
  if (D.nf_gw == 0 || D.c_pad == 0) return hipSuccess;
  switch (pt::chol_tiles(D.n_psr)) {
    case 8: return launch_fwd_t<128>(D, x, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_chol_bwd(const pt::Dev &D, const double *x, double *grad, hipStream_t s) {
  if (D.nf_gw == 0 || D.n_chains == 0) return hipSuccess;
  switch (pt::chol_tiles(D.n_psr)) {
    case 8: return launch_bwd_t<128>(D, x, grad, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace ptk
