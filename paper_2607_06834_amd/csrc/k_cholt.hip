// Dense per-frequency prior covariance on FP64 matrix cores: one 64-lane wave
// per (frequency, chain) holds the lower 16x16 tiles of the padded matrix in
// registers.  The factorisation takes arrays of up to 112 pulsars (seven
// tiles), the adjoint up to 80 (five tiles; beyond that k_chol's adjoint reads
// the same tile-major factor).
//
// Forward (Sec. IV.A, Eqs. HD, prior_cov; Sec. II.B, Eq.
// standardizing_transform with mu = 0): C = chol(rho_k Gamma + diag kappa_.k)
// by a right-looking blocked factorisation.  A block column is factorised by
// 16 rank-1 steps on the vector unit, with every operand moved between lanes
// by readlane, DPP and permlane swaps (no LDS); the trailing tiles are
// updated with 16x16x4 MFMAs.  Then a_.k,{sin,cos} = C z_.k,{sin,cos}.
//
// Backward, with abar from the TOA pass and v_c = C^T abar_c:
//   dz_c = v_c - z_c
//   W = C^-1 (block forward substitution on MFMA: W_II = C_II^-1 from a
//   16-lane substitution per diagonal tile, W_IJ = -W_II sum_K C_IK W_KJ)
//   M = W chol(Gamma)  (MFMA)
//   d/dkappa_I = w_I^T P w_I,  d/drho = sum_I m_I^T P m_I,  P = Phi(sum_c v_c z_c^T)
// The quadratic forms with the semiseparable P are prefix sums down each
// column, taken on the MFMA output layout.
//
// The launches also carry the diagonal-frequency work of the same stage
// (spec_dev.h) in a few extra workgroups after the dense ones, each taking a
// block of 16 chains and a segment of the frequencies: the two touch disjoint
// outputs, and the extra workgroups run on the compute units the dense
// problems leave free.
//
// Register layouts of a 16x16 block X (lane l = c + 16 q, item v or slice s):
//   forward, E(X):   X[c][q + 4s]       (operand A of X, operand B of X^T,
//                                         and the result layout of X^T)
//   backward, A(X):  X[pi(c)][4q + s]    operand A
//             B(X):  X[4q + v][c]        operand B and result layout
// with pi(c) = 4 (c mod 4) + c / 4, so that lane group q of a result holds the
// consecutive rows 4q .. 4q + 3 of every tile.
#include "common.h"
#include "spec_dev.h"

namespace {

using pt::Dev;
using pt::pk;
using v4d = double __attribute__((ext_vector_type(4)));

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/sqrt(a): hardware estimate refined by two Newton steps
__device__ inline double rsqrt_nr(double a) {
  double y = __builtin_amdgcn_rsq(a);
  y = y * (1.5 - 0.5 * a * y * y);
  y = y * (1.5 - 0.5 * a * y * y);
  return y;
}

// 1/a: hardware estimate refined by two Newton steps on e = 1 - a y
__device__ inline double rcp_nr(double a) {
  double y = __builtin_amdgcn_rcp(a);
  y = fma(y, fma(-a, y, 1.0), y);
  y = fma(y, fma(-a, y, 1.0), y);
  return y;
}

template <int N>
__device__ inline int dpp_row_share(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x150 + N, 0xF, 0xF, false);
}

// Lane n of every 16-lane row to all lanes of that row (DPP row broadcast);
// n is a constant once the caller's loop is unrolled.
__device__ inline double row_share_d(double v, int n) {
  const long long b = __double_as_longlong(v);
  int lo = (int)b, hi = (int)(b >> 32);
  switch (n) {
#define PT_ROW_SHARE(N)          \
  case N:                        \
    lo = dpp_row_share<N>(lo);   \
    hi = dpp_row_share<N>(hi);   \
    break;
    PT_ROW_SHARE(0) PT_ROW_SHARE(1) PT_ROW_SHARE(2) PT_ROW_SHARE(3)
    PT_ROW_SHARE(4) PT_ROW_SHARE(5) PT_ROW_SHARE(6) PT_ROW_SHARE(7)
    PT_ROW_SHARE(8) PT_ROW_SHARE(9) PT_ROW_SHARE(10) PT_ROW_SHARE(11)
    PT_ROW_SHARE(12) PT_ROW_SHARE(13) PT_ROW_SHARE(14) PT_ROW_SHARE(15)
#undef PT_ROW_SHARE
  }
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Row g (lanes 16g .. 16g + 15) to all four rows, lane for lane: a permlane16
// swap gives rows (g mod 2) and 2 + (g mod 2) twice each, a permlane32 swap
// then the chosen one four times.
__device__ inline unsigned row_bcast_u(unsigned v, int g) {
  const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  const unsigned y = (g & 1) ? p[1] : p[0];
  const auto r = __builtin_amdgcn_permlane32_swap(y, y, false, false);
  return (g & 2) ? r[1] : r[0];
}

__device__ inline double row_bcast_d(double v, int g) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = row_bcast_u((unsigned)b, g), hi = row_bcast_u((unsigned)(b >> 32), g);
  return __longlong_as_double(((long long)hi << 32) | lo);
}

// v of the same lane in the partner row (row q ^ 1, by the permlane16 swap)
// and in the partner half (row q ^ 2, by the permlane32 swap), q the caller's
// row: the swaps give every lane the value of the lower and of the upper
// member of its pair.
__device__ inline double xor16_d(double v, int q) {
  const long long b = __double_as_longlong(v);
  const auto pl = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
  const auto ph = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  const unsigned lo = (q & 1) ? pl[0] : pl[1], hi = (q & 1) ? ph[0] : ph[1];
  return __longlong_as_double(((long long)hi << 32) | lo);
}
__device__ inline double xor32_d(double v, int q) {
  const long long b = __double_as_longlong(v);
  const auto pl = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
  const auto ph = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  const unsigned lo = (q & 2) ? pl[0] : pl[1], hi = (q & 2) ? ph[0] : ph[1];
  return __longlong_as_double(((long long)hi << 32) | lo);
}

// The same through the LDS crossbar: every lane reads lane addr / 4 (addr =
// 4 (c + 16 g) for row g), two DS instructions instead of the VALU swaps.
__device__ inline double bperm_bcast_d(double v, int addr) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)b);
  const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// acc += X Y for one 16x16x16 product given the four k-slices of both operands
__device__ inline v4d mfma4(const v4d &a, const v4d &b, v4d acc) {
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], b[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], b[3], acc, 0, 0, 0);
  return acc;
}

__host__ __device__ constexpr int tidx(int I, int J) { return I * (I + 1) / 2 + J; }

// independent (frequency, chain) problems per workgroup, one wave each
constexpr int kProbPerGroup = 4;

// Work of the extra workgroups: G = nb * ns workgroups (spec_groups_fwd,
// spec_groups) for nb blocks of 16 chains and ns contiguous frequency
// segments.  The forward's segments hold equal numbers of frequencies (a
// split by the parts a frequency carries was measured slower); the adjoint's
// segments are balanced by cost, a frequency costing one unit per part it
// carries (diagonal red noise, DM).
struct spec_split {
  int G, nb, ns, kmax, nf_gw, ka, nf_dm;
  bool by_cost;
  __device__ spec_split(const Dev &D, int groups, int chains, bool balanced)
      : G(groups), nb((chains + pt::kCB - 1) / pt::kCB), ns(max(1, groups / nb)),
        kmax(max(D.ka, D.nf_dm)), nf_gw(D.nf_gw), ka(D.ka), nf_dm(D.nf_dm), by_cost(balanced) {}
  __device__ int cost(int k) const { return (k >= nf_gw && k < ka ? 1 : 0) + (k < nf_dm ? 1 : 0); }
  // first frequency of segment s (every segment keeps at least one: ns <= kmax)
  __device__ int k_lo(int s) const {
    if (s <= 0) return 0;
    if (s >= ns) return kmax;
    if (!by_cost) return kmax * s / ns;
    int total = 0;
    for (int k = 0; k < kmax; ++k) total += cost(k);
    int run = 0, k = 0;
    while (k < kmax && (long long)run * ns < (long long)total * s) run += cost(k++);
    return min(max(k, s), kmax - (ns - s));
  }
};

__device__ inline int pi16(int c) { return 4 * (c & 3) + (c >> 2); }

// ---------------------------------------------------------------------------
// Forward: one wave per (frequency, chain) problem, nf_gw * c_pad problems.
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(64 * kProbPerGroup) void k_cholt_fwd(Dev D, const double *__restrict__ x,
                                                                  int n_dense_groups) {
  if ((int)blockIdx.x >= n_dense_groups) {   // diagonal frequencies
    const spec_split sp(D, gridDim.x - n_dense_groups, D.c_pad, false);
    for (int it = blockIdx.x - n_dense_groups; it < sp.nb * sp.ns; it += sp.G) {
      const int b = it / sp.ns, s = it - b * sp.ns;
      pt::spec_fwd_cb(D, x, b * pt::kCB, sp.k_lo(s), sp.k_lo(s + 1), s, sp.ns);
      __syncthreads();
    }
    return;
  }
  constexpr int NP = 16 * NT;
  constexpr int NTILE = NT * (NT + 1) / 2;
  __shared__ double zb_[kProbPerGroup][NP][2];
  __shared__ double kb_[kProbPerGroup][NP];
  __shared__ double tb_[kProbPerGroup][16][17];   // tile transpose for the store of C
  // one wave per (frequency, chain) problem, kProbPerGroup problems per workgroup
  const int w = threadIdx.x >> 6;
  const int prob = blockIdx.x * kProbPerGroup + w;
  if (prob >= D.nf_gw * D.c_pad) return;
  const int k0 = prob % D.nf_gw, c = prob / D.nf_gw;
  const int l = threadIdx.x & 63, c16 = l & 15, q = l >> 4;
  double(*zb)[2] = zb_[w];
  double *kb = kb_[w];
  const int n = D.n_psr;
  const size_t cp = D.c_pad;
  const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
  auto coef = [&](int r, int sc) -> double & {
    return D.coef_rn[((size_t)r * D.rows_rn + (sc ? rc : rs)) * cp + c];
  };
  int32_t *flag = D.flag_dense + (size_t)c * D.nf_gw + k0;
  const double *xc = x + (size_t)(c < D.n_chains ? c : 0) * D.d;

  // Set-up: every global load (Gamma tiles, spectra parameters, z and the
  // prior box, which is checked here so nothing is read from k_spec_fwd) is
  // issued before the first of them is used, and the out-of-box exit comes
  // after the tiles are assembled, so the loads cost one round trip.
  // phi tiles in E layout: lane (c16, q), item v = phi[16I + c16][16J + q + 4v];
  // the padding is the identity.  The E layout of a tile is its column-major
  // image and the Gamma tiles are stored column-major, so every load reads
  // 512 contiguous bytes.
  v4d A[NTILE];
  const double *__restrict__ gt = D.gam_tile + l;
#pragma unroll
  for (int T = 0; T < NTILE; ++T)
#pragma unroll
    for (int v = 0; v < 4; ++v) A[T][v] = gt[T * 256 + 64 * v];
  constexpr int NR = (NP + 63) / 64;
  double kl[NR], kg[NR], zs[NR], zc[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const int r = l + 64 * j, rr = r < n ? r : n - 1;
    kl[j] = xc[D.off_rn + 2 * rr];
    kg[j] = xc[D.off_rn + 2 * rr + 1];
    const double *z = xc + D.off_z + (size_t)rr * 2 * D.ka + 2 * k0;
    zs[j] = z[0];
    zc[j] = z[1];
  }
  const double rho = pt::powerlaw_k(D, k0, xc[D.off_gw], xc[D.off_gw + 1]);
  const bool inbox = c < D.n_chains && pt::theta_in_box_wave(D, xc);
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const int r = l + 64 * j;
    if (r < NP) {
      const bool real = r < n;
      kb[r] = (real && k0 < D.nf_rn) ? pt::powerlaw_k(D, k0, kl[j], kg[j]) : 0.0;
      zb[r][0] = real ? zs[j] : 0.0;
      zb[r][1] = real ? zc[j] : 0.0;
    }
  }
  wave_sync();
#pragma unroll
  for (int T = 0; T < NTILE; ++T) A[T] *= rho;
#pragma unroll
  for (int I = 0; I < NT; ++I) {
    const int r = 16 * I + c16;
    const double dadd = (r < n) ? kb[r] : 1.0;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (c16 == q + 4 * v) A[tidx(I, I)][v] += dadd;
  }

  if (!inbox) {
    for (int r = l; r < n; r += 64) {
      coef(r, 0) = 0.0;
      coef(r, 1) = 0.0;
    }
    if (l == 0) *flag = 0;
    return;
  }

  bool pd = true;
#pragma unroll
  for (int J = 0; J < NT; ++J) {
    // ---- block column J: 16 rank-1 steps on the unscaled column a
    //      (a_r = A[r][cc]): A[r][c] -= a_r a_c / a_cc over the rows and
    //      columns after cc.  The diagonal tile is updated on both sides of
    //      its diagonal, so a_c for c > cc is also row cc of it, held by lane
    //      cc of every lane group (DPP row broadcast); a_r is column cc, held
    //      by lane group cc mod 4 (permlane broadcast).  Items v < cc / 4 of a
    //      lane are finished columns and are left alone.  A step's pivot is
    //      never touched by the later steps, so the scaling of the columns by
    //      1/sqrt(pivot) and the pivot checks wait for the end of the block
    //      column, where they are done four columns at a time.
    //      Each step is pipelined against the next: the diagonal tile is
    //      updated first, then the next pivot's reciprocal is started, and
    //      the tiles below (whose column arrived through the LDS crossbar
    //      during the previous step) are updated under its latency, their
    //      next column sent on its way.
    double ri_next = rcp_nr(readlane_d(A[tidx(J, J)][0], 0));
    double arn[NT];
#pragma unroll
    for (int I = J + 1; I < NT; ++I) arn[I] = bperm_bcast_d(A[tidx(I, J)][0], 4 * c16);
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      // padding columns of the last tile: pivot 1, zero column, nothing to do
      if (J == NT - 1 && 16 * J + cc >= n) continue;
      const int g0 = cc & 3, v0 = cc >> 2;
      const int g1 = (cc + 1) & 3, v1 = (cc + 1) >> 2;
      const double ri = ri_next;
      double lk[4];
#pragma unroll
      for (int v = v0; v < 4; ++v) {
        const double t = row_share_d(A[tidx(J, J)][v], cc) * ri;
        lk[v] = (v > v0 || q > g0) ? t : 0.0;
      }
      {
        double ar = row_bcast_d(A[tidx(J, J)][v0], g0);
        if (c16 <= cc) ar = 0.0;
#pragma unroll
        for (int v = v0; v < 4; ++v) A[tidx(J, J)][v] -= ar * lk[v];
      }
      if (cc + 1 < 16) ri_next = rcp_nr(readlane_d(A[tidx(J, J)][v1], cc + 1 + 16 * g1));
#pragma unroll
      for (int I = J + 1; I < NT; ++I) {
        const double ar = arn[I];
#pragma unroll
        for (int v = v0; v < 4; ++v) A[tidx(I, J)][v] -= ar * lk[v];
        if (cc + 1 < 16) arn[I] = bperm_bcast_d(A[tidx(I, J)][v1], 4 * (c16 + 16 * g1));
      }
    }
    // pivots of the lane's columns q + 4v (lane q + 4v of its own lane
    // group), then C[.][c] = a / sqrt(pivot_c); the padding pivots are 1
    {
      double rd[4];
      bool ok = true;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double piv = __shfl(A[tidx(J, J)][v], 17 * q + 4 * v, 64);
        ok = ok && (piv > 0.0) && isfinite(piv);
        rd[v] = rsqrt_nr(piv);
      }
      pd = pd && __all(ok);
#pragma unroll
      for (int I = J; I < NT; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) A[tidx(I, J)][v] *= rd[v];
    }
    // ---- trailing tiles: A_IK -= C_IJ C_KJ^T  (as A_IK^T -= C_KJ C_IJ^T)
#pragma unroll
    for (int K = J + 1; K < NT; ++K) {
      const v4d nk = -A[tidx(K, J)];
#pragma unroll
      for (int I = K; I < NT; ++I) A[tidx(I, K)] = mfma4(nk, A[tidx(I, J)], A[tidx(I, K)]);
    }
  }
  if (!pd) {
    for (int r = l; r < n; r += 64) {
      coef(r, 0) = 0.0;
      coef(r, 1) = 0.0;
    }
    if (l == 0) *flag = pt::kFlagNotPD;
    return;
  }
  if (l == 0) *flag = 0;
  // zero the upper part of the diagonal tiles
#pragma unroll
  for (int I = 0; I < NT; ++I)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (q + 4 * v > c16) A[tidx(I, I)][v] = 0.0;

  // a = C z: lane partial over its columns, then over the lane groups
#pragma unroll
  for (int I = 0; I < NT; ++I) {
    double as = 0.0, ac = 0.0;
#pragma unroll
    for (int J = 0; J <= I; ++J)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = 16 * J + q + 4 * v;
        as += A[tidx(I, J)][v] * zb[k][0];
        ac += A[tidx(I, J)][v] * zb[k][1];
      }
    as += __shfl_xor(as, 16, 64);
    ac += __shfl_xor(ac, 16, 64);
    as += __shfl_xor(as, 32, 64);
    ac += __shfl_xor(ac, 32, 64);
    const int r = 16 * I + c16;
    if (q == 0 && r < n) {
      coef(r, 0) = as;
      coef(r, 1) = ac;
    }
  }
  // keep C for the adjoint, tile-major with row-major tiles: each tile is
  // transposed through LDS so that every store writes 512 contiguous bytes
  double *dst = D.lstore + ((size_t)c * D.nf_gw + k0) * (NTILE * 256) + l;
  double(*tb)[17] = tb_[w];
#pragma unroll
  for (int T = 0; T < NTILE; ++T) {
#pragma unroll
    for (int v = 0; v < 4; ++v) tb[c16][q + 4 * v] = A[T][v];
    wave_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[T * 256 + 64 * v] = tb[4 * v + q][c16];
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// Backward: one wave per (frequency, chain) problem, nf_gw * n_chains problems.
// ---------------------------------------------------------------------------
struct ScanState {
  double rs, rc, q;   // running column sums of z x (sin, cos) and the quadratic form
};

// One 16-row tile of 16 columns (B layout: item v of lane group q is row
// row0 + 4q + v) added to the column quadratic forms x^T P x; vr[v] holds
// (v_sin, v_cos, z_sin, z_cos) of row row0 + 4q + v.
__device__ inline void scan_rows(const v4d &X, const double (&vr)[4][4], ScanState &st, int q) {
  double ls = 0.0, lc = 0.0, part = 0.0, sa = 0.0, ca = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double x = X[v];
    const double bs = vr[v][2] * x, bc = vr[v][3] * x;
    const double as = vr[v][0] * x, ac = vr[v][1] * x;
    part += as * (ls + 0.5 * bs) + ac * (lc + 0.5 * bc);
    ls += bs;
    lc += bc;
    sa += as;
    ca += ac;
  }
  // inclusive prefix of the lane sums over the four lane groups of a column
  // and their total, by the row swaps: with t the partner row's sum, the
  // pair total is p = x + t, the prefix x (+ t on odd rows) (+ the other
  // half's pair total on rows 2 and 3), the total p + that
  const double ts1 = xor16_d(ls, q), tc1 = xor16_d(lc, q);
  const double ps = ls + ts1, pc2 = lc + tc1;
  const double os = xor32_d(ps, q), oc = xor32_d(pc2, q);
  double is = (q & 1) ? ps : ls, ic = (q & 1) ? pc2 : lc;
  if (q >= 2) {
    is += os;
    ic += oc;
  }
  const double ts = ps + os, tc = pc2 + oc;
  st.q += part + (st.rs + (is - ls)) * sa + (st.rc + (ic - lc)) * ca;
  st.rs += ts;
  st.rc += tc;
}

// this lane's rows of v and z for the row tile at row0
__device__ inline void load_rows(const double (*vz)[4], int row0, int q, double (&vr)[4][4]) {
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int k = 0; k < 4; ++k) vr[v][k] = vz[row0 + 4 * q + v][k];
}

__device__ inline void scan_tile(const v4d &X, int row0, const double (*vz)[4], ScanState &st,
                                 int l, int c16, int q) {
  double vr[4][4];
  load_rows(vz, row0, q, vr);
  scan_rows(X, vr, st, q);
}

// Up to kTileMaxNT tiles all of W = C^-1 lives in registers and a problem
// has two waves, kBwdProbs problems per workgroup: wave 0 of a problem forms
// v = C^T abar and then the d/dkappa quadratic forms, wave 1 the diagonal
// inverses and W and then M = W G and the d/drho forms (the two halves are
// independent until W and v meet in LDS), at two waves a SIMD.  Beyond
// (COLW) the workgroup is one wave and one problem: W is built one block
// column at a time in registers and kept in LDS (the diagonal inverses in
// place of the diagonal tiles of C).
constexpr int kBwdProbs = 2;
template <int NT>
constexpr int bwd_probs() { return NT > pt::kTileMaxNT ? 1 : kBwdProbs; }
template <int NT>
constexpr int bwd_wpp() { return NT > pt::kTileMaxNT ? 1 : 2; }   // waves per problem
template <int NT>
constexpr int bwd_threads() { return 64 * bwd_probs<NT>() * bwd_wpp<NT>(); }

template <int NT>
__global__ __launch_bounds__(bwd_threads<NT>()) __attribute__((amdgpu_waves_per_eu(bwd_wpp<NT>())))
void k_cholt_bwd(Dev D, const double *__restrict__ x,
                                                  double *__restrict__ grad,
                                                  const double *__restrict__ lst,
                                                  const double *__restrict__ gch,
                                                  const double *__restrict__ bar,
                                                  int n_dense_groups) {
  constexpr bool COLW = NT > pt::kTileMaxNT;
  constexpr int PPG = bwd_probs<NT>();
  constexpr int WPP = bwd_wpp<NT>();
  static_assert(COLW || bwd_threads<NT>() == 256, "the diagonal-frequency work runs on 256 threads");
  if ((int)blockIdx.x >= n_dense_groups) {   // diagonal frequencies
    const spec_split sp(D, gridDim.x - n_dense_groups, D.n_chains, true);
    for (int it = blockIdx.x - n_dense_groups; it < sp.nb * sp.ns; it += sp.G) {
      const int b = it / sp.ns, s = it - b * sp.ns;
      pt::spec_bwd_cb(D, x, grad, b * pt::kCB, sp.k_lo(s), sp.k_lo(s + 1), s, sp.ns);
      __syncthreads();
    }
    return;
  }
  constexpr int NP = 16 * NT;
  constexpr int NTILE = NT * (NT + 1) / 2;
  constexpr int TS = 17;                              // LDS row stride of a tile
  constexpr int NTL = COLW ? NTILE : (NTILE > 2 * NT ? NTILE : 2 * NT);
  __shared__ double vz_[PPG][NP][4];                   // v_sin, v_cos, z_sin, z_cos
  __shared__ double tl_[PPG][NTL][16 * TS];
  __shared__ double ab_[PPG][NP][2];
  __shared__ int nbad_[PPG];
  const int w = (threadIdx.x >> 6) / WPP;          // problem slot
  const int role = (threadIdx.x >> 6) - w * WPP;   // 0: v and d/dkappa, 1: W and d/drho
  const bool do_v = COLW || role == 0;
  const int prob = blockIdx.x * PPG + w;
  if (prob >= D.nf_gw * D.n_chains) return;
  const int k0 = prob % D.nf_gw, c = prob / D.nf_gw;
  const int l = threadIdx.x & 63, c16 = l & 15, q = l >> 4;
  double(*vz)[4] = vz_[w];
  double(*tl)[16 * TS] = tl_[w];
  double(*ab)[2] = ab_[w];
  const int n = D.n_psr;
  const int kmax = max(D.ka, D.nf_dm);
  const size_t cp = D.c_pad;
  const int rs = pt::harm_row(k0 + 1, 0), rc = pt::harm_row(k0 + 1, 1);
  const int K2 = 2 * D.ka;
  const double *xc = x + (size_t)c * D.d;
  double *gz = grad + (size_t)c * D.d + D.off_z + 2 * k0;
  double *drn = pt::drn_at(D, c, 0, k0);   // pulsar I at drn[2 ka I]
  const size_t dI = 2 * (size_t)D.ka;
  double *dth = D.dth_k + ((size_t)c * D.ka + k0) * 2;
  const int fl0 = D.flag_k[(size_t)c * kmax + k0] | D.flag_dense[(size_t)c * D.nf_gw + k0];
  int32_t *fout = D.flag_out + (size_t)c * (kmax + pt::kSpecSeg) + k0;
  if (D.st_pre[c] != 0 || fl0 != 0) {
    if (!do_v) return;
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
  const double lnfy = D.lnfy[k0];   // for the outputs (loaded here, not after the barriers)
  const double *Cb = lst + ((size_t)c * D.nf_gw + k0) * (NTILE * 256);
  const int pc = pi16(c16);
  if constexpr (!COLW) {
    if (role == 1) {
      // ==== wave 1: W = C^-1, then M = W G and the d/drho quadratic forms
      const double rho_o = pt::powerlaw_k(D, k0, xc[D.off_gw], xc[D.off_gw + 1]);
      // ---- inverses of the diagonal tiles: lane group g solves tile J = g (+4)
      //      column c16 by forward substitution; C_JJ in tl[J], W_JJ in tl[NT + J]
#pragma unroll
      for (int J = 0; J < NT; ++J)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          tl[J][(4 * q + v) * TS + c16] = Cb[tidx(J, J) * 256 + (4 * q + v) * 16 + c16];
      // the off-diagonal factor tiles (A layout), issued now so that their
      // loads run under the substitutions and the products below never wait
      // on memory
      v4d Ca[NTILE];
#pragma unroll
      for (int I = 1; I < NT; ++I)
#pragma unroll
        for (int K = 0; K < I; ++K) {
          const double *t = Cb + tidx(I, K) * 256 + pc * 16 + 4 * q;
#pragma unroll
          for (int s = 0; s < 4; ++s) Ca[tidx(I, K)][s] = t[s];
        }
      wave_sync();
#pragma unroll
      for (int rnd = 0; rnd < (NT + 3) / 4; ++rnd) {
        const int J = 4 * rnd + q;
        if (J < NT) {
          const double *T = tl[J];
          // reciprocals of the diagonal first (independent of each other), so
          // the substitution's dependent chain has multiplies, not divisions
          double rdg[16];
#pragma unroll
          for (int r = 0; r < 16; ++r) rdg[r] = rcp_nr(T[r * TS + r]);
          double xs[16];
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            __builtin_amdgcn_sched_barrier(0);     // bound the live LDS reads to one row
            double s = (r == c16) ? 1.0 : 0.0;
#pragma unroll
            for (int m = 0; m < r; ++m) s -= T[r * TS + m] * xs[m];
            xs[r] = s * rdg[r];
          }
#pragma unroll
          for (int r = 0; r < 16; ++r) tl[NT + J][r * TS + c16] = xs[r];
        }
      }
      wave_sync();   // the diagonal inverses in LDS
      // ---- W = C^-1 (B layout) one block column at a time (the products of
      //      a column depend only on that column): W_IJ = -W_II sum_{J<=K<I}
      //      C_IK W_KJ, -W_II (A layout) read where it is used
      v4d Wb[NTILE];
#pragma unroll
      for (int J = 0; J < NT; ++J) {
        __builtin_amdgcn_sched_barrier(0);     // one block column live at a time
#pragma unroll
        for (int v = 0; v < 4; ++v) Wb[tidx(J, J)][v] = tl[NT + J][(4 * q + v) * TS + c16];
#pragma unroll
        for (int I = J + 1; I < NT; ++I) {
          v4d Wi;
#pragma unroll
          for (int v = 0; v < 4; ++v) Wi[v] = -tl[NT + I][pc * TS + 4 * q + v];
          v4d U = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int K = J; K < I; ++K) U = mfma4(Ca[tidx(I, K)], Wb[tidx(K, J)], U);
          Wb[tidx(I, J)] = mfma4(Wi, U, v4d{0.0, 0.0, 0.0, 0.0});
        }
      }
      wave_sync();   // every read of the diagonal inverses done before W overwrites them
#pragma unroll
      for (int T = 0; T < NTILE; ++T)
#pragma unroll
        for (int v = 0; v < 4; ++v) tl[T][(4 * q + v) * TS + c16] = Wb[T][v];
      __syncthreads();   // W (this wave) and v, z (wave 0) of every problem in LDS
      double dr = 0.0;
      // ---- d/drho: M = W G and its quadratic forms, row tile by row tile
      //      (each tile's rows of v and z read once); chol(Gamma) in
      //      registers, W in A layout from LDS
      v4d G[NTILE];
#pragma unroll
      for (int J = 0; J < NT; ++J)
#pragma unroll
        for (int K = J; K < NT; ++K) {
          const double *gt = gch + tidx(K, J) * 256 + 64 * q + c16;
#pragma unroll
          for (int v = 0; v < 4; ++v) G[tidx(K, J)][v] = gt[16 * v];
        }
      ScanState st[NT];
#pragma unroll
      for (int J = 0; J < NT; ++J) st[J] = ScanState{0.0, 0.0, 0.0};
#pragma unroll
      for (int I = 0; I < NT; ++I) {
        __builtin_amdgcn_sched_barrier(0);     // one row tile live at a time
        double vr[4][4];
        load_rows(vz, 16 * I, q, vr);
        v4d a[NT];
#pragma unroll
        for (int K = 0; K <= I; ++K)
#pragma unroll
          for (int s = 0; s < 4; ++s) a[K][s] = tl[tidx(I, K)][pc * TS + 4 * q + s];
#pragma unroll
        for (int J = 0; J <= I; ++J) {
          v4d Mt = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int K = J; K <= I; ++K) Mt = mfma4(a[K], G[tidx(K, J)], Mt);
          scan_rows(Mt, vr, st[J], q);
        }
      }
#pragma unroll
      for (int J = 0; J < NT; ++J) dr += st[J].q;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) dr += __shfl_xor(dr, o, 64);
      __syncthreads();   // wave 0's count of non-finite outputs
      if (l == 0) {
        dth[0] = dr * rho_o * 2.0 * pt::kLn10;
        dth[1] = dr * rho_o * (-lnfy);
        *fout = (nbad_[w] || !isfinite(dth[0]) || !isfinite(dth[1])) ? pt::kFlagOutNonfinite : 0;
      }
      return;
    }
  }
  // ==== wave 0 (the only wave in the column-wise form): v = C^T abar, then
  //      the d/dkappa quadratic forms and the pulsars' outputs
  // the spectra for the outputs, early (their loads and exponentials overlap the work below)
  double kapo[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int I = l + 64 * h;
    kapo[h] = (I < n && k0 < D.nf_rn) ? pt::powerlaw_k(D, k0, xc[D.off_rn + 2 * I], xc[D.off_rn + 2 * I + 1])
                                      : 0.0;
  }
  double vv[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  double zz[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  // ---- v_c = C^T abar_c: lane (c16, q) sums rows 16K + 4q + v of column
  //      16J + c16, then the four lane groups are added
  for (int m = l; m < NP; m += 64) {
    double as = 0.0, ac = 0.0;
    if (m < n) {
      as = bar[((size_t)m * D.rows_rn + rs) * cp + c];
      ac = bar[((size_t)m * D.rows_rn + rc) * cp + c];
    }
    ab[m][0] = as;
    ab[m][1] = ac;
  }
  wave_sync();
  double vcol[NT][2];
#pragma unroll
  for (int J = 0; J < NT; ++J) {
    if constexpr (!COLW) __builtin_amdgcn_sched_barrier(0);   // one column's loads in flight at a time
    double ss = 0.0, sc = 0.0;
#pragma unroll
    for (int K = J; K < NT; ++K) {
      const double *t = Cb + tidx(K, J) * 256 + 64 * q + c16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double e = t[16 * v];
        ss += e * ab[16 * K + 4 * q + v][0];
        sc += e * ab[16 * K + 4 * q + v][1];
      }
    }
    ss += xor16_d(ss, q);
    sc += xor16_d(sc, q);
    ss += xor32_d(ss, q);
    sc += xor32_d(sc, q);
    vcol[J][0] = ss;
    vcol[J][1] = sc;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int I = l + 64 * h;
#pragma unroll
    for (int J = 0; J < NT; ++J)
      if (J == (I >> 4)) {
        vv[h][0] = vcol[J][0];
        vv[h][1] = vcol[J][1];
      }
    if (I < n) {
      zz[h][0] = xc[D.off_z + (size_t)I * K2 + 2 * k0];
      zz[h][1] = xc[D.off_z + (size_t)I * K2 + 2 * k0 + 1];
    }
    if (I < NP) {
      vz[I][0] = vv[h][0];
      vz[I][1] = vv[h][1];
      vz[I][2] = zz[h][0];
      vz[I][3] = zz[h][1];
    }
  }

  double dkap[NT] = {};
  double dr = 0.0;
  if constexpr (COLW) {
    // ---- inverses of the diagonal tiles, in place: lane group g solves
    //      tile J = g (+4, ...) column c16 by forward substitution
#pragma unroll
    for (int J = 0; J < NT; ++J)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        tl[tidx(J, J)][(4 * q + v) * TS + c16] = Cb[tidx(J, J) * 256 + (4 * q + v) * 16 + c16];
    wave_sync();
#pragma unroll
    for (int rnd = 0; rnd < (NT + 3) / 4; ++rnd) {
      const int J = 4 * rnd + q;
      if (J < NT) {
        double *T = tl[tidx(J, J)];
        double xs[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          __builtin_amdgcn_sched_barrier(0);   // bound the live LDS reads to one row
          double s = (r == c16) ? 1.0 : 0.0;
#pragma unroll
          for (int m = 0; m < r; ++m) s -= T[r * TS + m] * xs[m];
          xs[r] = s / T[r * TS + r];
        }
        // (the lanes of a group read all of C_JJ before any of them writes)
#pragma unroll
        for (int r = 0; r < 16; ++r) T[r * TS + c16] = xs[r];
      }
    }
    wave_sync();
    // ---- W = C^-1 by block columns: W_IJ = -W_II sum_{J<=K<I} C_IK W_KJ
    //      (B layout), the column's d/dkappa, then the column into LDS
#pragma unroll
    for (int J = 0; J < NT; ++J) {
      __builtin_amdgcn_sched_barrier(0);       // one block column live at a time
      v4d Wc[NT];
#pragma unroll
      for (int v = 0; v < 4; ++v) Wc[J][v] = tl[tidx(J, J)][(4 * q + v) * TS + c16];
#pragma unroll
      for (int I = J + 1; I < NT; ++I) {
        __builtin_amdgcn_sched_barrier(0);
        v4d U = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int K = J; K < I; ++K) {
          v4d a;
          const double *t = Cb + tidx(I, K) * 256 + pc * 16 + 4 * q;
#pragma unroll
          for (int s = 0; s < 4; ++s) a[s] = t[s];
          U = mfma4(a, Wc[K], U);
        }
        v4d wi;
#pragma unroll
        for (int s = 0; s < 4; ++s) wi[s] = -tl[tidx(I, I)][pc * TS + 4 * q + s];
        Wc[I] = mfma4(wi, U, v4d{0.0, 0.0, 0.0, 0.0});
      }
      ScanState st{0.0, 0.0, 0.0};
#pragma unroll
      for (int I = J; I < NT; ++I) scan_tile(Wc[I], 16 * I, vz, st, l, c16, q);
      double qq = st.q;
      qq += xor16_d(qq, q);
      qq += xor32_d(qq, q);
      dkap[J] = qq;
#pragma unroll
      for (int I = J + 1; I < NT; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) tl[tidx(I, J)][(4 * q + v) * TS + c16] = Wc[I][v];
    }
    wave_sync();
    // ---- d/drho: M = W G column block by column block, W in A layout from LDS
#pragma unroll
    for (int J = 0; J < NT; ++J) {
      ScanState st{0.0, 0.0, 0.0};
#pragma unroll
      for (int I = J; I < NT; ++I) {
        __builtin_amdgcn_sched_barrier(0);     // one product tile live at a time
        v4d Mt = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int K = J; K <= I; ++K) {
          v4d a, g;
#pragma unroll
          for (int s = 0; s < 4; ++s) a[s] = tl[tidx(I, K)][pc * TS + 4 * q + s];
          const double *gt = gch + tidx(K, J) * 256 + 64 * q + c16;
#pragma unroll
          for (int v = 0; v < 4; ++v) g[v] = gt[16 * v];
          Mt = mfma4(a, g, Mt);
        }
        scan_tile(Mt, 16 * I, vz, st, l, c16, q);
      }
      dr += st.q;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dr += __shfl_xor(dr, o, 64);
  } else {
    __syncthreads();   // W (wave 1) and v, z (this wave) of every problem in LDS
      // ---- d/dkappa: quadratic forms down the columns of W (B layout), row
      //      tile by row tile, so that each tile's rows of v and z are read once
      ScanState st[NT];
#pragma unroll
      for (int J = 0; J < NT; ++J) st[J] = ScanState{0.0, 0.0, 0.0};
#pragma unroll
      for (int I = 0; I < NT; ++I) {
        __builtin_amdgcn_sched_barrier(0);       // one row tile live at a time
        double vr[4][4];
        load_rows(vz, 16 * I, q, vr);
        v4d Wr[NT];
#pragma unroll
        for (int J = 0; J <= I; ++J)
#pragma unroll
          for (int v = 0; v < 4; ++v) Wr[J][v] = tl[tidx(I, J)][(4 * q + v) * TS + c16];
#pragma unroll
        for (int J = 0; J <= I; ++J) scan_rows(Wr[J], vr, st[J], q);
      }
#pragma unroll
      for (int J = 0; J < NT; ++J) {
        double qq = st[J].q;
        qq += xor16_d(qq, q);
        qq += xor32_d(qq, q);
        dkap[J] = qq;
      }
  }

  // ---- outputs of the pulsars
  bool fin = true;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int I = l + 64 * h;
    if (I < n) {
      const double g0 = vv[h][0] - zz[h][0], g1 = vv[h][1] - zz[h][1];
      gz[(size_t)I * K2] = g0;
      gz[(size_t)I * K2 + 1] = g1;
      // column I = 16 (I / 16) + l % 16: this lane's entry of its column block
      double dk = 0.0;
#pragma unroll
      for (int J = 0; J < NT; ++J) dk = (J == (I >> 4)) ? dkap[J] : dk;
      const double kap = kapo[h];
      const double d0 = dk * kap * 2.0 * pt::kLn10, d1 = dk * kap * (-lnfy);
      drn[dI * I] = d0;
      drn[dI * I + 1] = d1;
      fin = fin && isfinite(g0) && isfinite(g1) && isfinite(d0) && isfinite(d1);
    }
  }
  const int nbad = __popcll(__ballot(!fin));
  if constexpr (!COLW) {
    if (l == 0) nbad_[w] = nbad;
    __syncthreads();   // read by wave 1, which writes d/drho and the flag
  } else {
    const double rho_o = pt::powerlaw_k(D, k0, xc[D.off_gw], xc[D.off_gw + 1]);
    if (l == 0) {
      dth[0] = dr * rho_o * 2.0 * pt::kLn10;
      dth[1] = dr * rho_o * (-lnfy);
      *fout = (nbad || !isfinite(dth[0]) || !isfinite(dth[1])) ? pt::kFlagOutNonfinite : 0;
    }
  }
}

// Workgroups for the diagonal-frequency work of `chains` chains next to ng
// dense workgroups, `per_cu` of which fill a compute unit: the workgroup
// slots those leave free, at least 8, split into blocks of 16 chains times
// frequency segments (spec_split).
int spec_groups(const Dev &D, int ng, int chains, int per_cu) {
  const int nb = (chains + pt::kCB - 1) / pt::kCB;
  const int kmax = max(D.ka, D.nf_dm);
  const int ns = max(1, min(min(kmax, pt::kSpecSeg), max(8, per_cu * D.n_cu - ng) / nb));
  return nb * ns;
}

// The forward's diagonal-frequency workgroups: up to one frequency segment
// per frequency, four per free compute unit's worth (the forward's segments
// write no per-segment flags, so their number is free).  A dense forward wave
// leaves room for one more wave on its SIMD; with fewer, longer segments these
// workgroups outlast the dense waves (measured: a segment of one or two
// frequencies of 16 chains and 67 pulsars takes about 30k-60k cycles, a
// dense wave about 48k).
int spec_groups_fwd(const Dev &D, int ng, int chains) {
  const int nb = (chains + pt::kCB - 1) / pt::kCB;
  const int kmax = max(D.ka, D.nf_dm);
  const int ns = max(1, min(kmax, 4 * max(8, D.n_cu - ng) / nb));
  return nb * ns;
}

// grid: the dense problems, kProbPerGroup per workgroup, then the
// diagonal-frequency workgroups
template <int NT>
hipError_t launch_fwd_t(const Dev &D, const double *x, hipStream_t s) {
  const int nprob = D.nf_gw * D.c_pad;
  const int ng = (nprob + kProbPerGroup - 1) / kProbPerGroup;
  hipLaunchKernelGGL(k_cholt_fwd<NT>, dim3(ng + spec_groups_fwd(D, ng, D.c_pad)),
                     dim3(64 * kProbPerGroup), 0, s, D, x, ng);
  return hipGetLastError();
}

// (beyond kTileMaxNT tiles the workgroups are single waves: the
// diagonal-frequency work runs in its own launch, k_spec_bwd)
template <int NT>
hipError_t launch_bwd_t(const Dev &D, const double *x, double *grad, hipStream_t s) {
  constexpr int P = bwd_probs<NT>();
  const int nprob = D.nf_gw * D.n_chains;
  const int ng = (nprob + P - 1) / P;
  // two tiled workgroups share a compute unit (half its LDS and registers each)
  const int ns = NT > pt::kTileMaxNT ? 0 : spec_groups(D, ng, D.n_chains, 2);
  hipLaunchKernelGGL(k_cholt_bwd<NT>, dim3(ng + ns), dim3(bwd_threads<NT>()), 0, s, D, x, grad,
                     (const double *)D.lstore, D.gtile, (const double *)D.bar_rn, ng);
  return hipGetLastError();
}

}  // namespace

namespace ptk {

hipError_t launch_cholt_fwd(const pt::Dev &D, const double *x, hipStream_t s) {
  switch (pt::chol_tiles(D.n_psr)) {
    case 1: return launch_fwd_t<1>(D, x, s);
    case 2: return launch_fwd_t<2>(D, x, s);
    case 3: return launch_fwd_t<3>(D, x, s);
    case 4: return launch_fwd_t<4>(D, x, s);
    case 5: return launch_fwd_t<5>(D, x, s);
    case 6: return launch_fwd_t<6>(D, x, s);
    case 7: return launch_fwd_t<7>(D, x, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_cholt_bwd(const pt::Dev &D, const double *x, double *grad, hipStream_t s) {
  switch (pt::chol_tiles(D.n_psr)) {
    case 1: return launch_bwd_t<1>(D, x, grad, s);
    case 2: return launch_bwd_t<2>(D, x, grad, s);
    case 3: return launch_bwd_t<3>(D, x, grad, s);
    case 4: return launch_bwd_t<4>(D, x, grad, s);
    case 5: return launch_bwd_t<5>(D, x, grad, s);
    case 6: return launch_bwd_t<6>(D, x, grad, s);
    case 7: return launch_bwd_t<7>(D, x, grad, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace ptk
