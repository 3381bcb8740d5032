// TOA pass: per-TOA residual, white-noise chi^2 and log-determinant, and the
// adjoint contractions, for every chain (Sec. IV, Eq. likelihood with the
// bases of Eqs. Fourier_series / RN=Fa, F_DM = w F of Sec. III.C and the
// timing model M = [1, tau, tau^2] of Eq. TM=Me; N of Eq. WN_cov):
//
//   r  = dt - F_tile . A - w (F_tile . A_dm) - h_cw   (A includes M b)
//   g  = r / N,  chi2 += r g,  logdet += ln N
//   Abar += F_tile^T g,  Abar_dm += F_tile^T (w g),  cwbar += g dh_cw/dtheta
//
// The batched form runs F.A and F^T.G as FP64 MFMA 16x16x4 contractions
// over 16-TOA x 16-chain tiles; the basis is generated in registers from one
// sincos per TOA and an angle-addition step, and transposed through LDS for
// the adjoint.  The plain form is a vector-ALU kernel launched per pulsar.
#include <type_traits>

#include "common.h"
#include "cw_dev.h"

namespace {

using pt::Dev;
using v4d = double __attribute__((ext_vector_type(4)));

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double tm_value(int i, double tau) {
  return i == 0 ? 1.0 : (i == 1 ? tau : (i == 2 ? tau * tau : 0.0));
}

// Map a hardware workgroup id to a work item so that consecutive items (the
// chain blocks of one chunk, then the next chunk of the same pulsar) land on
// the same XCD: workgroups are dispatched to the 8 XCDs round-robin.
__device__ inline int xcd_remap(int b, int G) {
  const int x = b & 7, idx = b >> 3;
  const int base = G >> 3, rem = G & 7;
  const int start = x * base + min(x, rem);
  return start + idx;
}

// ---------------------------------------------------------------------------
// Batched MFMA TOA pass.  grid = n_chunks * n_cb, block = 64 * WPB.
// Per-TOA inputs (padded by kToaPad so the one-tile-ahead prefetch never
// leaves the arrays): sin/cos of 2 pi t / T, tau, DM weight w, residual dt,
// and the per-call 1/N.
// ---------------------------------------------------------------------------
//
// With four waves per workgroup (SHB) the waves share the coefficient panels
// in LDS instead of holding them in registers, and keep one set of per-tile
// inputs, reloaded once the residuals are formed: three waves per SIMD (two
// with the CW terms, a few registers spilled).  With one or two waves per
// workgroup the panels live in registers and the inputs alternate between two
// register sets: two waves per SIMD, one with the CW terms.  (A single wave
// leaves the matrix core idle about half the time.)
template <int JTR, int JTD, int WPB, bool CW>
__global__ __launch_bounds__(64 * WPB, CW ? (WPB == 4 ? 2 : 1) : (WPB == 4 ? 3 : 2))
void k_toa_mfma(Dev D, int xcd_map) {
  constexpr int NSR = 4 * JTR;
  constexpr int NSD = 4 * JTD;
  constexpr int ROWS = 16 * JTR;
  constexpr int FS = ROWS + 1;                 // padded LDS row stride (doubles)
  constexpr bool SHB = WPB == 4;
  __shared__ double ftab[WPB][16 * FS];
  __shared__ double cred[WPB][16];
  __shared__ double cwred[CW ? WPB : 1][8][16];
  __shared__ double bop[SHB ? 4 * (NSR + NSD) * 16 : 1];   // panels [row][16 chains]

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, q = lane >> 4;
  int wg = blockIdx.x;
  if (D.wg_map) wg = D.wg_map[blockIdx.x];
  else if (xcd_map) wg = xcd_remap(wg, gridDim.x);
  const int chunk = wg / D.n_cb, cb = wg - chunk * D.n_cb;
  const int p = D.chunk_psr[chunk];
  const int tb = D.chunk_begin[chunk], te = D.chunk_end[chunk];
  const int chain = cb * 16 + col;
  const size_t cp = D.c_pad;
  const int kb = D.kb;

  // B operands: coefficient rows 4s + q for this lane's chain
  double cr[SHB ? 1 : NSR], cd[(SHB || NSD == 0) ? 1 : NSD];
  if constexpr (SHB) {
    const double *pr = D.coef_rn + (size_t)p * D.rows_rn * cp + cb * 16;
    for (int e = threadIdx.x; e < 4 * NSR * 16; e += 64 * WPB) bop[e] = pr[(size_t)(e >> 4) * cp + (e & 15)];
    const double *pd = D.coef_dm + (size_t)p * D.rows_dm * cp + cb * 16;
    for (int e = threadIdx.x; e < 4 * NSD * 16; e += 64 * WPB)
      bop[4 * NSR * 16 + e] = pd[(size_t)(e >> 4) * cp + (e & 15)];
    __syncthreads();
  } else {
    const double *pr = D.coef_rn + (size_t)p * D.rows_rn * cp + chain;
#pragma unroll
    for (int s = 0; s < NSR; ++s) cr[s] = pr[(size_t)(4 * s + q) * cp];
    if constexpr (NSD > 0) {
      const double *pd = D.coef_dm + (size_t)p * D.rows_dm * cp + chain;
#pragma unroll
      for (int s = 0; s < NSD; ++s) cd[s] = pd[(size_t)(4 * s + q) * cp];
    }
  }
  auto crs = [&](int s) -> double { return SHB ? bop[(4 * s + q) * 16 + col] : cr[SHB ? 0 : s]; };
  auto cds = [&](int s) -> double {
    return SHB ? bop[(4 * NSR + 4 * s + q) * 16 + col] : cd[(SHB || NSD == 0) ? 0 : s];
  };
  v4d ar[JTR];
  v4d ad[JTD > 0 ? JTD : 1];
#pragma unroll
  for (int t = 0; t < JTR; ++t) ar[t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < (JTD > 0 ? JTD : 1); ++t) ad[t] = v4d{0.0, 0.0, 0.0, 0.0};
  double chi = 0.0;
  pt::CwLane cwl;
  double cacc[8];
  if constexpr (CW) {
    cwl.load(D.cwc, cp, p, chain);
#pragma unroll
    for (int j = 0; j < 8; ++j) cacc[j] = 0.0;
  }
  double *ft = ftab[wv];
  const double *__restrict__ sth = D.sth;
  const double *__restrict__ cth = D.cth;
  const double *__restrict__ tau = D.tau;
  const double *__restrict__ dtp = D.dt;
  const double *__restrict__ ivn = D.invn;
  const double *__restrict__ wdm = D.wdm;

  // Per-tile inputs: forward-layout (sin, cos, tau) of TOA base + col and
  // output-layout (dt, 1/N, w, t) of TOAs base + q + 4v.
  struct TileIn {
    double s, c, t, dt[4], iv[4], w[4], tt[4];
  };
  auto load_in = [&](TileIn &in, int b) {
    in.s = sth[b + col];
    in.c = cth[b + col];
    in.t = tau[b + col];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      in.dt[v] = dtp[b + q + 4 * v];
      in.iv[v] = ivn[b + q + 4 * v];
      in.w[v] = wdm[b + q + 4 * v];
      if constexpr (CW) in.tt[v] = D.t[b + q + 4 * v];
    }
  };
  // Front of a tile: basis, forward contraction and residuals (G into gr, gd;
  // the transposed basis into ft); back: the adjoint contraction.
  double gr[4], gd[4];
  auto front = [&](const TileIn &in, int base) {
    const double s1 = in.s, c1 = in.c, tv = in.t;
    double cdt[4], civ[4], cw[4], ctt[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      cdt[v] = in.dt[v];
      civ[v] = (base + q + 4 * v < te) ? in.iv[v] : 0.0;   // rows past the chunk contribute nothing
      cw[v] = in.w[v];
      ctt[v] = in.tt[v];
    }
    // ---- forward layout: lane (col, q) walks harmonics q+1, q+5, ... of TOA base + col
    const double s2 = 2.0 * s1 * c1, c2 = (c1 - s1) * (c1 + s1);
    const double s4 = 2.0 * s2 * c2, c4 = (c2 - s2) * (c2 + s2);
    // harmonic q + 1 as base (0 or 2) plus step (1 or 2), both chosen by
    // selects: a divergent branch here would split the tile's code into
    // blocks the compiler schedules separately
    const bool upper = q >= 2, even_q = (q & 1) == 0;
    const double bs = upper ? s2 : 0.0, bc = upper ? c2 : 1.0;
    const double ss = even_q ? s1 : s2, sc = even_q ? c1 : c2;
    double sh = bs * sc + bc * ss;
    double ch = bc * sc - bs * ss;
    // ---- forward contraction R = F A, R_dm = F A_dm (16 TOA x 16 chains),
    //      each k-step issued as soon as its basis pair exists
    v4d rr = v4d{0.0, 0.0, 0.0, 0.0};
    v4d rd = v4d{0.0, 0.0, 0.0, 0.0};
    // raised wave priority while the forward's MFMAs issue: with several
    // waves per SIMD the others' loads, LDS and vector work then fill the
    // matrix core's gaps instead of delaying this chain
    __builtin_amdgcn_s_setprio(1);
    auto steps = [&](auto tail) {
      // the last TAIL steps may hold timing-model or zero columns, the others
      // hold harmonics in every lane group (TAIL 0: decided step by step)
#pragma unroll
      for (int m = 0; m < NSR / 2; ++m) {
        constexpr int TAIL = decltype(tail)::value;
        double fa, fb;
        if ((TAIL > 0 && m < NSR / 2 - TAIL) || (TAIL == 0 && 4 * m + 3 < kb)) {
          fa = sh;
          fb = ch;
        } else {                       // harmonic, timing-model column (1, tau, tau^2) or zero
          const int h = 4 * m + q;
          const double ta = (h == kb) ? 1.0 : ((h == kb + 1) ? tv * tv : 0.0);
          const double tb2 = (h == kb) ? tv : 0.0;
          fa = (h < kb) ? sh : ta;
          fb = (h < kb) ? ch : tb2;
        }
        ft[col * FS + 8 * m + q] = fa;
        ft[col * FS + 8 * m + 4 + q] = fb;
        const double sn = sh * c4 + ch * s4;
        ch = ch * c4 - sh * s4;
        sh = sn;
        rr = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, crs(2 * m), rr, 0, 0, 0);
        if (2 * m < NSD) rd = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, cds(2 * m), rd, 0, 0, 0);
        rr = __builtin_amdgcn_mfma_f64_16x16x4f64(fb, crs(2 * m + 1), rr, 0, 0, 0);
        if (2 * m + 1 < NSD) rd = __builtin_amdgcn_mfma_f64_16x16x4f64(fb, cds(2 * m + 1), rd, 0, 0, 0);
      }
    };
    // The first kb / 4 steps hold harmonics only.  With NSR = 4 ceil((kb + 2) / 8)
    // the rest is one to three steps, so the forward is always one branch-free
    // block, which lets the compiler schedule the panel loads and the
    // recurrence across steps (a branch per step keeps it from doing so).
    const int tail = NSR / 2 - kb / 4;
    if (tail == 1)
      steps(std::integral_constant<int, 1>{});
    else if (tail == 2)
      steps(std::integral_constant<int, 2>{});
    else if (tail == 3)
      steps(std::integral_constant<int, 3>{});
    else
      steps(std::integral_constant<int, 0>{});
    __builtin_amdgcn_s_setprio(0);
    wave_sync();
    // ---- residuals: lane (col, q) holds TOAs base + q + 4v, chain col
    // (v_mfma_f64_16x16x4f64 returns D[q + 4v][col] in item v of lane col + 16q)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double r = cdt[v] - rr[v] - cw[v] * rd[v];
      pt::CwToa cs;
      if constexpr (CW) {
        cs = cwl.delay(ctt[v]);
        r -= cs.h;
      }
      const double g = r * civ[v];
      chi += r * g;
      gr[v] = g;
      gd[v] = cw[v] * g;
      if constexpr (CW) cwl.adjoint(cs, g, cacc);
    }
  };
  auto back = [&]() {
    // ---- adjoint contraction: Abar += F^T G, Abar_dm += F^T (w G)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int t = 0; t < JTR; ++t) {
        const double fb = ft[(q + 4 * v) * FS + 16 * t + col];
        ar[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb, gr[v], ar[t], 0, 0, 0);
        if (t < JTD) ad[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb, gd[v], ad[t], 0, 0, 0);
      }
    }
    wave_sync();
  };

  // (the padding of the per-TOA arrays covers the load one tile past the chunk)
  int base = tb + 16 * wv;
  if constexpr (SHB) {
    // one input set, refilled for the next tile during the adjoint
    TileIn A;
    load_in(A, base);
    for (; base < te; base += 16 * WPB) {
      front(A, base);
      load_in(A, base + 16 * WPB);
      back();
    }
  } else {
    // two input sets: the next tile's inputs load into the idle one, a tile
    // ahead and with no copies between the sets
    TileIn A, B;
    load_in(A, base);
    for (;;) {
      if (base >= te) break;
      load_in(B, base + 16 * WPB);
      front(A, base);
      back();
      base += 16 * WPB;
      if (base >= te) break;
      load_in(A, base + 16 * WPB);
      front(B, base);
      back();
      base += 16 * WPB;
    }
  }

  // ---- per-wave chi^2 over the four lane groups (fixed order)
  chi += __shfl_xor(chi, 16, 64);
  chi += __shfl_xor(chi, 32, 64);
  if constexpr (CW) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      cacc[j] += __shfl_xor(cacc[j], 16, 64);
      cacc[j] += __shfl_xor(cacc[j], 32, 64);
    }
  }

  // ---- combine the waves of the block in LDS, then one partial per block
  double *pr = D.part_rn + (size_t)wg * D.rows_rn * 16;
  double *pd = D.part_dm + (size_t)wg * D.rows_dm * 16;
  if constexpr (WPB == 1) {
#pragma unroll
    for (int t = 0; t < JTR; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) pr[(16 * t + q + 4 * v) * 16 + col] = ar[t][v];
#pragma unroll
    for (int t = 0; t < JTD; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) pd[(16 * t + q + 4 * v) * 16 + col] = ad[t][v];
    if (q == 0) D.part_chi[(size_t)wg * 16 + col] = chi;
    if constexpr (CW) {
      if (q == 0) {
        double o[8];
        pt::cw_finish(D.cwc, cp, p, chain, cacc, o);
#pragma unroll
        for (int j = 0; j < 8; ++j) D.part_cw[((size_t)wg * 8 + j) * 16 + col] = o[j];
      }
    }
  } else {
    __syncthreads();
#pragma unroll
    for (int t = 0; t < JTR; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) ftab[wv][(16 * t + q + 4 * v) * 16 + col] = ar[t][v];
    if (q == 0) cred[wv][col] = chi;
    if constexpr (CW) {
      if (q == 0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) cwred[wv][j][col] = cacc[j];
      }
    }
    __syncthreads();
    if (wv == 0) {
      for (int e = lane; e < ROWS * 16; e += 64) {
        double s = ftab[0][e];
#pragma unroll
        for (int w = 1; w < WPB; ++w) s += ftab[w][e];
        pr[e] = s;
      }
      if (lane < 16) {
        double s = cred[0][lane];
#pragma unroll
        for (int w = 1; w < WPB; ++w) s += cred[w][lane];
        D.part_chi[(size_t)wg * 16 + lane] = s;
        if constexpr (CW) {
          double a[8], o[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            a[j] = cwred[0][j][lane];
#pragma unroll
            for (int w = 1; w < WPB; ++w) a[j] += cwred[w][j][lane];
          }
          pt::cw_finish(D.cwc, cp, p, cb * 16 + lane, a, o);
#pragma unroll
          for (int j = 0; j < 8; ++j) D.part_cw[((size_t)wg * 8 + j) * 16 + lane] = o[j];
        }
      }
    }
    if constexpr (JTD > 0) {
      __syncthreads();
#pragma unroll
      for (int t = 0; t < JTD; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) ftab[wv][(16 * t + q + 4 * v) * 16 + col] = ad[t][v];
      __syncthreads();
      if (wv == 0) {
        for (int e = lane; e < 16 * JTD * 16; e += 64) {
          double s = ftab[0][e];
#pragma unroll
          for (int w = 1; w < WPB; ++w) s += ftab[w][e];
          pd[e] = s;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Plain TOA pass: one launch per pulsar, one 64-lane wave per (TOA chunk,
// 16-chain block), lane = TOA, a loop over the block's chains, vector ALU only
// (no matrix cores).
// grid = (chunks of pulsar p, chain blocks), block = 64.  Per chain and 64-TOA group the lane
// forms the residual of its TOA (the basis by angle addition), then its
// contributions to the adjoint rows, 8 harmonics (16 rows of each block) at a
// time; those are summed over the 64 TOAs through an LDS transpose (lane l then
// holds row l / 2 of the group, half l % 2) and accumulated per lane over the
// chunk's TOA groups.
// LDS: the coefficient rows of the block's chains [rows_rn + rows_dm][16] and
// the transpose buffer [64 lanes][32 rows], rows padded to 33 so that the
// column reads of the sum fall on distinct banks.
// ---------------------------------------------------------------------------
constexpr int kPlainMaxGroups = 8;   // 16-row groups per block (rows <= 128)

__global__ __launch_bounds__(64) void k_toa_plain(Dev D, int p) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x;
  const int chunk = D.psr_chunk0[p] + blockIdx.x;
  const int nr = D.rows_rn, nd = D.rows_dm;
  const int gr = nr / 16, gd = nd / 16;
  double *cfb = lds;                // [nr + nd][16] coefficients of the block's chains
  double *tb = cfb + (nr + nd) * 16;   // [64][33] transpose buffer
  const size_t cp = D.c_pad;
  const int t_beg = D.chunk_begin[chunk], t_end = D.chunk_end[chunk];
  const double tc = D.tau_c[p], tsi = D.tau_sinv[p];
  const double wfac = pt::kTwoPi / D.tspan;
  const int kb = D.kb, kdm = D.nf_dm;
  const int t0 = pt::tm_row(0, kb), t1 = pt::tm_row(1, kb), t2 = pt::tm_row(2, kb);
  const int cb_row = lane >> 1, half = lane & 1;
  // the coefficient rows of the block's 16 chains (16 consecutive words per row)
  const int cb = blockIdx.y;
  for (int e = lane; e < (nr + nd) * 16; e += 64) {
    const int r = e >> 4, c16 = e & 15;
    cfb[e] = r < nr ? D.coef_rn[((size_t)p * nr + r) * cp + cb * 16 + c16]
                    : D.coef_dm[((size_t)p * nd + (r - nr)) * cp + cb * 16 + c16];
  }
  wave_sync();
  for (int col = 0; col < 16; ++col) {
    const int chain = cb * 16 + col;
    // row r of the chain at cfb[16 r + col]
    const double *cf = cfb + col;
    const bool cwon = D.has_cw;
    pt::CwLane cwl;
    if (cwon) cwl.load(D.cwc, cp, p, chain);
    double acc[2 * kPlainMaxGroups], chi = 0.0, cacc[8];
#pragma unroll
    for (int g = 0; g < 2 * kPlainMaxGroups; ++g) acc[g] = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) cacc[j] = 0.0;
    for (int i0 = t_beg; i0 < t_end; i0 += 64) {
      const int i = i0 + lane;
      const bool on = i < t_end;
      const int ii = on ? i : t_beg;
      const double t = D.t[ii];
      const int be = D.backend[ii];
      const double es = D.efac[be] * D.sigma[ii], eq = D.equad[be];
      const double N = es * es + eq * eq;
      const double w = D.dm_scale / (D.nu[ii] * D.nu[ii]);
      double s1, c1;
      sincos(wfac * t, &s1, &c1);
      const double tau = (t - tc) * tsi;
      // forward
      double R = cf[16 * t0] + tau * cf[16 * t1] + tau * tau * cf[16 * t2];
      double Rd = 0.0;
      double sk = s1, ck = c1;
      for (int k = 1; k <= kb; ++k) {
        const int rs = pt::harm_row(k, 0), rc = pt::harm_row(k, 1);
        R = fma(sk, cf[16 * rs], fma(ck, cf[16 * rc], R));
        if (k <= kdm) Rd = fma(sk, cf[16 * (nr + rs)], fma(ck, cf[16 * (nr + rc)], Rd));
        const double sn = sk * c1 + ck * s1;
        ck = ck * c1 - sk * s1;
        sk = sn;
      }
      double r = D.dt[ii] - R - w * Rd;
      pt::CwToa cs;
      if (cwon) {
        cs = cwl.delay(t);
        r -= cs.h;
      }
      const double g = on ? r / N : 0.0;
      chi = fma(r, g, chi);
      if (cwon && on) cwl.adjoint(cs, g, cacc);
      const double wg = w * g;
      // adjoint rows, 8 harmonics (16 rows per block) per group
      sk = s1;
      ck = c1;
      const int ng = gr > gd ? gr : gd;
#pragma unroll
      for (int grp = 0; grp < kPlainMaxGroups; ++grp) {
        if (grp >= ng) break;
        double hs[8], hc[8];
#pragma unroll
        for (int h = 0; h < 8; ++h) {
          hs[h] = sk;
          hc[h] = ck;
          const double sn = sk * c1 + ck * s1;
          ck = ck * c1 - sk * s1;
          sk = sn;
        }
        // the lane's 16 red-noise and 16 DM contributions of this group
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int row = 16 * grp + j;
          const int q = j & 3, sc = (j >> 2) & 1, mloc = j >> 3, hl = 4 * mloc + q;
          double vr = 0.0, vd = 0.0;
          if (grp < gr) {
            const pt::Slot sl = pt::rn_slot(row, kb);
            if (sl.kind == 0) vr = (sc ? hc[hl] : hs[hl]) * g;
            else if (sl.kind == 1) vr = (sl.tm == 0 ? 1.0 : (sl.tm == 1 ? tau : tau * tau)) * g;
          }
          if (grp < gd) {
            const pt::Slot sl = pt::dm_slot(row, kdm);
            if (sl.kind == 0) vd = (sc ? hc[hl] : hs[hl]) * wg;
          }
          tb[lane * 33 + j] = vr;
          tb[lane * 33 + 16 + j] = vd;
        }
        wave_sync();
        double sum = 0.0;
        const double *src = tb + 32 * half * 33 + cb_row;
#pragma unroll
        for (int l = 0; l < 32; ++l) sum += src[33 * l];
        sum += __shfl_xor(sum, 1, 64);
        wave_sync();
        if (cb_row < 16) {
          if (grp < gr) acc[grp] += sum;
        } else if (grp < gd) {
          acc[kPlainMaxGroups + grp] += sum;
        }
      }
    }
    // chi^2 and the CW sums over the chunk's TOAs
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) chi += __shfl_xor(chi, o, 64);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) cacc[j] += __shfl_xor(cacc[j], o, 64);
    }
    const size_t wg = (size_t)chunk * D.n_cb + cb;
    if (half == 0) {
      const int j = cb_row & 15;
#pragma unroll
      for (int grp = 0; grp < kPlainMaxGroups; ++grp) {
        if (cb_row < 16 && grp < gr) D.part_rn[(wg * nr + 16 * grp + j) * 16 + col] = acc[grp];
        if (cb_row >= 16 && grp < gd) D.part_dm[(wg * nd + 16 * grp + j) * 16 + col] = acc[kPlainMaxGroups + grp];
      }
    }
    if (lane == 0) {
      D.part_chi[wg * 16 + col] = chi;
      if (cwon) {
        double o[8];
        pt::cw_finish(D.cwc, cp, p, chain, cacc, o);
        for (int j = 0; j < 8; ++j) D.part_cw[(wg * 8 + j) * 16 + col] = o[j];
      }
    }
  }
}

// Sum of n strided values in index order, eight loads in flight at a time.
__device__ inline double sum_chunks(const double *src, size_t stride, int n) {
  double s = 0.0;
  for (int c0 = 0; c0 < n; c0 += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = (c0 + k < n) ? src[(size_t)(c0 + k) * stride] : 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
  }
  return s;
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of chunk partials into per-pulsar panels.
// grid = (n_psr, n_cb, row blocks of 256 elements), block = 256.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce(Dev D) {
  const int p = blockIdx.x, cb = blockIdx.y;
  const int c0 = D.psr_chunk0[p], c1 = D.psr_chunk0[p + 1];
  const int nr = D.rows_rn, nd = D.rows_dm;
  const size_t cp = D.c_pad;
  const size_t ncb = D.n_cb;
  const int e = blockIdx.z * 256 + threadIdx.x;
  const int ncw = D.has_cw ? 8 : 0;
  if (e < (nr + nd + ncw) * 16) {
    const int row = e >> 4, col = e & 15;
    if (row >= nr + nd) {
      const int e3 = e - (nr + nd) * 16, j = row - nr - nd;
      const double *src = D.part_cw + ((size_t)c0 * ncb + cb) * 8 * 16 + e3;
      D.cw_p[((size_t)p * 8 + j) * cp + cb * 16 + col] = sum_chunks(src, ncb * 8 * 16, c1 - c0);
    } else if (row < nr) {
      const double *src = D.part_rn + ((size_t)c0 * ncb + cb) * nr * 16 + e;
      D.bar_rn[((size_t)p * nr + row) * cp + cb * 16 + col] = sum_chunks(src, ncb * nr * 16, c1 - c0);
    } else {
      const int e2 = e - nr * 16, r2 = row - nr;
      const double *src = D.part_dm + ((size_t)c0 * ncb + cb) * nd * 16 + e2;
      D.bar_dm[((size_t)p * nd + r2) * cp + cb * 16 + col] = sum_chunks(src, ncb * nd * 16, c1 - c0);
    }
  }
  if (blockIdx.z == 0 && threadIdx.x < 16) {
    D.chi_p[(size_t)p * cp + cb * 16 + threadIdx.x] =
        sum_chunks(D.part_chi + ((size_t)c0 * ncb + cb) * 16 + threadIdx.x, ncb * 16, c1 - c0);
  }
}

template <int JTR, int JTD, int WPB>
hipError_t launch_mfma_t(const Dev &D, int xcd, hipStream_t s) {
  const int grid = D.n_chunks * D.n_cb;
  if (D.has_cw)
    hipLaunchKernelGGL((k_toa_mfma<JTR, JTD, WPB, true>), dim3(grid), dim3(64 * WPB), 0, s, D, xcd);
  else
    hipLaunchKernelGGL((k_toa_mfma<JTR, JTD, WPB, false>), dim3(grid), dim3(64 * WPB), 0, s, D, xcd);
  return hipGetLastError();
}

template <int JTR, int WPB>
hipError_t launch_mfma_d(const Dev &D, int xcd, hipStream_t s) {
  switch (D.jt_dm) {
    case 0: return launch_mfma_t<JTR, 0, WPB>(D, xcd, s);
    case 1: if constexpr (JTR >= 1) return launch_mfma_t<JTR, 1, WPB>(D, xcd, s); break;
    case 2: if constexpr (JTR >= 2) return launch_mfma_t<JTR, 2, WPB>(D, xcd, s); break;
    case 3: if constexpr (JTR >= 3) return launch_mfma_t<JTR, 3, WPB>(D, xcd, s); break;
    case 4: if constexpr (JTR >= 4) return launch_mfma_t<JTR, 4, WPB>(D, xcd, s); break;
  }
  return hipErrorInvalidValue;
}

template <int WPB>
hipError_t launch_mfma_r(const Dev &D, int xcd, hipStream_t s) {
  switch (D.jt_rn) {
    case 1: return launch_mfma_d<1, WPB>(D, xcd, s);
    case 2: return launch_mfma_d<2, WPB>(D, xcd, s);
    case 3: return launch_mfma_d<3, WPB>(D, xcd, s);
    case 4: return launch_mfma_d<4, WPB>(D, xcd, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

namespace ptk {

hipError_t launch_toa_mfma(const pt::Dev &D, int wpb, int xcd, hipStream_t s) {
  if (D.n_chunks == 0 || D.n_cb == 0) return hipSuccess;
  switch (wpb) {
    case 1: return launch_mfma_r<1>(D, xcd, s);
    case 2: return launch_mfma_r<2>(D, xcd, s);
    case 4: return launch_mfma_r<4>(D, xcd, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_toa_plain_psr(const pt::Dev &D, int p, int n_chunks_p, hipStream_t s) {
  if (D.rows_rn > 16 * kPlainMaxGroups || D.rows_dm > 16 * kPlainMaxGroups || D.rows_rn % 16 ||
      D.rows_dm % 16)
    return hipErrorInvalidValue;
  const size_t lds = (size_t)((D.rows_rn + D.rows_dm) * 16 + 64 * 33) * sizeof(double);
  hipLaunchKernelGGL(k_toa_plain, dim3(n_chunks_p, D.n_cb), dim3(64), lds, s, D, p);
  return hipGetLastError();
}

hipError_t launch_reduce_chunks(const pt::Dev &D, hipStream_t s) {
  if (D.n_psr == 0 || D.n_cb == 0) return hipSuccess;
  const int nz = ((D.rows_rn + D.rows_dm + (D.has_cw ? 8 : 0)) * 16 + 255) / 256;
  hipLaunchKernelGGL(k_reduce, dim3(D.n_psr, D.n_cb, nz), dim3(256), 0, s, D);
  return hipGetLastError();
}

hipError_t set_plain_lds_limit(size_t bytes) {
  return hipFuncSetAttribute((const void *)k_toa_plain, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace ptk
