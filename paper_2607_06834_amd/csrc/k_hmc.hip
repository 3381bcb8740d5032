// Fixed-step leapfrog HMC pieces (App. A: Eqs. Hamiltonian, Hamilton's_eq,
// Gaussian_momentum, HMC_acceptance) with a diagonal inverse mass.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten
// rounds of two 32x32->64-bit multiplications by fixed constants with the
// high halves xor-ed into the other counter words and the key, the key
// advanced by two Weyl increments between rounds.  Normals by Box-Muller.
#include "common.h"

namespace {

constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;

__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint32_t lo0 = kM0 * c[0], hi0 = __umulhi(kM0, c[0]);
    const uint32_t lo1 = kM1 * c[2], hi1 = __umulhi(kM1, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ inline double u53(uint32_t a, uint32_t b) {
  return (double)(((uint64_t)a << 21) | (uint64_t)(b >> 11));
}

// one workgroup of kHmcT threads per chain
constexpr int kHmcT = 1024;
constexpr int kHmcW = kHmcT / 64;

// grid = n_chains, block = kHmcT
__global__ __launch_bounds__(kHmcT) void k_hmc_begin(int d, double eps, const double *inv_mass,
                                                   uint64_t seed, const uint64_t *traj, double *x,
                                                   const double *logp, const double *grad,
                                                   double *p, double *x0, double *lp0, double *g0,
                                                   double *h0) {
  __shared__ double red[kHmcW];
  const int c = blockIdx.x, wg = blockIdx.y;   // chain, and which of its kHmcBeginG workgroups
  const uint32_t j = (uint32_t)(*traj);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const size_t off = (size_t)c * d;
  double kin = 0.0;
  const int npair = (d + 1) / 2;
  // the chain's pairs are dealt to its workgroups' threads (tg of TG); kB
  // pairs per thread per batch, their loads issued before the first use
  // (the pairs are independent; a plain loop would wait for each in turn)
  constexpr int kB = 3, TG = kHmcT * pt::kHmcBeginG;
  const int tg = wg * kHmcT + (int)threadIdx.x;
  for (int m0 = tg; m0 < npair; m0 += TG * kB) {
    double xv[kB][2], gv[kB][2], iv[kB][2];
#pragma unroll
    for (int b = 0; b < kB; ++b)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = 2 * (m0 + TG * b) + h;
        const bool in = i < d;
        xv[b][h] = in ? x[off + i] : 0.0;
        gv[b][h] = in ? grad[off + i] : 0.0;
        iv[b][h] = (in && inv_mass) ? inv_mass[i] : 1.0;
      }
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const int m = m0 + TG * b;
      if (m >= npair) continue;
      uint32_t ctr[4] = {(uint32_t)m, (uint32_t)c, j, 0u};
      philox10(ctr, k0, k1);
      const double u1 = (u53(ctr[0], ctr[1]) + 1.0) * 0x1.0p-53;
      const double u2 = u53(ctr[2], ctr[3]) * 0x1.0p-53;
      const double rad = sqrt(-2.0 * log(u1));
      double sn, cs;
      sincos(pt::kTwoPi * u2, &sn, &cs);
      const double nz[2] = {rad * cs, rad * sn};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = 2 * m + h;
        if (i >= d) break;
        const double im = iv[b][h];
        double pi = im > 0.0 ? nz[h] / sqrt(im) : 0.0;
        kin += 0.5 * im * pi * pi;
        const double xi = xv[b][h], gi = gv[b][h];
        x0[off + i] = xi;
        g0[off + i] = gi;
        pi += 0.5 * eps * gi;                  // half kick
        x[off + i] = xi + eps * im * pi;       // first drift
        p[off + i] = pi;
      }
    }
  }
  kin = pt::block_sum<kHmcW>(kin, red);
  if (threadIdx.x == 0) {
    if (wg == 0) lp0[c] = logp[c];
    h0[(size_t)c * pt::kHmcBeginG + wg] = kin;   // partial kinetic energy
  }
}

// final half kick, H1, accept / restore, optional sample
__global__ __launch_bounds__(kHmcT) void k_hmc_end(int d, double eps, const double *inv_mass,
                                                 uint64_t seed, const uint64_t *traj, int n_chains, double *x, double *logp, double *grad,
                                                 double *p, const double *x0, const double *lp0,
                                                 const double *g0, const double *h0,
                                                 int64_t *n_accept, double *samples,
                                                 const int32_t *status, int64_t *n_invalid) {
  __shared__ double red[kHmcW];
  __shared__ int acc_s;
  const int c = blockIdx.x;
  const uint64_t jj = traj[0];      // trajectory number; traj[1] = first of this run
  const uint32_t j = (uint32_t)jj;
  const size_t off = (size_t)c * d;
  // the accept test's inputs other than the kinetic energy, on thread 0
  // before the sum (its loads and the uniform draw overlap the loop)
  int st_c = 0;
  double lp_c = 0.0, lp0_c = 0.0, H0 = 0.0, log_u = 0.0;
  if (threadIdx.x == 0) {
    st_c = status[c];
    lp_c = logp[c];
    double kin0 = 0.0;
    for (int g = 0; g < pt::kHmcBeginG; ++g) kin0 += h0[(size_t)c * pt::kHmcBeginG + g];
    lp0_c = lp0[c];
    H0 = -lp0_c + kin0;
    uint32_t ctr[4] = {0u, (uint32_t)c, j, 1u};
    philox10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
    log_u = log((u53(ctr[0], ctr[1]) + 1.0) * 0x1.0p-53);
  }
  // kB elements per thread per batch, their loads issued together (one
  // pass up to 12288 parameters)
  constexpr int kB = 12;
  double kin = 0.0;
  for (int i0 = threadIdx.x; i0 < d; i0 += kHmcT * kB) {
    double pv[kB], gv[kB], iv[kB];
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const int i = i0 + kHmcT * b;
      const bool in = i < d;
      pv[b] = in ? p[off + i] : 0.0;
      gv[b] = in ? grad[off + i] : 0.0;
      iv[b] = (in && inv_mass) ? inv_mass[i] : 1.0;
    }
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      if (i0 + kHmcT * b >= d) continue;
      const double pi = pv[b] + 0.5 * eps * gv[b];
      kin += 0.5 * iv[b] * pi * pi;
    }
  }
  kin = pt::block_sum<kHmcW>(kin, red);
  if (threadIdx.x == 0) {
    if (n_invalid && st_c != 0) n_invalid[c] += 1;
    const double H1 = -lp_c + kin;
    const int a = (isfinite(H1) && log_u < H0 - H1) ? 1 : 0;
    acc_s = a;
    if (a) n_accept[c] += 1;
    else logp[c] = lp0_c;
  }
  __syncthreads();
  const int a = acc_s;
  double *smp = samples ? samples + ((size_t)(jj - traj[1]) * n_chains + c) * d : nullptr;
  for (int i0 = threadIdx.x; i0 < d; i0 += kHmcT * kB) {
    double xv[kB], gv[kB];
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const int i = i0 + kHmcT * b;
      const bool in = i < d;
      xv[b] = in ? (a ? x[off + i] : x0[off + i]) : 0.0;
      gv[b] = (in && !a) ? g0[off + i] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const int i = i0 + kHmcT * b;
      if (i >= d) continue;
      if (!a) {
        x[off + i] = xv[b];
        grad[off + i] = gv[b];
      }
      if (smp) smp[i] = xv[b];
    }
  }
}

__global__ void k_traj_inc(uint64_t *traj) { traj[0] += 1; }

// start of a run: trajectory counter and the number of its first trajectory
__global__ void k_traj_set(uint64_t *traj, uint64_t traj0) {
  traj[0] = traj0;
  traj[1] = traj0;
}

}  // namespace

namespace ptk {

hipError_t launch_hmc_begin(const pt::Dev &D, int d, double eps, const double *inv_mass,
                            uint64_t seed, const uint64_t *traj, double *x, const double *logp,
                            const double *grad, double *p, double *x0, double *lp0, double *g0,
                            double *h0, hipStream_t s) {
  hipLaunchKernelGGL(k_hmc_begin, dim3(D.n_chains, pt::kHmcBeginG), dim3(kHmcT), 0, s, d, eps, inv_mass, seed, traj,
                     x, logp, grad, p, x0, lp0, g0, h0);
  return hipGetLastError();
}

hipError_t launch_hmc_end(int n_chains, int d, double eps, const double *inv_mass, uint64_t seed,
                          const uint64_t *traj, double *x, double *logp,
                          double *grad, double *p, const double *x0, const double *lp0,
                          const double *g0, const double *h0, int64_t *n_accept, double *samples,
                          const int32_t *status, int64_t *n_invalid, hipStream_t s) {
  hipLaunchKernelGGL(k_hmc_end, dim3(n_chains), dim3(kHmcT), 0, s, d, eps, inv_mass, seed, traj,
                     n_chains, x, logp, grad, p, x0, lp0, g0, h0, n_accept, samples, status,
                     n_invalid);
  return hipGetLastError();
}

hipError_t launch_traj_inc(uint64_t *traj, hipStream_t s) {
  hipLaunchKernelGGL(k_traj_inc, dim3(1), dim3(1), 0, s, traj);
  return hipGetLastError();
}

hipError_t launch_traj_set(uint64_t *traj, uint64_t traj0, hipStream_t s) {
  hipLaunchKernelGGL(k_traj_set, dim3(1), dim3(1), 0, s, traj, traj0);
  return hipGetLastError();
}

}  // namespace ptk
