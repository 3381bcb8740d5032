// Per-chain kernels of the spectral side that need no dense factorisation:
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
#include "spec_dev.h"

namespace {

// grid (c_pad, segments), block 256
__global__ __launch_bounds__(256) void k_spec_fwd(pt::Dev D, const double *__restrict__ x) {
  pt::spec_fwd_block(D, x, blockIdx.x, blockIdx.y, blockIdx.y, pt::kSpecSeg);
}

// grid (n_chains, segments), block 256
__global__ __launch_bounds__(256) void k_spec_bwd(pt::Dev D, const double *__restrict__ x,
                                                  double *__restrict__ grad) {
  pt::spec_bwd_block(D, x, grad, blockIdx.x, blockIdx.y, pt::kSpecSeg, blockIdx.y);
}

}  // namespace

namespace ptk {

hipError_t launch_spec_fwd(const pt::Dev &D, const double *x, hipStream_t s) {
  const int kmax = max(D.ka, D.nf_dm);
  const int nseg = max(1, min(pt::kSpecSeg, kmax));
  if (D.c_pad == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spec_fwd, dim3(D.c_pad, nseg), dim3(256), 0, s, D, x);
  return hipGetLastError();
}

hipError_t launch_spec_bwd(const pt::Dev &D, const double *x, double *grad, hipStream_t s) {
  if (D.n_chains == 0) return hipSuccess;
  const int kmax = max(D.ka, D.nf_dm);
  const int nseg = max(1, min(pt::kSpecSeg, kmax));
  hipLaunchKernelGGL(k_spec_bwd, dim3(D.n_chains, nseg), dim3(256), 0, s, D, x, grad);
  return hipGetLastError();
}

}  // namespace ptk
