"""CPU oracle for the Fourier-space PTA log-posterior and its gradient.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: it is used by ``tests/``, by ``__graft_entry__.smoke()``
(to check the GPU result) and by the ``cpu_baseline`` leg of ``bench.py``.
It shares no code with the HIP library: it is a plain, slow NumPy/SciPy FP64
transcription of the paper's definitions, written to be checked by eye.

Modules
-------
model   log p and its hand-derived gradient (Eqs. likelihood, prior_cov, HD,
        power_law, a_prior with the whitening a = L z), plus the per-element
        magnitude companions used as tolerance floors.
cw      continuous-wave Earth-term delay and its parameter derivatives
        (Eqs. phase_evolve, CW_evolve).
dense   structurally different forms used as pins: the Gram (compressed)
        likelihood of Eq. posterior_implemented, the dense time-domain
        Gaussian marginal, the dense-phi whitened-prior identity.
philox  Philox4x32-10 counter-based generator (Salmon et al., SC'11).
hmc     fixed-step leapfrog HMC with Metropolis-Hastings accept (App. A).
std     the paper's standardized posterior: timing model marginalised
        (Eq. Gmatrix_proj), CURN standardizing transform a = a_hat + L z
        (Eqs. PTA_standard_transform_curn, standardized_stochastic_posterior),
        tempered likelihood (App. B), power-law or free spectra; PyTorch CPU
        FP64 with autograd for the gradient.
simulate  residuals drawn from the model (for tests that want them).
"""
