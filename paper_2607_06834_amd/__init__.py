"""MI355X-native Fourier-space PTA log-posterior and gradient (libptafs).

The HIP library (``libptafs.so``, C ABI in ``include/ptafs.h``) computes the
batched whitened log-posterior of a pulsar timing array and its gradient and
runs fixed-step HMC on it; ``paper_2607_06834_amd.api`` is its Python binding.
"""
