"""MI355X (gfx950) particle-filter likelihoods for stochastic reaction networks.

The compute path is liblik.so (HIP kernels behind a C ABI, see include/lik.h);
`lik` is its ctypes binding.  `workloads` builds seeded synthetic inputs.
"""
