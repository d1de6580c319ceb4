"""MI355X-native FK-table convolution (DIS and hadronic observables, their
adjoint and an FP64 chi2) behind a C-ABI library of hand-written HIP
kernels for gfx950."""
