"""lfft: lattice FFT and fast lattice wavelet decomposition on AMD MI355X.

The compute path is liblfft.so (host integer planner + gfx950 HIP kernels);
this package only marshals arguments to its C ABI (include/lfft.h).
"""
from .lfft import LatticePlan, WaveletPlan, forward, inverse, get_plan, lib, strerror  # noqa: F401
