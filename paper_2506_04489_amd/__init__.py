"""MI355X-native super-potential Gaussian-sum FFT solver for the 3D free-space
Poisson equation (C ABI in include/psp.h, HIP kernels in csrc/)."""
from .psp import Plan, Server, PspError, solve_batched, lib, PSP_F32, PSP_F64  # noqa: F401
