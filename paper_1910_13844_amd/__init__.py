"""MI355X-native Lippmann-Schwinger forward model, far field and gradient (arXiv 1910.13844).

The computation lives in libls.so (HIP kernels for gfx950 behind the C ABI in include/ls.h);
``api`` is a thin PyTorch/ctypes binding with the same names, ``workloads`` the seeded input
generators, ``autograd`` a torch.autograd.Function over ls_forward/ls_farfield/ls_vjp and
``serve`` a continuous-batching request loop over the slot API.
"""
__all__ = ["api", "workloads"]
