"""MI355X-native hot path of neural radiance caching (Mueller et al., arXiv 2106.12372).

The computation lives in the HIP library libnrc.so (C ABI: include/nrc.h);
``nrc`` is its Python binding and ``autograd`` wraps the fused
forward/backward kernels as a torch.autograd.Function.
"""
from . import nrc  # noqa: F401  (fails loudly if libnrc.so is missing)
