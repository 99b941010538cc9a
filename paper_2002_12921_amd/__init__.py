"""MI355X (gfx950) Vegas iteration: HIP kernels behind a C ABI (include/vegas.h).

Modules:
  _lib        ctypes loader of libvegas_gfx950.so (raises if it is not built)
  integrator  Vegas: one integration context (workspace = a torch uint8 tensor)
  autograd    VegasIntegral: torch.autograd.Function over the adjoint kernel
  batch       VegasBatch: many independent integrals in one graph launch
  workloads   seeded synthetic problem specifications (inputs only)
  build       hipcc build of the library
"""
from ._lib import VegasError, lib  # noqa: F401
from .integrator import Vegas, compile_user  # noqa: F401
