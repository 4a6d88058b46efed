"""MI355X (gfx950) fused subdomain training step for domain-decomposed PINN
flow reconstruction (arXiv 2602.15883).

The compute path is libddpinn.so (hand-written HIP kernels behind the C ABI
in include/ddpinn.h); this package is its thin Python binding.  Importing the
package does not touch the GPU; creating a Context does, and fails loudly if
the library is not built or no GPU is visible.
"""
from .abi import (PINN_CHECK_FINITE, PINN_NO_UPDATE, PINN_PER_SUBDOMAIN, PinnError,  # noqa: F401
                  lib, num_params)

__all__ = ["Context", "SubTensors", "context_from_problem", "subdomain_to_device", "PinnError",
           "lib", "num_params"]


def __getattr__(name):
    if name in ("Context", "SubTensors", "context_from_problem", "subdomain_to_device"):
        from . import context
        return getattr(context, name)
    raise AttributeError(name)
