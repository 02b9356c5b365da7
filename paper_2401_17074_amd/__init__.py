"""MI355X-native moment-only high-order thread-safe lattice Boltzmann update.

The solver is the C-ABI library ``libtslb.so`` (hand-written HIP for gfx950,
declared in include/tslb.h); this package binds it with ctypes and adds a
thin object wrapper and a ``torch.autograd.Function`` over the checkpointed
discrete adjoint.  torch provides device memory and streams only.
"""
from . import _binding as capi  # noqa: F401  (raises ImportError if the library is not built)
from ._binding import (TSLB_BF16, TSLB_D3Q27, TSLB_DEVICE, TSLB_FP16, TSLB_FP32, TSLB_INLET,  # noqa: F401
                       TSLB_OUTLET, TSLB_PERIODIC, TSLB_RHO_DEVIATION, TSLB_WALL, TslbError)
from .solver import Solver, TslbRollout  # noqa: F401
