"""libpifcm: the IFCM iteration of 3DPIFCM (arXiv 2002.01981) on MI355X.

The computation lives in libpifcm.so (HIP kernels for gfx950 behind the C ABI
of include/pifcm.h); this package is its thin Python binding.
"""
from .abi import (  # noqa: F401
    Context,
    Params,
    PifcmError,
    PIFCM_SWARM_BATCHED,
    PIFCM_SWARM_PLAIN,
    PIFCM_Q2_SQDIST,
    PIFCM_SHELL_SQDIST,
    load_library,
    header_symbols,
)
from .pipeline import ifcm_objective, refine, segment  # noqa: F401,E402
