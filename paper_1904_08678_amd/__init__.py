"""wcmg: Wilson-clover multigrid on AMD MI355X (gfx950).

The arithmetic lives in the HIP library ``libwcmg.so`` (C ABI in
``include/wcmg.h``); this package only marshals torch device tensors and the
current HIP stream into those calls.  There is no CPU fallback: without the
built library every call raises.
"""
from .wcmg import (  # noqa: F401
    F64, F32, BF16, Context, CoarseOperator, Network, WcmgError, coarse_apply_ragged, coarse_time_ragged,
    default_params, lib, library_path, solve_ragged, close_all,
)
