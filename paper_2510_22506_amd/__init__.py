"""MI355X-native trace-regularized FCTN tensor completion (PAM).

The compute path is libfctn.so (hand-written HIP for gfx950, C ABI in
include/fctn.h); ``fctn`` is its ctypes binding, ``serve`` a request loop on
top of it and ``schedule`` the rank-increasing driver.
"""

from .fctn import (  # noqa: F401
    Plan, Server, FctnError, make_desc, fctn_workspace_bytes, fctn_mode_sizes, fctn_status_str,
    sweep_many, factor_shape, lib, LIB_PATH,
)
from . import serve  # noqa: F401
from .schedule import complete_rank_increasing  # noqa: F401
