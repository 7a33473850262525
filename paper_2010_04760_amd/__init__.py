"""WENO5 / SSP-RK3 Teukolsky solver for AMD Instinct MI355X (gfx950).

The solver is the HIP library libteuk.so (C ABI in include/teuk.h); this
package is its thin Python binding.  See ``Solver`` and the ``teuk_*``
functions, which carry the C names.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import (EXPORTED, LIB_PATH, Group, Solver, TeukError, make_config, teuk_config,  # noqa: F401
                       teuk_device_ctx, teuk_group_info_t, teuk_group_tune_info_t, teuk_info_t, teuk_tune_info_t)
