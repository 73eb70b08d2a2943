"""MI355X-native synthesis step of iterative (Neumann-series) 2D Marchenko redatuming.

The work is done by hand-written HIP kernels in ``libmk.so`` behind the C ABI
of ``include/mk.h``; ``paper_2106_04649_amd.mk`` is the ctypes binding.
"""

from .mk import (  # noqa: F401
    FIELDS,
    MKError,
    MK_F1MINUS,
    MK_F1PLUS,
    MK_FLAG_GRAPH,
    MK_FLAG_PROFILE,
    MK_FLAG_AUTOTUNE,
    MK_GMINUS,
    MK_GPLUS,
    MK_R_BF16S,
    MK_R_C64,
    MK_R_F16S,
    Plan,
    load_library,
    mk_destroy,
    mk_get,
    mk_iterate,
    mk_load_R,
    mk_passes,
    mk_plan,
    mk_profile,
    mk_set_focal,
    mk_tune,
    mk_contract_variant,
)
