"""FP64 CPU oracle of iterative Marchenko redatuming (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The library and its Python binding never do: the HIP
path and this oracle share no code.
"""

from .marchenko import (  # noqa: F401
    SynthesisOperator,
    marchenko,
    mute_window,
    apply_mute,
    rev,
    signed_time,
    rel_l2,
)
from .imaging import double_focused, image  # noqa: F401,E402
