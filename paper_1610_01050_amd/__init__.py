"""MI355X-native RSFT: batched, fused high-dimensional sparse FFT detection.

The compute path is the HIP library librsft.so (C ABI in include/rsft.h);
this package is its thin ctypes binding. Loading fails loudly when the
library has not been built.
"""

from .binding import (  # noqa: F401
    DETECTION_DTYPE, OPT_ESTIMATE_WORKERS, OPT_GRAPH, OPT_TIMING, OPT_VOTE_WORDS,
    OPT_DFT_SPLIT, OPT_DFT_THREADS, STAGES, SYMBOLS, Plan, RsftError,
    chebyshev_window, design_thresholds, draw_sigma, flat_window, load_library, mod_inverse,
    stage1_probability,
)
