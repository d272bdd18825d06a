"""MI355X (gfx950) time-ordered-data simulator for KID integral-field
spectrometers (arXiv 2604.23305, section 2): HIP kernels behind the gtod
C-ABI (include/gtod.h), with a thin ctypes binding."""
from .binding import (GtodError, Outputs, ScenarioRun, abi_sizes,  # noqa
                      convolve_screen, convolve_source, counters, far_field,
                      free, load_filters, load_screen, memory,
                      philox, profile_enable, profile_read, release_stream,
                      sim_init,
                      reduce, simulate_to_disk, simulate_tod,
                      simulate_tod_noalloc, skydip,
                      spec_nep2_ref)
from ._abi import (PREC_FP32, PREC_SPLIT_BF16, OBJ_CTX, OBJ_SCREEN,  # noqa
                   OBJ_SPEC, LIB_PATH)
