"""MI355X (gfx950) on-the-fly multiple-tau correlator.

The per-step update of the multiple-tau correlator of the DL_POLY 5 paper
(Section 2.2; Appendix D, Algorithms 1 and 2), the k-space density producer
(Section "Currents") and the Green-Kubo readout (Section 2.3), implemented as
hand-written HIP kernels behind the C ABI of ``include/corr.h``.  This package
is the thin Python binding (``corr.Correlator``) and the build script.
"""
from .corr import (CorrError, Correlator, GroupDesc, Tuning, EXPORTS, LIB_PATH,  # noqa: F401
                   autotune, lib)
