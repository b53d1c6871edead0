"""MI355X-native Matsubara-time GW hot path (arXiv:1602.02313).

``Context`` is the thin ctypes binding of the C ABI in ``include/matsgw.h``
(libmatsgw.so, HIP kernels for gfx950); ``GWRun`` sequences the calls of one
G0W0 / GW0 / scGW run on one GPU.
"""
from ._lib import (BF16X3, BOSON, C64, C128, EXPORTS, FERMION, FP32, FP64, LIB_PATH,  # noqa: F401
                   MU_FIXED, MU_SEARCH, OP_POLARIZATION, OP_SELF_ENERGY, SIGMA_DIAG, SIGMA_FULL,
                   Context, MsgwError, load_library)
from .driver import GWRun, HostM, ResidentM, SynthM  # noqa: F401
