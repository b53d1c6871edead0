"""MI355X-native Matsubara-time GW hot path (arXiv:1602.02313).

``Context`` is the thin ctypes binding of the C ABI in ``include/matsgw.h``
(libmatsgw.so, HIP kernels for gfx950); ``GWRun`` sequences the calls of one
G0W0 / GW0 / scGW run on one GPU.
"""
from ._lib import (BF16X3, BOSON, C64, C128, EHIP, EINVAL, ENOMEM, ENOTSUP, ESHAPE, EXPORTS,  # noqa: F401
                   F16X3, FERMION, FLAG_NAN, FLAG_NOBRACKET, FLAG_NOCONV, FLAG_SINGULAR, FP32, FP64,
                   LIB_PATH, MU_FIXED, MU_SEARCH, OK, OP_POLARIZATION, OP_SELF_ENERGY, SIGMA_DIAG,
                   SIGMA_FULL, TS_DYSON, TS_WTILDE, Context, MsgwError, load_library)
from .driver import GWRun, HostM, ResidentM, SynthCubicM, SynthM  # noqa: F401
