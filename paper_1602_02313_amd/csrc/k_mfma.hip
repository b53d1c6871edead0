// Mixed-precision contractions on the matrix cores (placeholder until the MFMA kernels land).
#include "internal.h"

namespace msgw {

size_t mfma_scratch_bytes(const Host&, int) { return 0; }

int launch_pol_mfma(const Dev&, const Host&, hipStream_t, int, int, const void*, const double*, int,
                    void*) {
    return MSGW_ENOTSUP;
}

int launch_sig_mfma(const Dev&, const Host&, hipStream_t, int, int, const void*, const double*,
                    const void*, int, void*) {
    return MSGW_ENOTSUP;
}

}  // namespace msgw
