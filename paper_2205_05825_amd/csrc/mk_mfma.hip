// Int8-MFMA blind rotation (K3).  Placeholder until the kernel lands.
#include "mk_device_common.h"

namespace mk {

int mfma_upload(mk_ctx *, const std::vector<uint32_t> &, hipStream_t) { return MK_OK; }

int launch_br_mfma(mk_ctx *, const uint32_t *, uint32_t *, size_t, int, hipStream_t) {
    return fail(MK_EINVAL, "int8-MFMA path not built yet");
}

}  // namespace mk
