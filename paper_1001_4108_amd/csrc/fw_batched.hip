// Batched solves (placeholder until the persistent kernel lands).
#include "../../include/fwapsp.h"
#include "fw_internal.h"

extern "C" int fw_apsp_batched(void *const *, const int64_t *, const int64_t *, int64_t count,
                               int, int32_t *const *, const int64_t *, void *) {
    return count == 0 ? FW_OK : FW_ERR_UNSUPPORTED;
}

extern "C" int64_t fw_batched_max_n(int, int) { return 0; }
