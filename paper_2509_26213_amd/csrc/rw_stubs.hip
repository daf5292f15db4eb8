// Temporary entry points for the parts of the ABI still being written.
#include "rw_internal.h"
#include "rw_kernels.h"
using namespace rw;
extern "C" {
rw_status rw_downsample(rw_context*, const rw_volume*, const uint8_t*, float*, uint8_t*, void*) {
    return RW_ERR_UNSUPPORTED;
}
rw_status rw_classify_bricks(rw_context*, const float*, rw_dims, int32_t, int32_t, const uint8_t*,
                             rw_dims, const int32_t*, const int32_t*, double, double, rw_brick*,
                             int32_t, int32_t*, int32_t*, void*) {
    return RW_ERR_UNSUPPORTED;
}
size_t rw_bricks_workspace_bytes(const rw_brick*, int32_t, int32_t, int32_t, int32_t) { return 0; }
rw_status rw_solve_bricks(rw_context*, const rw_volume*, const rw_seeds*, const float*, rw_dims,
                          int32_t, const rw_brick*, int32_t, const rw_options*, float*, int32_t*,
                          void*, size_t, rw_stats*, void*) {
    return RW_ERR_UNSUPPORTED;
}
rw_status rw_fill_bricks(rw_context*, const float*, rw_dims, int32_t, int32_t, const uint8_t*,
                         rw_dims, const rw_brick*, int32_t, float*, void*) {
    return RW_ERR_UNSUPPORTED;
}
}
