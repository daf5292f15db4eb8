// Whole-volume time series solves of float data in mixed precision (float32 CG).
#include "rw_solve_impl.h"

namespace rw {

rw_status whole4_f32_f32(int R, rw_context* ctx, const rw_volume* vol, const uint8_t* lab,
                         const rw_options* o, int lab0, const double* x0, const GroupBuffers& B,
                         void* prob, rw_stats* st, int rb, int* worst, int tz) {
    return dispatch_r<float, float, true>(R, ctx, vol, lab, o, lab0, x0, B, prob, st,
                                                     rb, worst, tz);
}

}  // namespace rw
