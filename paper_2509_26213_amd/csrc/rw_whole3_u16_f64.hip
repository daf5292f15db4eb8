// Whole-3-D volume solves of uint16_t data in float64.
#include "rw_solve_impl.h"

namespace rw {

rw_status whole3_u16_f64(int R, rw_context* ctx, const rw_volume* vol, const uint8_t* lab,
                         const rw_options* o, int lab0, const double* x0, const GroupBuffers& B,
                         void* prob, rw_stats* st, int rb, int* worst, int tz) {
    return dispatch_r<uint16_t, double, false>(R, ctx, vol, lab, o, lab0, x0, B, prob, st,
                                                     rb, worst, tz);
}

}  // namespace rw
