// Batched brick solves for float volumes in mixed precision (float32 CG).
#include "rw_bricks.h"

namespace rw {

rw_status bricks_f32_f32(int R, rw_context* ctx, const rw_volume* fine, const rw_seeds* seeds,
                        const Shell& sh, const rw_brick* bricks, const rw_subvolume* sub, int n,
                        const rw_options* o, float* prob, int32_t* it, void* ws, rw_stats* st) {
    return bricks_r<float, float>(R, ctx, fine, seeds, sh, bricks, sub, n, o, prob, it, ws, st);
}

}  // namespace rw
