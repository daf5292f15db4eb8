// 4-D random walker: a volume time series [nt][nz][ny][nx] segmented as one
// grid in which every voxel is joined to its two neighbours along x, y, z
// and t (the paper's Sec. V-B applies the random walker to a cardiac MRI
// sequence this way).  The series is solved as the grid (nx, ny, nt * nz)
// with the z edges between time steps removed and time edges tz = nz planes
// apart added: the same matrix-free Jacobi-PCG, kernels and precisions as
// rw_solve.
#include "rw_solve_impl.h"

using namespace rw;

extern "C" {

size_t rw_solve4d_workspace_bytes(rw_dims dims, int32_t nt, int32_t num_labels,
                                  int32_t precision, int32_t solve_all_labels) {
    if (nt < 1 || dims.nz <= 0 || dims.nz > (int64_t(1) << 30) / nt) return 0;
    rw_dims f = dims;
    f.nz = dims.nz * nt;
    return rw_solve_workspace_bytes(f, num_labels, precision, solve_all_labels);
}

rw_status rw_solve4d(rw_context* ctx, const rw_volume* vol, int32_t nt, const rw_seeds* seeds,
                     const rw_options* opts, void* prob_out, uint8_t* argmax_out, void* ws,
                     size_t ws_bytes, rw_stats* stats, void* stream) {
    if (!vol) return invalid("volume is NULL");
    if (nt < 1) return invalid("nt must be >= 1");
    if (vol->dims.nz <= 0 || vol->dims.nz > (int64_t(1) << 30) / nt)
        return invalid("nz * nt must be in [1, 2^30]");
    rw_volume v = *vol;
    v.dims.nz = vol->dims.nz * nt;
    return solve_whole<true>(ctx, &v, int(vol->dims.nz), seeds, opts, prob_out, argmax_out, ws,
                             ws_bytes, stats, stream);
}

}  // extern "C"
