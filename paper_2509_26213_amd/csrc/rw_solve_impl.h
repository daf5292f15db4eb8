// The whole-volume solve, templated on the grid kind: a 3-D volume, or a
// volume time series (T4) stored as (nx, ny, nt * tz).  Shared by rw_solve
// and rw_solve4d, which live in their own translation units.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>

#include "rw_whole.h"

namespace rw {

rw_status check_options(const rw_options* o);
rw_status check_labels(rw_context* ctx, const uint8_t* lab, int64_t n, int K, int lab0,
                       int R_total, int64_t* unknowns);

template <typename V, typename T, int R, bool T4>
rw_status run_group(rw_context* ctx, const rw_volume* vol, const uint8_t* lab,
                    const rw_options* o, int lab0, const double* x0, const GroupBuffers& B,
                    void* prob_out, rw_stats* stats, int r_base, int* worst, int tz) {
    const TileChoice tc = choose_tiles(make_geom(vol->dims), o->precision, R);
    if constexpr (T4) {
        // time series: two columns per lane, 4 or 8 waves
        if (tc.by == 8)
            return run_group_vx<V, T, R, 2, 8, true>(ctx, vol, lab, o, lab0, x0, B, tc, prob_out,
                                                     stats, r_base, worst, tz);
        return run_group_vx<V, T, R, 2, 4, true>(ctx, vol, lab, o, lab0, x0, B, tc, prob_out, stats,
                                                 r_base, worst, tz);
    }
    if constexpr (std::is_same<T, float>::value) {
        if (tc.vx == 4)
            return run_group_vx<V, T, R, 4, 4, T4>(ctx, vol, lab, o, lab0, x0, B, tc, prob_out,
                                                   stats, r_base, worst, tz);
    }
    if constexpr (std::is_same<T, float>::value) {
        if (tc.vx == 2 && tc.by == 8 && tc.by2 == 4)
            return run_group_vx<V, T, R, 2, 8, T4, 4>(ctx, vol, lab, o, lab0, x0, B, tc, prob_out,
                                                      stats, r_base, worst, tz);
    }
    if (tc.vx == 2 && tc.by == 8)
        return run_group_vx<V, T, R, 2, 8, T4>(ctx, vol, lab, o, lab0, x0, B, tc, prob_out,
                                               stats, r_base, worst, tz);
    if (tc.vx == 2)
        return run_group_vx<V, T, R, 2, 4, T4>(ctx, vol, lab, o, lab0, x0, B, tc, prob_out,
                                               stats, r_base, worst, tz);
    return run_group_vx<V, T, R, 1, 4, T4>(ctx, vol, lab, o, lab0, x0, B, tc, prob_out, stats,
                                           r_base, worst, tz);
}

template <typename V, typename T, bool T4>
rw_status dispatch_r(int R, rw_context* ctx, const rw_volume* vol, const uint8_t* lab,
                     const rw_options* o, int lab0, const double* x0, const GroupBuffers& B,
                     void* prob, rw_stats* st, int rb, int* worst, int tz) {
    switch (R) {
        case 1: return run_group<V, T, 1, T4>(ctx, vol, lab, o, lab0, x0, B, prob, st, rb, worst, tz);
        case 2: return run_group<V, T, 2, T4>(ctx, vol, lab, o, lab0, x0, B, prob, st, rb, worst, tz);
        case 3: return run_group<V, T, 3, T4>(ctx, vol, lab, o, lab0, x0, B, prob, st, rb, worst, tz);
        case 4: return run_group<V, T, 4, T4>(ctx, vol, lab, o, lab0, x0, B, prob, st, rb, worst, tz);
    }
    return invalid("bad group size");
}

// One instantiation per (grid kind, volume type, precision):
// rw_whole<3|4>_<volume>_<precision>.hip (separate translation units, so
// they compile in parallel).
#define RW_WHOLE_DECL(NAME)                                                                  \
    rw_status NAME(int R, rw_context* ctx, const rw_volume* vol, const uint8_t* lab,         \
                   const rw_options* o, int lab0, const double* x0, const GroupBuffers& B,   \
                   void* prob, rw_stats* st, int rb, int* worst, int tz);
RW_WHOLE_DECL(whole3_u16_f32)
RW_WHOLE_DECL(whole3_u16_f64)
RW_WHOLE_DECL(whole3_f32_f32)
RW_WHOLE_DECL(whole3_f32_f64)
RW_WHOLE_DECL(whole3_f64_f32)
RW_WHOLE_DECL(whole3_f64_f64)
RW_WHOLE_DECL(whole4_u16_f32)
RW_WHOLE_DECL(whole4_u16_f64)
RW_WHOLE_DECL(whole4_f32_f32)
RW_WHOLE_DECL(whole4_f32_f64)
RW_WHOLE_DECL(whole4_f64_f32)
RW_WHOLE_DECL(whole4_f64_f64)
#undef RW_WHOLE_DECL

template <bool T4>
rw_status dispatch_group(int R, rw_context* ctx, const rw_volume* vol, const uint8_t* lab,
                         const rw_options* o, int lab0, const double* x0, const GroupBuffers& B,
                         void* prob, rw_stats* st, int rb, int* worst, int tz) {
    const bool m = o->precision == RW_PREC_MIXED;
    switch (vol->dtype) {
        case RW_DT_U16:
            return (T4 ? (m ? whole4_u16_f32 : whole4_u16_f64) : (m ? whole3_u16_f32 : whole3_u16_f64))(
                R, ctx, vol, lab, o, lab0, x0, B, prob, st, rb, worst, tz);
        case RW_DT_F32:
            return (T4 ? (m ? whole4_f32_f32 : whole4_f32_f64) : (m ? whole3_f32_f32 : whole3_f32_f64))(
                R, ctx, vol, lab, o, lab0, x0, B, prob, st, rb, worst, tz);
        default:
            return (T4 ? (m ? whole4_f64_f32 : whole4_f64_f64) : (m ? whole3_f64_f32 : whole3_f64_f64))(
                R, ctx, vol, lab, o, lab0, x0, B, prob, st, rb, worst, tz);
    }
}

// The whole-volume solve behind rw_solve (3-D grid, tz = 0) and rw_solve4d
// (volume time series stored as (nx, ny, nt * tz), T4).
template <bool T4>
rw_status solve_whole(rw_context* ctx, const rw_volume* vol, int tz, const rw_seeds* seeds,
                      const rw_options* o, void* prob_out, uint8_t* argmax_out, void* ws,
                      size_t ws_bytes, rw_stats* stats, void* stream) {
    if (!ctx) return invalid("context is NULL");
    rw_status e = check_volume(vol);
    if (e) return e;
    if ((e = check_options(o))) return e;
    if (!seeds || !seeds->labels) return invalid("seeds are NULL");
    const int K = seeds->num_labels;
    if (K < 1 || K > RW_MAX_LABELS) return invalid("num_labels must be in [1, 16]");
    if (!prob_out) return invalid("prob_out is NULL");
    const size_t need = rw_solve_workspace_bytes(vol->dims, K, o->precision, o->solve_all_labels);
    if (!ws || ws_bytes < need) {
        set_error("workspace needs " + std::to_string(need) + " bytes");
        return RW_ERR_WORKSPACE;
    }
    if (stats) memset(stats, 0, sizeof(*stats));
    const Geom G = make_geom(vol->dims);
    const int R_total = o->solve_all_labels ? K : K - 1;
    const int lab0 = o->solve_all_labels ? 1 : 2;
    if ((e = stream_enter(ctx, stream))) return e;
    RW_HIP(hipEventRecord(ctx->ev_begin, ctx->s));
    int64_t unknowns = 0;
    if ((e = check_labels(ctx, seeds->labels, G.n, K, lab0, R_total, &unknowns))) {
        (void)stream_leave(ctx, stream);
        return e;
    }
    int worst = RW_OK;
    for (int g0 = 0; g0 < R_total; g0 += 4) {
        const int Rg = std::min(4, R_total - g0);
        Carver cv(ws);
        GroupBuffers B;
        carve_group(cv, G, Rg, o->precision == RW_PREC_MIXED, &B);
        const double* x0 = o->x0 ? static_cast<const double*>(o->x0) + (int64_t)g0 * G.n : nullptr;
        e = dispatch_group<T4>(Rg, ctx, vol, seeds->labels, o, lab0 + g0, x0, B, prob_out, stats,
                               g0, &worst, tz);
        if (e) {
            (void)stream_leave(ctx, stream);
            return e;
        }
        if (worst < 0) break;
    }
    if (worst >= 0) {
        const int complement = o->solve_all_labels ? 0 : 1;
        if (o->precision == RW_PREC_MIXED)
            hipLaunchKernelGGL((k_finish<float>), dim3(grid1d(G.n)), dim3(256), 0, ctx->s,
                               seeds->labels, G.n, K, complement, (float*)prob_out, argmax_out);
        else
            hipLaunchKernelGGL((k_finish<double>), dim3(grid1d(G.n)), dim3(256), 0, ctx->s,
                               seeds->labels, G.n, K, complement, (double*)prob_out, argmax_out);
        RW_HIP(hipGetLastError());
    }
    RW_HIP(hipEventRecord(ctx->ev_end, ctx->s));
    RW_HIP(hipEventSynchronize(ctx->ev_end));
    if (stats) {
        float ms = 0.f;
        RW_HIP(hipEventElapsedTime(&ms, ctx->ev_begin, ctx->ev_end));
        stats->device_ms = ms;
        stats->num_solved = R_total;
        stats->unknowns = unknowns;
    }
    if ((e = stream_leave(ctx, stream))) return e;
    if (worst < 0) set_error(std::string("solve failed: ") + rw_status_string((rw_status)worst));
    return (rw_status)worst;
}

}  // namespace rw
