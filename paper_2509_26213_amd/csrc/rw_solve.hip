// Whole-volume Jacobi-PCG solve of the random-walker Dirichlet problem.
//
// Each label s solves, for every unseeded voxel i,
//     sum_j w_ij (x_i - x_j) = 0,   x_j = [label_j == s] on seeds,
// (random walker; the paper cites it in Sec. III-A and benchmarks the
// hierarchical form in Sec. IV-B), by Jacobi-preconditioned CG stopped at
// ||r|| <= tol ||b||.  The operator is never stored: every pass recomputes
// the six edge weights of each voxel from the raw intensities.
//
// Two passes per CG iteration (vectors x, z = D^-1 r, p; r is never stored,
// r = d * z is rebuilt where needed):
//   pass 1:  p <- z + beta p (formed on the fly at the voxel and its six
//            neighbours, written to the other p buffer); q = A p; sum p.q
//   pass 2:  q = A p again; x += alpha p; r = d z - alpha q; z = r / d;
//            sums r.z and r.r
// Between them one-block kernels turn the per-block float64 partials into
// alpha, beta and convergence flags, in a fixed order (deterministic).
// The host only polls the flags every `check_interval` iterations.
//
// Mixed precision: the CG runs in float32 (weights, vectors) with float64
// dot products, inside float64 iterative refinement: r64 = b - A64 x64 with
// float64 weights, inner float32 solve of A32 d = r64, x64 += d.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "rw_solve_impl.h"

namespace rw {

// ================================================================== kernels

rw_status check_options(const rw_options* o) {
    if (!o) return invalid("options is NULL");
    if (!(o->beta >= 0) || !std::isfinite(o->beta)) return invalid("beta must be finite and >= 0");
    if (!std::isfinite(o->w_eps)) return invalid("w_eps must be finite");
    if (!(o->tol > 0) || !std::isfinite(o->tol)) return invalid("tol must be > 0");
    if (o->precision != RW_PREC_FP64 && o->precision != RW_PREC_MIXED)
        return invalid("unknown precision");
    if (o->precision == RW_PREC_MIXED) {
        if (o->refine_mode != 0 && o->refine_mode != 1) return invalid("unknown refine_mode");
        if (o->refine_mode == 1 && !(o->inner_tol > 0 && o->inner_tol < 1))
            return invalid("inner_tol must be in (0, 1)");
        if (o->refine_mode == 0 && !(o->update_delta > 0 && o->update_delta < 1))
            return invalid("update_delta must be in (0, 1)");
    }
    if (o->max_iter <= 0) return invalid("max_iter must be > 0");
    if (o->max_refine < 0) return invalid("max_refine must be >= 0");
    if (o->check_interval <= 0 || o->check_interval > 1024)
        return invalid("check_interval must be in [1, 1024]");
    return RW_OK;
}

// Labels present (0..255) and their validity for a solve with K labels.
rw_status check_labels(rw_context* ctx, const uint8_t* lab, int64_t n, int K, int lab0,
                       int R_total, int64_t* unknowns) {
    unsigned int cnt[256];
    rw_status e = label_counts(ctx, lab, n, cnt);
    if (e) return e;
    for (int v = K + 1; v < 256; ++v)
        if (cnt[v]) return invalid("a seed label exceeds num_labels");
    uint64_t seeds = 0;
    for (int v = 1; v <= K; ++v) seeds += cnt[v];
    if (seeds == 0) {
        set_error("no seeds");
        return RW_ERR_NO_SEEDS;
    }
    for (int r = 0; r < R_total; ++r)
        if (cnt[lab0 + r] == 0) {
            set_error("label " + std::to_string(lab0 + r) + " has no seed");
            return RW_ERR_NO_SEEDS;
        }
    if (unknowns) *unknowns = cnt[0];
    return RW_OK;
}

template <typename V, typename T, int VX>
static rw_status apply_op_vx(rw_context* ctx, const rw_volume* vol, const WCoef& wc,
                             const TileChoice& tc, const void* p, void* q, void* ws) {
    constexpr int BY = 4;
    const Geom G = make_geom(vol->dims);
    const TileMap tm = make_tilemap(G, BY, tc.zc, tc.xcd, VX);
    Carver cv(ws);
    T* pnew = cv.take<T>(size_t(G.n));
    double* part = cv.take<double>(size_t(max_tiles(G)));
    RhsState* st = cv.take<RhsState>(1);
    RhsState h;
    memset(&h, 0, sizeof(h));
    h.active = 1;
    h.beta = 0.0;
    h.pcur = 0;
    RW_HIP(hipMemcpyAsync(st, &h, sizeof(h), hipMemcpyHostToDevice, ctx->s));
    // beta = 0: p_new = z = p; buffer 0 (p itself) is the old p, times 0
    WholeTiles ts;
    ts.tm = tm;
    ts.G = G;
    ts.ntiles = tm.tiles;
    hipLaunchKernelGGL((k_cg_pass1<V, T, 1, BY, PlaneBatch<T, VX>::value, VX, WholeTiles>),
                       dim3(unsigned(tm.blocks())), dim3(64, BY), 0, ctx->s, (const V*)vol->data,
                       wc, ts, (const T*)p, (T*)p, pnew, (T*)q, st, part);
    RW_HIP(hipGetLastError());
    RW_HIP(hipStreamSynchronize(ctx->s));
    return RW_OK;
}

template <typename V, typename T>
static rw_status apply_op(rw_context* ctx, const rw_volume* vol, const WCoef& wc, const void* p,
                          void* q, void* ws, int precision) {
    const TileChoice tc = choose_tiles(make_geom(vol->dims), precision, 1);
    if constexpr (std::is_same<T, float>::value) {
        if (tc.vx == 4) return apply_op_vx<V, T, 4>(ctx, vol, wc, tc, p, q, ws);
    }
    if (tc.vx == 2) return apply_op_vx<V, T, 2>(ctx, vol, wc, tc, p, q, ws);
    return apply_op_vx<V, T, 1>(ctx, vol, wc, tc, p, q, ws);
}

}  // namespace rw

using namespace rw;

extern "C" {

size_t rw_solve_workspace_bytes(rw_dims dims, int32_t num_labels, int32_t precision,
                                int32_t solve_all_labels) {
    if (!dims_supported(dims) || num_labels < 1) return 0;
    const int R_total = solve_all_labels ? num_labels : num_labels - 1;
    const int Rg = std::max(1, std::min(4, R_total));
    Carver cv(nullptr);
    return carve_group(cv, make_geom(dims), Rg, precision == RW_PREC_MIXED, nullptr);
}

rw_status rw_solve(rw_context* ctx, const rw_volume* vol, const rw_seeds* seeds,
                   const rw_options* o, void* prob_out, uint8_t* argmax_out, void* ws,
                   size_t ws_bytes, rw_stats* stats, void* stream) {
    return solve_whole<false>(ctx, vol, 0, seeds, o, prob_out, argmax_out, ws, ws_bytes, stats,
                              stream);
}

size_t rw_operator_workspace_bytes(rw_dims dims, int32_t precision) {
    if (!dims_supported(dims)) return 0;
    const Geom G = make_geom(dims);
    Carver cv(nullptr);
    cv.take<char>((precision == RW_PREC_MIXED ? 4 : 8) * size_t(G.n));
    cv.take<double>(size_t(max_tiles(G)));
    cv.take<RhsState>(1);
    return cv.bytes();
}

rw_status rw_apply_operator(rw_context* ctx, const rw_volume* vol, const rw_seeds* seeds,
                            double beta, double w_eps, int32_t precision, const void* p,
                            void* q_out, void* ws, size_t ws_bytes, void* stream) {
    (void)seeds;
    if (!ctx || !p || !q_out) return invalid("NULL argument");
    rw_status e = check_volume(vol);
    if (e) return e;
    if (!(beta >= 0) || !std::isfinite(beta)) return invalid("beta must be finite and >= 0");
    if (precision != RW_PREC_FP64 && precision != RW_PREC_MIXED) return invalid("bad precision");
    const size_t need = rw_operator_workspace_bytes(vol->dims, precision);
    if (!ws || ws_bytes < need) {
        set_error("workspace needs " + std::to_string(need) + " bytes");
        return RW_ERR_WORKSPACE;
    }
    const WCoef wc = make_wcoef(vol, beta, w_eps);
    if ((e = stream_enter(ctx, stream))) return e;
    const bool m = precision == RW_PREC_MIXED;
    switch (vol->dtype) {
        case RW_DT_U16:
            e = m ? apply_op<uint16_t, float>(ctx, vol, wc, p, q_out, ws, precision)
                  : apply_op<uint16_t, double>(ctx, vol, wc, p, q_out, ws, precision);
            break;
        case RW_DT_F32:
            e = m ? apply_op<float, float>(ctx, vol, wc, p, q_out, ws, precision)
                  : apply_op<float, double>(ctx, vol, wc, p, q_out, ws, precision);
            break;
        default:
            e = m ? apply_op<double, float>(ctx, vol, wc, p, q_out, ws, precision)
                  : apply_op<double, double>(ctx, vol, wc, p, q_out, ws, precision);
    }
    if (e) return e;
    return stream_leave(ctx, stream);
}

}  // extern "C"
