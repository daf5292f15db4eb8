// Adjoint gradient of a loss of the random-walker probabilities.
//
// Forward: A(w) x_U = b(w) with A = L_U symmetric, b from the seeds.  For a
// loss L(x), one solve of A lam = dL/dx_U (lam = 0 on seeds) gives, per edge
// e = (i, j),  dL/dw_e = -(lam_i - lam_j)(x_i - x_j), and with
// w_e = exp(-beta (g_i - g_j)^2):
//   dL/dbeta = sum_e (lam_i - lam_j)(x_i - x_j)(g_i - g_j)^2 w_e
//   dL/dg_i  = sum_{e=(i,j)} 2 beta (lam_i - lam_j)(x_i - x_j)(g_i - g_j) w_e.
// Every solved label contributes one adjoint solve; the contributions add.
// When the forward solve set the background (label 1) to 1 - sum of the
// solved labels, a loss of the background reaches label s through that sum:
// the adjoint right-hand side of label s is dL/dx^s - dL/dx^1.  The adjoint
// solves reuse the forward CG kernels (float64) with an explicit right-hand
// side and zero Dirichlet data.
#include "rw_whole.h"

namespace rw {

constexpr int GRAD_BLOCKS = 1024;

// Right-hand side of one label's adjoint system: dL/dx^s (minus dL/dx^1 when
// label 1 is the complement of the solved labels) on unseeded voxels, 0 on
// seeds.
__global__ __launch_bounds__(256) void k_adjoint_rhs(const uint8_t* __restrict__ lab, int64_t n,
                                                     const double* __restrict__ gs,
                                                     const double* __restrict__ g1,
                                                     double* __restrict__ rhs) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x)
        rhs[i] = lab[i] ? 0.0 : (g1 ? gs[i] - g1[i] : gs[i]);
}

// dL/dg per voxel and per-block partial sums of dL/dbeta (each edge counted
// once, by its low-side voxel) of one label; `accumulate` adds dL/dg to the
// previous labels'.  gscale = 1 / (hi - lo) turns raw differences into
// normalised ones.
template <typename V>
__global__ __launch_bounds__(256) void k_adjoint_grad(const V* __restrict__ vol,
                                                      const uint8_t* __restrict__ lab, Geom G,
                                                      WCoef wc, double gscale, double beta,
                                                      int label, const double* __restrict__ xf,
                                                      const double* __restrict__ lam,
                                                      double* __restrict__ grad_g, int accumulate,
                                                      double* __restrict__ part) {
    double acc_b = 0.0;
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < G.n; i += 256ll * gridDim.x) {
        const int z = int(i / G.plane);
        const int64_t rem = i - (int64_t)z * G.plane;
        const int y = int(rem / G.nx);
        const int x = int(rem - (int64_t)y * G.nx);
        const uint8_t li = lab[i];
        const double xi = li ? (li == label ? 1.0 : 0.0) : xf[i];
        const double ai = li ? 0.0 : lam[i];
        const double vi = (double)vol[i];
        const bool has[6] = {x > 0, x + 1 < G.nx, y > 0, y + 1 < G.ny, z > 0, z + 1 < G.nz};
        const int64_t nb[6] = {i - 1, i + 1, i - G.nx, i + G.nx, i - G.plane, i + G.plane};
        double acc_g = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            if (!has[k]) continue;
            const int64_t j = nb[k];
            const uint8_t lj = lab[j];
            const double xj = lj ? (lj == label ? 1.0 : 0.0) : xf[j];
            const double aj = lj ? 0.0 : lam[j];
            const double dv = vi - (double)vol[j];
            const double w = Weight<double>::of(dv, wc);
            const double ce = (ai - aj) * (xi - xj) * w;
            const double dg = gscale * dv;
            acc_g += 2.0 * beta * ce * dg;
            if (k & 1) acc_b += ce * dg * dg;  // +x, +y, +z: each edge once
        }
        if (grad_g) grad_g[i] = accumulate ? grad_g[i] + acc_g : acc_g;
    }
    double v[1] = {acc_b};
    block_sum_store<1, 4>(v, part + blockIdx.x, GRAD_BLOCKS);
}

// out = (accumulate ? out : 0) + sum of the partials, in a fixed order.
__global__ __launch_bounds__(FIN_THREADS) void k_sum1(const double* __restrict__ part, int nb,
                                                      double* __restrict__ out, int accumulate) {
    __shared__ double sums[1];
    sum_partials<1>(part, nb, sums);
    if (threadIdx.x == 0) out[0] = accumulate ? out[0] + sums[0] : sums[0];
}

// One solved label: its adjoint right-hand side, adjoint solve and edge
// sums, added to the previous labels' (slot = 0 for the first label).
template <typename V, int VX>
static rw_status backward_impl(rw_context* ctx, const rw_volume* vol, const uint8_t* lab,
                               const rw_options* o, int label, int slot, const double* x_full,
                               const double* grad_s, const double* grad_1, double* grad_g,
                               double* grad_beta, void* ws, rw_stats* stats) {
    const Geom G = make_geom(vol->dims);
    Carver cv(ws);
    GroupBuffers B;
    carve_group(cv, G, 1, false, &B);
    double* gpart = cv.take<double>(GRAD_BLOCKS + 1);
    double* rhs = cv.take<double>(G.n);
    hipLaunchKernelGGL(k_adjoint_rhs, dim3(GRAD_BLOCKS), dim3(256), 0, ctx->s, lab, G.n, grad_s,
                       grad_1, rhs);
    RW_HIP(hipGetLastError());
    const TileChoice tc = choose_tiles(G, RW_PREC_FP64, 1);
    rw_options fo = *o;
    fo.precision = RW_PREC_FP64;
    WholeSolve<V, double, 1, VX> S;
    S.ctx = ctx;
    S.vol = static_cast<const V*>(vol->data);
    S.lab = lab;
    S.G = G;
    S.wc = make_wcoef(vol, o->beta, o->w_eps);
    S.tm = make_tilemap(G, WholeSolve<V, double, 1, VX>::BY, tc.zc, tc.xcd, VX);
    S.lab0 = 0;  // zero Dirichlet data: lam = 0 on seeds
    S.mixed = false;
    S.reliable = false;
    S.o = &fo;
    S.rhs = rhs;
    S.B = B;
    S.zv = static_cast<double*>(B.z);
    S.p0 = static_cast<double*>(B.p0);
    S.p1 = static_cast<double*>(B.p1);
    S.xv = B.x64;
    rw_status e = S.run(nullptr);
    if (e) return e;
    const RhsState& h = S.host_st[0];
    int code = RW_OK;
    if (h.status == ST_MAXITER) code = RW_NOT_CONVERGED;
    else if (h.status == ST_SINGULAR) code = RW_ERR_SINGULAR;
    else if (h.status == ST_BREAKDOWN) code = RW_ERR_BREAKDOWN;
    else if (h.status == ST_NONFINITE) code = RW_ERR_NONFINITE;
    if (stats) {
        stats->iters[slot] = h.iter_total;
        stats->label_status[slot] = code;
        stats->rel_residual[slot] = h.bb > 0 ? std::sqrt(h.rr64 / h.bb) : 0.0;
        stats->num_solved = slot + 1;
        stats->loop_ms += S.loop_ms;
    }
    if (code < 0) {
        set_error("adjoint solve failed");
        return (rw_status)code;
    }
    const double span = vol->norm_hi - vol->norm_lo;
    const double gscale = span > 0 ? 1.0 / span : 0.0;
    hipLaunchKernelGGL((k_adjoint_grad<V>), dim3(GRAD_BLOCKS), dim3(256), 0, ctx->s,
                       static_cast<const V*>(vol->data), lab, G, S.wc, gscale, o->beta, label,
                       x_full, B.x64, grad_g, slot > 0 ? 1 : 0, gpart);
    hipLaunchKernelGGL(k_sum1, dim3(1), dim3(FIN_THREADS), 0, ctx->s, gpart, GRAD_BLOCKS,
                       grad_beta ? grad_beta : gpart + GRAD_BLOCKS, slot > 0 ? 1 : 0);
    RW_HIP(hipGetLastError());
    return (rw_status)code;
}

// Every solved label in turn (labels 2..K, or 1..K with solve_all_labels).
template <typename V>
static rw_status backward_v(rw_context* ctx, const rw_volume* vol, const uint8_t* lab, int K,
                            const rw_options* o, const double* prob, const double* grad_prob,
                            double* grad_g, double* grad_beta, void* ws, rw_stats* stats) {
    const Geom G = make_geom(vol->dims);
    const TileChoice tc = choose_tiles(G, RW_PREC_FP64, 1);
    const int first = o->solve_all_labels ? 1 : 2;
    const double* grad_1 = o->solve_all_labels ? nullptr : grad_prob;
    rw_status worst = RW_OK;
    for (int s = first; s <= K; ++s) {
        const int slot = s - first;
        const double* xs = prob + (int64_t)(s - 1) * G.n;
        const double* gs = grad_prob + (int64_t)(s - 1) * G.n;
        const rw_status e =
            tc.vx == 2 ? backward_impl<V, 2>(ctx, vol, lab, o, s, slot, xs, gs, grad_1, grad_g,
                                             grad_beta, ws, stats)
                       : backward_impl<V, 1>(ctx, vol, lab, o, s, slot, xs, gs, grad_1, grad_g,
                                             grad_beta, ws, stats);
        if (e < 0) return e;
        if (e > worst) worst = e;
    }
    RW_HIP(hipStreamSynchronize(ctx->s));
    return worst;
}

rw_status check_options(const rw_options* o);

}  // namespace rw

using namespace rw;

extern "C" {

size_t rw_backward_workspace_bytes(rw_dims dims) {
    if (!dims_supported(dims)) return 0;
    Carver cv(nullptr);
    const Geom G = make_geom(dims);
    carve_group(cv, G, 1, false, nullptr);
    cv.take<double>(GRAD_BLOCKS + 1);
    cv.take<double>(G.n);
    return cv.bytes();
}

rw_status rw_solve_backward(rw_context* ctx, const rw_volume* vol, const rw_seeds* seeds,
                            const rw_options* o, const double* prob, const double* grad_prob,
                            double* grad_g_out, double* grad_beta_out, void* ws, size_t ws_bytes,
                            rw_stats* stats, void* stream) {
    if (!ctx) return invalid("context is NULL");
    rw_status e = check_volume(vol);
    if (e) return e;
    if ((e = check_options(o))) return e;
    if (!seeds || !seeds->labels) return invalid("seeds are NULL");
    if (seeds->num_labels < 1 || seeds->num_labels > RW_MAX_LABELS)
        return invalid("num_labels must be in [1, 16]");
    if (seeds->num_labels < 2 && !o->solve_all_labels)
        return invalid("one label: solve_all_labels must be 1");
    if (!prob || !grad_prob) return invalid("prob and grad_prob are required");
    const size_t need = rw_backward_workspace_bytes(vol->dims);
    if (!ws || ws_bytes < need) {
        set_error("workspace needs " + std::to_string(need) + " bytes");
        return RW_ERR_WORKSPACE;
    }
    if (stats) memset(stats, 0, sizeof(*stats));
    if ((e = stream_enter(ctx, stream))) return e;
    unsigned int cnt[256];
    if ((e = label_counts(ctx, seeds->labels, make_geom(vol->dims).n, cnt))) return e;
    for (int v = seeds->num_labels + 1; v < 256; ++v)
        if (cnt[v]) {
            (void)stream_leave(ctx, stream);
            return invalid("a seed label exceeds num_labels");
        }
    const int K = seeds->num_labels;
    switch (vol->dtype) {
        case RW_DT_U16:
            e = backward_v<uint16_t>(ctx, vol, seeds->labels, K, o, prob, grad_prob, grad_g_out,
                                     grad_beta_out, ws, stats);
            break;
        case RW_DT_F32:
            e = backward_v<float>(ctx, vol, seeds->labels, K, o, prob, grad_prob, grad_g_out,
                                  grad_beta_out, ws, stats);
            break;
        default:
            e = backward_v<double>(ctx, vol, seeds->labels, K, o, prob, grad_prob, grad_g_out,
                                   grad_beta_out, ws, stats);
    }
    rw_status e2 = stream_leave(ctx, stream);
    return e ? e : e2;
}

}  // extern "C"
