// Whole-volume Jacobi-PCG driver: finalize kernels, elementwise kernels and
// the host-side iteration control shared by the forward and adjoint solves.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "rw_cg_kernels.h"
#include "rw_internal.h"
#include "rw_kernels.h"

namespace rw {

__device__ __forceinline__ bool any_active(const RhsState* st, int R) {
    bool a = false;
    for (int r = 0; r < R; ++r) a |= st[r].active != 0;
    return a;
}

// After pass 1: alpha = rho / p.q (or breakdown); the written p buffer
// becomes the current one.
template <int R>
__global__ __launch_bounds__(FIN_THREADS) void k_fin1(const double* __restrict__ part, int nb,
                                                      RhsState* __restrict__ st) {
    if (!any_active(st, R)) return;
    __shared__ double sums[R];
    sum_partials<R>(part, nb, sums);
    const int r = threadIdx.x;
    if (r < R && st[r].active) {
        RhsState& s = st[r];
        const double sigma = sums[r];
        s.pcur ^= 1;
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            s.status = ST_BREAKDOWN;
            s.active = 0;
            s.outer_active = 0;
        } else {
            s.alpha = s.rho / sigma;
        }
    }
}

// After pass 2: rho and beta for the next direction, convergence test on
// the recurrence residual, iteration cap.
template <int R>
__global__ __launch_bounds__(FIN_THREADS) void k_fin2(const double* __restrict__ part, int nb,
                                                      RhsState* __restrict__ st, int final_on_conv) {
    if (!any_active(st, R)) return;
    __shared__ double sums[2 * R];
    sum_partials<2 * R>(part, nb, sums);
    const int r = threadIdx.x;
    if (r < R && st[r].active) {
        RhsState& s = st[r];
        const double rz = sums[2 * r], rr = sums[2 * r + 1];
        s.iter += 1;
        s.iter_total += 1;
        s.rr = rr;
        if (!isfinite(rr) || !isfinite(rz)) {
            s.status = ST_NONFINITE;
            s.active = 0;
            s.outer_active = 0;
            return;
        }
        s.rho_prev = s.rho;
        s.rho = rz;
        s.beta = rz / s.rho_prev;
        if (rr <= s.thresh2) {
            s.active = 0;
            if (final_on_conv) {
                s.status = ST_CONVERGED;
                s.outer_active = 0;
            }
        } else if (s.iter_total >= s.max_iter) {
            s.active = 0;
            s.status = ST_MAXITER;
            s.outer_active = 0;
        }
    }
}

// After a residual evaluation that starts a CG run: record ||b|| (first
// call), test the float64 residual, set up the run.  thresh_mode 0 stops the
// run at ||r|| <= tol ||b||, 1 at ||r|| <= eta ||r_start|| (restarted
// refinement steps).
template <int R>
__global__ __launch_bounds__(FIN_THREADS) void k_fin_init(const double* __restrict__ part, int nb,
                                                          RhsState* __restrict__ st, double tol,
                                                          double eta, int first, int thresh_mode,
                                                          int max_iter) {
    constexpr int NQ = 4 * R + 2;
    __shared__ double sums[NQ];
    sum_partials<NQ>(part, nb, sums);
    const int r = threadIdx.x;
    if (r >= R) return;
    RhsState& s = st[r];
    if (first) {
        s.bb = sums[4 * r + 3];
        s.iter_total = 0;
        s.refreshes = 0;
        s.status = ST_RUNNING;
        s.outer_active = 1;
    }
    s.rr64 = sums[4 * r + 2];
    s.iter = 0;
    s.max_iter = max_iter;
    s.pcur = 0;
    if (s.status != ST_RUNNING || !s.outer_active) {
        s.active = 0;
        return;
    }
    if (sums[4 * R + 1] > 0) {
        s.status = ST_NONFINITE;
    } else if (sums[4 * R] > 0) {
        s.status = ST_SINGULAR;
    } else if (s.bb == 0.0 || s.rr64 <= tol * tol * s.bb) {
        s.status = ST_CONVERGED;
    }
    if (s.status != ST_RUNNING) {
        s.active = 0;
        s.outer_active = 0;
        return;
    }
    s.active = 1;
    s.rho = sums[4 * r + 0];
    s.rho_prev = s.rho;
    s.rr = sums[4 * r + 1];
    s.rr_ref = s.rr;
    s.beta = 0.0;
    s.alpha = 0.0;
    s.thresh2 = thresh_mode ? eta * eta * s.rr : tol * tol * s.bb;
}

// After a float64 residual refresh of the labels in `mask` (mixed precision,
// reliable updates): stop if the float64 residual meets the tolerance,
// otherwise continue the same CG run from the refreshed residual (beta
// recomputed with it, search direction kept).
template <int R>
__global__ __launch_bounds__(FIN_THREADS) void k_fin_refresh(const double* __restrict__ part,
                                                             int nb, RhsState* __restrict__ st,
                                                             double tol, int mask) {
    constexpr int NQ = 4 * R + 2;
    __shared__ double sums[NQ];
    sum_partials<NQ>(part, nb, sums);
    const int r = threadIdx.x;
    if (r >= R || !(mask & (1 << r))) return;
    RhsState& s = st[r];
    s.rr64 = sums[4 * r + 2];
    s.refreshes += 1;
    if (!isfinite(s.rr64) || !isfinite(sums[4 * r])) {
        s.status = ST_NONFINITE;
        s.active = 0;
        s.outer_active = 0;
        return;
    }
    if (s.rr64 <= tol * tol * s.bb) {
        s.status = ST_CONVERGED;
        s.active = 0;
        s.outer_active = 0;
        return;
    }
    if (s.iter_total >= s.max_iter) {
        s.status = ST_MAXITER;
        s.active = 0;
        s.outer_active = 0;
        return;
    }
    s.rho = sums[4 * r + 0];
    s.beta = s.rho / s.rho_prev;
    s.rr = sums[4 * r + 1];
    s.rr_ref = s.rr;
    s.active = 1;
    s.outer_active = 1;
}

// Flag the labels in `mask` for a float64 residual refresh.
template <int R>
__global__ void k_mark_refresh(RhsState* __restrict__ st, int mask) {
    const int r = threadIdx.x;
    if (r < R && (mask & (1 << r))) st[r].outer_active = 2;
}

// x64 += xi, xi = 0 for the labels in `mask`.  Seeds need no test: xi is 0
// there (never written but as 0), so their x64 keeps its value.
template <typename T, int R>
__global__ __launch_bounds__(256) void k_update64(int64_t n, T* __restrict__ xi,
                                                  double* __restrict__ x64, int mask) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (mask & (1 << r)) {
                x64[r * n + i] += (double)xi[r * n + i];
                xi[r * n + i] = T(0);
            }
    }
}

// Probabilities of the solved labels lab0..lab0+R-1, seeds exact.
template <typename TO, int R>
__global__ __launch_bounds__(256) void k_write_labels(const uint8_t* __restrict__ lab, int64_t n,
                                                      const double* __restrict__ x64, int lab0,
                                                      TO* __restrict__ prob) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
        const uint8_t lc = lab[i];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int L = lab0 + r;
            prob[(int64_t)(L - 1) * n + i] = lc ? TO(lc == L ? 1 : 0) : TO(x64[r * n + i]);
        }
    }
}

// Background label as the complement, and the argmax (lowest label on ties).
template <typename TO>
__global__ __launch_bounds__(256) void k_finish(const uint8_t* __restrict__ lab, int64_t n, int K,
                                                int complement, TO* __restrict__ prob,
                                                uint8_t* __restrict__ amax) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
        const uint8_t lc = lab[i];
        if (complement) {
            double s = 0.0;
            for (int L = 2; L <= K; ++L) s += (double)prob[(int64_t)(L - 1) * n + i];
            prob[i] = lc ? TO(lc == 1 ? 1 : 0) : TO(1.0 - s);
        }
        if (amax) {
            TO best = prob[i];
            int arg = 1;
            for (int L = 2; L <= K; ++L) {
                const TO v = prob[(int64_t)(L - 1) * n + i];
                if (v > best) {
                    best = v;
                    arg = L;
                }
            }
            amax[i] = uint8_t(arg);
        }
    }
}

// ================================================================== host

// Tile shape of a whole-volume solve: 64 vx x by columns (by = 8 with vx = 2
// only, else 4) by zc planes, from the tuning table (rw_tune.hip); zc
// shrinks until the grid has enough blocks.
inline TileChoice choose_tiles(const Geom& G, int precision, int R) {
    TileChoice c = tuned_tiles(G, precision, R);
    c.by = c.by == 8 && c.vx == 2 ? 8 : 4;
    // pass 2 on 4-row tiles beside 8-row pass-1 tiles (float32 only), else
    // the same tiles
    if (!(c.by == 8 && c.by2 == 4 && precision == RW_PREC_MIXED)) {
        c.by2 = c.by;
        c.zc2 = 0;
    }
    if (c.vx != 2 && c.vx != 4) c.vx = 1;
    if (precision != RW_PREC_MIXED && c.vx > 2) c.vx = 2;
    const int64_t cols =
        (int64_t)((G.nx + 64 * c.vx - 1) / (64 * c.vx)) * ((G.ny + c.by - 1) / c.by);
    while (c.zc > 4 && cols * ((G.nz + c.zc - 1) / c.zc) < 1024) c.zc = std::max(4, c.zc / 2);
    // the partial buffers are sized for 64 x 4 x 4 tiles
    c.zc = std::max(4, c.zc);
    if (c.zc2 <= 0) c.zc2 = c.zc;
    const int64_t cols2 =
        (int64_t)((G.nx + 64 * c.vx - 1) / (64 * c.vx)) * ((G.ny + c.by2 - 1) / c.by2);
    while (c.zc2 > 4 && cols2 * ((G.nz + c.zc2 - 1) / c.zc2) < 1024) c.zc2 = std::max(4, c.zc2 / 2);
    c.zc2 = std::max(4, c.zc2);
    return c;
}

inline int max_tiles(const Geom& G) { return make_tilemap(G, 4, 4, 0).tiles; }

inline int grid1d(int64_t n) { return int(std::min<int64_t>((n + 255) / 256, 8192)); }

struct GroupBuffers {
    double* x64;   // [R][n] float64 iterate (the CG x itself for FP64)
    void* xi;      // [R][n] inner float32 x (mixed only)
    void* z;       // [R][n]
    void* p0;      // [R][n]
    void* p1;      // [R][n]
    double* part;  // per-tile partials
    RhsState* st;  // [R]
};

inline size_t carve_group(Carver& cv, const Geom& G, int R, bool mixed, GroupBuffers* b) {
    const size_t vs = mixed ? sizeof(float) : sizeof(double);
    GroupBuffers t;
    t.x64 = cv.take<double>(size_t(R) * G.n);
    t.xi = mixed ? (void*)cv.take<char>(vs * R * G.n) : nullptr;
    t.z = cv.take<char>(vs * R * G.n);
    t.p0 = cv.take<char>(vs * R * G.n);
    t.p1 = cv.take<char>(vs * R * G.n);
    t.part = cv.take<double>(size_t(max_tiles(G)) * (4 * 4 + 2));
    t.st = cv.take<RhsState>(4);
    if (b) *b = t;
    return cv.bytes();
}

// Planes per batch of the CG passes: the registers of a batch hold U x VX
// values per operand, 4 in float32 and 2 in float64.
template <typename T, int VX>
struct PlaneBatch {
    static constexpr int per = std::is_same<T, double>::value ? 2 : 4;
    static constexpr int value = per / VX > 0 ? per / VX : 1;
};

// T4: the grid is a volume time series (G.tz planes per time step).  BY2:
// rows of pass 2's tiles (tm2), which may differ from pass 1's (tm): pass 2
// forms nothing on the halo, so it keeps its own best shape.
template <typename V, typename T, int R, int VX, int BY_ = 4, bool T4 = false, int BY2_ = BY_>
struct WholeSolve {
    static constexpr int BY = BY_;
    static constexpr int BY2 = BY2_;
    static constexpr int ZU = PlaneBatch<T, VX>::value;
    rw_context* ctx;
    const V* vol;
    const uint8_t* lab;
    Geom G;
    WCoef wc;
    TileMap tm;
    TileMap tm2{};  // pass 2 (tiles == 0: the same as tm)
    int lab0;
    bool mixed;
    bool reliable;
    const rw_options* o;
    const double* rhs = nullptr;  // explicit right-hand side (adjoint solves)
    GroupBuffers B;
    T* xv;  // CG x
    T* zv;
    T* p0;
    T* p1;
    RhsState host_st[R];
    double loop_ms = 0.0;
    double pass_ms[2] = {0, 0};
    int64_t launches[2] = {0, 0};
    int64_t rhs_iters = 0;
    int64_t box_vox = 0, rhs_vox = 0;

    dim3 grid() const { return dim3(unsigned(tm.blocks())); }
    WholeTiles ts() const {
        WholeTiles w;
        w.tm = tm;
        w.G = G;
        w.ntiles = tm.tiles;
        return w;
    }
    dim3 block() const { return dim3(64, BY); }
    const TileMap& map2() const { return tm2.tiles ? tm2 : tm; }
    dim3 grid2() const { return dim3(unsigned(map2().blocks())); }
    WholeTiles ts2() const {
        WholeTiles w;
        w.tm = map2();
        w.G = G;
        w.ntiles = map2().tiles;
        return w;
    }
    dim3 block2() const { return dim3(64, BY2); }

    rw_status launch_iteration(hipEvent_t* ev) {
        hipStream_t s = ctx->s;
        if (map2().by != BY2) return invalid("pass-2 tile map does not match its block shape");
        if (ev) RW_HIP(hipEventRecord(ev[0], s));
        hipLaunchKernelGGL((k_cg_pass1<V, T, R, BY, ZU, VX, WholeTiles, false, T4>), grid(), block(), 0, s, vol, wc, ts(), zv,
                           p0, p1, (T*)nullptr, B.st, B.part);
        if (ev) RW_HIP(hipEventRecord(ev[1], s));
        hipLaunchKernelGGL((k_fin1<R>), dim3(1), dim3(FIN_THREADS), 0, s, B.part, tm.tiles, B.st);
        if (ev) RW_HIP(hipEventRecord(ev[2], s));
        hipLaunchKernelGGL((k_cg_pass2<V, T, R, BY2, ZU, VX, WholeTiles, false, T4>), grid2(), block2(), 0, s, vol, lab, wc, ts2(),
                           xv, zv, (const T*)p0, (const T*)p1, B.st, B.part);
        if (ev) RW_HIP(hipEventRecord(ev[3], s));
        hipLaunchKernelGGL((k_fin2<R>), dim3(1), dim3(FIN_THREADS), 0, s, B.part, map2().tiles, B.st,
                           mixed ? 0 : 1);
        RW_HIP(hipGetLastError());
        return RW_OK;
    }

    rw_status read_state() {
        RW_HIP(hipMemcpyAsync(ctx->host_pinned, B.st, sizeof(RhsState) * R, hipMemcpyDeviceToHost,
                              ctx->s));
        RW_HIP(hipStreamSynchronize(ctx->s));
        memcpy(host_st, ctx->host_pinned, sizeof(RhsState) * R);
        return RW_OK;
    }

    rw_status launch_residual(int mode) {
        Shell none;
        memset(&none, 0, sizeof(none));
        hipLaunchKernelGGL((k_residual<V, T, R, BY, VX, WholeTiles, false, T4>), grid(), block(), 0, ctx->s, vol, lab,
                           wc, ts(), none, lab0, B.x64, rhs, zv, p0, p1,
                           mixed ? (T*)B.xi : (T*)nullptr, mode, B.st, B.part);
        RW_HIP(hipGetLastError());
        return RW_OK;
    }

    rw_status start(bool first, int thresh_mode, double eta, int mode = 1) {
        rw_status e = launch_residual(mode);
        if (e) return e;
        hipLaunchKernelGGL((k_fin_init<R>), dim3(1), dim3(FIN_THREADS), 0, ctx->s, B.part,
                           tm.tiles, B.st, o->tol, eta, first ? 1 : 0, thresh_mode, o->max_iter);
        RW_HIP(hipGetLastError());
        return read_state();
    }

    // Mixed precision, reliable updates: fold xi into x64 and refresh the
    // residual of the labels in `mask` in float64.
    rw_status refresh(int mask) {
        hipLaunchKernelGGL((k_mark_refresh<R>), dim3(1), dim3(64), 0, ctx->s, B.st, mask);
        hipLaunchKernelGGL((k_update64<T, R>), dim3(grid1d(G.n)), dim3(256), 0, ctx->s, G.n,
                           (T*)B.xi, B.x64, mask);
        rw_status e = launch_residual(2);
        if (e) return e;
        hipLaunchKernelGGL((k_fin_refresh<R>), dim3(1), dim3(FIN_THREADS), 0, ctx->s, B.part,
                           tm.tiles, B.st, o->tol, mask);
        RW_HIP(hipGetLastError());
        return read_state();
    }

    bool any_active() const {
        for (int r = 0; r < R; ++r)
            if (host_st[r].active) return true;
        return false;
    }

    int refresh_mask() const {
        if (!reliable) return 0;
        const double d2 = o->update_delta * o->update_delta;
        int mask = 0;
        for (int r = 0; r < R; ++r) {
            const RhsState& h = host_st[r];
            if (h.status != ST_RUNNING || !h.outer_active) continue;
            if (!h.active || h.rr < d2 * h.rr_ref) mask |= 1 << r;
        }
        return mask;
    }

    // CG iterations until every label of this group stops.
    rw_status inner() {
        hipStream_t s = ctx->s;
        const int m = o->check_interval;
        const bool timing = o->kernel_timing != 0;
        const bool graph = o->use_graph != 0 && !timing;
        if (timing) {
            rw_status e = ensure_events(ctx, size_t(4 * m));
            if (e) return e;
        }
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        RW_HIP(hipEventRecord(ctx->ev_loop0, s));
        int64_t done = 0;
        rw_status err = RW_OK;
        int prev_iter[R];
        for (int r = 0; r < R; ++r) prev_iter[r] = host_st[r].iter_total;
        while (true) {
            if (!any_active()) {
                const int mask = refresh_mask();
                if (!mask) break;
                if ((err = refresh(mask))) break;
                for (int r = 0; r < R; ++r) prev_iter[r] = host_st[r].iter_total;
                continue;
            }
            if (graph) {
                if (!ge) {
                    RW_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                    for (int k = 0; k < m && !err; ++k) err = launch_iteration(nullptr);
                    hipError_t e1 = hipStreamEndCapture(s, &g);
                    if (err) break;
                    RW_HIP(e1);
                    RW_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
                }
                RW_HIP(hipGraphLaunch(ge, s));
            } else {
                for (int k = 0; k < m && !err; ++k)
                    err = launch_iteration(timing ? &ctx->pool[4 * k] : nullptr);
                if (err) break;
            }
            if ((err = read_state())) break;
            // iterations each label made in this block; launches that did work
            int kmax = 0;
            for (int r = 0; r < R; ++r) {
                const int d = host_st[r].iter_total - prev_iter[r];
                rhs_iters += d;
                rhs_vox += (int64_t)d * G.n;
                kmax = std::max(kmax, d);
                prev_iter[r] = host_st[r].iter_total;
            }
            box_vox += (int64_t)kmax * G.n;
            if (timing) {
                for (int k = 0; k < kmax; ++k) {
                    float a = 0.f, b = 0.f;
                    RW_HIP(hipEventElapsedTime(&a, ctx->pool[4 * k], ctx->pool[4 * k + 1]));
                    RW_HIP(hipEventElapsedTime(&b, ctx->pool[4 * k + 2], ctx->pool[4 * k + 3]));
                    pass_ms[0] += a;
                    pass_ms[1] += b;
                }
                launches[0] += kmax;
                launches[1] += kmax;
            }
            done += m;
            const int mask = refresh_mask();
            if (mask) {
                if ((err = refresh(mask))) break;
                for (int r = 0; r < R; ++r) prev_iter[r] = host_st[r].iter_total;
            }
            if (done > (int64_t)o->max_iter + 4 * m) {
                set_error("CG loop did not stop at max_iter");
                err = RW_ERR_HIP;
                break;
            }
        }
        hipError_t e2 = hipEventRecord(ctx->ev_loop1, s);
        if (e2 == hipSuccess) e2 = hipEventSynchronize(ctx->ev_loop1);
        float ms = 0.f;
        if (e2 == hipSuccess) e2 = hipEventElapsedTime(&ms, ctx->ev_loop0, ctx->ev_loop1);
        loop_ms += ms;
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
        if (err) return err;
        RW_HIP(e2);
        return RW_OK;
    }

    int refreshes() const {
        int s = 0;
        for (int r = 0; r < R; ++r) s += host_st[r].refreshes;
        return s;
    }

    rw_status run(const double* x0) {
        hipStream_t s = ctx->s;
        const size_t vbytes = sizeof(double) * size_t(R) * G.n;
        if (x0)
            RW_HIP(hipMemcpyAsync(B.x64, x0, vbytes, hipMemcpyDeviceToDevice, s));
        else
            RW_HIP(hipMemsetAsync(B.x64, 0, vbytes, s));
        rw_status e;
        if (!mixed) {
            if ((e = start(true, 0, o->tol))) return e;
            if ((e = inner())) return e;
            // final float64 true residual, for the statistics only
            RhsState keep[R];
            memcpy(keep, host_st, sizeof(keep));
            if ((e = launch_residual(0))) return e;
            hipLaunchKernelGGL((k_fin_init<R>), dim3(1), dim3(FIN_THREADS), 0, s, B.part,
                               tm.tiles, B.st, o->tol, o->tol, 0, 0, o->max_iter);
            if ((e = read_state())) return e;
            for (int r = 0; r < R; ++r) keep[r].rr64 = host_st[r].rr64;
            memcpy(host_st, keep, sizeof(keep));
            return RW_OK;
        }
        if (reliable) {
            if ((e = start(true, 0, o->tol))) return e;
            if ((e = inner())) return e;
            // labels stopped by the iteration cap still hold their last
            // correction in xi
            hipLaunchKernelGGL((k_update64<T, R>), dim3(grid1d(G.n)), dim3(256), 0, s, G.n,
                               (T*)B.xi, B.x64, (1 << R) - 1);
            RW_HIP(hipGetLastError());
            return RW_OK;
        }
        // restarted iterative refinement around float32 CG runs
        for (int ref = 0;; ++ref) {
            if ((e = start(ref == 0, ref == 0 ? 0 : 1, o->inner_tol))) return e;
            if (!any_active()) break;
            if (ref > o->max_refine) {
                for (int r = 0; r < R; ++r)
                    if (host_st[r].outer_active && host_st[r].status == ST_RUNNING)
                        host_st[r].status = ST_MAXITER;
                break;
            }
            int mask = 0;
            for (int r = 0; r < R; ++r)
                if (host_st[r].active) mask |= 1 << r;
            if ((e = inner())) return e;
            hipLaunchKernelGGL((k_update64<T, R>), dim3(grid1d(G.n)), dim3(256), 0, s, G.n,
                               (T*)B.xi, B.x64, mask);
            RW_HIP(hipGetLastError());
            for (int r = 0; r < R; ++r) host_st[r].refreshes += (mask >> r) & 1;
        }
        return RW_OK;
    }
};

template <typename V, typename T, int R, int VX, int BY = 4, bool T4 = false, int BY2 = BY>
inline rw_status run_group_vx(rw_context* ctx, const rw_volume* vol, const uint8_t* lab,
                              const rw_options* o, int lab0, const double* x0,
                              const GroupBuffers& B, const TileChoice& tc, void* prob_out,
                              rw_stats* stats, int r_base, int* worst, int tz = 0) {
    WholeSolve<V, T, R, VX, BY, T4, BY2> S;
    S.ctx = ctx;
    S.vol = static_cast<const V*>(vol->data);
    S.lab = lab;
    S.G = make_geom(vol->dims);
    S.G.tz = tz;
    S.wc = make_wcoef(vol, o->beta, o->w_eps);
    S.tm = make_tilemap(S.G, BY, tc.zc, tc.xcd, VX);
    // a time series takes the step-interleaved XCD-aware order when its
    // tiles fit the workspace's partial slots (RW_SERIES_PLAIN=1: the plain
    // volume order, for comparison)
    if (T4 && tz > 0 && S.G.nz / tz > 1 && tc.series)
        make_tilemap_series(S.G, BY, VX, int(S.G.nz / tz), tz, max_tiles(S.G), S.tm);
    if (BY2 != BY) S.tm2 = make_tilemap(S.G, BY2, tc.zc2, tc.xcd, VX);
    S.lab0 = lab0;
    S.mixed = o->precision == RW_PREC_MIXED;
    S.reliable = S.mixed && o->refine_mode == 0;
    S.o = o;
    S.B = B;
    S.zv = static_cast<T*>(B.z);
    S.p0 = static_cast<T*>(B.p0);
    S.p1 = static_cast<T*>(B.p1);
    S.xv = S.mixed ? static_cast<T*>(B.xi) : reinterpret_cast<T*>(B.x64);
    rw_status e = S.run(x0);
    if (e) return e;
    for (int r = 0; r < R; ++r) {
        const RhsState& h = S.host_st[r];
        int code = RW_OK;
        switch (h.status) {
            case ST_CONVERGED: code = RW_OK; break;
            case ST_RUNNING: code = S.mixed ? RW_NOT_CONVERGED : RW_OK; break;
            case ST_MAXITER: code = RW_NOT_CONVERGED; break;
            case ST_SINGULAR: code = RW_ERR_SINGULAR; break;
            case ST_BREAKDOWN: code = RW_ERR_BREAKDOWN; break;
            default: code = RW_ERR_NONFINITE; break;
        }
        if (stats && r_base + r < RW_MAX_LABELS) {
            stats->iters[r_base + r] = h.iter_total;
            stats->label_status[r_base + r] = code;
            stats->rel_residual[r_base + r] = h.bb > 0 ? std::sqrt(h.rr64 / h.bb) : 0.0;
        }
        if (code < 0 && (*worst >= 0 || code < *worst)) *worst = code;
        if (code > 0 && *worst == RW_OK) *worst = code;
    }
    if (stats) {
        stats->loop_ms += S.loop_ms;
        stats->pass_ms[0] += S.pass_ms[0];
        stats->pass_ms[1] += S.pass_ms[1];
        stats->pass_launches[0] += S.launches[0];
        stats->pass_launches[1] += S.launches[1];
        stats->rhs_iterations += S.rhs_iters;
        stats->box_voxel_iterations += S.box_vox;
        stats->rhs_voxel_iterations += S.rhs_vox;
        stats->refinements += S.refreshes();
        stats->tile_by = S.tm.by;
        stats->tile_by2 = S.map2().by;
        stats->tile_zc2 = S.map2().zc;
        stats->tile_zc = S.tm.zc;
        stats->tile_vx = VX;
        stats->tile_xcd = S.tm.xcd;
        stats->tile_tuned = tc.tuned;
    }
    if (*worst < 0) return RW_OK;  // caller reports, outputs untouched
    const int64_t n = S.G.n;
    if (S.mixed)
        hipLaunchKernelGGL((k_write_labels<float, R>), dim3(grid1d(n)), dim3(256), 0, ctx->s, lab,
                           n, B.x64, lab0, (float*)prob_out);
    else
        hipLaunchKernelGGL((k_write_labels<double, R>), dim3(grid1d(n)), dim3(256), 0, ctx->s,
                           lab, n, B.x64, lab0, (double*)prob_out);
    RW_HIP(hipGetLastError());
    return RW_OK;
}

}  // namespace rw
