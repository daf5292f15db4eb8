// Batched brick solves of the coarse-to-fine random walker: per-brick
// finalize kernels, worklist compaction, brick set-up/fold/output kernels,
// the brick plan, and the driver (BrickSolve).  Instantiated per volume type
// and precision in rw_bricks_*.hip (separate translation units, so they
// compile in parallel); rw_hier.hip holds the entry points.
#pragma once

#include <algorithm>
#include <cstring>
#include <vector>

#include "rw_whole.h"

namespace rw {

template <int NQ>
__device__ __forceinline__ void brick_sums(const double* __restrict__ part, int ntiles,
                                           const BrickGeo& B, double* sums) {
    double a[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) a[q] = 0.0;
    for (int j = threadIdx.x; j < B.ntiles; j += 64) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) a[q] += part[(int64_t)q * ntiles + B.tile0 + j];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a[q] += __shfl_xor(a[q], off, 64);
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) sums[q] = a[q];
    }
    __syncthreads();
}

template <int R>
__device__ __forceinline__ bool brick_any(const RhsState* st, int b, bool need_active) {
    bool a = false;
    for (int r = 0; r < R; ++r)
        a |= need_active ? st[b * R + r].active != 0 : st[b * R + r].outer_active == 2;
    return a;
}

// The per-brick, per-label state updates between the passes (shared by the
// per-pass kernels below and the persistent brick kernel).  sums: the
// brick's sums of the pass's partials.

// Start of a brick's CG run from its residual (label r; sums [4R + 2]).
template <int R>
__device__ __forceinline__ void bfin_init_logic(RhsState& s, int r, const double* sums, double tol,
                                                int max_iter) {
    memset(&s, 0, sizeof(RhsState));
    s.bb = sums[4 * r + 3];
    s.rr64 = sums[4 * r + 2];
    s.max_iter = max_iter;
    s.status = ST_RUNNING;
    s.outer_active = 1;
    if (sums[4 * R + 1] > 0) s.status = ST_NONFINITE;
    else if (sums[4 * R] > 0) s.status = ST_SINGULAR;
    else if (s.bb == 0.0 || s.rr64 <= tol * tol * s.bb) s.status = ST_CONVERGED;
    if (s.status != ST_RUNNING) {
        s.outer_active = 0;
        return;
    }
    s.active = 1;
    s.rho = sums[4 * r + 0];
    s.rho_prev = s.rho;
    s.rr = sums[4 * r + 1];
    s.rr_ref = s.rr;
    s.thresh2 = tol * tol * s.bb;
}

// After pass 1 of an active label: alpha, or breakdown.
__device__ __forceinline__ void bfin1_logic(RhsState& s, double sigma) {
    s.pcur ^= 1;
    if (!(sigma > 0.0) || !isfinite(sigma)) {
        s.status = ST_BREAKDOWN;
        s.active = 0;
        s.outer_active = 0;
    } else {
        s.alpha = s.rho / sigma;
    }
}

// After pass 2 of an active label (mixed: a label whose recurrence
// residual has fallen by update_delta since the last refresh, or that met
// the tolerance, is flagged for a float64 refresh, outer_active = 2; it keeps
// iterating until then unless converged).
__device__ __forceinline__ void bfin2_logic(RhsState& s, double rz, double rr, int mixed,
                                            double delta2) {
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
        if (mixed) {
            s.outer_active = 2;
        } else {
            s.status = ST_CONVERGED;
            s.outer_active = 0;
        }
    } else if (s.iter_total >= s.max_iter) {
        s.active = 0;
        s.status = ST_MAXITER;
        s.outer_active = 0;
    } else if (mixed && rr < delta2 * s.rr_ref) {
        s.outer_active = 2;
    }
}

// After a float64 refresh of a flagged label (sums [4R + 2]).
template <int R>
__device__ __forceinline__ void bfin_refresh_logic(RhsState& s, int r, const double* sums,
                                                   double tol) {
    s.rr64 = sums[4 * r + 2];
    s.refreshes += 1;
    if (!isfinite(s.rr64) || !isfinite(sums[4 * r])) {
        s.status = ST_NONFINITE;
        s.active = 0;
        s.outer_active = 0;
    } else if (s.rr64 <= tol * tol * s.bb) {
        s.status = ST_CONVERGED;
        s.active = 0;
        s.outer_active = 0;
    } else if (s.iter_total >= s.max_iter) {
        s.status = ST_MAXITER;
        s.active = 0;
        s.outer_active = 0;
    } else {
        s.rho = sums[4 * r + 0];
        s.beta = s.rho / s.rho_prev;
        s.rr = sums[4 * r + 1];
        s.rr_ref = s.rr;
        s.active = 1;
        s.outer_active = 1;
    }
}

template <int R>
__global__ __launch_bounds__(64) void k_bfin_init(const double* __restrict__ part, int ntiles,
                                                  const BrickGeo* __restrict__ geo,
                                                  RhsState* __restrict__ st, double tol,
                                                  int max_iter) {
    constexpr int NQ = 4 * R + 2;
    __shared__ double sums[NQ];
    const BrickGeo B = geo[blockIdx.x];
    brick_sums<NQ>(part, ntiles, B, sums);
    const int r = threadIdx.x;
    if (r >= R) return;
    bfin_init_logic<R>(st[blockIdx.x * R + r], r, sums, tol, max_iter);
}

template <int R>
__global__ __launch_bounds__(64) void k_bfin1(const double* __restrict__ part, int ntiles,
                                              const BrickGeo* __restrict__ geo,
                                              RhsState* __restrict__ st) {
    if (!brick_any<R>(st, blockIdx.x, true)) return;
    __shared__ double sums[R];
    brick_sums<R>(part, ntiles, geo[blockIdx.x], sums);
    const int r = threadIdx.x;
    if (r < R) {
        RhsState& s = st[blockIdx.x * R + r];
        if (!s.active) return;
        bfin1_logic(s, sums[r]);
    }
}

template <int R>
__global__ __launch_bounds__(64) void k_bfin2(const double* __restrict__ part, int ntiles,
                                              const BrickGeo* __restrict__ geo,
                                              RhsState* __restrict__ st, int mixed, double delta2) {
    if (!brick_any<R>(st, blockIdx.x, true)) return;
    __shared__ double sums[2 * R];
    brick_sums<2 * R>(part, ntiles, geo[blockIdx.x], sums);
    const int r = threadIdx.x;
    if (r < R) {
        RhsState& s = st[blockIdx.x * R + r];
        if (!s.active) return;
        bfin2_logic(s, sums[2 * r], sums[2 * r + 1], mixed, delta2);
    }
}

template <int R>
__global__ __launch_bounds__(64) void k_bfin_refresh(const double* __restrict__ part, int ntiles,
                                                     const BrickGeo* __restrict__ geo,
                                                     RhsState* __restrict__ st, double tol) {
    constexpr int NQ = 4 * R + 2;
    if (!brick_any<R>(st, blockIdx.x, false)) return;
    __shared__ double sums[NQ];
    brick_sums<NQ>(part, ntiles, geo[blockIdx.x], sums);
    const int r = threadIdx.x;
    if (r >= R) return;
    RhsState& s = st[blockIdx.x * R + r];
    if (s.outer_active != 2) return;
    bfin_refresh_logic<R>(s, r, sums, tol);
}

// Worklists: the tiles of the bricks with a label iterating, and of the
// bricks with a label flagged for a refresh (bricks in order, tiles in
// order); counts = {active tiles, refresh tiles, labels iterating, labels
// flagged}.  One block.
template <int R>
__global__ __launch_bounds__(1024) void k_compact(const BrickGeo* __restrict__ geo, int nb,
                                                  const RhsState* __restrict__ st,
                                                  int* __restrict__ list_act,
                                                  int* __restrict__ list_ref,
                                                  int* __restrict__ counts) {
    __shared__ int sa[1024], sr[1024], pa[1024], pf[1024];
    const int tid = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
    int ta = 0, tr = 0, na = 0, nf = 0;
    for (int b = b0; b < b1; ++b) {
        bool a = false, f = false;
        for (int r = 0; r < R; ++r) {
            const RhsState& s = st[b * R + r];
            a |= s.active != 0;
            f |= s.outer_active == 2;
            na += s.active != 0;
            nf += s.outer_active == 2;
        }
        if (a) ta += geo[b].ntiles;
        if (f) tr += geo[b].ntiles;
    }
    sa[tid] = ta;
    sr[tid] = tr;
    pa[tid] = na;
    pf[tid] = nf;
    __syncthreads();
    // inclusive scans (Hillis-Steele, fixed order)
    for (int o = 1; o < 1024; o <<= 1) {
        const int va = tid >= o ? sa[tid - o] : 0, vr = tid >= o ? sr[tid - o] : 0;
        const int wa = tid >= o ? pa[tid - o] : 0, wf = tid >= o ? pf[tid - o] : 0;
        __syncthreads();
        sa[tid] += va;
        sr[tid] += vr;
        pa[tid] += wa;
        pf[tid] += wf;
        __syncthreads();
    }
    int oa = sa[tid] - ta, orf = sr[tid] - tr;
    for (int b = b0; b < b1; ++b) {
        bool a = false, f = false;
        for (int r = 0; r < R; ++r) {
            a |= st[b * R + r].active != 0;
            f |= st[b * R + r].outer_active == 2;
        }
        const int t0 = geo[b].tile0, nt = geo[b].ntiles;
        if (a)
            for (int j = 0; j < nt; ++j) list_act[oa++] = t0 + j;
        if (f)
            for (int j = 0; j < nt; ++j) list_ref[orf++] = t0 + j;
    }
    if (tid == 1023) {
        counts[0] = sa[1023];
        counts[1] = sr[1023];
        counts[2] = pa[1023];
        counts[3] = pf[1023];
    }
}

// x64 = upsampled coarse value on the unknowns of the boxes, xi = 0.
template <typename T, int R>
__global__ __launch_bounds__(256) void k_brick_init(BrickTiles ts, Shell sh, int lab0,
                                                    const uint8_t* __restrict__ lab,
                                                    const float* __restrict__ x0, int64_t x0_stride,
                                                    double* __restrict__ x64, T* __restrict__ xi) {
    const int cnt = ts.count();
    for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
        BoxTile bt;
        if (!ts.get(it, bt)) continue;
        const int lxb = bt.X0 + (threadIdx.x & 63), lyb = bt.Y0 + (threadIdx.x >> 6);
        for (int yy = lyb; yy < min(bt.Y0 + ts.by, bt.sy); yy += 4) {
            if (lxb >= bt.sx) break;
            for (int lz = bt.z0; lz < bt.z1; ++lz) {
                const int gx = bt.ox + lxb, gy = bt.oy + yy, gz = bt.oz + lz;
                const int64_t cb = ((int64_t)lz * bt.sy + yy) * bt.sx + lxb;
                const int64_t v = bt.voff + (int64_t)gz * bt.G.plane + (int64_t)gy * bt.G.nx + gx;
                const uint8_t l = lab[v];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t o = bt.vbase + r * bt.vstride + cb;
                    double xv = 0.0;
                    if (!l)
                        xv = x0 ? (double)x0[(int64_t)(lab0 - 1 + r) * x0_stride + v]
                                : upsample(sh, lab0 + r, bt.gox + gx, bt.goy + gy, bt.goz + gz);
                    x64[o] = xv;
                    if (xi) xi[o] = T(0);
                }
            }
        }
    }
}

// x64 += xi, xi = 0 on the cells of the listed tiles, for the labels
// flagged for a refresh (all labels when all = 1).
template <typename T, int R>
__global__ __launch_bounds__(256) void k_brick_fold(BrickTiles ts,
                                                    const RhsState* __restrict__ st,
                                                    double* __restrict__ x64, T* __restrict__ xi,
                                                    int all) {
    const int cnt = ts.count();
    for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
        BoxTile bt;
        if (!ts.get(it, bt)) continue;
        int mask = 0;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (all || st[bt.sidx * R + r].outer_active == 2) mask |= 1 << r;
        if (!mask) continue;
        // seeds need no test: xi is 0 there (never written but as 0), so
        // x64 keeps its value and the loads of a column pipeline freely
        const int lxb = bt.X0 + (threadIdx.x & 63);
        for (int yy = bt.Y0 + (threadIdx.x >> 6); yy < min(bt.Y0 + ts.by, bt.sy); yy += 4) {
            if (lxb >= bt.sx) break;
#pragma unroll 4
            for (int lz = bt.z0; lz < bt.z1; ++lz) {
                const int64_t cb = ((int64_t)lz * bt.sy + yy) * bt.sx + lxb;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (mask & (1 << r)) {
                        const int64_t o = bt.vbase + r * bt.vstride + cb;
                        x64[o] += (double)xi[o];
                        xi[o] = T(0);
                    }
            }
        }
    }
}

// Fine-grid output of the bricks: solved labels from x64 (seeds exact), the
// background as the complement when it was not solved.
template <int R>
__global__ __launch_bounds__(256) void k_brick_write(BrickTiles ts, Geom F,
                                                     const uint8_t* __restrict__ lab,
                                                     const double* __restrict__ x64, int lab0,
                                                     int K, int complement,
                                                     float* __restrict__ prob) {
    const int cnt = ts.count();
    for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
        BoxTile bt;
        if (!ts.get(it, bt)) continue;
        const int lxb = bt.X0 + (threadIdx.x & 63);
        for (int yy = bt.Y0 + (threadIdx.x >> 6); yy < min(bt.Y0 + ts.by, bt.sy); yy += 4) {
            if (lxb >= bt.sx) break;
            for (int lz = bt.z0; lz < bt.z1; ++lz) {
                const int64_t g = bt.voff + (int64_t)(bt.oz + lz) * bt.G.plane +
                                  (int64_t)(bt.oy + yy) * bt.G.nx + bt.ox + lxb;
                const int64_t cb = ((int64_t)lz * bt.sy + yy) * bt.sx + lxb;
                const uint8_t l = lab[g];
                double s = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int L = lab0 + r;
                    const double v = l ? (l == L ? 1.0 : 0.0) : x64[bt.vbase + r * bt.vstride + cb];
                    s += v;
                    prob[(int64_t)(L - 1) * F.n + g] = (float)v;
                }
                if (complement) prob[g] = l ? (l == 1 ? 1.f : 0.f) : (float)(1.0 - s);
            }
        }
    }
}

// ------------------------------------------------------------ persistent form

// Fixed-order sum of NQ per-thread values over the block (wave butterfly,
// then the wave totals in wave order); the totals land in red[NW * NQ + q],
// visible to every thread on return.  red: NW * NQ + NQ doubles of LDS.
template <int NQ, int NW>
__device__ __forceinline__ void block_sum_lds(double (&v)[NQ], double* __restrict__ red) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double a = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
        v[q] = a;
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) red[wid * NQ + q] = v[q];
    }
    __syncthreads();
    if (tid < NQ) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += red[w * NQ + tid];
        red[NW * NQ + tid] = s;
    }
    __syncthreads();
}

template <typename V, typename T, int R, int BY, int BVX>
struct PersistSmem {
    static constexpr bool YM = BVX > 1;
    static constexpr int ZU = PlaneBatch<T, BVX>::value;
    static constexpr size_t pass = PassSmem<T, R, BY, ZU, BVX, YM>::bytes;
    static constexpr size_t res = ResidualSmem<V, R, BY, BVX, YM>::bytes;
    static constexpr size_t bytes = pass > res ? pass : res;
};

// Every brick of a level in one launch: a block claims the next brick from
// an atomic queue (bricks in plan order, largest first), runs that brick's
// whole mixed-precision Jacobi-PCG (start, CG passes over the brick's tiles,
// float64 refreshes when the residual has fallen by update_delta, the final
// fold) with the brick's reductions and convergence state held in the block
// (LDS), then claims the next; no block waits for another.  The tile work is
// the per-pass kernels' own (cg_pass1_tile, cg_pass2_tile, residual_tile).
// Every loop is bounded (4 max_iter + 64 rounds per brick), so each block
// exits once the queue is empty.
template <typename V, typename T, int R, int BY, int BVX>
__global__ __launch_bounds__(64 * BY, 4) void k_bricks_persistent(
    const V* __restrict__ vol, const uint8_t* __restrict__ lab, WCoef wc, Shell sh, int lab0,
    const BrickGeo* __restrict__ geo, int nb, int zc, int* __restrict__ queue,
    const float* __restrict__ x0, int64_t x0_stride, double* __restrict__ x64, T* __restrict__ xi,
    T* __restrict__ zv, T* __restrict__ p0, T* __restrict__ p1, RhsState* __restrict__ st_out,
    double tol, int max_iter, double delta2) {
    using SM = PersistSmem<V, T, R, BY, BVX>;
    constexpr bool YM = SM::YM;
    constexpr int ZU = SM::ZU;
    constexpr int NQ = 4 * R + 2;
    __shared__ __align__(16) char smem[SM::bytes];
    __shared__ double red[BY * NQ + NQ];
    __shared__ RhsState sst[R];
    __shared__ int sb;
    const int tid = threadIdx.x + 64 * threadIdx.y;
    constexpr int NT = 64 * BY;
    const int rows = BY * BVX;
    for (;;) {
        __syncthreads();
        if (tid == 0) sb = atomicAdd(queue, 1);
        __syncthreads();
        const int b = sb;
        if (b >= nb) return;
        const BrickGeo B = geo[b];
        const int64_t vplane = (int64_t)B.vnx * B.vny;
        // x64 = the initial guess (x0, or the upsampled coarse value) on the
        // brick's unknowns, 0 on its seeds; xi = 0
        for (int64_t c = tid; c < B.vox; c += NT) {
            const int lxb = int(c % B.sx);
            const int yy = int((c / B.sx) % B.sy);
            const int lz = int(c / ((int64_t)B.sx * B.sy));
            const int gx = B.ox + lxb, gy = B.oy + yy, gz = B.oz + lz;
            const int64_t v = B.vvoff + (int64_t)gz * vplane + (int64_t)gy * B.vnx + gx;
            const uint8_t l = lab[v];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t o = B.voff + r * B.vox + c;
                double xv = 0.0;
                if (!l)
                    xv = x0 ? (double)x0[(int64_t)(lab0 - 1 + r) * x0_stride + v]
                            : upsample(sh, lab0 + r, B.gox + gx, B.goy + gy, B.goz + gz);
                x64[o] = xv;
                xi[o] = T(0);
            }
        }
        __syncthreads();
        BoxTile bt;
        {
            double acc[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
            for (int t = 0; t < B.ntiles; ++t) {
                BrickTiles::brick_tile(B, t, zc, rows, 0, 0, bt);
                residual_tile<V, T, R, BY, BVX, YM>(smem, bt, vol, lab, wc, sh, lab0, x64, nullptr,
                                                    zv, p0, p1, xi, 1, sst, acc);
            }
            block_sum_lds<NQ, BY>(acc, red);
            if (tid < R) bfin_init_logic<R>(sst[tid], tid, red + BY * NQ, tol, max_iter);
            __syncthreads();
        }
        for (int guard = 0; guard < 4 * max_iter + 64; ++guard) {
            bool act = false, ref = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                act |= sst[r].active != 0;
                ref |= sst[r].outer_active == 2;
            }
            if (!act && !ref) break;
            if (act) {
                double a1[R];
#pragma unroll
                for (int r = 0; r < R; ++r) a1[r] = 0.0;
                for (int t = 0; t < B.ntiles; ++t) {
                    BrickTiles::brick_tile(B, t, zc, rows, 0, 0, bt);
                    cg_pass1_tile<V, T, R, BY, ZU, BVX, YM>(smem, bt, vol, wc, zv, p0, p1,
                                                            (T*)nullptr, sst, a1);
                }
                block_sum_lds<R, BY>(a1, red);
                if (tid < R && sst[tid].active) bfin1_logic(sst[tid], red[BY * R + tid]);
                __syncthreads();
                double a2[2 * R];
#pragma unroll
                for (int q = 0; q < 2 * R; ++q) a2[q] = 0.0;
                for (int t = 0; t < B.ntiles; ++t) {
                    BrickTiles::brick_tile(B, t, zc, rows, 0, 0, bt);
                    cg_pass2_tile<V, T, R, BY, ZU, BVX, YM>(smem, bt, vol, lab, wc, xi, zv, p0, p1,
                                                            sst, a2);
                }
                block_sum_lds<2 * R, BY>(a2, red);
                if (tid < R && sst[tid].active)
                    bfin2_logic(sst[tid], red[2 * BY * R + 2 * tid], red[2 * BY * R + 2 * tid + 1],
                                1, delta2);
                __syncthreads();
                ref = false;
#pragma unroll
                for (int r = 0; r < R; ++r) ref |= sst[r].outer_active == 2;
            }
            if (ref) {
                // x64 += xi, xi = 0 for the flagged labels; then their float64
                // residual and the continuation (or end) of their CG runs
                for (int64_t c = tid; c < B.vox; c += NT) {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (sst[r].outer_active == 2) {
                            const int64_t o = B.voff + r * B.vox + c;
                            x64[o] += (double)xi[o];
                            xi[o] = T(0);
                        }
                }
                __syncthreads();
                double a3[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) a3[q] = 0.0;
                for (int t = 0; t < B.ntiles; ++t) {
                    BrickTiles::brick_tile(B, t, zc, rows, 0, 0, bt);
                    residual_tile<V, T, R, BY, BVX, YM>(smem, bt, vol, lab, wc, sh, lab0, x64,
                                                        nullptr, zv, p0, p1, xi, 2, sst, a3);
                }
                block_sum_lds<NQ, BY>(a3, red);
                if (tid < R && sst[tid].outer_active == 2)
                    bfin_refresh_logic<R>(sst[tid], tid, red + BY * NQ, tol);
                __syncthreads();
            }
        }
        // labels stopped by the iteration cap still hold their last
        // correction in xi
        for (int64_t c = tid; c < B.vox; c += NT) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t o = B.voff + r * B.vox + c;
                x64[o] += (double)xi[o];
                xi[o] = T(0);
            }
        }
        if (tid < R) st_out[b * R + tid] = sst[tid];
    }
}

static __global__ void k_zero_int(int* __restrict__ p) { *p = 0; }

struct BrickPlan {
    std::vector<BrickGeo> geo;
    std::vector<int> tile_brick;
    std::vector<int> order;  // solve order -> caller's brick index
    int ntiles = 0;
    int64_t vox = 0;
};

// Bricks sorted by decreasing size (stable), tiles of 64 x by x zc.
inline int64_t max_brick_voxels(const rw_brick* bricks, int n) {
    int64_t m = 0;
    for (int i = 0; i < n; ++i)
        m = std::max<int64_t>(m, (int64_t)bricks[i].sx * bricks[i].sy * bricks[i].sz);
    return m;
}

inline BrickPlan make_plan(const rw_brick* bricks, int n, int R, int by, int zc,
                           const rw_subvolume* sub = nullptr, rw_dims vol = rw_dims{1, 1, 1}) {
    BrickPlan P;
    P.order.resize(n);
    for (int i = 0; i < n; ++i) P.order[i] = i;
    std::stable_sort(P.order.begin(), P.order.end(), [&](int a, int b) {
        const int64_t va = (int64_t)bricks[a].sx * bricks[a].sy * bricks[a].sz;
        const int64_t vb = (int64_t)bricks[b].sx * bricks[b].sy * bricks[b].sz;
        return va > vb;
    });
    for (int i = 0; i < n; ++i) {
        const rw_brick& b = bricks[P.order[i]];
        BrickGeo g;
        if (sub) {
            const rw_subvolume& v = sub[P.order[i]];
            g.vnx = v.nx;
            g.vny = v.ny;
            g.vnz = v.nz;
            g.gox = v.gx;
            g.goy = v.gy;
            g.goz = v.gz;
            g.vvoff = v.offset;
        } else {
            g.vnx = int(vol.nx);
            g.vny = int(vol.ny);
            g.vnz = int(vol.nz);
            g.gox = g.goy = g.goz = 0;
            g.vvoff = 0;
        }
        g.ox = b.ox;
        g.oy = b.oy;
        g.oz = b.oz;
        g.sx = b.sx;
        g.sy = b.sy;
        g.sz = b.sz;
        g.gx = (b.sx + 63) / 64;
        g.gy = (b.sy + by - 1) / by;
        const int gz = (b.sz + zc - 1) / zc;
        g.tile0 = P.ntiles;
        g.ntiles = g.gx * g.gy * gz;
        g.vox = (int64_t)b.sx * b.sy * b.sz;
        g.voff = P.vox * R;
        P.vox += g.vox;
        for (int t = 0; t < g.ntiles; ++t) P.tile_brick.push_back(i);
        P.ntiles += g.ntiles;
        P.geo.push_back(g);
    }
    return P;
}

struct BrickBuffers {
    BrickGeo* geo;
    int* tile_brick;
    int* list_act;
    int* list_ref;
    int* list_all;
    int* counts;  // [0..3] worklist counts, [4] all tiles
    double* x64;
    void* xi;
    void* z;
    void* p0;
    void* p1;
    double* part;
    RhsState* st;
};

inline size_t carve_bricks(Carver& cv, const BrickPlan& P, int R, bool mixed, BrickBuffers* b) {
    const size_t nb = P.geo.size();
    const size_t vs = mixed ? 4 : 8;
    const size_t nv = size_t(R) * P.vox;
    BrickBuffers t;
    t.geo = cv.take<BrickGeo>(nb);
    t.tile_brick = cv.take<int>(P.ntiles);
    t.list_act = cv.take<int>(P.ntiles);
    t.list_ref = cv.take<int>(P.ntiles);
    t.list_all = cv.take<int>(P.ntiles);
    t.counts = cv.take<int>(8);
    t.x64 = cv.take<double>(nv);
    t.xi = mixed ? (void*)cv.take<char>(vs * nv) : nullptr;
    t.z = cv.take<char>(vs * nv);
    t.p0 = cv.take<char>(vs * nv);
    t.p1 = cv.take<char>(vs * nv);
    t.part = cv.take<double>(size_t(P.ntiles) * (4 * 4 + 2));
    t.st = cv.take<RhsState>(nb * R);
    if (b) *b = t;
    return cv.bytes();
}

// BVX = 2: each lane owns two rows BY apart (64 x 2 BY column tiles).
template <typename V, typename T, int R, int BY, int BVX = 1>
struct BrickSolve {
    static constexpr bool YM = BVX > 1;
    static constexpr int ZU = PlaneBatch<T, BVX>::value;
    rw_context* ctx;
    const V* vol;
    const uint8_t* lab;
    Geom F;
    WCoef wc;
    Shell sh;
    const rw_options* o;
    bool mixed;
    int lab0, zc, nb, xcd = 0;
    BrickPlan* P;
    BrickBuffers B;
    int grid;
    int counts[8];
    std::vector<RhsState> hst, prev;
    double loop_ms = 0.0, pass_ms[2] = {0, 0};
    int persist_blocks = 0;
    int64_t launches[2] = {0, 0}, rhs_iters = 0, box_vox = 0, rhs_vox = 0;

    BrickTiles tiles(const int* list, const int* count) const {
        BrickTiles t;
        t.bricks = B.geo;
        t.tile_brick = B.tile_brick;
        t.list = list;
        t.list_count = count;
        t.zc = zc;
        t.by = BY * BVX;  // rows per tile
        t.xcd = xcd;
        t.ntiles = P->ntiles;
        return t;
    }
    BrickTiles act() const { return tiles(B.list_act, B.counts + 0); }
    BrickTiles ref() const { return tiles(B.list_ref, B.counts + 1); }
    BrickTiles all() const { return tiles(B.list_all, B.counts + 4); }

    rw_status compact() {
        hipLaunchKernelGGL((k_compact<R>), dim3(1), dim3(1024), 0, ctx->s, B.geo, nb, B.st,
                           B.list_act, B.list_ref, B.counts);
        RW_HIP(hipGetLastError());
        RW_HIP(hipMemcpyAsync(ctx->host_pinned, B.counts, 4 * sizeof(int), hipMemcpyDeviceToHost,
                              ctx->s));
        RW_HIP(hipStreamSynchronize(ctx->s));
        memcpy(counts, ctx->host_pinned, 4 * sizeof(int));
        return RW_OK;
    }

    rw_status read_states() {
        const size_t bytes = sizeof(RhsState) * size_t(nb) * R;
        rw_status e = ensure_host_pinned(ctx, bytes);
        if (e) return e;
        RW_HIP(hipMemcpyAsync(ctx->host_pinned, B.st, bytes, hipMemcpyDeviceToHost, ctx->s));
        RW_HIP(hipStreamSynchronize(ctx->s));
        hst.resize(size_t(nb) * R);
        memcpy(hst.data(), ctx->host_pinned, bytes);
        return RW_OK;
    }

    // work accounting from the iteration counters (bricks x labels)
    int account() {
        int kmax = 0;
        for (int b = 0; b < nb; ++b) {
            int bmax = 0;
            for (int r = 0; r < R; ++r) {
                const int d = hst[b * R + r].iter_total - prev[b * R + r].iter_total;
                rhs_iters += d;
                rhs_vox += (int64_t)d * P->geo[b].vox;
                bmax = std::max(bmax, d);
            }
            box_vox += (int64_t)bmax * P->geo[b].vox;
            kmax = std::max(kmax, bmax);
        }
        prev = hst;
        return kmax;
    }

    rw_status launch_iteration(hipEvent_t* ev) {
        hipStream_t s = ctx->s;
        const BrickTiles ta = act();
        if (ev) RW_HIP(hipEventRecord(ev[0], s));
        hipLaunchKernelGGL((k_cg_pass1<V, T, R, BY, ZU, BVX, BrickTiles, YM>), dim3(grid), dim3(64, BY), 0,
                           s, vol, wc, ta, (const T*)B.z, (T*)B.p0, (T*)B.p1, (T*)nullptr, B.st,
                           B.part);
        if (ev) RW_HIP(hipEventRecord(ev[1], s));
        hipLaunchKernelGGL((k_bfin1<R>), dim3(nb), dim3(64), 0, s, B.part, P->ntiles, B.geo, B.st);
        if (ev) RW_HIP(hipEventRecord(ev[2], s));
        hipLaunchKernelGGL((k_cg_pass2<V, T, R, BY, ZU, BVX, BrickTiles, YM>), dim3(grid), dim3(64, BY), 0,
                           s, vol, lab, wc, ta, mixed ? (T*)B.xi : (T*)B.x64, (T*)B.z,
                           (const T*)B.p0, (const T*)B.p1, B.st, B.part);
        if (ev) RW_HIP(hipEventRecord(ev[3], s));
        hipLaunchKernelGGL((k_bfin2<R>), dim3(nb), dim3(64), 0, s, B.part, P->ntiles, B.geo, B.st,
                           mixed ? 1 : 0, o->update_delta * o->update_delta);
        RW_HIP(hipGetLastError());
        return RW_OK;
    }

    rw_status refresh() {
        hipStream_t s = ctx->s;
        const BrickTiles tr = ref();
        hipLaunchKernelGGL((k_brick_fold<T, R>), dim3(grid), dim3(256), 0, s, tr, B.st,
                           B.x64, (T*)B.xi, 0);
        hipLaunchKernelGGL((k_residual<V, T, R, BY, BVX, BrickTiles, YM>), dim3(grid), dim3(64, BY), 0, s,
                           vol, lab, wc, tr, sh, lab0, B.x64, (const double*)nullptr, (T*)B.z,
                           (T*)B.p0, (T*)B.p1, (T*)B.xi, 2, B.st, B.part);
        hipLaunchKernelGGL((k_bfin_refresh<R>), dim3(nb), dim3(64), 0, s, B.part, P->ntiles, B.geo,
                           B.st, o->tol);
        RW_HIP(hipGetLastError());
        return compact();
    }

    // The persistent form: one launch of k_bricks_persistent over every
    // brick (grid = the blocks the device holds at once, at most one per
    // brick), then the final states for the statistics.
    rw_status run_persistent() {
        hipStream_t s = ctx->s;
        std::vector<int> all_ids(P->ntiles);
        for (int i = 0; i < P->ntiles; ++i) all_ids[i] = i;
        int cnt_all[8] = {P->ntiles, 0, 0, 0, P->ntiles, 0, 0, 0};
        RW_HIP(hipMemcpyAsync(B.geo, P->geo.data(), sizeof(BrickGeo) * nb, hipMemcpyHostToDevice, s));
        RW_HIP(hipMemcpyAsync(B.tile_brick, P->tile_brick.data(), sizeof(int) * P->ntiles,
                              hipMemcpyHostToDevice, s));
        RW_HIP(hipMemcpyAsync(B.list_all, all_ids.data(), sizeof(int) * P->ntiles,
                              hipMemcpyHostToDevice, s));
        RW_HIP(hipMemcpyAsync(B.counts, cnt_all, sizeof(cnt_all), hipMemcpyHostToDevice, s));
        int* queue = B.counts + 6;
        hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, queue);
        auto kern = k_bricks_persistent<V, T, R, BY, BVX>;
        int per_cu = 0, cus = 0;
        RW_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                            64 * BY, 0));
        RW_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
        const int blocks = std::max(1, std::min(nb, std::max(1, per_cu) * std::max(1, cus)));
        RW_HIP(hipEventRecord(ctx->ev_loop0, s));
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(64, BY), 0, s, vol, lab, wc, sh, lab0, B.geo, nb,
                           zc, queue, static_cast<const float*>(o->x0), int64_t(F.n), B.x64,
                           (T*)B.xi, (T*)B.z, (T*)B.p0, (T*)B.p1, B.st, o->tol, o->max_iter,
                           o->update_delta * o->update_delta);
        RW_HIP(hipGetLastError());
        RW_HIP(hipEventRecord(ctx->ev_loop1, s));
        RW_HIP(hipEventSynchronize(ctx->ev_loop1));
        float ms = 0.f;
        RW_HIP(hipEventElapsedTime(&ms, ctx->ev_loop0, ctx->ev_loop1));
        loop_ms += ms;
        persist_blocks = blocks;
        rw_status e = read_states();
        if (e) return e;
        prev.assign(hst.size(), RhsState{});
        account();
        return RW_OK;
    }

    rw_status run() {
        hipStream_t s = ctx->s;
        // tables and the all-tiles list
        std::vector<int> all_ids(P->ntiles);
        for (int i = 0; i < P->ntiles; ++i) all_ids[i] = i;
        int cnt_all[8] = {P->ntiles, 0, 0, 0, P->ntiles, 0, 0, 0};
        RW_HIP(hipMemcpyAsync(B.geo, P->geo.data(), sizeof(BrickGeo) * nb, hipMemcpyHostToDevice, s));
        RW_HIP(hipMemcpyAsync(B.tile_brick, P->tile_brick.data(), sizeof(int) * P->ntiles,
                              hipMemcpyHostToDevice, s));
        RW_HIP(hipMemcpyAsync(B.list_all, all_ids.data(), sizeof(int) * P->ntiles,
                              hipMemcpyHostToDevice, s));
        RW_HIP(hipMemcpyAsync(B.counts, cnt_all, sizeof(cnt_all), hipMemcpyHostToDevice, s));
        // x0 = the caller's initial guess or the upsampled coarse solution,
        // then the brick residuals
        hipLaunchKernelGGL((k_brick_init<T, R>), dim3(grid), dim3(256), 0, s, all(), sh, lab0, lab,
                           static_cast<const float*>(o->x0), F.n, B.x64,
                           mixed ? (T*)B.xi : (T*)nullptr);
        hipLaunchKernelGGL((k_residual<V, T, R, BY, BVX, BrickTiles, YM>), dim3(grid), dim3(64, BY), 0, s,
                           vol, lab, wc, all(), sh, lab0, B.x64, (const double*)nullptr, (T*)B.z,
                           (T*)B.p0, (T*)B.p1, mixed ? (T*)B.xi : (T*)nullptr, 1, B.st, B.part);
        hipLaunchKernelGGL((k_bfin_init<R>), dim3(nb), dim3(64), 0, s, B.part, P->ntiles, B.geo, B.st,
                           o->tol, o->max_iter);
        RW_HIP(hipGetLastError());
        // the host tables must outlive the copies above
        RW_HIP(hipStreamSynchronize(s));
        rw_status e = compact();
        if (e) return e;
        if ((e = read_states())) return e;
        prev = hst;
        const int m = o->check_interval;
        const bool timing = o->kernel_timing != 0;
        const bool graph = o->use_graph != 0 && !timing;
        if (timing && (e = ensure_events(ctx, size_t(4 * m)))) return e;
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        RW_HIP(hipEventRecord(ctx->ev_loop0, s));
        int64_t done = 0;
        while (counts[2] > 0 || counts[3] > 0) {
            if (counts[2] > 0) {
                if (graph) {
                    if (!ge) {
                        RW_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                        for (int k = 0; k < m && !e; ++k) e = launch_iteration(nullptr);
                        hipError_t e1 = hipStreamEndCapture(s, &g);
                        if (e) break;
                        RW_HIP(e1);
                        RW_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
                    }
                    RW_HIP(hipGraphLaunch(ge, s));
                } else {
                    for (int k = 0; k < m && !e; ++k)
                        e = launch_iteration(timing ? &ctx->pool[4 * k] : nullptr);
                    if (e) break;
                }
                if ((e = compact())) break;
                if ((e = read_states())) break;
                const int kmax = account();
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
            }
            if (counts[3] > 0) {
                if ((e = refresh())) break;
                if ((e = read_states())) break;
                prev = hst;
            }
            if (done > (int64_t)o->max_iter + 4 * m) {
                set_error("brick CG loop did not stop at max_iter");
                e = RW_ERR_HIP;
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
        if (e) return e;
        RW_HIP(e2);
        if (mixed)
            hipLaunchKernelGGL((k_brick_fold<T, R>), dim3(grid), dim3(256), 0, s, all(), B.st,
                               B.x64, (T*)B.xi, 1);
        RW_HIP(hipGetLastError());
        return RW_OK;
    }
};

template <typename V, typename T, int R, int BY, int BVX = 1>
rw_status bricks_run(rw_context* ctx, const rw_volume* fine, const rw_seeds* seeds,
                            const Shell& sh, const rw_brick* bricks, const rw_subvolume* sub,
                            int n_bricks,
                            const rw_options* o, float* prob_out, int32_t* brick_iters, void* ws,
                            const TileChoice& tc, rw_stats* stats) {
    const bool mixed = o->precision == RW_PREC_MIXED;
    const int K = seeds->num_labels;
    const int lab0 = o->solve_all_labels ? 1 : 2;
    BrickPlan P = make_plan(bricks, n_bricks, R, BY * BVX, tc.zc, sub, fine->dims);
    BrickSolve<V, T, R, BY, BVX> S;
    S.ctx = ctx;
    S.vol = static_cast<const V*>(fine->data);
    S.lab = seeds->labels;
    S.F = make_geom(fine->dims);
    S.wc = make_wcoef(fine, o->beta, o->w_eps);
    S.sh = sh;
    S.o = o;
    S.mixed = mixed;
    S.lab0 = lab0;
    S.zc = tc.zc;
    S.xcd = tc.brick_xcd;
    S.nb = n_bricks;
    S.P = &P;
    S.grid = 8 * ((std::max(1, std::min(P.ntiles, 2048)) + 7) / 8);  // multiple of 8 (XCD order)
    Carver cv(ws);
    carve_bricks(cv, P, R, mixed, &S.B);
    rw_status e = RW_OK;
    bool persistent = false;
    if constexpr (std::is_same<T, float>::value && BVX == 2 && (BY == 8 || BY == 4)) {
        if (tc.persist && mixed && o->refine_mode == 0) {
            persistent = true;
            e = S.run_persistent();
        }
    }
    if (!persistent) e = S.run();
    if (e) return e;
    hipLaunchKernelGGL((k_brick_write<R>), dim3(S.grid), dim3(256), 0, ctx->s, S.all(), S.F,
                       seeds->labels, S.B.x64, lab0, K, o->solve_all_labels ? 0 : 1, prob_out);
    RW_HIP(hipGetLastError());
    if ((e = S.read_states())) return e;
    int worst = RW_OK;
    int64_t refreshes = 0;
    for (int i = 0; i < n_bricks; ++i)
        for (int r = 0; r < R; ++r) {
            const RhsState& h = S.hst[size_t(i) * R + r];
            int code = RW_OK;
            if (h.status == ST_MAXITER || h.status == ST_RUNNING) code = RW_NOT_CONVERGED;
            else if (h.status == ST_SINGULAR) code = RW_ERR_SINGULAR;
            else if (h.status == ST_BREAKDOWN) code = RW_ERR_BREAKDOWN;
            else if (h.status == ST_NONFINITE) code = RW_ERR_NONFINITE;
            if (code < 0 && (worst >= 0 || code < worst)) worst = code;
            if (code > 0 && worst == RW_OK) worst = code;
            if (brick_iters) brick_iters[size_t(P.order[i]) * R + r] = h.iter_total;
            refreshes += h.refreshes;
            if (stats && r < RW_MAX_LABELS) stats->iters[r] = std::max(stats->iters[r], h.iter_total);
        }
    if (stats) {
        stats->num_solved = R;
        stats->loop_ms = S.loop_ms;
        stats->pass_ms[0] = S.pass_ms[0];
        stats->pass_ms[1] = S.pass_ms[1];
        stats->pass_launches[0] = S.launches[0];
        stats->pass_launches[1] = S.launches[1];
        stats->rhs_iterations = S.rhs_iters;
        stats->box_voxel_iterations = S.box_vox;
        stats->rhs_voxel_iterations = S.rhs_vox;
        stats->active_bricks = n_bricks;
        stats->unknowns = P.vox;
        stats->refinements = int32_t(std::min<int64_t>(refreshes, INT32_MAX));
        stats->tile_by = BY;
        stats->tile_by2 = BY;
        stats->tile_zc2 = tc.zc;
        stats->tile_zc = tc.zc;
        stats->tile_vx = BVX;
        stats->tile_xcd = tc.brick_xcd;
        stats->brick_blocks = S.persist_blocks;
        stats->tile_tuned = tc.tuned;
    }
    if (worst < 0) set_error(std::string("brick solve failed: ") + rw_status_string((rw_status)worst));
    return (rw_status)worst;
}

template <typename V, typename T, int R>
rw_status bricks_by(rw_context* ctx, const rw_volume* fine, const rw_seeds* seeds,
                           const Shell& sh, const rw_brick* bricks, const rw_subvolume* sub, int n,
                           const rw_options* o, float* prob, int32_t* it, void* ws, rw_stats* st) {
    const TileChoice tc = brick_tiles(
        o->precision, R, o->brick_voxels > 0 ? o->brick_voxels : max_brick_voxels(bricks, n));
    if (tc.vx == 2) {
        if (tc.by == 8)
            return bricks_run<V, T, R, 8, 2>(ctx, fine, seeds, sh, bricks, sub, n, o, prob, it, ws,
                                             tc, st);
        return bricks_run<V, T, R, 4, 2>(ctx, fine, seeds, sh, bricks, sub, n, o, prob, it, ws, tc,
                                         st);
    }
    if (tc.by == 8)
        return bricks_run<V, T, R, 8>(ctx, fine, seeds, sh, bricks, sub, n, o, prob, it, ws, tc, st);
    if (tc.by == 16)
        return bricks_run<V, T, R, 16>(ctx, fine, seeds, sh, bricks, sub, n, o, prob, it, ws, tc, st);
    return bricks_run<V, T, R, 4>(ctx, fine, seeds, sh, bricks, sub, n, o, prob, it, ws, tc, st);
}

template <typename V, typename T>
rw_status bricks_r(int R, rw_context* ctx, const rw_volume* fine, const rw_seeds* seeds,
                          const Shell& sh, const rw_brick* bricks, const rw_subvolume* sub, int n,
                          const rw_options* o, float* prob, int32_t* it, void* ws, rw_stats* st) {
    switch (R) {
        case 1: return bricks_by<V, T, 1>(ctx, fine, seeds, sh, bricks, sub, n, o, prob, it, ws, st);
        case 2: return bricks_by<V, T, 2>(ctx, fine, seeds, sh, bricks, sub, n, o, prob, it, ws, st);
        case 3: return bricks_by<V, T, 3>(ctx, fine, seeds, sh, bricks, sub, n, o, prob, it, ws, st);
        case 4: return bricks_by<V, T, 4>(ctx, fine, seeds, sh, bricks, sub, n, o, prob, it, ws, st);
    }
    set_error("brick solves support 1 to 4 solved labels");
    return RW_ERR_UNSUPPORTED;
}


// One instantiation per (volume type, precision): rw_bricks_<v>_<t>.hip.
#define RW_BRICKS_DECL(NAME)                                                                  \
    rw_status NAME(int R, rw_context* ctx, const rw_volume* fine, const rw_seeds* seeds,      \
                   const Shell& sh, const rw_brick* bricks, const rw_subvolume* sub, int n,   \
                   const rw_options* o, float* prob, int32_t* it, void* ws, rw_stats* st);
RW_BRICKS_DECL(bricks_u16_f32)
RW_BRICKS_DECL(bricks_u16_f64)
RW_BRICKS_DECL(bricks_f32_f32)
RW_BRICKS_DECL(bricks_f32_f64)
RW_BRICKS_DECL(bricks_f64_f32)
RW_BRICKS_DECL(bricks_f64_f64)
#undef RW_BRICKS_DECL

}  // namespace rw
