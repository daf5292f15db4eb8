// Coarse-to-fine random walker (the hierarchical method benchmarked in the
// paper's Sec. IV-B, Table III; levels of detail of Sec. III-D; bricks are
// the chunks of Sec. II's chunk mapping):
//   rw_downsample       one LOD step of intensities and seed labels
//   rw_classify_bricks  which fine bricks the coarse solution leaves uncertain
//   rw_fill_bricks      upsampled coarse probabilities for the certain bricks
//   rw_solve_bricks     batched Jacobi-PCG of many bricks, Dirichlet shell
//                       from the upsampled coarse solution
#include <algorithm>
#include <cstring>
#include <vector>

#include "rw_whole.h"

namespace rw {

rw_status check_options(const rw_options* o);

// ================================================================== LOD step

template <typename V, typename TO>
__global__ __launch_bounds__(256) void k_downsample(const V* __restrict__ vol, Geom F, double lo,
                                                    double scale, Geom C, TO* __restrict__ g_out,
                                                    const uint8_t* __restrict__ lab,
                                                    uint8_t* __restrict__ lab_out) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < C.n; i += 256ll * gridDim.x) {
        const int cz = int(i / C.plane);
        const int64_t rem = i - (int64_t)cz * C.plane;
        const int cy = int(rem / C.nx);
        const int cx = int(rem - (int64_t)cy * C.nx);
        double s = 0.0;
        int cnt = 0, first = 0;
        bool conflict = false;
        for (int dz = 0; dz < 2; ++dz) {
            const int z = 2 * cz + dz;
            if (z >= F.nz) continue;
            for (int dy = 0; dy < 2; ++dy) {
                const int y = 2 * cy + dy;
                if (y >= F.ny) continue;
                for (int dx = 0; dx < 2; ++dx) {
                    const int x = 2 * cx + dx;
                    if (x >= F.nx) continue;
                    const int64_t f = (int64_t)z * F.plane + (int64_t)y * F.nx + x;
                    s += ((double)vol[f] - lo) * scale;
                    ++cnt;
                    if (lab) {
                        const int l = lab[f];
                        if (l) {
                            if (!first) first = l;
                            else if (l != first) conflict = true;
                        }
                    }
                }
            }
        }
        g_out[i] = (TO)(s / cnt);
        if (lab_out) lab_out[i] = conflict ? 0 : (uint8_t)first;
    }
}

// ================================================================== classify / fill

struct DevBrick {
    int ox, oy, oz, sx, sy, sz;     // box in its volume
    int vnx, vny;                   // its volume's row / plane sizes
    int gox, goy, goz;              // global position of the volume's origin
    int64_t voff;                   // offset of the volume in the label / output arrays
};

// One block per candidate brick; flags[b] = 1 if active.
__global__ __launch_bounds__(256) void k_classify(Shell sh, int K, Geom F,
                                                  const uint8_t* __restrict__ lab,
                                                  const DevBrick* __restrict__ cand, double lo,
                                                  double hi, uint8_t* __restrict__ flags) {
    __shared__ int found;
    const DevBrick b = cand[blockIdx.x];
    if (threadIdx.x == 0) found = 0;
    __syncthreads();
    const int64_t inner = (int64_t)b.sx * b.sy * b.sz;
    // face shell: six faces, each the brick's face moved one voxel outwards
    const int64_t fxy = (int64_t)b.sx * b.sy, fxz = (int64_t)b.sx * b.sz, fyz = (int64_t)b.sy * b.sz;
    const int64_t total = inner + 2 * (fxy + fxz + fyz);
    for (int64_t i = threadIdx.x; i < total; i += 256) {
        if (*(volatile int*)&found) break;
        int x, y, z;
        bool in_brick = i < inner;
        if (in_brick) {
            z = int(i / fxy);
            const int64_t r = i - (int64_t)z * fxy;
            y = int(r / b.sx);
            x = int(r - (int64_t)y * b.sx);
            x += b.ox;
            y += b.oy;
            z += b.oz;
        } else {
            int64_t j = i - inner;
            if (j < 2 * fxy) {
                const int side = int(j / fxy);
                j -= side * fxy;
                y = b.oy + int(j / b.sx);
                x = b.ox + int(j % b.sx);
                z = side ? b.oz + b.sz : b.oz - 1;
            } else if ((j -= 2 * fxy) < 2 * fxz) {
                const int side = int(j / fxz);
                j -= side * fxz;
                z = b.oz + int(j / b.sx);
                x = b.ox + int(j % b.sx);
                y = side ? b.oy + b.sy : b.oy - 1;
            } else {
                j -= 2 * fxz;
                const int side = int(j / fyz);
                j -= side * fyz;
                z = b.oz + int(j / b.sy);
                y = b.oy + int(j % b.sy);
                x = side ? b.ox + b.sx : b.ox - 1;
            }
            if (x < 0 || x >= F.nx || y < 0 || y >= F.ny || z < 0 || z >= F.nz) continue;
        }
        const uint8_t l = in_brick ? lab[(int64_t)z * F.plane + (int64_t)y * F.nx + x] : 0;
        double best = -1.0;
        int arg = 1;
        bool unc = false;
        for (int L = 1; L <= K; ++L) {
            const double p = upsample(sh, L, x, y, z);
            unc |= (p > lo && p < hi);
            if (p > best) {
                best = p;
                arg = L;
            }
        }
        if (unc || (l != 0 && l != arg)) atomicOr(&found, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) flags[blockIdx.x] = found ? 1 : 0;
}

// Upsampled probabilities (seeds exact) for every voxel of the listed bricks
// (each in its volume; n = voxels of the label / output arrays).
__global__ __launch_bounds__(256) void k_fill(Shell sh, int K, int64_t n,
                                              const uint8_t* __restrict__ lab,
                                              const DevBrick* __restrict__ bricks,
                                              float* __restrict__ prob) {
    const DevBrick b = bricks[blockIdx.y];
    const int64_t inner = (int64_t)b.sx * b.sy * b.sz;
    const int64_t fxy = (int64_t)b.sx * b.sy;
    const int64_t plane = (int64_t)b.vnx * b.vny;
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < inner; i += 256ll * gridDim.x) {
        const int z = b.oz + int(i / fxy);
        const int64_t r = i % fxy;
        const int y = b.oy + int(r / b.sx);
        const int x = b.ox + int(r % b.sx);
        const int64_t g = b.voff + (int64_t)z * plane + (int64_t)y * b.vnx + x;
        const uint8_t l = lab[g];
        for (int L = 1; L <= K; ++L)
            prob[(int64_t)(L - 1) * n + g] =
                l ? (l == L ? 1.f : 0.f)
                  : (float)upsample(sh, L, b.gox + x, b.goy + y, b.goz + z);
    }
}

static rw_status make_shell(const void* coarse, int32_t cdt, rw_dims cd, int32_t factor, Shell* sh) {
    if (!coarse) return invalid("coarse probabilities are NULL");
    if (cdt != RW_DT_F32 && cdt != RW_DT_F64) return invalid("coarse dtype must be F32 or F64");
    if (!dims_supported(cd)) return invalid("coarse dims must be positive and supported");
    if (factor < 1) return invalid("factor must be >= 1");
    sh->coarse = coarse;
    sh->cdt = cdt == RW_DT_F64 ? 1 : 0;
    sh->cnx = int(cd.nx);
    sh->cny = int(cd.ny);
    sh->cnz = int(cd.nz);
    sh->cn = cd.nx * cd.ny * cd.nz;
    sh->factor = factor;
    return RW_OK;
}

static std::vector<std::pair<int, int>> cuts(int n, int b, int o) {
    std::vector<std::pair<int, int>> out;
    int e = 0;
    if (o > 0) {
        out.push_back({0, std::min(o, n)});
        e = std::min(o, n);
    }
    while (e < n) {
        const int s = std::min(b, n - e);
        out.push_back({e, s});
        e += s;
    }
    return out;
}

// ================================================================== brick solve

// Per-brick finalize kernels: one 64-thread block per brick sums its tiles'
// partials (layout [NQ][ntiles]) in a fixed order.
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
    RhsState& s = st[blockIdx.x * R + r];
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

// mixed: a label whose recurrence residual has fallen by update_delta since
// the last refresh, or that met the tolerance, is flagged for a float64
// refresh (outer_active = 2); it keeps iterating until then unless converged.
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

struct BrickPlan {
    std::vector<BrickGeo> geo;
    std::vector<int> tile_brick;
    std::vector<int> order;  // solve order -> caller's brick index
    int ntiles = 0;
    int64_t vox = 0;
};

// Bricks sorted by decreasing size (stable), tiles of 64 x by x zc.
static int64_t max_brick_voxels(const rw_brick* bricks, int n) {
    int64_t m = 0;
    for (int i = 0; i < n; ++i)
        m = std::max<int64_t>(m, (int64_t)bricks[i].sx * bricks[i].sy * bricks[i].sz);
    return m;
}

static BrickPlan make_plan(const rw_brick* bricks, int n, int R, int by, int zc,
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

static size_t carve_bricks(Carver& cv, const BrickPlan& P, int R, bool mixed, BrickBuffers* b) {
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
static rw_status bricks_run(rw_context* ctx, const rw_volume* fine, const rw_seeds* seeds,
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
    rw_status e = S.run();
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
        stats->tile_zc = tc.zc;
        stats->tile_vx = BVX;
        stats->tile_xcd = tc.brick_xcd;
    }
    if (worst < 0) set_error(std::string("brick solve failed: ") + rw_status_string((rw_status)worst));
    return (rw_status)worst;
}

template <typename V, typename T, int R>
static rw_status bricks_by(rw_context* ctx, const rw_volume* fine, const rw_seeds* seeds,
                           const Shell& sh, const rw_brick* bricks, const rw_subvolume* sub, int n,
                           const rw_options* o, float* prob, int32_t* it, void* ws, rw_stats* st) {
    const TileChoice tc = brick_tiles(o->precision, R, max_brick_voxels(bricks, n));
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
static rw_status bricks_r(int R, rw_context* ctx, const rw_volume* fine, const rw_seeds* seeds,
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

}  // namespace rw

using namespace rw;

extern "C" {

rw_status rw_downsample(rw_context* ctx, const rw_volume* fine, const uint8_t* fine_labels,
                        int32_t out_dtype, void* g_out, uint8_t* labels_out, void* stream) {
    if (!ctx || !g_out) return invalid("NULL argument");
    rw_status e = check_volume(fine);
    if (e) return e;
    if (out_dtype != RW_DT_F32 && out_dtype != RW_DT_F64) return invalid("out_dtype must be F32 or F64");
    if (labels_out && !fine_labels) return invalid("labels_out needs fine_labels");
    const Geom F = make_geom(fine->dims);
    rw_dims cd{(fine->dims.nx + 1) / 2, (fine->dims.ny + 1) / 2, (fine->dims.nz + 1) / 2};
    const Geom C = make_geom(cd);
    const double span = fine->norm_hi - fine->norm_lo;
    const double scale = span > 0 ? 1.0 / span : 0.0;
    if ((e = stream_enter(ctx, stream))) return e;
    const dim3 grid(unsigned(std::min<int64_t>((C.n + 255) / 256, 16384)));
#define RW_DS(V, TO)                                                                           \
    hipLaunchKernelGGL((k_downsample<V, TO>), grid, dim3(256), 0, ctx->s, (const V*)fine->data, F, \
                       fine->norm_lo, scale, C, (TO*)g_out, fine_labels, labels_out)
    if (out_dtype == RW_DT_F32) {
        if (fine->dtype == RW_DT_U16) RW_DS(uint16_t, float);
        else if (fine->dtype == RW_DT_F32) RW_DS(float, float);
        else RW_DS(double, float);
    } else {
        if (fine->dtype == RW_DT_U16) RW_DS(uint16_t, double);
        else if (fine->dtype == RW_DT_F32) RW_DS(float, double);
        else RW_DS(double, double);
    }
#undef RW_DS
    RW_HIP(hipGetLastError());
    return stream_leave(ctx, stream);
}

rw_status rw_classify_bricks(rw_context* ctx, const void* coarse_prob, int32_t coarse_dtype,
                             rw_dims coarse_dims, int32_t num_labels, int32_t factor,
                             const uint8_t* fine_labels, rw_dims fine_dims,
                             const int32_t brick_size[3], const int32_t grid_offset[3],
                             double lo_thr, double hi_thr, rw_brick* bricks_out,
                             uint8_t* active_out, int32_t capacity, int32_t* n_candidates,
                             void* stream) {
    if (!ctx || !fine_labels || !brick_size || !grid_offset || !n_candidates)
        return invalid("NULL argument");
    if (num_labels < 1 || num_labels > RW_MAX_LABELS) return invalid("num_labels must be in [1, 16]");
    if (!dims_supported(fine_dims)) return invalid("fine dims must be positive and supported");
    for (int a = 0; a < 3; ++a)
        if (brick_size[a] < 1 || grid_offset[a] < 0) return invalid("bad brick size or offset");
    Shell sh;
    rw_status e = make_shell(coarse_prob, coarse_dtype, coarse_dims, factor, &sh);
    if (e) return e;
    const auto cx = cuts(int(fine_dims.nx), brick_size[0], grid_offset[0]);
    const auto cy = cuts(int(fine_dims.ny), brick_size[1], grid_offset[1]);
    const auto cz = cuts(int(fine_dims.nz), brick_size[2], grid_offset[2]);
    const int64_t n = (int64_t)cx.size() * cy.size() * cz.size();
    *n_candidates = int32_t(n);
    if (!bricks_out || !active_out || capacity < n) {
        set_error("capacity must hold " + std::to_string(n) + " candidate bricks");
        return RW_ERR_INVALID_ARG;
    }
    std::vector<DevBrick> cand;
    cand.reserve(n);
    for (auto& z : cz)
        for (auto& y : cy)
            for (auto& x : cx)
                cand.push_back(DevBrick{x.first, y.first, z.first, x.second, y.second, z.second,
                                        int(fine_dims.nx), int(fine_dims.ny), 0, 0, 0, 0});
    if ((e = ensure_dev_small(ctx, sizeof(DevBrick) * n + n + 256))) return e;
    if ((e = stream_enter(ctx, stream))) return e;
    DevBrick* dc = static_cast<DevBrick*>(ctx->dev_small);
    uint8_t* flags = reinterpret_cast<uint8_t*>(dc + n);
    RW_HIP(hipMemcpyAsync(dc, cand.data(), sizeof(DevBrick) * n, hipMemcpyHostToDevice, ctx->s));
    hipLaunchKernelGGL(k_classify, dim3(unsigned(n)), dim3(256), 0, ctx->s, sh, num_labels,
                       make_geom(fine_dims), fine_labels, dc, lo_thr, hi_thr, flags);
    RW_HIP(hipGetLastError());
    if ((e = ensure_host_pinned(ctx, size_t(n)))) return e;
    RW_HIP(hipMemcpyAsync(ctx->host_pinned, flags, n, hipMemcpyDeviceToHost, ctx->s));
    RW_HIP(hipStreamSynchronize(ctx->s));
    memcpy(active_out, ctx->host_pinned, n);
    for (int64_t i = 0; i < n; ++i)
        bricks_out[i] = rw_brick{cand[i].ox, cand[i].oy, cand[i].oz, cand[i].sx, cand[i].sy, cand[i].sz};
    return stream_leave(ctx, stream);
}

static rw_status check_subvolumes(const rw_brick* bricks, const rw_subvolume* sub, int n,
                                  rw_dims pool);

static rw_status check_bricks(const rw_brick* bricks, int n, rw_dims d) {
    if (n < 0 || (n > 0 && !bricks)) return invalid("bad brick list");
    for (int i = 0; i < n; ++i) {
        const rw_brick& b = bricks[i];
        if (b.sx < 1 || b.sy < 1 || b.sz < 1 || b.ox < 0 || b.oy < 0 || b.oz < 0 ||
            b.ox + b.sx > d.nx || b.oy + b.sy > d.ny || b.oz + b.sz > d.nz)
            return invalid("brick " + std::to_string(i) + " does not lie inside the volume");
    }
    return RW_OK;
}

rw_status rw_fill_bricks(rw_context* ctx, const void* coarse_prob, int32_t coarse_dtype,
                         rw_dims coarse_dims, int32_t num_labels, int32_t factor,
                         const uint8_t* fine_labels, rw_dims fine_dims, const rw_brick* bricks,
                         const rw_subvolume* subvols, int32_t n_bricks, float* prob_out,
                         void* stream) {
    if (!ctx || !fine_labels || !prob_out) return invalid("NULL argument");
    if (num_labels < 1 || num_labels > RW_MAX_LABELS) return invalid("num_labels must be in [1, 16]");
    Shell sh;
    rw_status e = make_shell(coarse_prob, coarse_dtype, coarse_dims, factor, &sh);
    if (e) return e;
    if (n_bricks < 0 || (n_bricks > 0 && !bricks)) return invalid("bad brick list");
    if (subvols) {
        if ((e = check_subvolumes(bricks, subvols, n_bricks, fine_dims))) return e;
    } else if ((e = check_bricks(bricks, n_bricks, fine_dims))) {
        return e;
    }
    if (n_bricks == 0) return RW_OK;
    if ((e = ensure_dev_small(ctx, sizeof(DevBrick) * size_t(n_bricks)))) return e;
    if ((e = stream_enter(ctx, stream))) return e;
    std::vector<DevBrick> v(n_bricks);
    for (int i = 0; i < n_bricks; ++i) {
        const rw_brick& b = bricks[i];
        DevBrick d{b.ox, b.oy, b.oz, b.sx, b.sy, b.sz, int(fine_dims.nx), int(fine_dims.ny), 0, 0, 0, 0};
        if (subvols) {
            const rw_subvolume& s = subvols[i];
            d.vnx = s.nx;
            d.vny = s.ny;
            d.gox = s.gx;
            d.goy = s.gy;
            d.goz = s.gz;
            d.voff = s.offset;
        }
        v[i] = d;
    }
    DevBrick* db = static_cast<DevBrick*>(ctx->dev_small);
    RW_HIP(hipMemcpyAsync(db, v.data(), sizeof(DevBrick) * n_bricks, hipMemcpyHostToDevice, ctx->s));
    // the host vector must stay valid until the copy has run
    RW_HIP(hipStreamSynchronize(ctx->s));
    const int64_t n = fine_dims.nx * fine_dims.ny * fine_dims.nz;
    for (int b0 = 0; b0 < n_bricks; b0 += 65535) {
        const int nb = std::min(65535, n_bricks - b0);
        hipLaunchKernelGGL(k_fill, dim3(64, unsigned(nb)), dim3(256), 0, ctx->s, sh, num_labels, n,
                           fine_labels, db + b0, prob_out);
    }
    RW_HIP(hipGetLastError());
    return stream_leave(ctx, stream);
}

size_t rw_bricks_workspace_bytes(const rw_brick* bricks, int32_t n_bricks, int32_t num_labels,
                                 int32_t precision, int32_t solve_all_labels) {
    if (n_bricks <= 0 || !bricks || num_labels < 1) return 0;
    const int R = solve_all_labels ? num_labels : num_labels - 1;
    if (R < 1 || R > 4) return 0;
    // enough for the shape in use and for every shape the autotuner may pick
    std::vector<TileChoice> shapes = brick_candidates();
    shapes.push_back(brick_tiles(precision, R, max_brick_voxels(bricks, n_bricks)));
    size_t need = 0;
    for (const TileChoice& tc : shapes) {
        BrickPlan P = make_plan(bricks, n_bricks, R, tc.by * tc.vx, tc.zc);
        Carver cv(nullptr);
        need = std::max(need, carve_bricks(cv, P, R, precision == RW_PREC_MIXED, nullptr));
    }
    return need;
}

static rw_status check_subvolumes(const rw_brick* bricks, const rw_subvolume* sub, int n,
                                  rw_dims pool) {
    const int64_t total = pool.nx * pool.ny * pool.nz;
    for (int i = 0; i < n; ++i) {
        const rw_subvolume& v = sub[i];
        if (!dims_supported(rw_dims{v.nx, v.ny, v.nz}))
            return invalid("sub-volume " + std::to_string(i) + " is too large");
        if (v.nx < 1 || v.ny < 1 || v.nz < 1 || v.offset < 0 ||
            v.offset + (int64_t)v.nx * v.ny * v.nz > total || v.gx < 0 || v.gy < 0 || v.gz < 0)
            return invalid("sub-volume " + std::to_string(i) + " does not fit the pool");
        const rw_brick& b = bricks[i];
        if (b.sx < 1 || b.sy < 1 || b.sz < 1 || b.ox < 0 || b.oy < 0 || b.oz < 0 ||
            b.ox + b.sx > v.nx || b.oy + b.sy > v.ny || b.oz + b.sz > v.nz)
            return invalid("brick " + std::to_string(i) + " does not lie inside its sub-volume");
    }
    return RW_OK;
}

rw_status rw_solve_bricks(rw_context* ctx, const rw_volume* fine, const rw_seeds* seeds,
                          const void* coarse_prob, int32_t coarse_dtype, rw_dims coarse_dims,
                          int32_t factor, const rw_brick* bricks, const rw_subvolume* subvols,
                          int32_t n_bricks, const rw_options* o, float* prob_out,
                          int32_t* brick_iters, void* ws, size_t ws_bytes, rw_stats* stats,
                          void* stream) {
    if (!ctx || !prob_out) return invalid("NULL argument");
    rw_status e = check_volume(fine, subvols != nullptr);
    if (e) return e;
    if ((e = check_options(o))) return e;
    if (!seeds || !seeds->labels) return invalid("seeds are NULL");
    const int K = seeds->num_labels;
    if (K < 1 || K > RW_MAX_LABELS) return invalid("num_labels must be in [1, 16]");
    const int R = o->solve_all_labels ? K : K - 1;
    if (R < 1 || R > 4) {
        set_error("brick solves support 1 to 4 solved labels");
        return RW_ERR_UNSUPPORTED;
    }
    Shell sh;
    if ((e = make_shell(coarse_prob, coarse_dtype, coarse_dims, factor, &sh))) return e;
    if (n_bricks < 0 || (n_bricks > 0 && !bricks)) return invalid("bad brick list");
    if (subvols) {
        if ((e = check_subvolumes(bricks, subvols, n_bricks, fine->dims))) return e;
    } else if ((e = check_bricks(bricks, n_bricks, fine->dims))) {
        return e;
    }
    if (stats) memset(stats, 0, sizeof(*stats));
    if (n_bricks == 0) return RW_OK;
    const size_t need = rw_bricks_workspace_bytes(bricks, n_bricks, K, o->precision, o->solve_all_labels);
    if (!ws || ws_bytes < need) {
        set_error("workspace needs " + std::to_string(need) + " bytes");
        return RW_ERR_WORKSPACE;
    }
    if ((e = stream_enter(ctx, stream))) return e;
    RW_HIP(hipEventRecord(ctx->ev_begin, ctx->s));
    unsigned int cnt[256];
    if ((e = label_counts(ctx, seeds->labels, make_geom(fine->dims).n, cnt))) return e;
    for (int v = K + 1; v < 256; ++v)
        if (cnt[v]) {
            (void)stream_leave(ctx, stream);
            return invalid("a seed label exceeds num_labels");
        }
    const bool mixed = o->precision == RW_PREC_MIXED;
    switch (fine->dtype) {
        case RW_DT_U16:
            e = mixed ? bricks_r<uint16_t, float>(R, ctx, fine, seeds, sh, bricks, subvols, n_bricks, o, prob_out,
                                                  brick_iters, ws, stats)
                      : bricks_r<uint16_t, double>(R, ctx, fine, seeds, sh, bricks, subvols, n_bricks, o,
                                                   prob_out, brick_iters, ws, stats);
            break;
        case RW_DT_F32:
            e = mixed ? bricks_r<float, float>(R, ctx, fine, seeds, sh, bricks, subvols, n_bricks, o, prob_out,
                                               brick_iters, ws, stats)
                      : bricks_r<float, double>(R, ctx, fine, seeds, sh, bricks, subvols, n_bricks, o, prob_out,
                                                brick_iters, ws, stats);
            break;
        default:
            e = mixed ? bricks_r<double, float>(R, ctx, fine, seeds, sh, bricks, subvols, n_bricks, o, prob_out,
                                                brick_iters, ws, stats)
                      : bricks_r<double, double>(R, ctx, fine, seeds, sh, bricks, subvols, n_bricks, o, prob_out,
                                                 brick_iters, ws, stats);
    }
    RW_HIP(hipEventRecord(ctx->ev_end, ctx->s));
    RW_HIP(hipEventSynchronize(ctx->ev_end));
    if (stats) {
        float ms = 0.f;
        RW_HIP(hipEventElapsedTime(&ms, ctx->ev_begin, ctx->ev_end));
        stats->device_ms = ms;
    }
    rw_status e2 = stream_leave(ctx, stream);
    return e ? e : e2;
}

}  // extern "C"
