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

#include "rw_bricks.h"

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
        const uint8_t l = in_brick && lab ? lab[(int64_t)z * F.plane + (int64_t)y * F.nx + x] : 0;
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

// Index of the candidate brick holding coordinate p along one axis: cuts at
// o (if o > 0), then every b voxels.
__device__ __forceinline__ int cut_index(int p, int b, int o) {
    return o > 0 ? (p < o ? 0 : 1 + (p - o) / b) : p / b;
}

// The seed rule of the activity test from a seed list: a brick is active if
// one of its seeds has a label other than the upsampled argmax (lowest label
// on ties) at that voxel.  One thread per seed; seeds outside the grid are
// ignored.
__global__ __launch_bounds__(256) void k_seed_bricks(Shell sh, int K, Geom F,
                                                     const int64_t* __restrict__ sidx,
                                                     const uint8_t* __restrict__ slab, int64_t ns,
                                                     int bx, int by, int bz, int ox, int oy,
                                                     int oz, int ncx, int ncy,
                                                     uint8_t* __restrict__ flags) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < ns; i += 256ll * gridDim.x) {
        const int64_t g = sidx[i];
        const uint8_t l = slab[i];
        if (g < 0 || g >= F.n || l == 0) continue;
        const int z = int(g / F.plane);
        const int64_t r = g - (int64_t)z * F.plane;
        const int y = int(r / F.nx);
        const int x = int(r - (int64_t)y * F.nx);
        double best = -1.0;
        int arg = 1;
        for (int L = 1; L <= K; ++L) {
            const double p = upsample(sh, L, x, y, z);
            if (p > best) {
                best = p;
                arg = L;
            }
        }
        if (l != arg) {
            const int64_t b = ((int64_t)cut_index(z, bz, oz) * ncy + cut_index(y, by, oy)) * ncx +
                              cut_index(x, bx, ox);
            flags[b] = 1;
        }
    }
}

// Bricks a seed edit reaches: for every fine voxel whose label changed, the
// brick holding it and the bricks holding one of its six face neighbours
// (the bricks whose face shell holds it).  Grid-stride over the voxels.
__global__ __launch_bounds__(256) void k_edit_bricks(const uint8_t* __restrict__ old_l,
                                                     const uint8_t* __restrict__ new_l, Geom F,
                                                     int bx, int by, int bz, int ox, int oy,
                                                     int oz, int ncx, int ncy,
                                                     uint8_t* __restrict__ flags) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < F.n; i += 256ll * gridDim.x) {
        if (old_l[i] == new_l[i]) continue;
        const int z = int(i / F.plane);
        const int64_t r = i - (int64_t)z * F.plane;
        const int y = int(r / F.nx);
        const int x = int(r - (int64_t)y * F.nx);
        const int dx[7] = {0, -1, 1, 0, 0, 0, 0}, dy[7] = {0, 0, 0, -1, 1, 0, 0},
                  dz[7] = {0, 0, 0, 0, 0, -1, 1};
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const int px = x + dx[k], py = y + dy[k], pz = z + dz[k];
            if (px < 0 || px >= F.nx || py < 0 || py >= F.ny || pz < 0 || pz >= F.nz) continue;
            const int64_t b = ((int64_t)cut_index(pz, bz, oz) * ncy + cut_index(py, by, oy)) * ncx +
                              cut_index(px, bx, ox);
            flags[b] = 1;
        }
    }
}

// How far the coarse solution moved under each brick: the largest
// |new - old| over the labels and over the coarse cells of the brick's
// footprint and one cell around it.  One block per candidate brick.
__global__ __launch_bounds__(256) void k_coarse_moved(Shell olds, Shell news, int K,
                                                      const DevBrick* __restrict__ cand,
                                                      double* __restrict__ moved) {
    const DevBrick b = cand[blockIdx.x];
    const int f = news.factor;
    const int x0 = max(0, b.ox / f - 1), x1 = min(news.cnx, (b.ox + b.sx + f - 1) / f + 1);
    const int y0 = max(0, b.oy / f - 1), y1 = min(news.cny, (b.oy + b.sy + f - 1) / f + 1);
    const int z0 = max(0, b.oz / f - 1), z1 = min(news.cnz, (b.oz + b.sz + f - 1) / f + 1);
    const int64_t wx = x1 - x0, wy = y1 - y0, cells = wx * wy * (z1 - z0);
    double m = 0.0;
    for (int64_t c = threadIdx.x; c < cells * K; c += 256) {
        const int L = int(c / cells);
        const int64_t j = c - (int64_t)L * cells;
        const int z = z0 + int(j / (wx * wy));
        const int64_t r = j % (wx * wy);
        const int y = y0 + int(r / wx), x = x0 + int(r % wx);
        const int64_t idx = (int64_t)L * news.cn + ((int64_t)z * news.cny + y) * news.cnx + x;
        m = fmax(m, fabs(coarse_at(news, idx) - coarse_at(olds, idx)));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    __shared__ double wmax[4];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) moved[blockIdx.x] = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
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

}  // extern "C"

// Brick activity from the coarse probabilities, with the seed rule taken
// from a dense fine label map (labels) or from a seed list (sidx, slab).
static rw_status classify_impl(rw_context* ctx, const void* coarse_prob, int32_t coarse_dtype,
                               rw_dims coarse_dims, int32_t num_labels, int32_t factor,
                               const uint8_t* labels, const int64_t* sidx, const uint8_t* slab,
                               int64_t n_seeds, rw_dims fine_dims, const int32_t brick_size[3],
                               const int32_t grid_offset[3], double lo_thr, double hi_thr,
                               rw_brick* bricks_out, uint8_t* active_out, int32_t capacity,
                               int32_t* n_candidates, void* stream) {
    if (!ctx || !brick_size || !grid_offset || !n_candidates) return invalid("NULL argument");
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
    const Geom F = make_geom(fine_dims);
    RW_HIP(hipMemcpyAsync(dc, cand.data(), sizeof(DevBrick) * n, hipMemcpyHostToDevice, ctx->s));
    hipLaunchKernelGGL(k_classify, dim3(unsigned(n)), dim3(256), 0, ctx->s, sh, num_labels, F,
                       labels, dc, lo_thr, hi_thr, flags);
    if (n_seeds > 0)
        hipLaunchKernelGGL(k_seed_bricks, dim3(unsigned(std::min<int64_t>((n_seeds + 255) / 256, 4096))),
                           dim3(256), 0, ctx->s, sh, num_labels, F, sidx, slab, n_seeds,
                           brick_size[0], brick_size[1], brick_size[2], grid_offset[0],
                           grid_offset[1], grid_offset[2], int(cx.size()), int(cy.size()), flags);
    RW_HIP(hipGetLastError());
    if ((e = ensure_host_pinned(ctx, size_t(n)))) return e;
    RW_HIP(hipMemcpyAsync(ctx->host_pinned, flags, n, hipMemcpyDeviceToHost, ctx->s));
    RW_HIP(hipStreamSynchronize(ctx->s));
    memcpy(active_out, ctx->host_pinned, n);
    for (int64_t i = 0; i < n; ++i)
        bricks_out[i] = rw_brick{cand[i].ox, cand[i].oy, cand[i].oz, cand[i].sx, cand[i].sy, cand[i].sz};
    return stream_leave(ctx, stream);
}

extern "C" {

rw_status rw_classify_bricks(rw_context* ctx, const void* coarse_prob, int32_t coarse_dtype,
                             rw_dims coarse_dims, int32_t num_labels, int32_t factor,
                             const uint8_t* fine_labels, rw_dims fine_dims,
                             const int32_t brick_size[3], const int32_t grid_offset[3],
                             double lo_thr, double hi_thr, rw_brick* bricks_out,
                             uint8_t* active_out, int32_t capacity, int32_t* n_candidates,
                             void* stream) {
    if (!fine_labels) return invalid("fine_labels is NULL");
    return classify_impl(ctx, coarse_prob, coarse_dtype, coarse_dims, num_labels, factor,
                         fine_labels, nullptr, nullptr, 0, fine_dims, brick_size, grid_offset,
                         lo_thr, hi_thr, bricks_out, active_out, capacity, n_candidates, stream);
}

rw_status rw_seed_edit_bricks(rw_context* ctx, const uint8_t* old_labels,
                              const uint8_t* new_labels, rw_dims fine_dims,
                              const void* old_coarse, const void* new_coarse,
                              int32_t coarse_dtype, rw_dims coarse_dims, int32_t num_labels,
                              int32_t factor, const int32_t brick_size[3],
                              const int32_t grid_offset[3], uint8_t* edited_out,
                              double* moved_out, int32_t capacity, int32_t* n_candidates,
                              void* stream) {
    if (!ctx || !old_labels || !new_labels || !brick_size || !grid_offset || !n_candidates)
        return invalid("NULL argument");
    if (num_labels < 1 || num_labels > RW_MAX_LABELS) return invalid("num_labels must be in [1, 16]");
    if (!dims_supported(fine_dims)) return invalid("fine dims must be positive and supported");
    for (int a = 0; a < 3; ++a)
        if (brick_size[a] < 1 || grid_offset[a] < 0) return invalid("bad brick size or offset");
    Shell so, sn;
    rw_status e = make_shell(old_coarse, coarse_dtype, coarse_dims, factor, &so);
    if (e) return e;
    if ((e = make_shell(new_coarse, coarse_dtype, coarse_dims, factor, &sn))) return e;
    const auto cx = cuts(int(fine_dims.nx), brick_size[0], grid_offset[0]);
    const auto cy = cuts(int(fine_dims.ny), brick_size[1], grid_offset[1]);
    const auto cz = cuts(int(fine_dims.nz), brick_size[2], grid_offset[2]);
    const int64_t n = (int64_t)cx.size() * cy.size() * cz.size();
    *n_candidates = int32_t(n);
    if (!edited_out || !moved_out || capacity < n) {
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
    const size_t bytes = sizeof(DevBrick) * n + sizeof(double) * n + n + 256;
    if ((e = ensure_dev_small(ctx, bytes))) return e;
    if ((e = ensure_host_pinned(ctx, sizeof(double) * n + n))) return e;
    if ((e = stream_enter(ctx, stream))) return e;
    DevBrick* dc = static_cast<DevBrick*>(ctx->dev_small);
    double* moved = reinterpret_cast<double*>(dc + n);
    uint8_t* flags = reinterpret_cast<uint8_t*>(moved + n);
    const Geom F = make_geom(fine_dims);
    RW_HIP(hipMemcpyAsync(dc, cand.data(), sizeof(DevBrick) * n, hipMemcpyHostToDevice, ctx->s));
    RW_HIP(hipMemsetAsync(flags, 0, n, ctx->s));
    hipLaunchKernelGGL(k_edit_bricks, dim3(unsigned(std::min<int64_t>((F.n + 255) / 256, 8192))),
                       dim3(256), 0, ctx->s, old_labels, new_labels, F, brick_size[0],
                       brick_size[1], brick_size[2], grid_offset[0], grid_offset[1],
                       grid_offset[2], int(cx.size()), int(cy.size()), flags);
    hipLaunchKernelGGL(k_coarse_moved, dim3(unsigned(n)), dim3(256), 0, ctx->s, so, sn,
                       num_labels, dc, moved);
    RW_HIP(hipGetLastError());
    char* hp = static_cast<char*>(ctx->host_pinned);
    RW_HIP(hipMemcpyAsync(hp, moved, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->s));
    RW_HIP(hipMemcpyAsync(hp + sizeof(double) * n, flags, n, hipMemcpyDeviceToHost, ctx->s));
    RW_HIP(hipStreamSynchronize(ctx->s));
    memcpy(moved_out, hp, sizeof(double) * n);
    memcpy(edited_out, hp + sizeof(double) * n, n);
    return stream_leave(ctx, stream);
}

rw_status rw_classify_bricks_sparse(rw_context* ctx, const void* coarse_prob,
                                    int32_t coarse_dtype, rw_dims coarse_dims, int32_t num_labels,
                                    int32_t factor, const int64_t* seed_index,
                                    const uint8_t* seed_label, int64_t n_seeds, rw_dims fine_dims,
                                    const int32_t brick_size[3], const int32_t grid_offset[3],
                                    double lo_thr, double hi_thr, rw_brick* bricks_out,
                                    uint8_t* active_out, int32_t capacity, int32_t* n_candidates,
                                    void* stream) {
    if (n_seeds < 0 || (n_seeds > 0 && (!seed_index || !seed_label)))
        return invalid("bad seed list");
    return classify_impl(ctx, coarse_prob, coarse_dtype, coarse_dims, num_labels, factor, nullptr,
                         seed_index, seed_label, n_seeds, fine_dims, brick_size, grid_offset,
                         lo_thr, hi_thr, bricks_out, active_out, capacity, n_candidates, stream);
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
            e = (mixed ? bricks_u16_f32 : bricks_u16_f64)(R, ctx, fine, seeds, sh, bricks, subvols,
                                                          n_bricks, o, prob_out, brick_iters, ws,
                                                          stats);
            break;
        case RW_DT_F32:
            e = (mixed ? bricks_f32_f32 : bricks_f32_f64)(R, ctx, fine, seeds, sh, bricks, subvols,
                                                          n_bricks, o, prob_out, brick_iters, ws,
                                                          stats);
            break;
        default:
            e = (mixed ? bricks_f64_f32 : bricks_f64_f64)(R, ctx, fine, seeds, sh, bricks, subvols,
                                                          n_bricks, o, prob_out, brick_iters, ws,
                                                          stats);
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
