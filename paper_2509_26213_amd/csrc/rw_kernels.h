// Host helpers shared by the translation units, and the device-side
// reduction helpers of the CG kernels.
#pragma once

#include "rw_internal.h"

namespace rw {

rw_status invalid(const std::string& msg);
// pool: the volume is a flat pool of brick sub-volumes (dims (n, 1, 1)), which
// the kernels address per sub-volume, so only its total size is limited.
rw_status check_volume(const rw_volume* vol, bool pool = false);
// Grids the kernels can address: every side in [1, 2^30], a plane of at most
// 2^29 voxels (in-plane offsets are 32-bit byte offsets of 8-byte values)
// and at most 2^40 voxels (tile counts are 32-bit).
bool dims_supported(rw_dims d);
Geom make_geom(rw_dims d);
WCoef make_wcoef(const rw_volume* vol, double beta, double w_eps);
rw_status stream_enter(rw_context* ctx, void* user);
rw_status stream_leave(rw_context* ctx, void* user);
rw_status label_counts(rw_context* ctx, const uint8_t* lab, int64_t n, unsigned int* host256);
rw_status ensure_events(rw_context* ctx, size_t n);
// Grow the context's pinned host buffer / small device scratch (contents lost).
rw_status ensure_host_pinned(rw_context* ctx, size_t bytes);
rw_status ensure_dev_small(rw_context* ctx, size_t bytes);
// Looks up the device address of the no-allocation solve's static scratch on
// `device` (which must be current); once per device.
rw_status noalloc_register_device(int device);

// Tile shape of the stencil kernels, from the tuning table or the
// environment.  Whole volumes: 64 vx columns (each lane owns vx of them, 64
// apart) by `by` rows by zc planes, XCD-aware tile order or not; vx in {1,
// 2, 4}, by = 8 with vx = 2 only, else 4.  Bricks: 64 columns by `by` vx rows
// (each lane owns vx rows, by apart), vx in {1, 2}, by in {4, 8, 16}.
struct TileChoice {
    int by, zc, xcd, vx;
    int brick_xcd = 0;  // brick solves: XCD-aware order of the tile worklist
    int persist = 0;    // brick solves: one persistent launch (one block per brick)
    int tuned = 0;      // 1: from the autotuner's table
    int series = 1;     // time series: step-interleaved order (RW_SERIES_PLAIN=1: off)
    int by2 = 0;        // whole volumes: rows of pass 2's tiles (0 or by: pass 1's)
    int zc2 = 0;        // whole volumes: planes of pass 2's tiles (0: zc)
};
// Reads the autotuner's table file once per process (rw_context_create).
void load_tuning();
TileChoice tuned_tiles(const Geom& G, int precision, int R);
// Tile shape of batched brick solves: 64 x (by vx) column tiles, vx rows
// per lane (1 or 2), by in {4, 8, 16}.
// Brick tile shape for a batch whose largest brick has max_brick_vox voxels:
// the autotuner's choice for (precision, R, floor(log2 max_brick_vox)) if it
// ran, else the measured default with RW_BRICK_* overrides.
TileChoice brick_tiles(int precision, int R, int64_t max_brick_vox);
// The shapes the brick autotuner times (every one a brick solve supports).
const std::vector<TileChoice>& brick_candidates();

// Sum NQ per-thread values over a block of NW waves in a fixed order (wave
// butterfly, then the wave totals in wave order); threads 0..NQ-1 write
// out[q * stride].  Every thread of the block must call it.
template <int NQ, int NW>
__device__ __forceinline__ void block_sum_store(double (&v)[NQ], double* __restrict__ out,
                                                int64_t stride) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double a = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
        v[q] = a;
    }
    __shared__ double sh[NW][NQ];
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) sh[wid][q] = v[q];
    }
    __syncthreads();
    if (tid < NQ) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += sh[w][tid];
        out[tid * stride] = s;
    }
}

// Fixed-order sum over blocks of partials laid out [NQ][nblocks]; result in
// sums[] (shared) visible to every thread after return.  One block of
// FIN_THREADS threads.
constexpr int FIN_THREADS = 1024;

template <int NQ>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int nblocks,
                                             double* sums) {
    constexpr int NW = FIN_THREADS / 64;
    __shared__ double sh[NW][NQ];
    const int tid = threadIdx.x;
    double a[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) a[q] = 0.0;
    for (int b = tid; b < nblocks; b += FIN_THREADS) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) a[q] += part[(int64_t)q * nblocks + b];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a[q] += __shfl_xor(a[q], off, 64);
    }
    if ((tid & 63) == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) sh[tid >> 6][q] = a[q];
    }
    __syncthreads();
    if (tid < NQ) {
        double s = 0.0;
        for (int w = 0; w < NW; ++w) s += sh[w][tid];
        sums[tid] = s;
    }
    __syncthreads();
}

// Tile order of the 2.5D stencil kernels: tiles of 64 x BY columns by zc
// planes, tx fastest, then ty, then tz.  With xcd = 1 the grid has 8 * per
// blocks and block b takes slot (b % 8) * per + b / 8: the hardware deals
// blocks to the eight XCDs round-robin, so each XCD walks one contiguous
// range of slots and the neighbour rows a tile re-reads were fetched into
// the same XCD's L2 by the tile before it.
//
// Volume time series (nt > 0): the planes are nt steps of nzs, each step cut
// into cz chunks of at most zc planes (no chunk straddles two steps; tz =
// step * cz + chunk), and slot j holds step j % nt of column and chunk j / nt:
// the tiles of one column and chunk in consecutive steps, whose own planes
// are each other's time neighbours, are neighbours in the slot order and so
// run side by side in one XCD.  Slot -> tile is a bijection; a tile's
// partial slot is its tile index, so the order changes no reduction.
struct TileMap {
    int gx, gy, gz, zc, tiles, per, xcd, by, vx;
    int nt, nzs, cz;  // time series order (nt = 0: plain volume)
    __host__ __device__ __forceinline__ int tile(int b) const {
        int j;
        if (!xcd) {
            j = b < tiles ? b : -1;
        } else {
            j = (b & 7) * per + (b >> 3);
            if (j >= tiles) j = -1;
        }
        if (j < 0 || nt == 0) return j;
        const int s = j % nt, k = j / nt;
        const int tx = k % gx, ty = (k / gx) % gy, c = k / (gx * gy);
        return ((s * cz + c) * gy + ty) * gx + tx;
    }
    // first and one-past-last plane of tile layer tz
    __host__ __device__ __forceinline__ void planes(int tz, int nz, int& z0, int& z1) const {
        if (nt == 0) {
            z0 = tz * zc;
            z1 = z0 + zc < nz ? z0 + zc : nz;
            return;
        }
        const int s = tz / cz, c = tz - s * cz;
        z0 = s * nzs + c * zc;
        z1 = z0 + zc < (s + 1) * nzs ? z0 + zc : (s + 1) * nzs;
    }
    __host__ __device__ int blocks() const { return xcd ? 8 * per : tiles; }
};

inline TileMap make_tilemap(const Geom& G, int by, int zc, int xcd, int vx = 1) {
    TileMap m;
    m.by = by;
    m.vx = vx;
    m.zc = zc;
    m.gx = (G.nx + 64 * vx - 1) / (64 * vx);
    m.gy = (G.ny + by - 1) / by;
    m.gz = (G.nz + zc - 1) / zc;
    m.tiles = m.gx * m.gy * m.gz;
    m.per = (m.tiles + 7) / 8;
    m.xcd = xcd;
    m.nt = m.nzs = m.cz = 0;
    return m;
}

// Time-series order for nt steps of nzs planes (G.nz = nt * nzs), XCD-aware:
// chunks of at most 64 planes, equal within a step, halved while the grid
// has fewer than 1024 tiles (down to 4 planes).  Returns false (m untouched)
// if the tiles would outnumber max_tiles, the partial slots a solve's
// workspace holds.
inline bool make_tilemap_series(const Geom& G, int by, int vx, int nt, int nzs, int max_tiles,
                                TileMap& m) {
    if (nt < 2 || nzs < 1 || (int64_t)nt * nzs != G.nz) return false;
    TileMap t = make_tilemap(G, by, 4, 1, vx);
    const int64_t cols = (int64_t)t.gx * t.gy;
    int zc = (nzs + ((nzs + 63) / 64) - 1) / ((nzs + 63) / 64);
    while (zc > 4 && cols * nt * ((nzs + zc - 1) / zc) < 1024) zc = std::max(4, zc / 2);
    zc = std::max(4, zc);
    t.zc = zc;
    t.nt = nt;
    t.nzs = nzs;
    t.cz = (nzs + zc - 1) / zc;
    const int64_t tiles = cols * nt * t.cz;
    if (tiles > max_tiles) return false;
    t.gz = nt * t.cz;
    t.tiles = int(tiles);
    t.per = (t.tiles + 7) / 8;
    m = t;
    return true;
}

}  // namespace rw
