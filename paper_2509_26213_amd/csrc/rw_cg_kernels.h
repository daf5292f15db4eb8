// The 2.5D stencil kernels of the matrix-free Jacobi-PCG.
//
// A system is solved on a box of the grid: the whole volume, or one brick of
// the fine level (whose face shell then carries Dirichlet data).  A box is cut
// into tiles of 64 VX x BY columns by zc planes; a block of 64 x BY threads
// walks a tile's planes in batches of U, each lane owning VX columns 64 apart
// (so every load instruction of a wave reads 64 consecutive values).  Per batch it issues every global load
// (unconditionally, from clamped addresses, values outside the volume or box
// replaced by selects), then publishes the batch's planes of intensity and CG
// operand, with their one-voxel x/y halo, to LDS; in-plane neighbours come
// from LDS, z neighbours from registers.  Vectors of a box are stored
// box-locally, [label][z][y][x] from the box's vector offset.
//
// Tile sources: WholeTiles (one tile per block, optional XCD-aware order) and
// BrickTiles (blocks stride over a compacted list of the tiles of the bricks
// that still iterate).
#pragma once

#include <type_traits>

#include "rw_kernels.h"

namespace rw {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Element i of a row/plane whose base is wave-uniform, addressed by a 32-bit
// byte offset (the loads then take the base in scalar registers and only the
// 32-bit offset per lane).
template <typename P>
__device__ __forceinline__ P ldu(const P* __restrict__ base, uint32_t i) {
    return *reinterpret_cast<const P*>(reinterpret_cast<const char*>(base) + i * uint32_t(sizeof(P)));
}
template <typename P>
__device__ __forceinline__ void stu(P* __restrict__ base, uint32_t i, P v) {
    *reinterpret_cast<P*>(reinterpret_cast<char*>(base) + i * uint32_t(sizeof(P))) = v;
}
// The same store marked non-temporal: pass 2's outputs (x, z) are not read
// again before the next iteration, so they need not displace the halo rows
// that the running tiles re-read from L2 (measured: pass 2 +1.5 % on 512^3;
// pass 1's p_new, which pass 2 reads right after, loses with it).
template <typename P>
__device__ __forceinline__ void stnt(P* __restrict__ base, uint32_t i, P v) {
    __builtin_nontemporal_store(v, reinterpret_cast<P*>(reinterpret_cast<char*>(base) +
                                                        i * uint32_t(sizeof(P))));
}

struct BoxTile {
    Geom G;                  // the volume the box lives in
    int64_t voff;            // offset of that volume in the intensity / label arrays
    int gox, goy, goz;       // global position of that volume's origin (coarse upsampling)
    int ox, oy, oz;          // box origin in the volume
    int sx, sy, sz;          // box size
    int X0, Y0, z0, z1;      // tile origin (box-local) and plane range [z0, z1)
    int tw;                  // tile width in columns (64 vx)
    int64_t vbase, vstride;  // vector offset of the box's first label, label stride
    int sidx;                // box index: RhsState rows sidx*R .. sidx*R+R-1
    int pidx;                // partial slot of the tile
};

struct WholeTiles {
    TileMap tm;
    Geom G;
    int ntiles;  // partial stride
    __device__ __forceinline__ int count() const { return tm.xcd ? 8 * tm.per : tm.tiles; }
    __device__ __forceinline__ bool get(int i, BoxTile& b) const {
        const int t = tm.tile(i);
        if (t < 0) return false;
        const int tx = t % tm.gx, ty = (t / tm.gx) % tm.gy, tz = t / (tm.gx * tm.gy);
        b.G = G;
        b.voff = 0;
        b.gox = b.goy = b.goz = 0;
        b.ox = b.oy = b.oz = 0;
        b.sx = G.nx;
        b.sy = G.ny;
        b.sz = G.nz;
        b.tw = 64 * tm.vx;
        b.X0 = tx * b.tw;
        b.Y0 = ty * tm.by;
        tm.planes(tz, G.nz, b.z0, b.z1);
        b.vbase = 0;
        b.vstride = G.n;
        b.sidx = 0;
        b.pidx = t;
        return true;
    }
};

// One brick of a batched solve: the box inside its volume, and that volume
// (the whole fine grid, or the brick's own sub-volume in a pool).
struct BrickGeo {
    int vnx, vny, vnz;   // volume dims
    int gox, goy, goz;   // global position of the volume's origin
    int64_t vvoff;       // offset of the volume in the intensity / label arrays
    int ox, oy, oz, sx, sy, sz;
    int gx, gy;         // tiles per row of columns / per column of rows
    int tile0, ntiles;  // its tiles in the global tile table
    int64_t voff;       // vector offset of its first label
    int64_t vox;        // sx * sy * sz
};

struct BrickTiles {
    const BrickGeo* bricks;
    const int* tile_brick;  // global tile -> brick
    const int* list;        // compacted tiles to work on
    const int* list_count;
    int zc, by;
    int ntiles;  // partial stride (all tiles)
    int xcd;    // 1: XCD-aware order
    // XCD-aware order: slot `it` runs on XCD it % 8 (the grid is a multiple of
    // 8 blocks, handed to the XCDs round-robin), and each XCD walks its own
    // contiguous eighth of the list in order, so the tiles of one brick
    // (consecutive in the list) meet in one L2.  Plain order: slot = index.
    __device__ __forceinline__ int count() const {
        return xcd ? 8 * ((*list_count + 7) / 8) : *list_count;
    }
    __device__ __forceinline__ bool get(int it, BoxTile& b) const {
        int i = it;
        if (xcd) {
            const int n = *list_count;
            const int per = (n + 7) / 8;
            const int pos = it >> 3;
            i = (it & 7) * per + pos;
            if (pos >= per || i >= n) return false;
        }
        const int g = list[i];
        const int bi = tile_brick[g];
        brick_tile(bricks[bi], g - bricks[bi].tile0, zc, by, bi, g, b);
        return true;
    }

    // Tile t of brick B (tiles of 64 x by columns by zc planes, x fastest,
    // then y, then z); its RhsState rows are sidx * R.., its partial slot pidx.
    static __device__ __forceinline__ void brick_tile(const BrickGeo& B, int t, int zc, int by,
                                                      int sidx, int pidx, BoxTile& b) {
        const int tx = t % B.gx, ty = (t / B.gx) % B.gy, tz = t / (B.gx * B.gy);
        b.G.nx = B.vnx;
        b.G.ny = B.vny;
        b.G.nz = B.vnz;
        b.G.plane = (int64_t)B.vnx * B.vny;
        b.G.n = b.G.plane * B.vnz;
        b.voff = B.vvoff;
        b.gox = B.gox;
        b.goy = B.goy;
        b.goz = B.goz;
        b.ox = B.ox;
        b.oy = B.oy;
        b.oz = B.oz;
        b.sx = B.sx;
        b.sy = B.sy;
        b.sz = B.sz;
        b.tw = 64;
        b.X0 = tx * 64;
        b.Y0 = ty * by;
        b.z0 = tz * zc;
        b.z1 = min(b.z0 + zc, B.sz);
        b.vbase = B.voff;
        b.vstride = B.vox;
        b.sidx = sidx;
        b.pidx = pidx;
    }
};

// Dirichlet data of the face shell of a brick: the coarse probabilities,
// upsampled trilinearly (cell centred, edge clamped) to the fine voxel.
struct Shell {
    const void* coarse;  // [K][cnz][cny][cnx], float32 (cdt 0) or float64 (cdt 1); NULL: none
    int cdt;
    int cnx, cny, cnz;
    int64_t cn;
    int factor;
};

__device__ __forceinline__ double coarse_at(const Shell& s, int64_t i) {
    return s.cdt ? static_cast<const double*>(s.coarse)[i]
                 : (double)static_cast<const float*>(s.coarse)[i];
}

// Fine index i <-> coarse coordinate u = (i + 0.5)/f - 0.5, clamped to
// [0, n-1]; linear weights (1 - t, t) of the two nearest coarse cells.
__device__ __forceinline__ void axis_lerp(int i, int f, int nc, int& i0, int& i1, double& t) {
    double u = __dsub_rn(__ddiv_rn((double)i + 0.5, (double)f), 0.5);
    u = fmin(fmax(u, 0.0), (double)(nc - 1));
    i0 = min((int)floor(u), nc - 1);
    i1 = min(i0 + 1, nc - 1);
    t = __dsub_rn(u, (double)i0);
}

// Corner products ((wz wy) wx) c summed z-major, y, then x, without fused
// multiply-adds.
__device__ __forceinline__ double upsample(const Shell& s, int label, int x, int y, int z) {
    int x0, x1, y0, y1, z0, z1;
    double tx, ty, tz;
    axis_lerp(x, s.factor, s.cnx, x0, x1, tx);
    axis_lerp(y, s.factor, s.cny, y0, y1, ty);
    axis_lerp(z, s.factor, s.cnz, z0, z1, tz);
    const int64_t base = (int64_t)(label - 1) * s.cn;
    const int zi[2] = {z0, z1}, yi[2] = {y0, y1}, xi[2] = {x0, x1};
    const double wz[2] = {__dsub_rn(1.0, tz), tz}, wy[2] = {__dsub_rn(1.0, ty), ty},
                 wx[2] = {__dsub_rn(1.0, tx), tx};
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double w = __dmul_rn(__dmul_rn(wz[a], wy[b]), wx[c]);
                const int64_t idx = base + ((int64_t)zi[a] * s.cny + yi[b]) * s.cnx + xi[c];
                acc = __dadd_rn(acc, __dmul_rn(w, coarse_at(s, idx)));
            }
    return acc;
}

// ---------------------------------------------------------------- CG passes

// Lane geometry of a tile.  Each lane owns VX cells per plane: VX columns 64
// apart (YM = false: the tile is 64 VX x BY columns) or VX rows BY apart
// (YM = true: 64 x BY VX, for 64-wide boxes).  lr/lc: the cells' LDS row and
// column (one halo row/column on each side).
template <int BY, int U, int VX, bool YM = false>
struct TileLanes {
    static constexpr int TR = YM ? BY * VX : BY;  // tile rows
    static constexpr int TC = YM ? 64 : 64 * VX;  // tile columns
    static constexpr int HR = YM ? VX : 1;        // rows per lane
    static constexpr int HV = YM ? 1 : VX;        // columns per lane
    static constexpr int NYH = (2 * U + BY - 1) / BY;  // y-halo rows per wave per batch
    static constexpr int TW = TC;
    int lx, ly;
    int gx[VX], gy[VX];               // own cells, global column / row
    int lr[VX], lc[VX];               // own cells in LDS
    bool in_box[VX], in_vol[VX];      // own cell's column inside the box / the volume
    uint32_t colv[VX], colb[VX];      // clamped in-plane offsets in the volume / the box
    bool hx_use, hx_vol, hx_box;
    int hx_k, hx_col_lds, hx_row_lds, hx_gx, hx_gy;
    uint32_t hx_colv, hx_colb;
    bool hy_use[NYH];
    int hy_gy[NYH];
    bool hy_vol[NYH][HV], hy_box[NYH][HV];
    int hy_k[NYH], hy_row_lds[NYH];
    uint32_t hy_colv[NYH][HV], hy_colb[NYH][HV];

    __device__ __forceinline__ void init(const Geom& G, const BoxTile& b) {
        lx = threadIdx.x;
        ly = threadIdx.y;
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const int xl = b.X0 + lx + (YM ? 0 : 64 * v);  // box-local
            const int yl = b.Y0 + ly + (YM ? BY * v : 0);
            gx[v] = b.ox + xl;
            gy[v] = b.oy + yl;
            lr[v] = ly + 1 + (YM ? BY * v : 0);
            lc[v] = lx + 1 + (YM ? 0 : 64 * v);
            in_box[v] = xl < b.sx && yl < b.sy;
            in_vol[v] = gx[v] < G.nx && gy[v] < G.ny;
            colv[v] = uint32_t(min(gy[v], G.ny - 1)) * uint32_t(G.nx) + uint32_t(min(gx[v], G.nx - 1));
            colb[v] = uint32_t(min(yl, b.sy - 1)) * uint32_t(b.sx) + uint32_t(min(xl, b.sx - 1));
        }
        // x halo: lanes 0 .. 2 U HR - 1, one value each: side = lane parity,
        // plane = (lane / 2) % U, own row = (lane / 2) / U
        const int side = lx & 1;
        const int t = lx >> 1;
        hx_use = lx < 2 * U * HR;
        hx_k = min(t % U, U - 1);
        const int vr = min(t / U, HR - 1);
        const int yl = b.Y0 + ly + (YM ? BY * vr : 0);
        const int xl = side ? b.X0 + TC : b.X0 - 1;
        hx_gx = b.ox + xl;
        hx_gy = b.oy + yl;
        hx_vol = hx_use && hx_gx >= 0 && hx_gx < G.nx && hx_gy < G.ny;
        hx_box = hx_use && xl >= 0 && xl < b.sx && yl < b.sy;
        hx_colv = uint32_t(min(hx_gy, G.ny - 1)) * uint32_t(G.nx) +
                  uint32_t(clampi(hx_gx, 0, G.nx - 1));
        hx_colb = uint32_t(min(yl, b.sy - 1)) * uint32_t(b.sx) + uint32_t(clampi(xl, 0, b.sx - 1));
        hx_col_lds = side ? TC + 1 : 0;
        hx_row_lds = ly + 1 + (YM ? BY * vr : 0);
        // y halo: 2U rows (side, plane) spread over the waves, TC values each
#pragma unroll
        for (int j = 0; j < NYH; ++j) {
            const int i = ly + j * BY;
            hy_use[j] = i < 2 * U;
            const int sy = i & 1;
            hy_k[j] = min(i >> 1, U - 1);
            const int ybl = sy ? b.Y0 + TR : b.Y0 - 1;
            const int gyh = b.oy + ybl;
            hy_gy[j] = gyh;
            const uint32_t rv = uint32_t(clampi(gyh, 0, G.ny - 1)) * uint32_t(G.nx);
            const uint32_t rb = uint32_t(clampi(ybl, 0, b.sy - 1)) * uint32_t(b.sx);
#pragma unroll
            for (int h = 0; h < HV; ++h) {
                const int xl2 = b.X0 + lx + 64 * h;
                const int gxh = b.ox + xl2;
                hy_vol[j][h] = hy_use[j] && gyh >= 0 && gyh < G.ny && gxh < G.nx;
                hy_box[j][h] = hy_use[j] && ybl >= 0 && ybl < b.sy && xl2 < b.sx;
                hy_colv[j][h] = rv + uint32_t(min(gxh, G.nx - 1));
                hy_colb[j][h] = rb + uint32_t(min(xl2, b.sx - 1));
            }
            hy_row_lds[j] = sy ? TR + 1 : 0;
        }
    }
};

// Offsets of box-local plane lz in the volume and in the box (both clamped),
// and whether lz lies in the box.
struct PlaneOff {
    int64_t v, b;
    bool inb;
};

__device__ __forceinline__ PlaneOff plane_off(const Geom& G, const BoxTile& bt, int lz) {
    PlaneOff p;
    const int gz = bt.oz + lz;
    p.v = (int64_t)clampi(gz, 0, G.nz - 1) * G.plane;
    p.b = (int64_t)clampi(lz, 0, bt.sz - 1) * bt.sx * bt.sy;
    p.inb = lz >= 0 && lz < bt.sz;
    return p;
}

// Labels of a box that iterate, and the label each one reads its operands
// from: one that does not iterate reads an iterating label's operands (no
// extra HBM traffic) and writes nothing.  Returns -1 if none iterates.
template <int R>
__device__ __forceinline__ int box_labels(const RhsState* __restrict__ st, int sidx,
                                          bool (&act)[R], int (&src)[R]) {
    int first = -1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        act[r] = st[sidx * R + r].active != 0;
        if (act[r] && first < 0) first = r;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) src[r] = act[r] ? r : max(first, 0);
    return first;
}

// Whether plane Z has a neighbour at Z + 1 (a time series has no z edge
// between the last plane of a time step and the first of the next).
template <bool T4>
__device__ __forceinline__ bool has_zp(const Geom& G, int gz) {
    return gz + 1 < G.nz && (!T4 || (gz + 1) % G.tz != 0);
}

// The five edge weights of a voxel in plane k, column v of the LDS tile:
// -x, +x, -y, +y read from the batch's edge-weight planes (each in-plane
// edge evaluated once, by the cell on its low side: publish_edge_weights),
// +z from the registers, zero across the volume border; d adds the -z
// weight carried from the previous plane.  T4 (volume
// time series): eval_t adds the two time edges (the same voxel in the
// previous and next time step, tz planes away) to d.
template <typename T, typename Lanes, int U, bool T4 = false>
struct Stencil {
    using Tile = T[U][Lanes::TR + 2][Lanes::TC + 2];
    T wxm, wxp, wym, wyp, wzp, d;
    T wtm, wtp;
    // SW: the in-plane weights from the edge-weight planes swx / swy
    // (publish_edge_weights), else evaluated here from the intensity plane sg
    template <bool SW>
    __device__ __forceinline__ void eval(const Tile& sg, const Tile& swx, const Tile& swy, int k,
                                         int v, const Lanes& L, const Geom& G, int gz, T gc,
                                         T gzn, T wzm, const WCoef& wc) {
        const int r = L.lr[v], c = L.lc[v];
        if constexpr (SW) {
            wxm = L.gx[v] > 0 ? swx[k][r][c - 1] : T(0);
            wxp = swx[k][r][c];
            wym = L.gy[v] > 0 ? swy[k][r - 1][c] : T(0);
            wyp = swy[k][r][c];
        } else {
            wxm = L.gx[v] > 0 ? Weight<T>::of(gc - sg[k][r][c - 1], wc) : T(0);
            wxp = L.gx[v] + 1 < G.nx ? Weight<T>::of(gc - sg[k][r][c + 1], wc) : T(0);
            wym = L.gy[v] > 0 ? Weight<T>::of(gc - sg[k][r - 1][c], wc) : T(0);
            wyp = L.gy[v] + 1 < G.ny ? Weight<T>::of(gc - sg[k][r + 1][c], wc) : T(0);
        }
        wzp = has_zp<T4>(G, gz) ? Weight<T>::of(gc - gzn, wc) : T(0);
        d = wxm + wxp + wym + wyp + wzm + wzp;
    }
    __device__ __forceinline__ void eval_t(const Geom& G, int gz, T gc, T gtm, T gtp,
                                           const WCoef& wc) {
        wtm = gz >= G.tz ? Weight<T>::of(gc - gtm, wc) : T(0);
        wtp = gz + G.tz < G.nz ? Weight<T>::of(gc - gtp, wc) : T(0);
        d = d + wtm + wtp;
    }
    // q = d p - sum_j w_j p_j
    __device__ __forceinline__ T apply(const Tile& sp, int k, int v, const Lanes& L, T wzm, T pc,
                                       T pzm, T pzp) const {
        const int r = L.lr[v], c = L.lc[v];
        return d * pc - (wxm * sp[k][r][c - 1] + wxp * sp[k][r][c + 1] + wym * sp[k][r - 1][c] +
                         wyp * sp[k][r + 1][c] + wzm * pzm + wzp * pzp);
    }
    __device__ __forceinline__ T apply_t(const Tile& sp, int k, int v, const Lanes& L, T wzm,
                                         T pc, T pzm, T pzp, T ptm, T ptp) const {
        const int r = L.lr[v], c = L.lc[v];
        return d * pc - (wxm * sp[k][r][c - 1] + wxp * sp[k][r][c + 1] + wym * sp[k][r - 1][c] +
                         wyp * sp[k][r + 1][c] + wzm * pzm + wzp * pzp + wtm * ptm + wtp * ptp);
    }
};

// The +x and +y edge weights of a batch's cells into the edge-weight planes
// (swx, swy: same layout as the intensity planes sg): every own cell
// evaluates the edges to its +x and +y neighbours, the x-halo lanes of the
// low side the edge from the left halo cell into the tile, and the lanes of
// the top y-halo row the edges from that row into the tile.  A cell then
// reads its -x / -y weight where its neighbour wrote the +x / +y one: three
// exponentials per cell instead of five, the same values (an edge's weight
// depends on the squared difference only).  Zero across the volume border
// on the high side, as the cells' own tests give on the low side.  Called
// between the barrier after the planes are published and another barrier.
template <typename T, typename Lanes, int U, int VX>
__device__ __forceinline__ void publish_edge_weights(T (&swx)[U][Lanes::TR + 2][Lanes::TC + 2],
                                                     T (&swy)[U][Lanes::TR + 2][Lanes::TC + 2],
                                                     const T (&sg)[U][Lanes::TR + 2][Lanes::TC + 2],
                                                     const Lanes& L, const Geom& G,
                                                     const T (&Gv)[U + 2][VX], const WCoef& wc) {
    constexpr int NYH = Lanes::NYH;
    constexpr int HV = Lanes::HV;
#pragma unroll
    for (int k = 0; k < U; ++k) {
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const int r = L.lr[v], c = L.lc[v];
            const T gc = Gv[k + 1][v];
            swx[k][r][c] = L.gx[v] + 1 < G.nx ? Weight<T>::of(gc - sg[k][r][c + 1], wc) : T(0);
            swy[k][r][c] = L.gy[v] + 1 < G.ny ? Weight<T>::of(gc - sg[k][r + 1][c], wc) : T(0);
        }
    }
    if (L.hx_use && L.hx_col_lds == 0) {
        const int k = L.hx_k, r = L.hx_row_lds;
        swx[k][r][0] = Weight<T>::of(sg[k][r][0] - sg[k][r][1], wc);
    }
#pragma unroll
    for (int j = 0; j < NYH; ++j) {
        if (L.hy_use[j] && L.hy_row_lds[j] == 0) {
#pragma unroll
            for (int h = 0; h < HV; ++h) {
                const int k = L.hy_k[j], c = 64 * h + L.lx + 1;
                swy[k][0][c] = Weight<T>::of(sg[k][0][c] - sg[k][1][c], wc);
            }
        }
    }
}

// Pass 1: p_new = z + beta p_old (formed on the fly for the voxel and its
// neighbours; zero on seeds and outside the box), q = A p_new, partial
// p_new.q per label.  Label r reads p_old from buffer st.pcur of pb0/pb1 and
// writes p_new to the other one.  qout (optional) receives q.  T4: a volume
// time series (whole volume only); the two time neighbours of each own cell
// are read directly, tz planes away.
template <typename T, int R, int BY, int U, int VX, bool YM, bool SW = false>
struct PassSmem {
    using Lanes = TileLanes<BY, U, VX, YM>;
    static constexpr size_t plane = size_t(U) * (Lanes::TR + 2) * (Lanes::TC + 2);
    // intensity, p per label, and (SW) the +x / +y edge weights
    static constexpr size_t bytes = sizeof(T) * plane * (1 + R + (SW ? 2 : 0));
};

// One tile of pass 1, accumulated into acc (per label p_new.q); false if no
// label of the tile's box iterates (uniform over the block).  smem: at least
// PassSmem<T, R, BY, U, VX, YM>::bytes of LDS.
template <typename V, typename T, int R, int BY, int U, int VX, bool YM = false, bool T4 = false,
          bool SW = false>
__device__ __forceinline__ bool cg_pass1_tile(char* __restrict__ smem, const BoxTile& bt,
                                              const V* __restrict__ volp, WCoef wc,
                                              const T* __restrict__ zv, T* __restrict__ pb0,
                                              T* __restrict__ pb1, T* __restrict__ qout,
                                              const RhsState* __restrict__ st,
                                              double (&acc)[R]) {
    using Lanes = TileLanes<BY, U, VX, YM>;
    constexpr int NYH = Lanes::NYH;
    constexpr int HV = Lanes::HV;
    using Plane = T[U][Lanes::TR + 2][Lanes::TC + 2];
    Plane& sg = *reinterpret_cast<Plane*>(smem);
    Plane(&sp)[R] = *reinterpret_cast<Plane(*)[R]>(smem + sizeof(Plane));
    // the edge-weight planes exist with SW only (else they alias sg, unread)
    Plane& swx = *reinterpret_cast<Plane*>(smem + (SW ? (1 + R) * sizeof(Plane) : 0));
    Plane& swy = *reinterpret_cast<Plane*>(smem + (SW ? (2 + R) * sizeof(Plane) : 0));
    bool act[R];
    int src[R];
    if (box_labels<R>(st, bt.sidx, act, src) < 0) return false;  // uniform over the block
    const Geom& G = bt.G;
    const V* __restrict__ vol = volp + bt.voff;
    T bet[R];
    const T* zr[R];
    const T* po[R];
    T* pw[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const RhsState& s = st[bt.sidx * R + src[r]];
        bet[r] = (T)s.beta;
        zr[r] = zv + bt.vbase + src[r] * bt.vstride;
        po[r] = (s.pcur ? pb1 : pb0) + bt.vbase + src[r] * bt.vstride;
        pw[r] = (st[bt.sidx * R + r].pcur ? pb0 : pb1) + bt.vbase + r * bt.vstride;
    }
    Lanes L;
    L.init(G, bt);
    // halo cells of the vectors outside the box read as zero: on brick tiles
    // (not SW) a wave none of whose halo lanes lies in the box (the x-halo of
    // a brick-wide tile, the y-halo at the brick's faces) issues none of
    // those loads; whole-volume tiles load them (their halo is outside the
    // box only at the volume border, and the test costs them registers)
    const bool hx_vec = SW || __ballot(L.hx_box) != 0;
    bool hy_vec[Lanes::NYH];
#pragma unroll
    for (int j = 0; j < Lanes::NYH; ++j) {
        bool any = false;
#pragma unroll
        for (int h = 0; h < Lanes::HV; ++h) any = any || L.hy_box[j][h];
        hy_vec[j] = SW || __ballot(any) != 0;
    }
    const int64_t bplane = (int64_t)bt.sx * bt.sy;

    T Gv[U + 2][VX], Pv[U + 2][R][VX];  // own columns: planes z-1, z, z+1 .. z+U
    {
        const PlaneOff om = plane_off(G, bt, bt.z0 - 1), oc = plane_off(G, bt, bt.z0);
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            Gv[0][v] = (T)ldu(vol + om.v, L.colv[v]);
            Gv[1][v] = (T)ldu(vol + oc.v, L.colv[v]);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T a = ldu(zr[r] + om.b, L.colb[v]) + bet[r] * ldu(po[r] + om.b, L.colb[v]);
                Pv[0][r][v] = om.inb ? a : T(0);
                Pv[1][r][v] = ldu(zr[r] + oc.b, L.colb[v]) + bet[r] * ldu(po[r] + oc.b, L.colb[v]);
            }
        }
    }
    T wzm[VX];
#pragma unroll
    for (int v = 0; v < VX; ++v)
        wzm[v] = (L.in_box[v] && bt.oz + bt.z0 > 0 && has_zp<T4>(G, bt.oz + bt.z0 - 1))
                     ? Weight<T>::of(Gv[1][v] - Gv[0][v], wc)
                     : T(0);

    for (int zb = bt.z0; zb < bt.z1; zb += U) {
        // (1) every read of the batch
        T zN[U][R][VX], oN[U][R][VX];
        bool nin[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const PlaneOff o = plane_off(G, bt, zb + 1 + k);
            nin[k] = o.inb;
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                Gv[k + 2][v] = (T)ldu(vol + o.v, L.colv[v]);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    zN[k][r][v] = ldu(zr[r] + o.b, L.colb[v]);
                    oN[k][r][v] = ldu(po[r] + o.b, L.colb[v]);
                }
            }
        }
        // T4: g and p_new of the previous and next time step of the
        // batch's own cells
        T Gtm[T4 ? U : 1][VX], Gtp[T4 ? U : 1][VX], Ptm[T4 ? U : 1][R][VX],
            Ptp[T4 ? U : 1][R][VX];
        if constexpr (T4) {
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int lz = zb + k;
                const PlaneOff om = plane_off(G, bt, lz - G.tz), op = plane_off(G, bt, lz + G.tz);
                const bool im = lz - G.tz >= 0, ip = lz + G.tz < bt.sz;
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    Gtm[k][v] = (T)ldu(vol + om.v, L.colv[v]);
                    Gtp[k][v] = (T)ldu(vol + op.v, L.colv[v]);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const T am = ldu(zr[r] + om.b, L.colb[v]) +
                                     bet[r] * ldu(po[r] + om.b, L.colb[v]);
                        const T ap = ldu(zr[r] + op.b, L.colb[v]) +
                                     bet[r] * ldu(po[r] + op.b, L.colb[v]);
                        Ptm[k][r][v] = im ? am : T(0);
                        Ptp[k][r][v] = ip ? ap : T(0);
                    }
                }
            }
        }
        T hxg, hxz[R], hxo[R];
        {
            const PlaneOff o = plane_off(G, bt, zb + L.hx_k);
            hxg = (T)ldu(vol + o.v, L.hx_colv);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                hxz[r] = hx_vec ? ldu(zr[r] + o.b, L.hx_colb) : T(0);
                hxo[r] = hx_vec ? ldu(po[r] + o.b, L.hx_colb) : T(0);
            }
        }
        T hyg[NYH][HV], hyz[NYH][R][HV], hyo[NYH][R][HV];
#pragma unroll
        for (int j = 0; j < NYH; ++j) {
            const PlaneOff o = plane_off(G, bt, zb + L.hy_k[j]);
#pragma unroll
            for (int h = 0; h < HV; ++h) {
                hyg[j][h] = (T)ldu(vol + o.v, L.hy_colv[j][h]);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    hyz[j][r][h] = hy_vec[j] ? ldu(zr[r] + o.b, L.hy_colb[j][h]) : T(0);
                    hyo[j][r][h] = hy_vec[j] ? ldu(po[r] + o.b, L.hy_colb[j][h]) : T(0);
                }
            }
        }
        // (2) the previous batch (or tile) is done with the LDS planes
        __syncthreads();
        // (3) publish planes zb..zb+U-1
#pragma unroll
        for (int k = 0; k < U; ++k) {
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                if (k > 0) {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        Pv[k + 1][r][v] =
                            nin[k - 1] ? zN[k - 1][r][v] + bet[r] * oN[k - 1][r][v] : T(0);
                }
                sg[k][L.lr[v]][L.lc[v]] = L.in_vol[v] ? Gv[k + 1][v] : T(0);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    sp[r][k][L.lr[v]][L.lc[v]] = L.in_box[v] ? Pv[k + 1][r][v] : T(0);
            }
        }
        if (L.hx_use) {
            sg[L.hx_k][L.hx_row_lds][L.hx_col_lds] = L.hx_vol ? hxg : T(0);
#pragma unroll
            for (int r = 0; r < R; ++r)
                sp[r][L.hx_k][L.hx_row_lds][L.hx_col_lds] =
                    L.hx_box ? hxz[r] + bet[r] * hxo[r] : T(0);
        }
#pragma unroll
        for (int j = 0; j < NYH; ++j) {
            if (L.hy_use[j]) {
#pragma unroll
                for (int h = 0; h < HV; ++h) {
                    const int c = 64 * h + L.lx + 1;
                    sg[L.hy_k[j]][L.hy_row_lds[j]][c] = L.hy_vol[j][h] ? hyg[j][h] : T(0);
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        sp[r][L.hy_k[j]][L.hy_row_lds[j]][c] =
                            L.hy_box[j][h] ? hyz[j][r][h] + bet[r] * hyo[j][r][h] : T(0);
                }
            }
        }
#pragma unroll
        for (int v = 0; v < VX; ++v)
#pragma unroll
            for (int r = 0; r < R; ++r)
                Pv[U + 1][r][v] =
                    nin[U - 1] ? zN[U - 1][r][v] + bet[r] * oN[U - 1][r][v] : T(0);
        __syncthreads();
        if constexpr (SW) {
            publish_edge_weights<T, Lanes, U, VX>(swx, swy, sg, L, G, Gv, wc);
            __syncthreads();
        }
        // (4) stencil on planes zb..zb+U-1
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int lz = zb + k;
            const int gz = bt.oz + lz;
            const bool zin = lz < bt.z1;
            T* __restrict__ prow[R];
#pragma unroll
            for (int r = 0; r < R; ++r) prow[r] = pw[r] + (int64_t)lz * bplane;
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                Stencil<T, Lanes, U, T4> S;
                S.template eval<SW>(sg, swx, swy, k, v, L, G, gz, Gv[k + 1][v], Gv[k + 2][v],
                                    wzm[v], wc);
                if constexpr (T4) S.eval_t(G, gz, Gv[k + 1][v], Gtm[k][v], Gtp[k][v], wc);
                const bool valid = L.in_box[v] && zin;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const T pc = Pv[k + 1][r][v];
                    T q;
                    if constexpr (T4)
                        q = S.apply_t(sp[r], k, v, L, wzm[v], pc, Pv[k][r][v], Pv[k + 2][r][v],
                                      Ptm[k][r][v], Ptp[k][r][v]);
                    else
                        q = S.apply(sp[r], k, v, L, wzm[v], pc, Pv[k][r][v], Pv[k + 2][r][v]);
                    if (valid && act[r]) {
                        stu(prow[r], L.colb[v], pc);
                        if (qout) qout[bt.vbase + r * bt.vstride + (int64_t)lz * bplane + L.colb[v]] = q;
                        acc[r] += (double)pc * (double)q;
                    }
                }
                wzm[v] = S.wzp;
            }
        }
        // (5) carry planes zb+U-1 and zb+U
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            Gv[0][v] = Gv[U][v];
            Gv[1][v] = Gv[U + 1][v];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                Pv[0][r][v] = Pv[U][r][v];
                Pv[1][r][v] = Pv[U + 1][r][v];
            }
        }
    }
    return true;
}

// The passes keep four waves per SIMD (at most 128 VGPRs): their loads of a
// batch are in flight while other waves compute, and with fewer waves the
// latency shows.
// Minimum waves per SIMD the compiler keeps for a pass (1: no constraint).
// 128 x 4 float32 whole-volume tiles of one or two labels otherwise land a
// few VGPRs above 128, one wave per SIMD short of four (with the cap: about
// 110, no spills).
template <typename T, int R, int BY, int U, int VX, bool T4, bool SW>
constexpr int pass_min_waves() {
    return SW && sizeof(T) == 4 && BY == 4 && U * VX == 4 && VX <= 2 && (R == 1 || (R == 2 && !T4))
               ? 4
               : 1;
}

template <typename V, typename T, int R, int BY, int U, int VX, typename TS, bool YM = false,
          bool T4 = false>
__global__ __launch_bounds__(64 * BY) __attribute__((
    amdgpu_waves_per_eu(pass_min_waves<T, R, BY, U, VX, T4, std::is_same<TS, WholeTiles>::value>()))) void k_cg_pass1(
    const V* __restrict__ volp, WCoef wc, TS ts, const T* __restrict__ zv,
    T* __restrict__ pb0, T* __restrict__ pb1, T* __restrict__ qout,
    const RhsState* __restrict__ st, double* __restrict__ part) {
    // whole volumes share each in-plane edge weight through LDS; brick
    // tiles (more planes per batch, one column per lane) run faster
    // evaluating all five per cell
    constexpr bool SW = std::is_same<TS, WholeTiles>::value;
    __shared__ __align__(16) char smem[PassSmem<T, R, BY, U, VX, YM, SW>::bytes];
    const int cnt = ts.count();
    for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
        BoxTile bt;
        if (!ts.get(it, bt)) continue;
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        if (!cg_pass1_tile<V, T, R, BY, U, VX, YM, T4, SW>(smem, bt, volp, wc, zv, pb0, pb1, qout, st,
                                                       acc))
            continue;
        block_sum_store<R, BY>(acc, part + bt.pidx, ts.ntiles);
    }
}

// Pass 2: q = A p (p = buffer st.pcur, just written by pass 1); on unknowns
// x += alpha p, r = d z - alpha q, z = r / d; partials r.z and r.r per label
// ([2R][ntiles]).  T4 as in pass 1.
// One tile of pass 2, accumulated into acc (per label r.z, r.r); false if
// no label of the tile's box iterates.  smem as for pass 1.
template <typename V, typename T, int R, int BY, int U, int VX, bool YM = false, bool T4 = false,
          bool SW = false>
__device__ __forceinline__ bool cg_pass2_tile(char* __restrict__ smem, const BoxTile& bt,
                                              const V* __restrict__ volp,
                                              const uint8_t* __restrict__ labp, WCoef wc,
                                              T* __restrict__ xv, T* __restrict__ zv,
                                              const T* __restrict__ pb0, const T* __restrict__ pb1,
                                              const RhsState* __restrict__ st,
                                              double (&acc)[2 * R]) {
    using Lanes = TileLanes<BY, U, VX, YM>;
    constexpr int NYH = Lanes::NYH;
    constexpr int HV = Lanes::HV;
    using Plane = T[U][Lanes::TR + 2][Lanes::TC + 2];
    Plane& sg = *reinterpret_cast<Plane*>(smem);
    Plane(&sp)[R] = *reinterpret_cast<Plane(*)[R]>(smem + sizeof(Plane));
    // the edge-weight planes exist with SW only (else they alias sg, unread)
    Plane& swx = *reinterpret_cast<Plane*>(smem + (SW ? (1 + R) * sizeof(Plane) : 0));
    Plane& swy = *reinterpret_cast<Plane*>(smem + (SW ? (2 + R) * sizeof(Plane) : 0));
    bool act[R];
    int src[R];
    if (box_labels<R>(st, bt.sidx, act, src) < 0) return false;
    const Geom& G = bt.G;
    const V* __restrict__ vol = volp + bt.voff;
    const uint8_t* __restrict__ lab = labp + bt.voff;
    T alp[R];
    const T* pr[R];
    T* xr[R];
    T* zr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        alp[r] = (T)st[bt.sidx * R + r].alpha;
        const int64_t vb = bt.vbase + src[r] * bt.vstride;
        pr[r] = (st[bt.sidx * R + src[r]].pcur ? pb1 : pb0) + vb;
        xr[r] = xv + vb;
        zr[r] = zv + vb;
    }
    Lanes L;
    L.init(G, bt);
    // halo cells of the vectors outside the box read as zero: on brick tiles
    // (not SW) a wave none of whose halo lanes lies in the box (the x-halo of
    // a brick-wide tile, the y-halo at the brick's faces) issues none of
    // those loads; whole-volume tiles load them (their halo is outside the
    // box only at the volume border, and the test costs them registers)
    const bool hx_vec = SW || __ballot(L.hx_box) != 0;
    bool hy_vec[Lanes::NYH];
#pragma unroll
    for (int j = 0; j < Lanes::NYH; ++j) {
        bool any = false;
#pragma unroll
        for (int h = 0; h < Lanes::HV; ++h) any = any || L.hy_box[j][h];
        hy_vec[j] = SW || __ballot(any) != 0;
    }

    T Gv[U + 2][VX], Pv[U + 2][R][VX];
    {
        const PlaneOff om = plane_off(G, bt, bt.z0 - 1), oc = plane_off(G, bt, bt.z0);
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            Gv[0][v] = (T)ldu(vol + om.v, L.colv[v]);
            Gv[1][v] = (T)ldu(vol + oc.v, L.colv[v]);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T a = ldu(pr[r] + om.b, L.colb[v]);
                Pv[0][r][v] = om.inb ? a : T(0);
                Pv[1][r][v] = ldu(pr[r] + oc.b, L.colb[v]);
            }
        }
    }
    T wzm[VX];
#pragma unroll
    for (int v = 0; v < VX; ++v)
        wzm[v] = (L.in_box[v] && bt.oz + bt.z0 > 0 && has_zp<T4>(G, bt.oz + bt.z0 - 1))
                     ? Weight<T>::of(Gv[1][v] - Gv[0][v], wc)
                     : T(0);

    for (int zb = bt.z0; zb < bt.z1; zb += U) {
        T Xv[U][R][VX], Zv[U][R][VX];
        uint8_t Lv[U][VX];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const PlaneOff o = plane_off(G, bt, zb + 1 + k);
            const PlaneOff oc = plane_off(G, bt, zb + k);
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                Gv[k + 2][v] = (T)ldu(vol + o.v, L.colv[v]);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const T a = ldu(pr[r] + o.b, L.colb[v]);
                    Pv[k + 2][r][v] = o.inb ? a : T(0);
                }
                Lv[k][v] = ldu(lab + oc.v, L.colv[v]);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    Xv[k][r][v] = ldu(xr[r] + oc.b, L.colb[v]);
                    Zv[k][r][v] = ldu(zr[r] + oc.b, L.colb[v]);
                }
            }
        }
        T Gtm[T4 ? U : 1][VX], Gtp[T4 ? U : 1][VX], Ptm[T4 ? U : 1][R][VX],
            Ptp[T4 ? U : 1][R][VX];
        if constexpr (T4) {
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int lz = zb + k;
                const PlaneOff om = plane_off(G, bt, lz - G.tz), op = plane_off(G, bt, lz + G.tz);
                const bool im = lz - G.tz >= 0, ip = lz + G.tz < bt.sz;
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    Gtm[k][v] = (T)ldu(vol + om.v, L.colv[v]);
                    Gtp[k][v] = (T)ldu(vol + op.v, L.colv[v]);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const T am = ldu(pr[r] + om.b, L.colb[v]);
                        const T ap = ldu(pr[r] + op.b, L.colb[v]);
                        Ptm[k][r][v] = im ? am : T(0);
                        Ptp[k][r][v] = ip ? ap : T(0);
                    }
                }
            }
        }
        T hxg, hxp[R];
        {
            const PlaneOff o = plane_off(G, bt, zb + L.hx_k);
            hxg = (T)ldu(vol + o.v, L.hx_colv);
#pragma unroll
            for (int r = 0; r < R; ++r) hxp[r] = hx_vec ? ldu(pr[r] + o.b, L.hx_colb) : T(0);
        }
        T hyg[NYH][HV], hyp[NYH][R][HV];
#pragma unroll
        for (int j = 0; j < NYH; ++j) {
            const PlaneOff o = plane_off(G, bt, zb + L.hy_k[j]);
#pragma unroll
            for (int h = 0; h < HV; ++h) {
                hyg[j][h] = (T)ldu(vol + o.v, L.hy_colv[j][h]);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    hyp[j][r][h] = hy_vec[j] ? ldu(pr[r] + o.b, L.hy_colb[j][h]) : T(0);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < U; ++k)
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                sg[k][L.lr[v]][L.lc[v]] = L.in_vol[v] ? Gv[k + 1][v] : T(0);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    sp[r][k][L.lr[v]][L.lc[v]] = L.in_box[v] ? Pv[k + 1][r][v] : T(0);
            }
        if (L.hx_use) {
            sg[L.hx_k][L.hx_row_lds][L.hx_col_lds] = L.hx_vol ? hxg : T(0);
#pragma unroll
            for (int r = 0; r < R; ++r)
                sp[r][L.hx_k][L.hx_row_lds][L.hx_col_lds] = L.hx_box ? hxp[r] : T(0);
        }
#pragma unroll
        for (int j = 0; j < NYH; ++j) {
            if (L.hy_use[j]) {
#pragma unroll
                for (int h = 0; h < HV; ++h) {
                    const int c = 64 * h + L.lx + 1;
                    sg[L.hy_k[j]][L.hy_row_lds[j]][c] = L.hy_vol[j][h] ? hyg[j][h] : T(0);
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        sp[r][L.hy_k[j]][L.hy_row_lds[j]][c] =
                            L.hy_box[j][h] ? hyp[j][r][h] : T(0);
                }
            }
        }
        __syncthreads();
        if constexpr (SW) {
            publish_edge_weights<T, Lanes, U, VX>(swx, swy, sg, L, G, Gv, wc);
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int lz = zb + k;
            const int gz = bt.oz + lz;
            const bool zin = lz < bt.z1;
            const int64_t ob = (int64_t)lz * bt.sx * bt.sy;
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                Stencil<T, Lanes, U, T4> S;
                S.template eval<SW>(sg, swx, swy, k, v, L, G, gz, Gv[k + 1][v], Gv[k + 2][v],
                                    wzm[v], wc);
                if constexpr (T4) S.eval_t(G, gz, Gv[k + 1][v], Gtm[k][v], Gtp[k][v], wc);
                const T dinv = T(1) / S.d;
                const bool valid = L.in_box[v] && zin && Lv[k][v] == 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const T pc = Pv[k + 1][r][v];
                    T q;
                    if constexpr (T4)
                        q = S.apply_t(sp[r], k, v, L, wzm[v], pc, Pv[k][r][v], Pv[k + 2][r][v],
                                      Ptm[k][r][v], Ptp[k][r][v]);
                    else
                        q = S.apply(sp[r], k, v, L, wzm[v], pc, Pv[k][r][v], Pv[k + 2][r][v]);
                    const T xn = Xv[k][r][v] + alp[r] * pc;
                    const T rres = S.d * Zv[k][r][v] - alp[r] * q;
                    const T zn = dinv * rres;
                    if (valid && act[r]) {
                        T* __restrict__ xo = xv + bt.vbase + r * bt.vstride + ob;
                        T* __restrict__ zo = zv + bt.vbase + r * bt.vstride + ob;
                        stnt(xo, L.colb[v], xn);
                        stnt(zo, L.colb[v], zn);
                        acc[2 * r] += (double)rres * (double)zn;
                        acc[2 * r + 1] += (double)rres * (double)rres;
                    }
                }
                wzm[v] = S.wzp;
            }
        }
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            Gv[0][v] = Gv[U][v];
            Gv[1][v] = Gv[U + 1][v];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                Pv[0][r][v] = Pv[U][r][v];
                Pv[1][r][v] = Pv[U + 1][r][v];
            }
        }
    }
    return true;
}

template <typename V, typename T, int R, int BY, int U, int VX, typename TS, bool YM = false,
          bool T4 = false>
__global__ __launch_bounds__(64 * BY) __attribute__((
    amdgpu_waves_per_eu(pass_min_waves<T, R, BY, U, VX, T4, std::is_same<TS, WholeTiles>::value>()))) void k_cg_pass2(
    const V* __restrict__ volp, const uint8_t* __restrict__ labp, WCoef wc, TS ts,
    T* __restrict__ xv, T* __restrict__ zv, const T* __restrict__ pb0,
    const T* __restrict__ pb1, const RhsState* __restrict__ st, double* __restrict__ part) {
    // whole volumes share each in-plane edge weight through LDS; brick
    // tiles (more planes per batch, one column per lane) run faster
    // evaluating all five per cell
    constexpr bool SW = std::is_same<TS, WholeTiles>::value;
    __shared__ __align__(16) char smem[PassSmem<T, R, BY, U, VX, YM, SW>::bytes];
    const int cnt = ts.count();
    for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
        BoxTile bt;
        if (!ts.get(it, bt)) continue;
        double acc[2 * R];
#pragma unroll
        for (int q = 0; q < 2 * R; ++q) acc[q] = 0.0;
        if (!cg_pass2_tile<V, T, R, BY, U, VX, YM, T4, SW>(smem, bt, volp, labp, wc, xv, zv, pb0, pb1,
                                                       st, acc))
            continue;
        block_sum_store<2 * R, BY>(acc, part + bt.pidx, ts.ntiles);
    }
}


// ---------------------------------------------------------------- residual

// Value of one cell of the full-grid embedding x~ of label lab0 + r for the
// float64 residual: the iterate on unknowns of the box, 1 on the label's
// seeds and 0 on other seeds (lab0 = 0: 0 on every seed), the upsampled
// coarse value on non-seed voxels outside the box (the brick shell), 0
// outside the volume.  dir: the cell carries Dirichlet data.  The intensity
// is kept in GT, the volume's own precision (float for uint16 and float32
// volumes, which it holds exactly).
template <typename GT, int R>
struct XCell {
    GT g;
    double xt[R];
    bool dir;

    // lmask: the labels whose values are wanted (the others are left 0).
    // shv (optional): the cell's shell values per label, interpolated
    // beforehand (else interpolated here).
    __device__ __forceinline__ void make(double gv, uint8_t lb, const double (&xb)[R], bool in_vol,
                                         bool in_box, const Shell& sh, int lab0, int gx, int gy,
                                         int gz, int lmask, const double* shv = nullptr) {
        g = in_vol ? (GT)gv : GT(0);
        dir = !(in_box && lb == 0);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double v = 0.0;
            if (!in_vol || !(lmask & (1 << r))) v = 0.0;
            else if (lb != 0) v = (lab0 > 0 && lb == lab0 + r) ? 1.0 : 0.0;
            else if (in_box) v = xb[r];
            else if (sh.coarse && lab0 > 0) v = shv ? shv[r] : upsample(sh, lab0 + r, gx, gy, gz);
            xt[r] = v;
        }
    }
};

// Float64 residual r = b - A x64 of the current iterate with float64
// weights, and the start of a CG run: z = r / d written in T (d from
// T-precision weights, summed in the passes' order, so the passes rebuild
// r = d z with the same d).  Dirichlet data as in XCell; rhs (optional) adds
// an explicit right-hand side.  Partials per tile [4R + 2][ntiles]: per label
// r.z, r.r (in T), r64.r64, b.b; then the number of unknowns with a
// non-positive and with a non-finite degree.  mode 0 only measures; mode 1
// starts a CG run for every label (p buffers and xi zeroed); mode 2
// refreshes z of the labels flagged for it (st.outer_active == 2).
// Tiled like the passes (one plane per batch): every cell's x~ is formed once
// by the lane that loads it and shared through LDS.  T4 (volume time series,
// whole volume): the two time neighbours of an own cell, tz planes away, are
// loaded and formed by its lane.
// SHX (brick tiles): LDS slots for the x-halo shell cache, per wave, row
// of the wave, side and plane of a batch of RES_HZ planes, and label.
constexpr int RES_HZ = 32;
template <typename V, int R, int BY, int VX, bool YM, bool SHX = false>
struct ResidualSmem {
    using Lanes = TileLanes<BY, 1, VX, YM>;
    using GT = typename std::conditional<std::is_same<V, double>::value, double, float>::type;
    static constexpr size_t cells = size_t(Lanes::TR + 2) * (Lanes::TC + 2);
    static constexpr size_t base = ((8 * R + sizeof(GT) + 1) * cells + 15) / 16 * 16;
    static constexpr size_t shx = SHX ? sizeof(double) * BY * Lanes::HR * 2 * RES_HZ * R : 0;
    static constexpr size_t bytes = base + shx;
};

// One tile of the float64 residual, accumulated into acc; false if a refresh
// (mode 2) has no flagged label in the tile's box.  smem: at least
// ResidualSmem<V, R, BY, VX, YM>::bytes of LDS.
template <typename V, typename T, int R, int BY, int VX, bool YM = false, bool T4 = false,
          bool SHX = false>
__device__ __forceinline__ bool residual_tile(
    char* __restrict__ smem, const BoxTile& bt, const V* __restrict__ volp,
    const uint8_t* __restrict__ labp, WCoef wc, const Shell& sh, int lab0,
    const double* __restrict__ x64, const double* __restrict__ rhs, T* __restrict__ zv,
    T* __restrict__ p0, T* __restrict__ p1, T* __restrict__ xi, int mode,
    const RhsState* __restrict__ st, double (&acc)[4 * R + 2]) {
    constexpr int NQ = 4 * R + 2;
    using Lanes = TileLanes<BY, 1, VX, YM>;
    constexpr int NYH = Lanes::NYH;
    constexpr int HV = Lanes::HV;
    constexpr int LR = Lanes::TR + 2, LC = Lanes::TC + 2;
    using GT = typename std::conditional<std::is_same<V, double>::value, double, float>::type;
    using XCells = double[R][LR][LC];
    using GCells = GT[LR][LC];
    using DCells = uint8_t[LR][LC];
    XCells& sx = *reinterpret_cast<XCells*>(smem);
    GCells& sg = *reinterpret_cast<GCells*>(smem + sizeof(XCells));
    DCells& sdir = *reinterpret_cast<DCells*>(smem + sizeof(XCells) + sizeof(GCells));
    (void)NQ;
    const Geom& G = bt.G;
    const V* __restrict__ vol = volp + bt.voff;
    const uint8_t* __restrict__ lab = labp + bt.voff;
    int wmask = 0;
    if (mode == 2) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (st[bt.sidx * R + r].outer_active == 2) wmask |= 1 << r;
        if (!wmask) return false;  // uniform over the block
    }
    // labels computed: a refresh (mode 2) needs only the flagged ones,
    // whose partials alone are read back
    const int lmask = mode == 2 ? wmask : (1 << R) - 1;
    Lanes L;
    L.init(G, bt);
    const int64_t bplane = (int64_t)bt.sx * bt.sy;

    // SHX: the x-halo cells of a brick tile lie in the brick's Dirichlet
    // shell, and every wave needs one interpolated coarse value per side and
    // plane.  Formed on the plane loop's path these cost a dependent round of
    // coarse loads per plane; instead every lane of the wave forms one
    // (plane, side) entry per row for RES_HZ planes at a time, kept in the
    // wave's own LDS slots, and the halo lanes read them.
    constexpr int HRW = Lanes::HR;
    double* shx = nullptr;
    if constexpr (SHX)
        shx = reinterpret_cast<double*>(smem + ResidualSmem<V, R, BY, VX, YM, true>::base);
    auto fill_shx = [&](int lz0) {
        const int k = L.lx >> 1, side = L.lx & 1;
        const int lz = lz0 + k;
        const int xl = side ? bt.X0 + Lanes::TC : bt.X0 - 1;
        const int gxh = bt.ox + xl;
#pragma unroll
        for (int vr = 0; vr < HRW; ++vr) {
            const int yl = bt.Y0 + L.ly + (YM ? BY * vr : 0);
            const int gyh = bt.oy + yl;
            const bool shell = sh.coarse && lab0 > 0 && lz < bt.z1 && gxh >= 0 && gxh < G.nx &&
                               gyh < G.ny && !(xl >= 0 && xl < bt.sx && yl < bt.sy);
            double* e = shx + ((((size_t)L.ly * HRW + vr) * 2 + side) * RES_HZ + k) * R;
#pragma unroll
            for (int r = 0; r < R; ++r)
                e[r] = shell && (lmask & (1 << r))
                           ? upsample(sh, lab0 + r, bt.gox + gxh, bt.goy + gyh, bt.goz + bt.oz + lz)
                           : 0.0;
        }
    };
    // this lane's x-halo entry (side, row) in the cache
    const double* shx_lane = nullptr;
    if constexpr (SHX)
        shx_lane = shx + (((size_t)L.ly * HRW + min(L.lx >> 1, HRW - 1)) * 2 + (L.lx & 1)) *
                             RES_HZ * R;

    // Raw values of a cell (intensity, label, float64 iterates); loads
    // are issued one plane (halo cells) or two planes (own cells) ahead of
    // the plane being computed, and the cells of the embedding are formed
    // from them one iteration later, so the loads overlap a plane's work.
    struct Raw {
        V g;
        uint8_t lb;
        double xb[R];
    };
    auto load_raw = [&](int64_t ov, int64_t ob, uint32_t cv, uint32_t cb, Raw& w) {
        w.g = ldu(vol + ov, cv);
        w.lb = ldu(lab + ov, cv);
#pragma unroll
        for (int r = 0; r < R; ++r)
            w.xb[r] = x64 && (lmask & (1 << r)) ? ldu(x64 + bt.vbase + r * bt.vstride + ob, cb)
                                                : 0.0;
    };
    auto load_own = [&](int lz, Raw (&w)[VX]) {
        const PlaneOff o = plane_off(G, bt, lz);
#pragma unroll
        for (int v = 0; v < VX; ++v) load_raw(o.v, o.b, L.colv[v], L.colb[v], w[v]);
    };
    auto load_halo = [&](int lz, Raw& wx, Raw (&wy)[NYH][HV]) {
        const PlaneOff o = plane_off(G, bt, lz);
        load_raw(o.v, o.b, L.hx_colv, L.hx_colb, wx);
#pragma unroll
        for (int j = 0; j < NYH; ++j)
#pragma unroll
            for (int h = 0; h < HV; ++h) load_raw(o.v, o.b, L.hy_colv[j][h], L.hy_colb[j][h], wy[j][h]);
    };
    auto make_own = [&](int lz, const Raw (&w)[VX], XCell<GT, R> (&c)[VX], uint8_t (&lb)[VX]) {
        const int gz = bt.oz + lz;
        const bool zvol = gz >= 0 && gz < G.nz;
        const bool inb = lz >= 0 && lz < bt.sz;
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            lb[v] = w[v].lb;
            c[v].make((double)w[v].g, w[v].lb, w[v].xb, L.in_vol[v] && zvol, L.in_box[v] && inb,
                      sh, lab0, bt.gox + L.gx[v], bt.goy + L.gy[v], bt.goz + gz, lmask);
        }
    };

    XCell<GT, R> cm[VX], cc[VX], cp[VX];
    uint8_t lbm[VX], lbc[VX], lbp[VX];
    Raw own1[VX], own2[VX], hx0, hx1, hy0[NYH][HV], hy1[NYH][HV];
    load_own(bt.z0 - 1, own1);
    make_own(bt.z0 - 1, own1, cm, lbm);
    load_own(bt.z0, own1);
    make_own(bt.z0, own1, cc, lbc);
    load_own(bt.z0 + 1, own1);
    load_halo(bt.z0, hx0, hy0);
    for (int lz = bt.z0; lz < bt.z1; ++lz) {
        const int gz = bt.oz + lz;
        const bool zvol = gz >= 0 && gz < G.nz;
        const bool inb = lz >= 0 && lz < bt.sz;
        // (A) the next loads: own cells of plane lz+2, halo cells of lz+1
        load_own(lz + 2, own2);
        load_halo(lz + 1, hx1, hy1);
        // (B) cells of plane lz+1 (own) and of plane lz's halo
        make_own(lz + 1, own1, cp, lbp);
        const double* shv = nullptr;
        if constexpr (SHX) {
            const int kz = (lz - bt.z0) % RES_HZ;
            if (kz == 0) {
                fill_shx(lz);
                __syncthreads();
            }
            shv = shx_lane + (size_t)kz * R;
        }
        XCell<GT, R> hx;
        hx.make((double)hx0.g, hx0.lb, hx0.xb, L.hx_vol && zvol, L.hx_box && inb, sh, lab0,
                bt.gox + L.hx_gx, bt.goy + L.hx_gy, bt.goz + gz, lmask, shv);
        XCell<GT, R> hy[NYH][HV];
#pragma unroll
        for (int j = 0; j < NYH; ++j)
#pragma unroll
            for (int h = 0; h < HV; ++h)
                hy[j][h].make((double)hy0[j][h].g, hy0[j][h].lb, hy0[j][h].xb,
                              L.hy_vol[j][h] && zvol, L.hy_box[j][h] && inb, sh, lab0,
                              bt.gox + L.gx[0] + 64 * h, bt.goy + L.hy_gy[j], bt.goz + gz,
                              lmask);
        __syncthreads();
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            sg[L.lr[v]][L.lc[v]] = cc[v].g;
            sdir[L.lr[v]][L.lc[v]] = cc[v].dir;
#pragma unroll
            for (int r = 0; r < R; ++r) sx[r][L.lr[v]][L.lc[v]] = cc[v].xt[r];
        }
        if (L.hx_use) {
            sg[L.hx_row_lds][L.hx_col_lds] = hx.g;
            sdir[L.hx_row_lds][L.hx_col_lds] = hx.dir;
#pragma unroll
            for (int r = 0; r < R; ++r) sx[r][L.hx_row_lds][L.hx_col_lds] = hx.xt[r];
        }
#pragma unroll
        for (int j = 0; j < NYH; ++j)
            if (L.hy_use[j]) {
#pragma unroll
                for (int h = 0; h < HV; ++h) {
                    const int c = 64 * h + L.lx + 1;
                    sg[L.hy_row_lds[j]][c] = hy[j][h].g;
                    sdir[L.hy_row_lds[j]][c] = hy[j][h].dir;
#pragma unroll
                    for (int r = 0; r < R; ++r) sx[r][L.hy_row_lds[j]][c] = hy[j][h].xt[r];
                }
            }
        __syncthreads();
        const bool zin = lz < bt.z1;
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            if (!(L.in_box[v] && zin)) continue;
            const uint32_t cb = L.colb[v];
            const int64_t ob = (int64_t)lz * bplane;
            if (lbc[v] != 0) {
                if (mode == 1) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int64_t vb = bt.vbase + r * bt.vstride + ob;
                        stu(zv + vb, cb, T(0));
                        stu(p0 + vb, cb, T(0));
                        stu(p1 + vb, cb, T(0));
                        if (xi) stu(xi + vb, cb, T(0));
                    }
                }
                continue;
            }
            const int c = L.lc[v], rr = L.lr[v];
            // neighbour order -x, +x, -y, +y, -z, +z (T4: then -t, +t; the
            // passes sum d in this order)
            constexpr int NB = T4 ? 8 : 6;
            XCell<GT, R> ct[2];
            bool hv[NB];
            hv[0] = L.gx[v] > 0;
            hv[1] = L.gx[v] + 1 < G.nx;
            hv[2] = L.gy[v] > 0;
            hv[3] = L.gy[v] + 1 < G.ny;
            hv[4] = gz > 0 && has_zp<T4>(G, gz - 1);
            hv[5] = has_zp<T4>(G, gz);
            if constexpr (T4) {
                hv[6] = gz - G.tz >= 0;
                hv[7] = gz + G.tz < G.nz;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int lt = h ? lz + G.tz : lz - G.tz;
                    const PlaneOff ot = plane_off(G, bt, lt);
                    Raw wt;
                    load_raw(ot.v, ot.b, L.colv[v], L.colb[v], wt);
                    ct[h].make((double)wt.g, wt.lb, wt.xb, L.in_vol[v] && hv[6 + h],
                               L.in_box[v] && ot.inb, sh, lab0, bt.gox + L.gx[v],
                               bt.goy + L.gy[v], bt.goz + bt.oz + lt, lmask);
                }
            }
            const int ry[6] = {rr, rr, rr - 1, rr + 1, 0, 0};
            const int rx[6] = {c - 1, c + 1, c, c, 0, 0};
            double gn[NB];
            bool dn[NB];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                gn[k] = sg[ry[k]][rx[k]];
                dn[k] = sdir[ry[k]][rx[k]] != 0;
            }
            gn[4] = cm[v].g;
            dn[4] = cm[v].dir;
            gn[5] = cp[v].g;
            dn[5] = cp[v].dir;
            if constexpr (T4) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    gn[6 + h] = ct[h].g;
                    dn[6 + h] = ct[h].dir;
                }
            }
            const double gc = cc[v].g;
            double w[NB];
            double d = 0.0;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                w[k] = hv[k] ? Weight<double>::of(gc - gn[k], wc) : 0.0;
                d += w[k];
            }
            T dT;
            if constexpr (std::is_same<T, double>::value) {
                dT = d;
            } else {
                T wT[NB];
#pragma unroll
                for (int k = 0; k < NB; ++k)
                    wT[k] = hv[k] ? Weight<T>::of((T)gc - (T)gn[k], wc) : T(0);
                dT = wT[0] + wT[1] + wT[2] + wT[3] + wT[4] + wT[5];
                if constexpr (T4) dT = dT + wT[6] + wT[7];
            }
            if (!(d > 0.0)) acc[4 * R] += 1.0;
            if (!isfinite(d)) acc[4 * R + 1] += 1.0;
            const T dinv = T(1) / dT;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!(lmask & (1 << r))) continue;  // uniform over the block
                const int64_t vb = bt.vbase + r * bt.vstride + ob;
                double xn[NB];
#pragma unroll
                for (int k = 0; k < 4; ++k) xn[k] = sx[r][ry[k]][rx[k]];
                xn[4] = cm[v].xt[r];
                xn[5] = cp[v].xt[r];
                if constexpr (T4) {
                    xn[6] = ct[0].xt[r];
                    xn[7] = ct[1].xt[r];
                }
                const double xc = cc[v].xt[r];
                double b = rhs ? ldu(rhs + vb, cb) : 0.0;
                double res = b;
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    if (!hv[k]) continue;
                    if (dn[k]) b += w[k] * xn[k];
                    res += w[k] * (xn[k] - xc);
                }
                const T rT = (T)res;
                const T zval = dinv * rT;
                acc[4 * r + 0] += (double)rT * (double)zval;
                acc[4 * r + 1] += (double)rT * (double)rT;
                acc[4 * r + 2] += res * res;
                acc[4 * r + 3] += b * b;
                if (mode == 1) {
                    stu(zv + vb, cb, zval);
                    stu(p0 + vb, cb, T(0));
                    stu(p1 + vb, cb, T(0));
                    if (xi) stu(xi + vb, cb, T(0));
                } else if (mode == 2 && (wmask & (1 << r))) {
                    stu(zv + vb, cb, zval);
                }
            }
        }
        // carry planes lz, lz+1 and the loads in flight
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            cm[v] = cc[v];
            cc[v] = cp[v];
            lbc[v] = lbp[v];
            own1[v] = own2[v];
        }
        hx0 = hx1;
#pragma unroll
        for (int j = 0; j < NYH; ++j)
#pragma unroll
            for (int h = 0; h < HV; ++h) hy0[j][h] = hy1[j][h];
    }
    return true;
}

template <typename V, typename T, int R, int BY, int VX, typename TS, bool YM = false,
          bool T4 = false>
__global__ __launch_bounds__(64 * BY) void k_residual(
    const V* __restrict__ volp, const uint8_t* __restrict__ labp, WCoef wc, TS ts,
    Shell sh, int lab0, const double* __restrict__ x64, const double* __restrict__ rhs,
    T* __restrict__ zv, T* __restrict__ p0, T* __restrict__ p1, T* __restrict__ xi, int mode,
    const RhsState* __restrict__ st, double* __restrict__ part) {
    constexpr int NQ = 4 * R + 2;
    constexpr bool SHX = std::is_same<TS, BrickTiles>::value;  // bricks: shell cache
    __shared__ __align__(16) char smem[ResidualSmem<V, R, BY, VX, YM, SHX>::bytes];
    const int cnt = ts.count();
    for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
        BoxTile bt;
        if (!ts.get(it, bt)) continue;
        double acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
        if (!residual_tile<V, T, R, BY, VX, YM, T4, SHX>(smem, bt, volp, labp, wc, sh, lab0, x64, rhs,
                                                    zv, p0, p1, xi, mode, st, acc))
            continue;
        block_sum_store<NQ, BY>(acc, part + bt.pidx, ts.ntiles);
    }
}

}  // namespace rw
