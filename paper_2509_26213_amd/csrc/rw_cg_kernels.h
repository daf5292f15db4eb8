// The 2.5D stencil kernels of the matrix-free Jacobi-PCG.
//
// A system is solved on a box of the grid: the whole volume, or one brick of
// the fine level (whose face shell then carries Dirichlet data).  A box is cut
// into tiles of 64 x BY columns by zc planes; a block of 64 x BY threads walks
// a tile's planes in batches of U.  Per batch it issues every global load
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

struct BoxTile {
    Geom G;                  // the volume the box lives in
    int64_t voff;            // offset of that volume in the intensity / label arrays
    int gox, goy, goz;       // global position of that volume's origin (coarse upsampling)
    int ox, oy, oz;          // box origin in the volume
    int sx, sy, sz;          // box size
    int X0, Y0, z0, z1;      // tile origin (box-local) and plane range [z0, z1)
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
        b.X0 = tx * 64;
        b.Y0 = ty * tm.by;
        b.z0 = tz * tm.zc;
        b.z1 = min(b.z0 + tm.zc, G.nz);
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
    __device__ __forceinline__ int count() const { return *list_count; }
    __device__ __forceinline__ bool get(int i, BoxTile& b) const {
        const int g = list[i];
        const int bi = tile_brick[g];
        const BrickGeo B = bricks[bi];
        const int t = g - B.tile0;
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
        b.X0 = tx * 64;
        b.Y0 = ty * by;
        b.z0 = tz * zc;
        b.z1 = min(b.z0 + zc, B.sz);
        b.vbase = B.voff;
        b.vstride = B.vox;
        b.sidx = bi;
        b.pidx = g;
        return true;
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

// ---------------------------------------------------------------- residual

// Float64 residual r = b - A x64 of the current iterate with float64
// weights, and the start of a CG run: z = r / d written in T (d from
// T-precision weights, the ones the passes use).  Dirichlet data of label
// lab0 + r: 1 on its seeds, 0 on other seeds (lab0 = 0: 0 on every seed),
// the upsampled coarse value on non-seed shell voxels; rhs (optional) adds an
// explicit right-hand side.  Partials per tile [4R + 2][ntiles]: per label
// r.z, r.r (in T), r64.r64, b.b; then the number of unknowns with a
// non-positive and with a non-finite degree.  mode 0 only measures; mode 1
// starts a CG run for every label (p buffers and xi zeroed); mode 2
// refreshes z of the labels flagged for it (st.outer_active == 2).
template <typename V, typename T, int R, int BY, typename TS>
__global__ __launch_bounds__(64 * BY) void k_residual(
    const V* __restrict__ volp, const uint8_t* __restrict__ labp, WCoef wc, TS ts,
    Shell sh, int lab0, const double* __restrict__ x64, const double* __restrict__ rhs,
    T* __restrict__ zv, T* __restrict__ p0, T* __restrict__ p1, T* __restrict__ xi, int mode,
    const RhsState* __restrict__ st, double* __restrict__ part) {
    constexpr int NQ = 4 * R + 2;
    const int cnt = ts.count();
    for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
        BoxTile bt;
        if (!ts.get(it, bt)) continue;
        const Geom& G = bt.G;
        const V* __restrict__ vol = volp + bt.voff;
        const uint8_t* __restrict__ lab = labp + bt.voff;
        int wmask = 0;
        if (mode == 2) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (st[bt.sidx * R + r].outer_active == 2) wmask |= 1 << r;
            if (!wmask) continue;
        }
        double acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
        const int lxb = bt.X0 + threadIdx.x, lyb = bt.Y0 + threadIdx.y;
        if (lxb < bt.sx && lyb < bt.sy) {
            const int gx = bt.ox + lxb, gy = bt.oy + lyb;
            for (int lz = bt.z0; lz < bt.z1; ++lz) {
                const int gz = bt.oz + lz;
                const int64_t c = (int64_t)gz * G.plane + (int64_t)gy * G.nx + gx;
                const int64_t cb = ((int64_t)lz * bt.sy + lyb) * bt.sx + lxb;
                const uint8_t lc = lab[c];
                if (lc != 0) {
                    if (mode == 1) {
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const int64_t o = bt.vbase + r * bt.vstride + cb;
                            zv[o] = T(0);
                            p0[o] = T(0);
                            p1[o] = T(0);
                            if (xi) xi[o] = T(0);
                        }
                    }
                    continue;
                }
                // neighbour order -x, +x, -y, +y, -z, +z (the passes sum d in this order)
                const bool hv[6] = {gx > 0, gx + 1 < G.nx, gy > 0, gy + 1 < G.ny, gz > 0,
                                    gz + 1 < G.nz};
                const int64_t nb[6] = {c - 1, c + 1, c - G.nx, c + G.nx, c - G.plane, c + G.plane};
                const int dxl[6] = {-1, 1, 0, 0, 0, 0}, dyl[6] = {0, 0, -1, 1, 0, 0},
                          dzl[6] = {0, 0, 0, 0, -1, 1};
                const double vc = (double)vol[c];
                double w[6];
                double d = 0.0;
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    w[k] = hv[k] ? Weight<double>::of(vc - (double)vol[nb[k]], wc) : 0.0;
                    d += w[k];
                }
                T dT;
                if constexpr (std::is_same<T, double>::value) {
                    dT = d;
                } else {
                    const T vcT = (T)vol[c];
                    T wT[6];
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        wT[k] = hv[k] ? Weight<T>::of(vcT - (T)vol[nb[k]], wc) : T(0);
                    dT = wT[0] + wT[1] + wT[2] + wT[3] + wT[4] + wT[5];
                }
                uint8_t ln[6];
                bool inb[6];
                int64_t nbb[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    ln[k] = hv[k] ? lab[nb[k]] : 0;
                    const int xx = lxb + dxl[k], yy = lyb + dyl[k], zz = lz + dzl[k];
                    inb[k] = xx >= 0 && xx < bt.sx && yy >= 0 && yy < bt.sy && zz >= 0 && zz < bt.sz;
                    nbb[k] = ((int64_t)zz * bt.sy + yy) * bt.sx + xx;
                }
                if (!(d > 0.0)) acc[4 * R] += 1.0;
                if (!isfinite(d)) acc[4 * R + 1] += 1.0;
                const T dinv = T(1) / dT;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int L = lab0 + r;
                    const int64_t vb = bt.vbase + r * bt.vstride;
                    const double xc = x64 ? x64[vb + cb] : 0.0;
                    double b = rhs ? rhs[vb + cb] : 0.0;
                    double res = b;
#pragma unroll
                    for (int k = 0; k < 6; ++k) {
                        if (!hv[k]) continue;
                        double xj;
                        if (ln[k] != 0) {
                            xj = (lab0 > 0 && ln[k] == L) ? 1.0 : 0.0;
                            b += w[k] * xj;
                        } else if (inb[k]) {
                            xj = x64 ? x64[vb + nbb[k]] : 0.0;
                        } else {
                            xj = (sh.coarse && lab0 > 0)
                                     ? upsample(sh, L, bt.gox + gx + dxl[k], bt.goy + gy + dyl[k],
                                                bt.goz + gz + dzl[k])
                                     : 0.0;
                            b += w[k] * xj;
                        }
                        res += w[k] * (xj - xc);
                    }
                    const T rT = (T)res;
                    const T zval = dinv * rT;
                    acc[4 * r + 0] += (double)rT * (double)zval;
                    acc[4 * r + 1] += (double)rT * (double)rT;
                    acc[4 * r + 2] += res * res;
                    acc[4 * r + 3] += b * b;
                    const int64_t o = vb + cb;
                    if (mode == 1) {
                        zv[o] = zval;
                        p0[o] = T(0);
                        p1[o] = T(0);
                        if (xi) xi[o] = T(0);
                    } else if (mode == 2 && (wmask & (1 << r))) {
                        zv[o] = zval;
                    }
                }
            }
        }
        block_sum_store<NQ, BY>(acc, part + bt.pidx, ts.ntiles);
    }
}

// ---------------------------------------------------------------- CG passes

template <int BY, int U>
struct TileLanes {
    static constexpr int NYH = (2 * U + BY - 1) / BY;  // y-halo rows per wave per batch
    int lx, ly;
    int lxb, lyb;         // own position, box-local
    int gx, gy;           // own position, global
    bool in_box, in_vol;  // own column inside the box / the volume
    int64_t colv, colb;   // clamped own column offset in the volume / in the box
    bool hx_use, hx_vol, hx_box;
    int hx_k, hx_col_lds;
    int64_t hx_colv, hx_colb;
    bool hy_use[NYH], hy_vol[NYH], hy_box[NYH];
    int hy_k[NYH], hy_row_lds[NYH];
    int64_t hy_colv[NYH], hy_colb[NYH];

    __device__ __forceinline__ void init(const Geom& G, const BoxTile& b) {
        lx = threadIdx.x;
        ly = threadIdx.y;
        lxb = b.X0 + lx;
        lyb = b.Y0 + ly;
        gx = b.ox + lxb;
        gy = b.oy + lyb;
        in_box = lxb < b.sx && lyb < b.sy;
        in_vol = gx < G.nx && gy < G.ny;
        const int cgx = min(gx, G.nx - 1), cgy = min(gy, G.ny - 1);
        const int cbx = min(lxb, b.sx - 1), cby = min(lyb, b.sy - 1);
        colv = (int64_t)cgy * G.nx + cgx;
        colb = (int64_t)cby * b.sx + cbx;
        const int side = lx & 1;
        hx_k = min(lx >> 1, U - 1);
        hx_use = lx < 2 * U;
        const int hxb = side ? b.X0 + 64 : b.X0 - 1;
        const int hgx = b.ox + hxb;
        hx_vol = hx_use && hgx >= 0 && hgx < G.nx && gy < G.ny;
        hx_box = hx_use && hxb >= 0 && hxb < b.sx && lyb < b.sy;
        hx_colv = (int64_t)cgy * G.nx + clampi(hgx, 0, G.nx - 1);
        hx_colb = (int64_t)cby * b.sx + clampi(hxb, 0, b.sx - 1);
        hx_col_lds = side ? 65 : 0;
#pragma unroll
        for (int j = 0; j < NYH; ++j) {
            const int i = ly + j * BY;
            hy_use[j] = i < 2 * U;
            const int s = i & 1;
            hy_k[j] = min(i >> 1, U - 1);
            const int yb = s ? b.Y0 + BY : b.Y0 - 1;
            const int gyh = b.oy + yb;
            hy_vol[j] = hy_use[j] && gyh >= 0 && gyh < G.ny && gx < G.nx;
            hy_box[j] = hy_use[j] && yb >= 0 && yb < b.sy && lxb < b.sx;
            hy_colv[j] = (int64_t)clampi(gyh, 0, G.ny - 1) * G.nx + cgx;
            hy_colb[j] = (int64_t)clampi(yb, 0, b.sy - 1) * b.sx + cbx;
            hy_row_lds[j] = s ? BY + 1 : 0;
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

// Pass 1: p_new = z + beta p_old (formed on the fly for the voxel and its
// neighbours; zero on seeds and outside the box), q = A p_new, partial
// p_new.q per label.  Label r reads p_old from buffer st.pcur of pb0/pb1 and
// writes p_new to the other one.  qout (optional) receives q.
template <typename V, typename T, int R, int BY, int U, typename TS>
__global__ __launch_bounds__(64 * BY) void k_cg_pass1(
    const V* __restrict__ volp, WCoef wc, TS ts, const T* __restrict__ zv,
    T* __restrict__ pb0, T* __restrict__ pb1, T* __restrict__ qout,
    const RhsState* __restrict__ st, double* __restrict__ part) {
    constexpr int NYH = TileLanes<BY, U>::NYH;
    __shared__ T sg[U][BY + 2][66];
    __shared__ T sp[R][U][BY + 2][66];
    const int cnt = ts.count();
    for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
        BoxTile bt;
        if (!ts.get(it, bt)) continue;
        bool act[R];
        int src[R];
        if (box_labels<R>(st, bt.sidx, act, src) < 0) continue;  // uniform over the block
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
        TileLanes<BY, U> L;
        L.init(G, bt);

        T Gv[U + 2], Pv[U + 2][R];  // own column: planes z-1, z, z+1 .. z+U
        {
            const PlaneOff om = plane_off(G, bt, bt.z0 - 1), oc = plane_off(G, bt, bt.z0);
            Gv[0] = (T)vol[om.v + L.colv];
            Gv[1] = (T)vol[oc.v + L.colv];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T a = zr[r][om.b + L.colb] + bet[r] * po[r][om.b + L.colb];
                Pv[0][r] = om.inb ? a : T(0);
                Pv[1][r] = zr[r][oc.b + L.colb] + bet[r] * po[r][oc.b + L.colb];
            }
        }
        T wzm = (L.in_box && bt.oz + bt.z0 > 0) ? Weight<T>::of(Gv[1] - Gv[0], wc) : T(0);
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;

        for (int zb = bt.z0; zb < bt.z1; zb += U) {
            // (1) every read of the batch
            T zN[U][R], oN[U][R];
            bool nin[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const PlaneOff o = plane_off(G, bt, zb + 1 + k);
                nin[k] = o.inb;
                Gv[k + 2] = (T)vol[o.v + L.colv];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    zN[k][r] = zr[r][o.b + L.colb];
                    oN[k][r] = po[r][o.b + L.colb];
                }
            }
            T hxg, hxz[R], hxo[R];
            {
                const PlaneOff o = plane_off(G, bt, zb + L.hx_k);
                hxg = (T)vol[o.v + L.hx_colv];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    hxz[r] = zr[r][o.b + L.hx_colb];
                    hxo[r] = po[r][o.b + L.hx_colb];
                }
            }
            T hyg[NYH], hyz[NYH][R], hyo[NYH][R];
#pragma unroll
            for (int j = 0; j < NYH; ++j) {
                const PlaneOff o = plane_off(G, bt, zb + L.hy_k[j]);
                hyg[j] = (T)vol[o.v + L.hy_colv[j]];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    hyz[j][r] = zr[r][o.b + L.hy_colb[j]];
                    hyo[j][r] = po[r][o.b + L.hy_colb[j]];
                }
            }
            // (2) the previous batch (or tile) is done with the LDS planes
            __syncthreads();
            // (3) publish planes zb..zb+U-1
#pragma unroll
            for (int k = 0; k < U; ++k) {
                if (k > 0) {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        Pv[k + 1][r] = nin[k - 1] ? zN[k - 1][r] + bet[r] * oN[k - 1][r] : T(0);
                }
                sg[k][L.ly + 1][L.lx + 1] = L.in_vol ? Gv[k + 1] : T(0);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    sp[r][k][L.ly + 1][L.lx + 1] = L.in_box ? Pv[k + 1][r] : T(0);
            }
            if (L.hx_use) {
                sg[L.hx_k][L.ly + 1][L.hx_col_lds] = L.hx_vol ? hxg : T(0);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    sp[r][L.hx_k][L.ly + 1][L.hx_col_lds] =
                        L.hx_box ? hxz[r] + bet[r] * hxo[r] : T(0);
            }
#pragma unroll
            for (int j = 0; j < NYH; ++j) {
                if (L.hy_use[j]) {
                    sg[L.hy_k[j]][L.hy_row_lds[j]][L.lx + 1] = L.hy_vol[j] ? hyg[j] : T(0);
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        sp[r][L.hy_k[j]][L.hy_row_lds[j]][L.lx + 1] =
                            L.hy_box[j] ? hyz[j][r] + bet[r] * hyo[j][r] : T(0);
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r)
                Pv[U + 1][r] = nin[U - 1] ? zN[U - 1][r] + bet[r] * oN[U - 1][r] : T(0);
            __syncthreads();
            // (4) stencil on planes zb..zb+U-1
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int lz = zb + k;
                const int gz = bt.oz + lz;
                const T gc = Gv[k + 1];
                const T wxm = L.gx > 0 ? Weight<T>::of(gc - sg[k][L.ly + 1][L.lx], wc) : T(0);
                const T wxp = L.gx + 1 < G.nx ? Weight<T>::of(gc - sg[k][L.ly + 1][L.lx + 2], wc) : T(0);
                const T wym = L.gy > 0 ? Weight<T>::of(gc - sg[k][L.ly][L.lx + 1], wc) : T(0);
                const T wyp = L.gy + 1 < G.ny ? Weight<T>::of(gc - sg[k][L.ly + 2][L.lx + 1], wc) : T(0);
                const T wzp = gz + 1 < G.nz ? Weight<T>::of(gc - Gv[k + 2], wc) : T(0);
                const T d = wxm + wxp + wym + wyp + wzm + wzp;
                const bool valid = L.in_box && lz < bt.z1;
                const int64_t ob = (int64_t)lz * bt.sx * bt.sy + L.colb;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const T pc = Pv[k + 1][r];
                    const T q = d * pc - (wxm * sp[r][k][L.ly + 1][L.lx] + wxp * sp[r][k][L.ly + 1][L.lx + 2] +
                                          wym * sp[r][k][L.ly][L.lx + 1] + wyp * sp[r][k][L.ly + 2][L.lx + 1] +
                                          wzm * Pv[k][r] + wzp * Pv[k + 2][r]);
                    if (valid && act[r]) {
                        pw[r][ob] = pc;
                        if (qout) qout[bt.vbase + r * bt.vstride + ob] = q;
                        acc[r] += (double)pc * (double)q;
                    }
                }
                wzm = wzp;
            }
            // (5) carry planes zb+U-1 and zb+U
            Gv[0] = Gv[U];
            Gv[1] = Gv[U + 1];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                Pv[0][r] = Pv[U][r];
                Pv[1][r] = Pv[U + 1][r];
            }
        }
        block_sum_store<R, BY>(acc, part + bt.pidx, ts.ntiles);
    }
}

// Pass 2: q = A p (p = buffer st.pcur, just written by pass 1); on unknowns
// x += alpha p, r = d z - alpha q, z = r / d; partials r.z and r.r per label
// ([2R][ntiles]).
template <typename V, typename T, int R, int BY, int U, typename TS>
__global__ __launch_bounds__(64 * BY) void k_cg_pass2(
    const V* __restrict__ volp, const uint8_t* __restrict__ labp, WCoef wc, TS ts,
    T* __restrict__ xv, T* __restrict__ zv, const T* __restrict__ pb0,
    const T* __restrict__ pb1, const RhsState* __restrict__ st, double* __restrict__ part) {
    constexpr int NYH = TileLanes<BY, U>::NYH;
    __shared__ T sg[U][BY + 2][66];
    __shared__ T sp[R][U][BY + 2][66];
    const int cnt = ts.count();
    for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
        BoxTile bt;
        if (!ts.get(it, bt)) continue;
        bool act[R];
        int src[R];
        if (box_labels<R>(st, bt.sidx, act, src) < 0) continue;
        const Geom& G = bt.G;
        const V* __restrict__ vol = volp + bt.voff;
        const uint8_t* __restrict__ lab = labp + bt.voff;
        T alp[R];
        const T* pr[R];
        const T* xr[R];
        const T* zr[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            alp[r] = (T)st[bt.sidx * R + r].alpha;
            const int64_t vb = bt.vbase + src[r] * bt.vstride;
            pr[r] = (st[bt.sidx * R + src[r]].pcur ? pb1 : pb0) + vb;
            xr[r] = xv + vb;
            zr[r] = zv + vb;
        }
        TileLanes<BY, U> L;
        L.init(G, bt);

        T Gv[U + 2], Pv[U + 2][R];
        {
            const PlaneOff om = plane_off(G, bt, bt.z0 - 1), oc = plane_off(G, bt, bt.z0);
            Gv[0] = (T)vol[om.v + L.colv];
            Gv[1] = (T)vol[oc.v + L.colv];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T a = pr[r][om.b + L.colb];
                Pv[0][r] = om.inb ? a : T(0);
                Pv[1][r] = pr[r][oc.b + L.colb];
            }
        }
        T wzm = (L.in_box && bt.oz + bt.z0 > 0) ? Weight<T>::of(Gv[1] - Gv[0], wc) : T(0);
        double acc[2 * R];
#pragma unroll
        for (int q = 0; q < 2 * R; ++q) acc[q] = 0.0;

        for (int zb = bt.z0; zb < bt.z1; zb += U) {
            T Xv[U][R], Zv[U][R];
            uint8_t Lv[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const PlaneOff o = plane_off(G, bt, zb + 1 + k);
                Gv[k + 2] = (T)vol[o.v + L.colv];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const T a = pr[r][o.b + L.colb];
                    Pv[k + 2][r] = o.inb ? a : T(0);
                }
                const PlaneOff oc = plane_off(G, bt, zb + k);
                Lv[k] = lab[oc.v + L.colv];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    Xv[k][r] = xr[r][oc.b + L.colb];
                    Zv[k][r] = zr[r][oc.b + L.colb];
                }
            }
            T hxg, hxp[R];
            {
                const PlaneOff o = plane_off(G, bt, zb + L.hx_k);
                hxg = (T)vol[o.v + L.hx_colv];
#pragma unroll
                for (int r = 0; r < R; ++r) hxp[r] = pr[r][o.b + L.hx_colb];
            }
            T hyg[NYH], hyp[NYH][R];
#pragma unroll
            for (int j = 0; j < NYH; ++j) {
                const PlaneOff o = plane_off(G, bt, zb + L.hy_k[j]);
                hyg[j] = (T)vol[o.v + L.hy_colv[j]];
#pragma unroll
                for (int r = 0; r < R; ++r) hyp[j][r] = pr[r][o.b + L.hy_colb[j]];
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < U; ++k) {
                sg[k][L.ly + 1][L.lx + 1] = L.in_vol ? Gv[k + 1] : T(0);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    sp[r][k][L.ly + 1][L.lx + 1] = L.in_box ? Pv[k + 1][r] : T(0);
            }
            if (L.hx_use) {
                sg[L.hx_k][L.ly + 1][L.hx_col_lds] = L.hx_vol ? hxg : T(0);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    sp[r][L.hx_k][L.ly + 1][L.hx_col_lds] = L.hx_box ? hxp[r] : T(0);
            }
#pragma unroll
            for (int j = 0; j < NYH; ++j) {
                if (L.hy_use[j]) {
                    sg[L.hy_k[j]][L.hy_row_lds[j]][L.lx + 1] = L.hy_vol[j] ? hyg[j] : T(0);
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        sp[r][L.hy_k[j]][L.hy_row_lds[j]][L.lx + 1] = L.hy_box[j] ? hyp[j][r] : T(0);
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int lz = zb + k;
                const int gz = bt.oz + lz;
                const T gc = Gv[k + 1];
                const T wxm = L.gx > 0 ? Weight<T>::of(gc - sg[k][L.ly + 1][L.lx], wc) : T(0);
                const T wxp = L.gx + 1 < G.nx ? Weight<T>::of(gc - sg[k][L.ly + 1][L.lx + 2], wc) : T(0);
                const T wym = L.gy > 0 ? Weight<T>::of(gc - sg[k][L.ly][L.lx + 1], wc) : T(0);
                const T wyp = L.gy + 1 < G.ny ? Weight<T>::of(gc - sg[k][L.ly + 2][L.lx + 1], wc) : T(0);
                const T wzp = gz + 1 < G.nz ? Weight<T>::of(gc - Gv[k + 2], wc) : T(0);
                const T d = wxm + wxp + wym + wyp + wzm + wzp;
                const T dinv = T(1) / d;
                const bool valid = L.in_box && lz < bt.z1 && Lv[k] == 0;
                const int64_t ob = (int64_t)lz * bt.sx * bt.sy + L.colb;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const T pc = Pv[k + 1][r];
                    const T q = d * pc - (wxm * sp[r][k][L.ly + 1][L.lx] + wxp * sp[r][k][L.ly + 1][L.lx + 2] +
                                          wym * sp[r][k][L.ly][L.lx + 1] + wyp * sp[r][k][L.ly + 2][L.lx + 1] +
                                          wzm * Pv[k][r] + wzp * Pv[k + 2][r]);
                    const T xn = Xv[k][r] + alp[r] * pc;
                    const T rres = d * Zv[k][r] - alp[r] * q;
                    const T zn = dinv * rres;
                    if (valid && act[r]) {
                        const int64_t o = bt.vbase + r * bt.vstride + ob;
                        xv[o] = xn;
                        zv[o] = zn;
                        acc[2 * r] += (double)rres * (double)zn;
                        acc[2 * r + 1] += (double)rres * (double)rres;
                    }
                }
                wzm = wzp;
            }
            Gv[0] = Gv[U];
            Gv[1] = Gv[U + 1];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                Pv[0][r] = Pv[U][r];
                Pv[1][r] = Pv[U + 1][r];
            }
        }
        block_sum_store<2 * R, BY>(acc, part + bt.pidx, ts.ntiles);
    }
}

}  // namespace rw
