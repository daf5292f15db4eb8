// Tile shapes of the stencil kernels: the measured default, the table filled
// by the autotuner, and overrides.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "rw_internal.h"
#include "rw_kernels.h"

namespace rw {

namespace {

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, TileChoice> g_tuned;  // (precision, R, size class)
thread_local bool g_forced = false;
thread_local TileChoice g_force{4, 32, 0, 1};

int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}

int size_class(const Geom& G) {
    return G.n > 0 ? int(std::floor(std::log2(double(G.n)))) : 0;
}

}  // namespace

TileChoice tuned_tiles(const Geom& G, int precision, int R) {
    if (g_forced) return g_force;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(std::make_tuple(precision, R, size_class(G)));
        if (it != g_tuned.end()) return it->second;
    }
    // measured on MI355X: two columns per lane (128-wide tiles) beat one and
    // four in both precisions.  Float32 passes of two labels run fastest on
    // 128 x 8 x 64 tiles (8 waves; 2 % over 128 x 4 x 32 on 512^3, whose
    // y-halo rows, half of the tile again, all miss L2) when the volume holds
    // at least 1024 of them; with three or more labels the passes fit three
    // or fewer waves per SIMD, so an 8-wave tile leaves a slot idle (three
    // labels on 512 x 512 x 256: 4 % slower) and 128 x 4 x 32 in XCD-aware
    // order stays.  Float64 passes: 128 x 4 x 32 in plain order (128 x 8
    // loses 6-10 %).
    TileChoice c{4, 32, 0, 2};
    if (precision == RW_PREC_MIXED) {
        const int64_t tall = int64_t((G.nx + 127) / 128) * ((G.ny + 7) / 8) * ((G.nz + 63) / 64);
        c = R == 2 && tall >= 1024 ? TileChoice{8, 64, 0, 2} : TileChoice{4, 32, 1, 2};
    }
    c.vx = env_int("RW_TILE_VX", c.vx);
    c.zc = env_int("RW_TILE_ZC", c.zc);
    c.xcd = env_int("RW_TILE_XCD", c.xcd);
    c.by = env_int("RW_TILE_BY", c.by);
    if (c.zc < 4) c.zc = 4;
    return c;
}

TileChoice brick_tiles(int precision) {
    (void)precision;
    // measured on MI355X (4850 uneven 64^3 bricks of a 1024^3 uint16 volume,
    // mixed): 64 x 16 column tiles of a whole brick depth, 8 waves with two
    // rows per lane, beat 64 x 8 (one row per lane) by 4 % and 64 x 4 x 32 by
    // 11 %; 64 x 16 with one row per lane loses occupancy; the XCD-aware
    // worklist order loses
    TileChoice c{8, 64, 0, 2};
    c.by = env_int("RW_BRICK_BY", c.by);
    c.vx = env_int("RW_BRICK_VX", c.vx) == 2 ? 2 : 1;  // rows per lane
    c.zc = env_int("RW_BRICK_ZC", c.zc);
    c.brick_xcd = env_int("RW_BRICK_XCD", 0) ? 1 : 0;
    if (c.by != 4 && c.by != 8 && c.by != 16) c.by = 8;
    if (c.vx == 2 && c.by == 16) c.by = 8;
    if (c.zc < 4) c.zc = 4;
    return c;
}

}  // namespace rw

using namespace rw;

extern "C" {

rw_status rw_autotune(rw_context* ctx, const rw_volume* vol, const rw_seeds* seeds,
                      const rw_options* opts, void* prob_scratch, void* ws, size_t ws_bytes,
                      int32_t* best, void* stream) {
    if (!ctx || !vol || !seeds || !opts || !prob_scratch) return invalid("NULL argument");
    rw_status e = check_volume(vol);
    if (e) return e;
    const Geom G = make_geom(vol->dims);
    const int K = seeds->num_labels;
    const int R = std::max(1, std::min(4, opts->solve_all_labels ? K : K - 1));
    static const int vxs[] = {1, 2, 4};
    static const int bys[] = {4, 8};
    static const int zcs[] = {16, 32, 64};
    static const int xcds[] = {0, 1};
    rw_options o = *opts;
    o.kernel_timing = 1;
    o.use_graph = 0;
    o.max_iter = std::max(2, o.check_interval) * 2;
    o.x0 = nullptr;
    double best_t = INFINITY;
    TileChoice win = tuned_tiles(G, opts->precision, R);
    for (int vx : vxs)
        for (int by : bys)
            for (int zc : zcs)
                for (int xcd : xcds) {
                    if (vx == 4 && opts->precision != RW_PREC_MIXED) continue;
                    if (by != 4 && vx != 2) continue;
                    const TileChoice cand{by, zc, xcd, vx};
                    g_forced = true;
                    g_force = cand;
                    rw_stats st;
                    memset(&st, 0, sizeof(st));
                    // every candidate writes the scratch output
                    e = rw_solve(ctx, vol, seeds, &o, prob_scratch, nullptr, ws, ws_bytes, &st,
                                 stream);
                    g_forced = false;
                    if (e < 0) return e;
                    const int64_t l = st.pass_launches[0] + st.pass_launches[1];
                    if (l <= 0) continue;
                    const double t = (st.pass_ms[0] + st.pass_ms[1]) / double(l);
                    if (t < best_t) {
                        best_t = t;
                        win = cand;
                    }
                }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[std::make_tuple(opts->precision, R, size_class(G))] = win;
    }
    if (best) {
        best[0] = win.vx;
        best[1] = win.zc;
        best[2] = win.xcd;
        best[3] = win.by;
    }
    return RW_OK;
}

}  // extern "C"
