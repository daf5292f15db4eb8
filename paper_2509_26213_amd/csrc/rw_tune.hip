// Tile shapes of the stencil kernels: the measured default, the table filled
// by the autotuner (kept in a text file next to librw.so, so later processes
// use it), and overrides.
#include <dlfcn.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
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

std::map<std::tuple<int, int, int>, TileChoice> g_brick_tuned;  // (precision, R, size class)
bool g_table_loaded = false;

// The tuning table file: RW_TUNE_FILE if set (empty: none), else librw.tune
// beside the loaded librw.so.
std::string tune_path() {
    const char* env = std::getenv("RW_TUNE_FILE");
    if (env) return std::string(env);
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&tune_path), &info) && info.dli_fname) {
        const std::string p = info.dli_fname;
        const size_t slash = p.rfind('/');
        return (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) +
               "/librw.tune";
    }
    return std::string();
}

bool valid_whole(const TileChoice& c) {
    return (c.vx == 1 || c.vx == 2 || c.vx == 4) && (c.by == 4 || (c.by == 8 && c.vx == 2)) &&
           c.zc >= 4 && c.zc <= 1024 && (c.xcd == 0 || c.xcd == 1);
}

bool valid_brick(const TileChoice& c) {
    return (c.vx == 1 || c.vx == 2) && (c.by == 4 || c.by == 8 || (c.by == 16 && c.vx == 1)) &&
           c.zc >= 4 && c.zc <= 1024 && (c.brick_xcd == 0 || c.brick_xcd == 1) &&
           (c.persist == 0 || (c.persist == 1 && c.vx == 2 && c.by != 16));
}

// Lines "whole|brick precision R class by zc xcd vx brick_xcd persist";
// '#' starts a comment; malformed or invalid lines are skipped.  Called with
// g_tune_mu held; reads the file once per process.
void load_table_locked() {
    if (g_table_loaded) return;
    g_table_loaded = true;
    const std::string path = tune_path();
    if (path.empty()) return;
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof(line), f)) {
        if (line[0] == '#') continue;
        char kind[16];
        int prec, R, cls;
        TileChoice c{4, 32, 0, 1};
        if (std::sscanf(line, "%15s %d %d %d %d %d %d %d %d %d", kind, &prec, &R, &cls, &c.by,
                        &c.zc, &c.xcd, &c.vx, &c.brick_xcd, &c.persist) != 10)
            continue;
        if ((prec != RW_PREC_FP64 && prec != RW_PREC_MIXED) || R < 1 || R > 4 || cls < 0 ||
            cls > 62)
            continue;
        c.tuned = 1;
        const auto key = std::make_tuple(prec, R, cls);
        if (!std::strcmp(kind, "whole") && valid_whole(c)) g_tuned[key] = c;
        if (!std::strcmp(kind, "brick") && valid_brick(c)) g_brick_tuned[key] = c;
    }
    std::fclose(f);
}

// Rewrite the file with the whole table (called with g_tune_mu held after a
// tuner run); failures to write leave the in-process table in place.
void save_table_locked() {
    const std::string path = tune_path();
    if (path.empty()) return;
    const std::string tmp = path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "# librw tile table, written by rw_autotune / rw_autotune_bricks\n");
    std::fprintf(f, "# kind precision(0 fp64, 1 mixed) solved_labels size_class(floor log2 "
                    "voxels) by zc xcd vx brick_xcd persist\n");
    for (const auto& kv : g_tuned)
        std::fprintf(f, "whole %d %d %d %d %d %d %d %d %d\n", std::get<0>(kv.first),
                     std::get<1>(kv.first), std::get<2>(kv.first), kv.second.by, kv.second.zc,
                     kv.second.xcd, kv.second.vx, kv.second.brick_xcd, kv.second.persist);
    for (const auto& kv : g_brick_tuned)
        std::fprintf(f, "brick %d %d %d %d %d %d %d %d %d\n", std::get<0>(kv.first),
                     std::get<1>(kv.first), std::get<2>(kv.first), kv.second.by, kv.second.zc,
                     kv.second.xcd, kv.second.vx, kv.second.brick_xcd, kv.second.persist);
    const bool ok = std::fclose(f) == 0;
    if (ok) std::rename(tmp.c_str(), path.c_str());
    else std::remove(tmp.c_str());
}

bool env_set(const char* name) {
    const char* v = std::getenv(name);
    return v && *v;
}

}  // namespace

void load_tuning() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_table_locked();
}

// Precedence: a shape forced by the autotuner while it times candidates,
// then RW_TILE_* overrides, then the autotuner's table, then the measured
// default.
TileChoice tuned_tiles(const Geom& G, int precision, int R) {
    if (g_forced) return g_force;
    TileChoice c{4, 32, 0, 2};
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_table_locked();
        auto it = g_tuned.find(std::make_tuple(precision, R, size_class(G)));
        if (it != g_tuned.end()) {
            c = it->second;
            have = true;
        }
    }
    if (!have && precision == RW_PREC_MIXED) {
        // measured on MI355X: two columns per lane (128-wide tiles) beat one and
        // four in both precisions.  Float32 passes of two labels run fastest on
        // 128 x 8 x 64 tiles (8 waves; 2 % over 128 x 4 x 32 on 512^3, whose
        // y-halo rows, half of the tile again, all miss L2) when the volume holds
        // at least 1024 of them; with three or more labels the passes fit three
        // or fewer waves per SIMD, so an 8-wave tile leaves a slot idle (three
        // labels on 512 x 512 x 256: 4 % slower) and 128 x 4 x 32 in XCD-aware
        // order stays.  Float64 passes: 128 x 4 x 32 in plain order (128 x 8
        // loses 6-10 %).
        const int64_t tall = int64_t((G.nx + 127) / 128) * ((G.ny + 7) / 8) * ((G.nz + 63) / 64);
        c = R == 2 && tall >= 1024 ? TileChoice{8, 64, 0, 2} : TileChoice{4, 32, 1, 2};
        // pass 2 reads two fields through the stencil where pass 1 reads
        // three, and runs fastest on 128 x 4 x 32 tiles (512^3, two labels:
        // 1113 us per launch against 1156 us on pass 1's 128 x 8 x 64; pass
        // 1 loses 7 % on 4-row tiles)
        if (c.by == 8) {
            c.by2 = 4;
            c.zc2 = 32;
        }
    }
    if (env_set("RW_TILE_VX") || env_set("RW_TILE_ZC") || env_set("RW_TILE_XCD") ||
        env_set("RW_TILE_BY")) {
        c.vx = env_int("RW_TILE_VX", c.vx);
        c.zc = env_int("RW_TILE_ZC", c.zc);
        c.xcd = env_int("RW_TILE_XCD", c.xcd);
        c.by = env_int("RW_TILE_BY", c.by);
        c.by2 = c.zc2 = 0;
        c.tuned = 0;
    }
    if (env_set("RW_TILE_BY2")) c.by2 = env_int("RW_TILE_BY2", c.by);
    if (env_set("RW_TILE_ZC2")) c.zc2 = env_int("RW_TILE_ZC2", c.zc);
    if (c.zc < 4) c.zc = 4;
    c.series = env_set("RW_SERIES_PLAIN") ? 0 : 1;
    return c;
}

namespace {

thread_local bool g_brick_forced = false;
thread_local TileChoice g_brick_force{8, 64, 0, 2};

int brick_class(int64_t max_vox) {
    return max_vox > 0 ? int(std::floor(std::log2(double(max_vox)))) : 0;
}

}  // namespace

// Precedence as for tuned_tiles: a candidate forced by the autotuner, then
// RW_BRICK_* overrides, then the autotuner's table, then the default.
TileChoice brick_tiles(int precision, int R, int64_t max_brick_vox) {
    if (g_brick_forced) return g_brick_force;
    const bool env = env_set("RW_BRICK_BY") || env_set("RW_BRICK_VX") || env_set("RW_BRICK_ZC") ||
                     env_set("RW_BRICK_XCD") || env_set("RW_BRICK_PERSIST");
    if (!env) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_table_locked();
        auto it = g_brick_tuned.find(std::make_tuple(precision, R, brick_class(max_brick_vox)));
        if (it != g_brick_tuned.end()) return it->second;
    }
    // measured on MI355X (4850 uneven 64^3 bricks of a 1024^3 uint16 volume,
    // mixed, two labels): 64 x 16 column tiles of a whole brick depth, 8
    // waves with two rows per lane, beat 64 x 8 (one row per lane) by 4 % and
    // 64 x 4 x 32 by 11 %; 64 x 16 with one row per lane loses occupancy; the
    // XCD-aware worklist order loses.  With three or more labels the passes
    // fit three waves per SIMD, so 8-wave blocks leave a slot idle: 64 x 8
    // tiles of 4 waves (two rows per lane) are 1.7 % faster (2048 128^3
    // bricks, three labels)
    TileChoice c{R >= 3 ? 4 : 8, 64, 0, 2};
    c.by = env_int("RW_BRICK_BY", c.by);
    c.vx = env_int("RW_BRICK_VX", c.vx) == 2 ? 2 : 1;  // rows per lane
    c.zc = env_int("RW_BRICK_ZC", c.zc);
    c.brick_xcd = env_int("RW_BRICK_XCD", 0) ? 1 : 0;
    c.persist = env_int("RW_BRICK_PERSIST", c.persist) ? 1 : 0;
    if (c.by != 4 && c.by != 8 && c.by != 16) c.by = 8;
    if (c.vx == 2 && c.by == 16) c.by = 8;
    if (c.zc < 4) c.zc = 4;
    return c;
}

const std::vector<TileChoice>& brick_candidates() {
    static const std::vector<TileChoice> cands = [] {
        std::vector<TileChoice> v;
        const int shapes[][2] = {{8, 2}, {4, 2}, {16, 1}, {8, 1}, {4, 1}};  // (by, rows per lane)
        for (const auto& sh : shapes)
            for (int zc : {16, 32, 64})
                for (int xcd : {0, 1}) {
                    TileChoice c{sh[0], zc, 0, sh[1]};
                    c.brick_xcd = xcd;
                    v.push_back(c);
                }
        return v;
    }();
    return cands;
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
        load_table_locked();
        win.tuned = 1;
        g_tuned[std::make_tuple(opts->precision, R, size_class(G))] = win;
        save_table_locked();
    }
    if (best) {
        best[0] = win.vx;
        best[1] = win.zc;
        best[2] = win.xcd;
        best[3] = win.by;
    }
    return RW_OK;
}

rw_status rw_autotune_bricks(rw_context* ctx, const rw_volume* fine, const rw_seeds* seeds,
                             const void* coarse_prob, int32_t coarse_dtype, rw_dims coarse_dims,
                             int32_t factor, const rw_brick* bricks, const rw_subvolume* subvols,
                             int32_t n_bricks, const rw_options* opts, float* prob_scratch,
                             void* ws, size_t ws_bytes, int32_t* best, void* stream) {
    if (!ctx || !seeds || !opts || !prob_scratch) return invalid("NULL argument");
    if (n_bricks <= 0 || !bricks) return invalid("no bricks to tune on");
    const int K = seeds->num_labels;
    const int R = std::max(1, std::min(4, opts->solve_all_labels ? K : K - 1));
    int64_t max_vox = 0;
    for (int i = 0; i < n_bricks; ++i)
        max_vox = std::max<int64_t>(max_vox, (int64_t)bricks[i].sx * bricks[i].sy * bricks[i].sz);
    if (opts->brick_voxels > 0) max_vox = opts->brick_voxels;
    rw_options o = *opts;
    o.kernel_timing = 1;
    o.max_iter = std::max(2, o.check_interval) * 2;
    double best_t = INFINITY;
    TileChoice win = brick_tiles(opts->precision, R, max_vox);
    for (const TileChoice& cand : brick_candidates()) {
        g_brick_forced = true;
        g_brick_force = cand;
        rw_stats st;
        memset(&st, 0, sizeof(st));
        // every candidate writes the scratch output
        rw_status e = rw_solve_bricks(ctx, fine, seeds, coarse_prob, coarse_dtype, coarse_dims,
                                      factor, bricks, subvols, n_bricks, &o, prob_scratch, nullptr,
                                      ws, ws_bytes, &st, stream);
        g_brick_forced = false;
        if (e < 0) return e;
        if (st.rhs_voxel_iterations <= 0) continue;
        const double t = (st.pass_ms[0] + st.pass_ms[1]) / double(st.rhs_voxel_iterations);
        if (t < best_t) {
            best_t = t;
            win = cand;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_table_locked();
        win.tuned = 1;
        g_brick_tuned[std::make_tuple(opts->precision, R, brick_class(max_vox))] = win;
        save_table_locked();
    }
    if (best) {
        best[0] = win.by;
        best[1] = win.vx;
        best[2] = win.zc;
        best[3] = win.brick_xcd;
    }
    return RW_OK;
}

}  // extern "C"
