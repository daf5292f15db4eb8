// Tile shapes of the stencil kernels: the tuned table and its overrides.
#include <cstdlib>

#include "rw_internal.h"
#include "rw_kernels.h"

namespace rw {

static int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}

TileChoice tuned_tiles(const Geom& G, int precision, int R) {
    (void)G;
    (void)precision;
    (void)R;
    // measured on MI355X (512^3, two labels): float32 passes prefer the
    // XCD-aware tile order, float64 passes the plain one
    TileChoice c{4, 32, precision == RW_PREC_MIXED ? 1 : 0};
    c.by = env_int("RW_TILE_BY", c.by);
    c.zc = env_int("RW_TILE_ZC", c.zc);
    c.xcd = env_int("RW_TILE_XCD", c.xcd);
    if (c.by != 4 && c.by != 8) c.by = 4;
    if (c.zc < 4) c.zc = 4;
    return c;
}

}  // namespace rw
