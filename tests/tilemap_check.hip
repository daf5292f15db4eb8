// Host-side check of the stencil kernels' tile orders (compiled by
// tests/test_tilemap_host.py): every block slot maps to a distinct tile, the
// tiles cover every plane of every column once, and the time-series order
// keeps each chunk inside one time step.
#include <cstdio>
#include <vector>
#include "rw_kernels.h"
using namespace rw;
int main() {
    int bad = 0, cases = 0;
    for (int nx : {5, 70, 128, 224, 300})
    for (int ny : {3, 11, 224})
    for (int nzs : {1, 3, 9, 50, 64, 65, 130, 200})
    for (int nt : {2, 3, 7, 20})
    for (int by : {4, 8})
    for (int vx : {1, 2, 4}) {
        Geom G{};
        G.nx = nx; G.ny = ny; G.nz = nt * nzs;
        G.plane = (int64_t)nx * ny; G.n = G.plane * G.nz;
        const int maxt = make_tilemap(G, 4, 4, 0).tiles;
        // the plain volume order, both tile orders, two plane counts
        for (int zc : {4, 32})
        for (int xcd : {0, 1}) {
            const TileMap p = make_tilemap(G, by, zc, xcd, vx);
            std::vector<int> seen(p.tiles, 0);
            std::vector<int> cover((size_t)G.nz * p.gx * p.gy, 0);
            for (int b = 0; b < p.blocks(); ++b) {
                const int t = p.tile(b);
                if (t < 0) continue;
                if (t >= p.tiles) { ++bad; continue; }
                seen[t]++;
                const int tx = t % p.gx, ty = (t / p.gx) % p.gy, tz = t / (p.gx * p.gy);
                int z0, z1;
                p.planes(tz, G.nz, z0, z1);
                for (int z = z0; z < z1; ++z) cover[((size_t)z * p.gy + ty) * p.gx + tx]++;
            }
            for (int v : seen) if (v != 1) ++bad;
            for (int v : cover) if (v != 1) ++bad;
            ++cases;
        }
        TileMap m;
        if (!make_tilemap_series(G, by, vx, nt, nzs, maxt, m)) continue;
        ++cases;
        std::vector<int> seen(m.tiles, 0);
        std::vector<int> cover((size_t)G.nz * m.gx * m.gy, 0);
        for (int b = 0; b < m.blocks(); ++b) {
            const int t = m.tile(b);
            if (t < 0) continue;
            if (t >= m.tiles) { ++bad; continue; }
            seen[t]++;
            const int tx = t % m.gx, ty = (t / m.gx) % m.gy, tz = t / (m.gx * m.gy);
            int z0, z1;
            m.planes(tz, G.nz, z0, z1);
            if (z0 < 0 || z1 > G.nz || z0 >= z1) { ++bad; continue; }
            if (z0 / nzs != (z1 - 1) / nzs) ++bad;  // straddles a step
            if (z1 - z0 > m.zc) ++bad;
            for (int z = z0; z < z1; ++z) cover[((size_t)z * m.gy + ty) * m.gx + tx]++;
        }
        for (int v : seen) if (v != 1) ++bad;
        for (int v : cover) if (v != 1) ++bad;
    }
    printf("cases %d bad %d\n", cases, bad);
    return bad != 0;
}
