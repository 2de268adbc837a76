// Brute-force check of df_neighbour (paper_2303_08163_amd/csrc/tile_deps.hpp):
// for many slot geometries, every tile that owns a node of a two-step tile's
// read footprint (its nodes and two columns and rows around them, periodic)
// is among that tile's polled candidates, and every candidate is a tile of the
// slot.  The dependency is symmetric, so this also covers the tiles that read
// what the tile overwrites.  Prints "ok <cases>" or the first failure.
#include <cstdio>
#include <cstdlib>
#include <set>

#include "tile_deps.hpp"

using lbm::df_neighbour;

static int check(int nx, int ny, int w, int rr, int tx, int rows) {
    const int tiles_x = w > 0 ? 1 : (nx + tx - 1) / tx;
    const int tiles_y = w > 0 ? (ny + rr - 1) / rr : (ny + rows - 1) / rows;
    const int tiles = tiles_x * tiles_y;
    auto owner = [&](int x, int y) { return w > 0 ? y / rr : (y / rows) * tiles_x + x / tx; };
    for (int tt = 0; tt < tiles; ++tt) {
        std::set<int> cand;
        for (int l = 0; l < 64; ++l) {
            const int c = df_neighbour(l, nx, ny, w, rr, tx, rows, tt);
            if (c < -1 || c >= tiles) {
                std::printf("candidate %d out of range: nx %d ny %d w %d rr %d tx %d rows %d tile %d\n", c, nx, ny, w,
                            rr, tx, rows, tt);
                return 1;
            }
            if (c >= 0)
                cand.insert(c);
        }
        int x0, x1, y0, y1;
        if (w > 0) {
            x0 = 0;
            x1 = nx;
            y0 = tt * rr;
            y1 = y0 + rr < ny ? y0 + rr : ny;
        } else {
            x0 = (tt % tiles_x) * tx;
            x1 = x0 + tx < nx ? x0 + tx : nx;
            y0 = (tt / tiles_x) * rows;
            y1 = y0 + rows < ny ? y0 + rows : ny;
        }
        for (int y = y0 - 2; y < y1 + 2; ++y)
            for (int x = x0 - 2; x < x1 + 2; ++x) {
                const int o = owner(lbm::df_wrap(x, nx), lbm::df_wrap(y, ny));
                if (!cand.count(o)) {
                    std::printf("missing dependency: nx %d ny %d w %d rr %d tx %d rows %d tile %d node (%d, %d) owner %d\n",
                                nx, ny, w, rr, tx, rows, tt, x, y, o);
                    return 1;
                }
            }
    }
    return 0;
}

int main() {
    std::srand(2303);
    long cases = 0;
    // whole-row tiles: row width w (64 m) >= nx, rr = sub-tiles x rows
    for (int n = 0; n < 3000; ++n) {
        const int block = n % 2 ? 1024 : 512;  // two-step launches, tile-ordered form
        const int w = 64 * (1 + std::rand() % (block / 64));
        const int nx = 1 + std::rand() % w;
        const int ny = 1 + std::rand() % 300;
        const int sub = block / w;
        const int R = 1 + std::rand() % 40;
        if (check(nx, ny, w, sub * R, 0, 0))
            return 1;
        ++cases;
    }
    // column tiles of tx x rows (the last ones partial), small grids included; tiles
    // of 1 .. 3 columns make every candidate column matter
    const int txs[7] = {128, 512, 1024, 64, 1, 2, 3};
    for (int n = 0; n < 3000; ++n) {
        const int tx = txs[std::rand() % 7];
        const int nx = 1 + std::rand() % (n < 1500 ? 3 * tx + 2 : 8);
        const int ny = 1 + std::rand() % (n % 2 ? 200 : 6);
        const int rows = 1 + std::rand() % 33;
        if (check(nx, ny, 0, 0, tx, rows))
            return 1;
        ++cases;
    }
    // a last tile of one or two columns, whose left neighbour across the wrap is two
    // tiles away from tile 0 (nx = k tx + 1 or + 2)
    for (int tx : {64, 128, 512, 1024})
        for (int k = 1; k <= 3; ++k)
            for (int extra = 1; extra <= 2; ++extra)
                for (int rows : {1, 2, 16})
                    for (int ny : {1, 2, 5, 40}) {
                        if (check(k * tx + extra, ny, 0, 0, tx, rows))
                            return 1;
                        ++cases;
                    }
    std::printf("ok %ld\n", cases);
    return 0;
}
