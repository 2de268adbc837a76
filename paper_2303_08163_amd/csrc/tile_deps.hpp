// tile_deps.hpp -- the two-step tiles that one tile's iteration depends on, in
// the tile-ordered persistent pool form (k_pool_df2).  Plain C++: the
// functions are constexpr, so device code calls them and a host program
// checks them against a brute-force footprint.
//
// Iteration k of a two-step tile reads the previous state at its own nodes and
// at the nodes up to two columns and two rows around them (periodic wrap), and
// writes its own nodes only.  The tiles it depends on are therefore those that
// own a node of that dilated box; since tiles are rectangles on a regular grid,
// those are the tiles holding the box's rows y0 - 2, y0 - 1, y0 (the tile's
// own), y1, y1 + 1 crossed with its columns x0 - 2, x0 - 1, x0, x0 + nv,
// x0 + nv + 1 -- 25 candidates, 5 for whole-row tiles (some repeated when the
// slot has few tiles).
#pragma once

namespace lbm {

constexpr int df_wrap(int c, int n) { return ((c % n) + n) % n; }

// Candidate l of two-step tile tt of a slot of nx x ny nodes: whole-row tiles of
// rr rows when w > 0 (l < 5), else column tiles of tx columns x rows rows
// (l < 25, x index l % 5, y index l / 5).  -1 when l names no candidate.
constexpr int df_neighbour(int l, int nx, int ny, int w, int rr, int tx, int rows, int tt) {
    if (w > 0) {
        if (l < 0 || l >= 5)
            return -1;
        const int y0 = tt * rr, y1 = y0 + rr < ny ? y0 + rr : ny;
        const int ry[5] = {y0 - 2, y0 - 1, y0, y1, y1 + 1};
        return df_wrap(ry[l], ny) / rr;
    }
    if (l < 0 || l >= 25)
        return -1;
    const int tiles_x = (nx + tx - 1) / tx;
    const int x0 = (tt % tiles_x) * tx, nv = tx < nx - x0 ? tx : nx - x0;
    const int y0 = (tt / tiles_x) * rows, y1 = y0 + rows < ny ? y0 + rows : ny;
    const int cx[5] = {x0 - 2, x0 - 1, x0, x0 + nv, x0 + nv + 1};
    const int ry[5] = {y0 - 2, y0 - 1, y0, y1, y1 + 1};
    return (df_wrap(ry[l / 5], ny) / rows) * tiles_x + df_wrap(cx[l % 5], nx) / tx;
}

}  // namespace lbm
