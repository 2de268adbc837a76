// kernels_t2.hpp -- several LBGK steps per launch (temporal blocking): two on
// D2Q9, K = 2, 4 or 8 on D1Q3 (k_stream_collide_t1, further below).
//
// A step reads and writes every population once, so a one-step kernel moves
// 2 Q s bytes per node update whatever its tiling.  Two steps in one sweep
// halve that: the intermediate state f*(t + 1) never leaves the chip.
//
// Each workgroup owns tx consecutive columns [x0, x0 + tx) (fewer in the last
// tile of a ragged row) of `rows` consecutive rows [y0, y1) and sweeps its
// rows in y order.  At sweep row r
// (r = y0 - 1 .. y1) it
//   1. pulls f(t + 1) at row r for the tx + 2 columns [x0 - 1, x0 + tx + 1)
//      from the source buffer, collides, and puts the post-collision values
//      (rounded to the storage type, exactly what a one-step launch would
//      store) into a ring of four LDS rows;
//   2. once rows r - 2 .. r are in the ring, pulls f(t + 2) at row r - 1 for
//      the tx owned columns from the ring, collides, and stores f*(t + 2).
// A D2Q9 population moves at most one row and one column per step, so the
// halo of one column on each side and one row above and below is all that
// step 2 needs.  The halo nodes are also computed by the neighbouring
// workgroups; every node runs the same collision code as in the one-step
// kernels, so the results are bitwise those of two one-step launches.  A
// workgroup reads the populations of (tx + 2) x (rows + 2) step-1 node
// updates and writes those of its tx x rows nodes once.
//
// A D3Q27 node holds 27 populations, so the ring would need (tx + 2) x 27 x 4
// rows of a 2-D tile (and the x-y halo grows the re-read area); in 160 KB of
// LDS that does not fit at any useful tile size, so D3Q27 stays one step per
// launch.
#pragma once

#include "kernels.hpp"

namespace lbm {

struct Step2Args {
    const void *src;  // f*(t), row-interleaved layout
    void *dst;        // f*(t + 2)
    int nx, ny;
    int tx;           // columns per workgroup tile (64 .. 1024; the last tile of a row may be partial)
    int rows;         // owned rows per workgroup
    int tiles_x, tiles_y;
    int64_t ps, rs;
    Relax relax;
    int *flag;
};

// Non-temporal output stores pay when the two population buffers exceed the
// 256 MB last-level (Infinity) cache: 4096^2 D2Q9, us per step, FP64 212.4
// against 224.4 with plain stores.  When both fit, the next launch reads the
// output from that cache, and non-temporal stores lose it (1024^2 FP64: 20.3
// against 16.3).  A compile-time choice (the NT parameter of the kernels): as
// a run-time branch the compiler merges the two store sequences and drops
// the hint.
__host__ __device__ constexpr bool t2_nt_stores(size_t buf_bytes) { return 2 * buf_bytes > ((size_t)192 << 20); }

constexpr int kT2Ring = 4;  // LDS rows in the ring (see the barrier note below)

// The two step-1 halo columns of a row: with float storage wavefront 0
// computes them for a chunk of 32 sweep rows at a time (2 x 32 nodes, one
// wavefront), into a small LDS area copied into the ring row by row; with
// double storage an extra wavefront per workgroup computes them every row.
// (Measured at 4096^2, us per step: float 143.2 with chunks against 148.3
// with the extra wavefront; double 265.2 against 225.9 -- the double
// workgroups of tx = 128 keep only two wavefronts without it, too few loads
// in flight.)
__host__ __device__ constexpr bool t2_halo_wave(size_t elem) { return elem == 8; }
constexpr int kT2Chunk = 32;

// Threads per workgroup and LDS bytes for tx owned columns and elements of
// `elem` bytes: the ring [4][9][tx + 2], and the halo chunk [32][2][9].
__host__ __device__ constexpr int t2_threads(int tx, size_t elem) { return tx + (t2_halo_wave(elem) ? 64 : 0); }
__host__ __device__ constexpr size_t t2_lds_bytes(int tx, size_t elem) {
    return ((size_t)kT2Ring * 9 * (size_t)(tx + 2) + (t2_halo_wave(elem) ? 0 : (size_t)kT2Chunk * 2 * 9)) * elem;
}

// Population buffers live in global memory.  The sweeps load and store them
// through these helpers, which name the global address space at the access
// for float storage: where the compiler sees only a generic pointer (one read
// from a slot descriptor in memory, in the pool kernels) it otherwise emits
// flat accesses, which count against the LDS counter too, so that every LDS
// wait of a sweep also waits for the next rows' loads in flight (batched
// workload, float: 313 -> 309 us per step).  Double storage keeps generic
// accesses: its pool sweeps measured slower with global ones (547 -> 558).
template <typename T>
__device__ __forceinline__ T gload(const T *p) {
    if constexpr (sizeof(T) == 4)
        return *(const __attribute__((address_space(1))) T *)p;
    else
        return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void gstore(T *p, T v) {
    if constexpr (sizeof(T) == 4) {
        auto *q = (__attribute__((address_space(1))) T *)p;
        if constexpr (NT)
            __builtin_nontemporal_store(v, q);
        else
            *q = v;
    } else {
        if constexpr (NT)
            __builtin_nontemporal_store(v, p);
        else
            *p = v;
    }
}

// Pull f_i(x, y) = f*_i(x - c_x, y - c_y) of one D2Q9 node from a buffer
// (periodic wrap; 0 <= x < nx, 0 <= y < ny).
template <typename T>
__device__ __forceinline__ void pull_d2q9(const T *__restrict__ src, int nx, int ny, int64_t ps, int64_t rs, int x,
                                          int y, T (&f)[9]) {
    const int xs[3] = {x + 1 == nx ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};  // x - c_x
    const int ys[3] = {y + 1 == ny ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};  // y - c_y
#pragma unroll
    for (int cy = 0; cy < 3; ++cy)
#pragma unroll
        for (int cx = 0; cx < 3; ++cx) {
            const int i = cx + 3 * cy;
            f[i] = gload(src + (int64_t)ys[cy] * rs + i * ps + xs[cx]);
        }
}

// The same pull for a row y common to the wavefront: the (row, population)
// bases are wavefront-uniform (scalar registers) and the lane's part is a
// byte offset xb[cx] of its source column x - c_x, fixed for the whole sweep,
// so the loads need no per-lane 64-bit address arithmetic.
template <typename T>
__device__ __forceinline__ void pull_row_d2q9(const T *__restrict__ src, int ny, int64_t ps, int64_t rs, int y,
                                              const uint32_t (&xb)[3], T (&f)[9]) {
    const int ys[3] = {y + 1 == ny ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};  // y - c_y
#pragma unroll
    for (int cy = 0; cy < 3; ++cy)
#pragma unroll
        for (int cx = 0; cx < 3; ++cx) {
            const int i = cx + 3 * cy;
            const char *base = reinterpret_cast<const char *>(src + (int64_t)ys[cy] * rs + (int64_t)i * ps);
            f[i] = gload(reinterpret_cast<const T *>(base + xb[cx]));
        }
}

// Grid: tiles_x * tiles_y workgroups of t2_threads(tx, sizeof(T)) threads,
// dynamic LDS t2_lds_bytes(tx, sizeof(T)).  A tile owns nv = min(tx, nx - x0)
// columns (fewer than tx in the last tile of a ragged row).  Ring column c
// holds step-1 column x0 - 1 + c, c = 0 .. nv + 1.  With chunks, lane t < nv
// computes step 1 and step 2 at column x0 + t; with the halo wavefront, lane
// t < nv + 2 computes step 1 at x0 - 1 + t and lane t < nv step 2 at x0 + t.
// Other lanes load a valid node, discard the result, and keep to the barriers.
template <int DT, bool CORR, int EQ, bool NT>
__device__ __forceinline__ void two_step_tile(const Step2Args &a, int tile) {
    using T = store_t<DT>;
    constexpr bool HW = t2_halo_wave(sizeof(T));
    constexpr int CH = kT2Chunk;
    extern __shared__ __align__(16) unsigned char t2_lds[];
    const T *__restrict__ src = static_cast<const T *>(a.src);
    T *__restrict__ dst = static_cast<T *>(a.dst);

    const int t = (int)threadIdx.x;
    const int w1 = a.tx + 2;  // ring columns: x0 - 1 .. x0 + tx
    T *ring = reinterpret_cast<T *>(t2_lds);
    T *hal = ring + (size_t)kT2Ring * 9 * w1;  // [CH][2][9]
    const int x0 = (tile % a.tiles_x) * a.tx;
    const int y0 = (tile / a.tiles_x) * a.rows;
    const int y1 = min(y0 + a.rows, a.ny);
    const int nsweep = y1 - y0 + 2;  // sweep rows y0 - 1 .. y1 (offsets 0 .. nsweep - 1)
    const int nv = min(a.tx, a.nx - x0);  // owned columns of this tile
    const int x = x0 + t;                  // step-2 column
    const bool s2 = t < nv;
    // step-1 column: x0 + t, or with the halo wavefront x0 - 1 + t wrapped (x0 + nv <= nx:
    // one wrap suffices); lanes past them read column x0 and discard the result
    const bool s1 = HW ? t < nv + 2 : t < nv;
    int x1 = s1 ? x : x0;
    if (HW) {
        x1 = s1 ? x0 - 1 + t : x0;
        x1 = x1 < 0 ? x1 + a.nx : (x1 >= a.nx ? x1 - a.nx : x1);
    }
    // byte offsets of the step-1 lane's source columns x1 - c_x
    const uint32_t xb[3] = {(uint32_t)((x1 + 1 == a.nx ? 0 : x1 + 1) * (int)sizeof(T)), (uint32_t)(x1 * (int)sizeof(T)),
                            (uint32_t)((x1 == 0 ? a.nx - 1 : x1 - 1) * (int)sizeof(T))};
    // sweep rows run from y0 - 1 to y1 <= ny: one wrap at either end
    auto wrap_row = [&](int r) { return r < 0 ? r + a.ny : (r >= a.ny ? r - a.ny : r); };

    // halo lanes of wavefront 0: sweep offset k0 + (t >> 1), column t & 1 (x0 - 1 or x0 + nv,
    // wrapped); lanes past the chunk or the sweep load a valid row and discard it
    const bool w0 = !HW && t < 64;
    const int hx = (t & 1) ? (x0 + nv == a.nx ? 0 : x0 + nv) : (x0 == 0 ? a.nx - 1 : x0 - 1);
    T h[9];
    auto halo_load = [&](int k0) {
        const int k = min(k0 + ((t & 63) >> 1), nsweep - 1);
        pull_d2q9<T>(src, a.nx, a.ny, a.ps, a.rs, hx, wrap_row(y0 - 1 + k), h);
    };

    if constexpr (HW) {
        // Double storage: one sweep row after another, step 2 behind the barrier of
        // the row it needs.  (The pipelined form below ran 1.8 % slower here:
        // 215.7 against 211.9 us per step at 4096^2.)
        // One sweep row: (at a chunk start, the halo chunk) step 1 at row r from f
        // (pulled two rows earlier), then the loads of row r + 2 into f, then
        // step 2 at row r - 1.
        auto sweep_row = [&](T (&f)[9], int r) {
            const int k = r - y0 + 1;  // sweep offset
            if (!HW && k % CH == 0) {
                if (w0) {
                    const bool valid = t < 2 * CH && k + (t >> 1) < nsweep;
                    const bool badh = collide_dt<2, DT, CORR, EQ>(h, a.relax);
                    raise_flag(a.flag, badh && valid);
                    if (valid) {
    #pragma unroll
                        for (int i = 0; i < 9; ++i)
                            hal[t * 9 + i] = h[i];
                    }
                    if (k + CH < nsweep)  // the next chunk's loads
                        halo_load(k + CH);
                }
                // The chunk is complete before any lane copies from it; the
                // previous chunk was last read before the barrier of row r - 1.
                __syncthreads();
            }
            // step 1 at sweep row r into ring slot k mod 4 (column c <-> x0 - 1 + c)
            const bool bad1 = collide_dt<2, DT, CORR, EQ>(f, a.relax);
            raise_flag(a.flag, bad1 && s1);
            T *slot = ring + (size_t)(k & (kT2Ring - 1)) * 9 * w1;
            if (s1) {
    #pragma unroll
                for (int i = 0; i < 9; ++i)
                    slot[i * w1 + (HW ? t : t + 1)] = f[i];
            }
            if (!HW && t < 2) {
                const T *hv = hal + ((k % CH) * 2 + t) * 9;
                const int c = t == 0 ? 0 : nv + 1;
    #pragma unroll
                for (int i = 0; i < 9; ++i)
                    slot[i * w1 + c] = hv[i];
            }
            // Slot r + 1 (written in the next row) is slot r - 3, last read by
            // step 2 of row r - 2 in the previous row, which every lane finished
            // before passing this barrier: one barrier per row suffices.
            __syncthreads();
            if (r + 2 <= y1)  // keep two rows of loads in flight
                pull_row_d2q9<T>(src, a.ny, a.ps, a.rs, wrap_row(r + 2), xb, f);
            if (r > y0 && s2) {
                // step 2 at row y = r - 1: f_i(x, y) = f*_i(x - c_x, y - c_y) from
                // sweep row y + 1 - cy, ring column (x + 1 - cx) - (x0 - 1)
                const int y = r - 1;
                T g[9];
    #pragma unroll
                for (int cy = 0; cy < 3; ++cy) {
                    const T *srow = ring + (size_t)((y + 2 - cy - y0) & (kT2Ring - 1)) * 9 * w1;
    #pragma unroll
                    for (int cx = 0; cx < 3; ++cx) {
                        const int i = cx + 3 * cy;
                        g[i] = srow[i * w1 + t + 2 - cx];
                    }
                }
                const bool bad2 = collide_dt<2, DT, CORR, EQ>(g, a.relax);
                raise_flag(a.flag, bad2);
                const uint32_t ob = (uint32_t)(x * (int)sizeof(T));
    #pragma unroll
                for (int i = 0; i < 9; ++i) {
                    char *base = reinterpret_cast<char *>(dst + (int64_t)y * a.rs + (int64_t)i * a.ps);
                    gstore<NT>(reinterpret_cast<T *>(base + ob), g[i]);
                }
            }
        };

        // sweep rows y0 - 1 .. y1 (at least three), alternating two register sets
        T fa[9], fb[9];
        if (w0)
            halo_load(0);
        pull_row_d2q9<T>(src, a.ny, a.ps, a.rs, wrap_row(y0 - 1), xb, fa);
        pull_row_d2q9<T>(src, a.ny, a.ps, a.rs, y0, xb, fb);
        for (int r = y0 - 1;;) {
            sweep_row(fa, r);
            if (++r > y1)
                break;
            sweep_row(fb, r);
            if (++r > y1)
                break;
        }
    } else {
        // The sweep in intervals between barriers.  Interval k (sweep offset k,
        // sweep row y0 - 1 + k) holds step 1 at offset k (from f, pulled two
        // offsets earlier) into ring slot k mod 4, and step 2 at row y0 - 3 + k from
        // the slots k - 3 .. k - 1, which the barrier before it completed; slot k
        // is slot k - 4, last read by step 2 in interval k - 1.  The two collisions
        // are independent and sit in one straight-line block, so the compiler can
        // interleave their dependency chains: every lane runs step 2 (lanes past
        // the tile on its last column, results discarded), and the first three
        // intervals (step 1 only) and the last (step 2 only) are separate
        // instances of the body.
        const int c2 = s2 ? t : nv - 1;  // step-2 ring column base of the lane
        // with the halo wavefront (FP64), that wavefront takes no step 2 (uniform per wavefront)
        const bool w2 = !HW || t < a.tx;
        // The lane's domain checks are collected over the sweep and raised once at
        // the end (the flag is read after the launch): a flag store per collision
        // is a branch, which would split the block the two collisions share.
        bool bad_any = false;
        auto interval = [&](T (&f)[9], int k, auto do1_, auto do2_) {
            constexpr bool DO1 = decltype(do1_)::value, DO2 = decltype(do2_)::value;
            if constexpr (DO1) {
                if (!HW && k % CH == 0) {
                    if (w0) {
                        const bool valid = t < 2 * CH && k + (t >> 1) < nsweep;
                        const bool badh = collide_dt<2, DT, CORR, EQ>(h, a.relax);
                        bad_any |= badh && valid;
                        if (valid) {
    #pragma unroll
                            for (int i = 0; i < 9; ++i)
                                hal[t * 9 + i] = h[i];
                        }
                        if (k + CH < nsweep)  // the next chunk's loads
                            halo_load(k + CH);
                    }
                    // The chunk is complete before any lane copies from it; the
                    // previous chunk was last read before the previous barrier.
                    __syncthreads();
                }
            }
            // step 2 at row y = y0 - 3 + k: f_i(x, y) = f*_i(x - c_x, y - c_y) from sweep
            // row y + 1 - cy (slot k - 1 - cy), ring column (x + 1 - cx) - (x0 - 1)
            T g[9];
            if (DO2 && w2) {
    #pragma unroll
                for (int cy = 0; cy < 3; ++cy) {
                    const T *srow = ring + (size_t)((k - 1 - cy) & (kT2Ring - 1)) * 9 * w1;
    #pragma unroll
                    for (int cx = 0; cx < 3; ++cx) {
                        const int i = cx + 3 * cy;
                        g[i] = srow[i * w1 + c2 + 2 - cx];
                    }
                }
            }
            bool bad1 = false, bad2 = false;
            if constexpr (DO1)
                bad1 = collide_dt<2, DT, CORR, EQ>(f, a.relax);
            if (DO2 && w2)
                bad2 = collide_dt<2, DT, CORR, EQ>(g, a.relax);
            // Both results are used below only by lanes that own them; an empty asm
            // (no instruction, values unchanged) uses them here, so that neither
            // collision is sunk into its lanes' conditional store and the two stay
            // in one block.
    #pragma unroll
            for (int i = 0; i < 9; ++i) {
                if constexpr (DO1)
                    asm("" : "+v"(f[i]));
                if (DO2 && w2)
                    asm("" : "+v"(g[i]));
            }
            bad_any |= (bad1 && s1) | (bad2 && s2);
            if constexpr (DO2) {
                if (s2) {
                    const int y = y0 - 3 + k;
                    const uint32_t ob = (uint32_t)(x * (int)sizeof(T));
    #pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        char *base = reinterpret_cast<char *>(dst + (int64_t)y * a.rs + (int64_t)i * a.ps);
                        gstore<NT>(reinterpret_cast<T *>(base + ob), g[i]);
                    }
                }
            }
            if constexpr (DO1) {
                // step 1 into ring slot k mod 4 (column c <-> x0 - 1 + c)
                T *slot = ring + (size_t)(k & (kT2Ring - 1)) * 9 * w1;
                if (s1) {
    #pragma unroll
                    for (int i = 0; i < 9; ++i)
                        slot[i * w1 + (HW ? t : t + 1)] = f[i];
                }
                if (!HW && t < 2) {
                    const T *hv = hal + ((k % CH) * 2 + t) * 9;
                    const int c = t == 0 ? 0 : nv + 1;
    #pragma unroll
                    for (int i = 0; i < 9; ++i)
                        slot[i * w1 + c] = hv[i];
                }
                if (k + 2 < nsweep)  // two offsets of loads in flight
                    pull_row_d2q9<T>(src, a.ny, a.ps, a.rs, wrap_row(y0 + 1 + k), xb, f);
                __syncthreads();
            }
        };
        using Y = std::true_type;
        using N = std::false_type;

        // offsets 0 .. nsweep - 1 (nsweep >= 3), alternating two register sets
        T fa[9], fb[9];
        if (w0)
            halo_load(0);
        pull_row_d2q9<T>(src, a.ny, a.ps, a.rs, wrap_row(y0 - 1), xb, fa);
        pull_row_d2q9<T>(src, a.ny, a.ps, a.rs, y0, xb, fb);
        interval(fa, 0, Y{}, N{});
        interval(fb, 1, Y{}, N{});
        interval(fa, 2, Y{}, N{});
        for (int k = 3;;) {
            if (k >= nsweep)
                break;
            interval(fb, k, Y{}, Y{});
            if (++k >= nsweep)
                break;
            interval(fa, k, Y{}, Y{});
            ++k;
        }
        interval(fa, nsweep, N{}, Y{});
        raise_flag(a.flag, bad_any);
    }
}

// Whole-row two-step tiles, for rows no wider than a workgroup.  The
// workgroup's B threads form S sub-tiles of w = 64 m lanes (w >= nx, S w <= B,
// so no wavefront straddles two sub-tiles); sub-tile s of workgroup tile
// `tile` owns the rows [(tile S + s) R, + R) of the whole width and sweeps
// them as two_step_tile does, with a ring of four LDS rows of w + 2 columns
// of its own.  The row is whole, so the x neighbours of step 2 at the ends of
// the row are the row's own columns across the periodic wrap, already in the
// ring: no halo column is loaded or computed, and no node of step 1 is
// computed twice along x.  Lane t < nx computes column t; lanes past the row
// load column 0 and discard the result.  Wavefronts of sub-tiles without rows
// (past S, or past the last row) only keep to the barriers.  Every node runs
// the same collision code as the one-step kernels, so the results are
// bitwise those of two one-step launches.  Dynamic LDS:
// t2_rows_lds_bytes(S, w, elem).
__host__ __device__ constexpr size_t t2_rows_lds_bytes(int S, int w, size_t elem) {
    return (size_t)S * kT2Ring * 9 * (size_t)(w + 2) * elem;
}

template <int DT, bool CORR, int EQ, bool NT>
__device__ __forceinline__ void two_step_rows_tile(const Step2Args &a, int tile, int w, int S, int R) {
    using T = store_t<DT>;
    extern __shared__ __align__(16) unsigned char t2_lds[];
    const T *__restrict__ src = static_cast<const T *>(a.src);
    T *__restrict__ dst = static_cast<T *>(a.dst);

    const int tid = (int)threadIdx.x;
    const int sub = tid / w;      // uniform per wavefront (w is a multiple of 64)
    const int t = tid - sub * w;  // column
    const int w1 = w + 2;         // ring columns: column c holds x = c - 1 (1 .. nx)
    const int y0 = (tile * S + sub) * R;
    const int y1 = min(y0 + R, a.ny);
    const bool active = sub < S && y0 < a.ny;  // uniform per wavefront
    const int my_sweep = active ? y1 - y0 + 2 : 0;  // sweep rows y0 - 1 .. y1
    T *ring = reinterpret_cast<T *>(t2_lds) + (size_t)(active ? sub : 0) * kT2Ring * 9 * w1;
    const bool valid = t < a.nx;
    const int x = valid ? t : 0;
    // byte offsets of the source columns x - c_x (c_x = -1, 0, +1), wrapped
    const uint32_t xb[3] = {(uint32_t)((x + 1 == a.nx ? 0 : x + 1) * (int)sizeof(T)), (uint32_t)(x * (int)sizeof(T)),
                            (uint32_t)((x == 0 ? a.nx - 1 : x - 1) * (int)sizeof(T))};
    // ring columns of the same sources for step 2, wrapped inside the row
    const int cc[3] = {x + 1 == a.nx ? 1 : x + 2, x + 1, x == 0 ? a.nx : x};
    auto wrap_row = [&](int r) { return r < 0 ? r + a.ny : (r >= a.ny ? r - a.ny : r); };

    // The sweep in intervals between barriers, as in two_step_tile's float
    // form: interval k holds step 1 at offset k (row y0 - 1 + k) into ring slot
    // k mod 4 and step 2 at row y0 - 3 + k from the slots k - 3 .. k - 1, the two
    // collisions in one block; the domain checks are raised once at the end.
    // A wavefront's sub-tile takes my_sweep offsets (fewer, or none, at the end
    // of the slot); every wavefront passes R + 2 barriers, one after each of
    // the intervals 0 .. R + 1.
    bool bad_any = false;
    auto interval = [&](T (&f)[9], int k, auto do1_, auto do2_) {
        constexpr bool DO1 = decltype(do1_)::value, DO2 = decltype(do2_)::value;
        T g[9];
        if constexpr (DO2) {
#pragma unroll
            for (int cy = 0; cy < 3; ++cy) {
                const T *srow = ring + (size_t)((k - 1 - cy) & (kT2Ring - 1)) * 9 * w1;
#pragma unroll
                for (int cx = 0; cx < 3; ++cx)
                    g[cx + 3 * cy] = srow[(cx + 3 * cy) * w1 + cc[cx]];
            }
        }
        bool bad1 = false, bad2 = false;
        if constexpr (DO1)
            bad1 = collide_dt<2, DT, CORR, EQ>(f, a.relax);
        if constexpr (DO2)
            bad2 = collide_dt<2, DT, CORR, EQ>(g, a.relax);
        // (an empty asm uses both results, so that neither collision is sunk into its
        // lanes' conditional store; no instruction, values unchanged)
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            if constexpr (DO1)
                asm("" : "+v"(f[i]));
            if constexpr (DO2)
                asm("" : "+v"(g[i]));
        }
        bad_any |= (bad1 | bad2) && valid;
        if constexpr (DO2) {
            if (valid) {
                const int y = y0 - 3 + k;
                const uint32_t ob = (uint32_t)(x * (int)sizeof(T));
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    char *base = reinterpret_cast<char *>(dst + (int64_t)y * a.rs + (int64_t)i * a.ps);
                    gstore<NT>(reinterpret_cast<T *>(base + ob), g[i]);
                }
            }
        }
        if constexpr (DO1) {
            T *slot = ring + (size_t)(k & (kT2Ring - 1)) * 9 * w1;
            if (valid) {
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    slot[i * w1 + t + 1] = f[i];
            }
            if (k + 2 < my_sweep)  // two offsets of loads in flight
                pull_row_d2q9<T>(src, a.ny, a.ps, a.rs, wrap_row(y0 + 1 + k), xb, f);
        }
        // slot k + 1 (written in the next interval) is slot k - 3, last read here
        if (k <= R + 1)
            __syncthreads();
    };
    using Y = std::true_type;
    using N = std::false_type;

    int k = 0;
    if (active) {  // uniform per wavefront; my_sweep >= 3
        T fa[9], fb[9];
        pull_row_d2q9<T>(src, a.ny, a.ps, a.rs, wrap_row(y0 - 1), xb, fa);
        pull_row_d2q9<T>(src, a.ny, a.ps, a.rs, y0, xb, fb);
        interval(fa, 0, Y{}, N{});
        interval(fb, 1, Y{}, N{});
        interval(fa, 2, Y{}, N{});
        for (k = 3;;) {
            if (k >= my_sweep)
                break;
            interval(fb, k, Y{}, Y{});
            if (++k >= my_sweep)
                break;
            interval(fa, k, Y{}, Y{});
            ++k;
        }
        interval(fa, k, N{}, Y{});  // k = my_sweep: the last step 2
        ++k;
    }
    for (; k <= R + 1; ++k)  // the workgroup's remaining barriers
        __syncthreads();
    raise_flag(a.flag, bad_any);
}

template <int DT, bool CORR, int EQ = kEqEntropic, bool NT = false>
__global__ __launch_bounds__(1024) void k_stream_collide2(Step2Args a) {
    two_step_tile<DT, CORR, EQ, NT>(a, xcd_tile((int)blockIdx.x, (int)gridDim.x));
}

// ---------------------------------------------------------------------------
// D1Q3, K steps per launch.  A workgroup owns tx consecutive nodes [x0, x0 +
// tx) and keeps the segment [x0 - K, x0 + tx + K) in LDS, as two buffers
// [3][tx + 2K] used in turn.  Step 1 pulls from HBM for the positions
// 1 .. tx + 2K - 2 of the segment, step j for j .. tx + 2K - 1 - j from the
// previous step's buffer, and step K, on the owned positions, stores to HBM:
// a population moves one node per step, so K nodes of halo on each side are
// all that K steps need.  The halo nodes are also computed by the
// neighbouring workgroups, with the same per-node code, so the results are
// bitwise those of K one-step launches.  Needs nx >= tx + K (one periodic
// wrap); the last workgroup's positions past nx are the nodes from x = 0 on,
// computed but not stored.
struct StepKArgs {
    const void *src;  // f*(t)
    void *dst;        // f*(t + K)
    int nx;
    int tx;           // owned nodes per workgroup
    int K;            // steps per launch (2 .. 8)
    int64_t ps;       // population stride (the one row's pitch)
    Relax relax;
    int *flag;
};

constexpr int kT1MaxK = 8;

__host__ __device__ constexpr size_t t1_lds_bytes(int tx, int K, size_t elem) {
    return (size_t)2 * 3 * (size_t)(tx + 2 * K) * elem;
}

template <int DT, bool CORR, int EQ = kEqEntropic, bool NT = false>
__global__ __launch_bounds__(256) void k_stream_collide_t1(StepKArgs a) {
    using T = store_t<DT>;
    extern __shared__ __align__(16) unsigned char t1_lds[];
    const T *__restrict__ src = static_cast<const T *>(a.src);
    T *__restrict__ dst = static_cast<T *>(a.dst);
    const int w = a.tx + 2 * a.K;  // segment length
    // the two buffers at offsets 0 and 3 w of the LDS array: offsets, not a
    // chosen pointer, so that every access keeps the LDS address space (a
    // pointer picked from an array of two compiles to flat accesses)
    T *lds = reinterpret_cast<T *>(t1_lds);
    const int x0 = (int)blockIdx.x * a.tx;
    const int nthr = (int)blockDim.x;
    auto wrap = [&](int x) { return x < 0 ? x + a.nx : (x >= a.nx ? x - a.nx : x); };

    // step 1: positions m = 1 .. w - 2 (x = x0 - K + m) pull f*_i(x - c_i) from HBM
    for (int m = 1 + (int)threadIdx.x; m < w - 1; m += nthr) {
        const int x = x0 - a.K + m;
        T f[3];
#pragma unroll
        for (int cx = 0; cx < 3; ++cx)
            f[cx] = src[cx * a.ps + wrap(x + 1 - cx)];
        const bool bad = collide_dt<1, DT, CORR, EQ>(f, a.relax);
        raise_flag(a.flag, bad);
        if (a.K == 1) {
            if (m >= 1 && m < 1 + a.tx && x < a.nx)
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    dst[i * a.ps + x] = f[i];
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i)
                lds[i * w + m] = f[i];
        }
    }
    // steps 2 .. K from LDS; the last one stores the owned positions
    for (int j = 2; j <= a.K; ++j) {
        __syncthreads();
        const int in = j & 1 ? 3 * w : 0, out = 3 * w - in;
        for (int m = j + (int)threadIdx.x; m < w - j; m += nthr) {
            T f[3];
#pragma unroll
            for (int cx = 0; cx < 3; ++cx)
                f[cx] = lds[in + cx * w + m + 1 - cx];
            const bool bad = collide_dt<1, DT, CORR, EQ>(f, a.relax);
            raise_flag(a.flag, bad);
            if (j == a.K) {
                const int x = x0 - a.K + m;  // m in [K, K + tx): x0 <= x < x0 + tx
                if (x < a.nx) {
                    if constexpr (NT) {
#pragma unroll
                        for (int i = 0; i < 3; ++i)
                            __builtin_nontemporal_store(f[i], dst + i * a.ps + x);
                    } else {
#pragma unroll
                        for (int i = 0; i < 3; ++i)
                            dst[i * a.ps + x] = f[i];
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    lds[out + i * w + m] = f[i];
            }
        }
    }
}

}  // namespace lbm
