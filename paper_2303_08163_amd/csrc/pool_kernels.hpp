// pool_kernels.hpp -- kernels that advance many independent domains together.
//
// A pool holds slots; each slot is one periodic domain with its own two
// population buffers.  For a run, the active slots of one (lattice, storage,
// bulk correction) class -- all compile-time choices of the per-node code, so
// the kernel carries one variant only and keeps the single-domain kernel's
// register budget -- are listed in order of decreasing remaining steps, with the running
// sum of their workgroup tiles.  At step s of the run exactly the slots with
// more than s remaining steps are active, and they form a prefix of the list,
// so the active tiles are [0, P(s)).  A workgroup finds its slot by binary
// search in the running sum.  Every node goes through the same step_node
// function as the single-domain kernels, so a slot's populations are bitwise
// the same as when it runs alone.
//
// Two launch forms:
//   - one kernel launch per step over the active prefix (the kernel boundary
//     orders the steps);
//   - one persistent cooperative launch for all steps of a run: each
//     workgroup takes a contiguous share of the active prefix, then waits at a
//     grid barrier before the next step.  The barrier spins on a device
//     counter with a bound; past the bound it raises an error flag that makes
//     every workgroup leave, so the grid always drains.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "kernels_t2.hpp"
#include "tile_deps.hpp"

namespace lbm {

struct SlotDesc {
    void *buf[2];
    int nx, ny, nz;
    int tiles_x, tiles_y;
    int parity;    // buffer holding the state at the start of the run
    int tw_shift;  // > 0: tiles are rows of 1 << tw_shift threads (row fit); 0: blockDim's shape
    int t2_w;      // two-step launches: > 0: whole-row sub-tiles of t2_w lanes, t2_sub per
    int t2_sub;    //   workgroup (two_step_rows_tile); 0: column tiles (two_step_tile)
    int run_steps; // tile-ordered persistent form: steps of this slot in the launch
    int64_t ps, rs;
    Relax relax;
    int *flag;
    int64_t *tdone;  // tile-ordered persistent form: one completion counter per two-step tile
};

struct PoolRunArgs {
    const SlotDesc *slots;    // n slots, remaining steps decreasing
    const int *tile_start;    // n + 1 running tile counts, tile_start[0] = 0
    const int64_t *remaining; // n remaining step counts at the start of the run
    int n;
    int step0;                // first step of this launch within the run
    int nsteps;               // steps done by this launch
    unsigned *barrier;        // persistent form: arrival counter, zero at launch
    int *error;               // persistent form: set on a barrier timeout
    long long spin_limit;
    int flat;                 // 1: a tile is blockDim.x * blockDim.y consecutive nodes of its slot
    int t2_tx, t2_rows;       // two-step form: columns and rows of a column tile
    int t2_R;                 // two-step form: rows of a whole-row sub-tile
    int tile_base;            // the launch's first tile (its blocks cover tile_base + [0, grid))
    int64_t base;             // tile-ordered form: counter value of a tile with no iteration of this launch done
};

// Active tiles at step s: the tile count of the slots with remaining > s.
__device__ __forceinline__ int active_tiles(const PoolRunArgs &a, int s) {
    int lo = 0, hi = a.n;  // first index with remaining <= s
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a.remaining[mid] > s)
            lo = mid + 1;
        else
            hi = mid;
    }
    return a.tile_start[lo];
}

template <int DIM, int DT, bool CORR>
__device__ __forceinline__ void pool_tile(const PoolRunArgs &a, int t, int s) {
    int lo = 0, hi = a.n - 1;  // last slot k with tile_start[k] <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.tile_start[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    // Copy the descriptor into locals before any store: the stores below could
    // alias the descriptor table as far as the compiler knows, and reading the
    // fields through a reference makes it keep them in vector registers
    // (124 VGPRs instead of 70 for D3Q27).
    const SlotDesc &dd = a.slots[lo];
    const int nx = dd.nx, ny = dd.ny, nz = dd.nz, tiles_x = dd.tiles_x, tiles_y = dd.tiles_y;
    const int tw_shift = dd.tw_shift;
    const int64_t ps = dd.ps, rs = dd.rs;
    const Relax relax = dd.relax;
    int *flag = dd.flag;
    const int p = (dd.parity + s) & 1;
    using T = store_t<DT>;
    const T *src = static_cast<const T *>(dd.buf[p]);
    T *dst = static_cast<T *>(dd.buf[p ^ 1]);
    const int tile = t - a.tile_start[lo];
    int x, y, z;
    bool pad = false;
    if (a.flat) {
        // consecutive nodes of the slot, x fastest, across rows and planes
        const int64_t n = (int64_t)tile * (blockDim.x * blockDim.y) + threadIdx.y * blockDim.x + threadIdx.x;
        if (n >= (int64_t)nx * ny * nz)
            return;
        const int row = (int)(n / nx);
        x = (int)(n - (int64_t)row * nx);
        y = row % ny;
        z = row / ny;
    } else {
        const int tx = tile % tiles_x;
        const int ty = (tile / tiles_x) % tiles_y;
        z = tile / (tiles_x * tiles_y);
        int lx = (int)threadIdx.x, ly = (int)threadIdx.y, bw = (int)blockDim.x, bh = (int)blockDim.y;
        if (tw_shift > 0) {  // the slot's own row width: consecutive threads along x
            const int tid = (int)(threadIdx.y * blockDim.x + threadIdx.x);
            lx = tid & ((1 << tw_shift) - 1);
            ly = tid >> tw_shift;
            bw = 1 << tw_shift;
            bh = (int)(blockDim.x * blockDim.y) >> tw_shift;
        }
        x = tx * bw + lx;
        y = ty * bh + ly;
        pad = x >= nx;
        if (y >= ny || (pad && !in_padding<DIM>(ps, rs, x)))
            return;
    }
    step_node<DIM, DT, CORR>(src, dst, nx, ny, nz, ps, rs, relax, flag, x, y, z, pad);
}

// Two steps per launch (D2Q9): tile_start counts each slot's two-step tiles --
// ceil(ny / (t2_sub t2_R)) whole-row tiles when the row fits the workgroup
// (t2_w > 0), else ceil(nx / t2_tx) x ceil(ny / t2_rows) column tiles -- and
// the launch covers the tiles [tile_base, tile_base + grid): a prefix of the
// slots that still take two steps at this point of the run.  a.step0 is the
// launch's index in the run, the number of launches (of either kind) each
// covered slot has had before (one buffer swap per launch).  The per-tile
// code is the single-domain two-step kernel's, or its whole-row form, so a
// slot's populations are bitwise those of one-step launches.  Block
// t2_threads(t2_tx, elem) threads, which the whole-row form splits into
// sub-tiles; dynamic LDS the larger of the two forms' needs.
template <int DT, bool CORR, bool NT>
__global__ __launch_bounds__(1024) void k_pool_step2(PoolRunArgs a) {
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x) + a.tile_base;
    int lo = 0, hi = a.n - 1;  // last slot k with tile_start[k] <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.tile_start[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    const SlotDesc &dd = a.slots[lo];
    const int nx = dd.nx, ny = dd.ny;
    const int p = (dd.parity + a.step0) & 1;
    Step2Args s{dd.buf[p], dd.buf[p ^ 1], nx, ny, a.t2_tx, a.t2_rows, (nx + a.t2_tx - 1) / a.t2_tx,
                (ny + a.t2_rows - 1) / a.t2_rows, dd.ps, dd.rs, dd.relax, dd.flag};
    const int w = dd.t2_w, sub = dd.t2_sub;  // copied before any store (see pool_tile)
    if (w > 0)  // uniform per workgroup
        two_step_rows_tile<DT, CORR, kEqEntropic, NT>(s, t - a.tile_start[lo], w, sub, a.t2_R);
    else
        two_step_tile<DT, CORR, kEqEntropic, NT>(s, t - a.tile_start[lo]);
}

// One step (a.step0) over the tiles [tile_base, tile_base + grid): the active
// prefix, or the range of slots whose last step of the run is a single one.
template <int DIM, int DT, bool CORR>
__global__ __launch_bounds__(256) void k_pool_step(PoolRunArgs a) {
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x) + a.tile_base;
    pool_tile<DIM, DT, CORR>(a, t, a.step0);
}

// Bounded grid barrier.  A workgroup-scope barrier does not wait for stores,
// so every wave first waits for its own; one thread then writes the XCD's L2
// back (agent-scope release), arrives, and spins; after it, every wave drops
// stale L1/L2 lines (agent-scope acquire).  Returns false when the wait
// timed out or another workgroup reported a timeout; the caller then leaves.
__device__ __forceinline__ bool grid_barrier(unsigned *counter, unsigned target, int *error, long long spin_limit) {
    __shared__ int ok;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int good = 1;
        long long spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                ++spins > spin_limit) {
                __hip_atomic_fetch_or(error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                good = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        ok = good;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok != 0;
}

// All nsteps steps of a run in one cooperative launch.  Workgroup w covers
// the contiguous share [L P / G, (L + 1) P / G) of the P active tiles, with
// L = xcd_tile(w, G) so that each XCD walks one contiguous range.
template <int DIM, int DT, bool CORR>
__global__ __launch_bounds__(256) void k_pool_persistent(PoolRunArgs a) {
    const int G = (int)gridDim.x;
    const int L = xcd_tile((int)blockIdx.x, G);
    for (int s = 0; s < a.nsteps; ++s) {
        const int step = a.step0 + s;
        const int P = active_tiles(a, step);
        const int lo = (int)(((int64_t)L * P) / G), hi = (int)(((int64_t)(L + 1) * P) / G);
        for (int t = lo; t < hi; ++t)
            pool_tile<DIM, DT, CORR>(a, t, step);
        if (s + 1 < a.nsteps && !grid_barrier(a.barrier, (unsigned)G * (unsigned)(s + 1), a.error, a.spin_limit))
            return;
    }
}

// ---------------------------------------------------------------------------
// Tile-ordered persistent form (D2Q9 two-step classes): every iteration of a
// run in one cooperative launch, with no grid-wide barrier.  Slot j takes its
// s_j = run_steps steps as n_j = ceil(s_j / 2) iterations over its two-step
// tiles: two steps each and, for odd s_j, a last iteration of one step over
// the tile's own nodes.  Iteration k of a tile reads buffer (parity + k) & 1
// at the tile's nodes and the two columns and rows around them, and writes
// the other buffer at its own nodes only.  It may therefore start once every
// tile whose nodes lie within two nodes of it (itself included, periodic wrap)
// has finished iteration k - 1: the state it reads is then complete, and the
// state it overwrites (that of iteration k - 1's input) has no reader left.
// The relation is symmetric and stays inside a slot.
//
// Each tile has a completion counter; iteration k done is base + k + 1, and
// base exceeds every value an earlier launch stored, so the counters need no
// clearing between runs (they are zeroed once, at admission).
//
// Workgroup L (XCD-ordered) owns the tiles L, L + G, L + 2 G, ... of the
// class and takes them in that order for iteration 0, then for iteration 1,
// and so on.  At any moment the workgroups therefore work on about G
// consecutive tiles, each XCD on a contiguous part of them, as the hardware
// dispatcher would order one launch per iteration: neighbouring tiles share
// halo lines in L2 and the pages in use stay few.  (Contiguous ranges per
// workgroup spread the grid over the whole footprint at once; on the batched
// shear-wave workload that ran 17% slower, fences aside.)  A workgroup
// publishes an iteration once, after all its tiles of it: one agent-scope
// release (a write-back of the XCD's L2), then the counters of those tiles.
// One release per tile cost FP64 half its rate: on MI355X each release waits
// for the L2 write-back.  Every workgroup is resident (cooperative launch), and
// a tile's wait at iteration k needs only iteration k - 1 of other workgroups,
// which they publish without waiting on anything later, so every wait ends.
// Each is nevertheless bounded like the grid barrier's: past the bound, or
// once another workgroup has reported a timeout, the workgroup leaves.

// Wait until the tiles within two nodes of tile tt of a slot (whole-row tiles
// of rr rows when w > 0, else column tiles of tx x rows) have counters >=
// need.  Wavefront 0 polls, lane l the candidate df_neighbour(l, ...) (every
// tile that the dilated box [x0 - 2, x0 + nv + 2) x [y0 - 2, y1 + 2) meets,
// some of them repeatedly; tile_deps.hpp).  Wavefront 0
// then acquires at agent scope (dropping stale L1 and L2 lines), and the
// workgroup barrier orders the other wavefronts' loads after it.  Returns
// false (the same in every thread) when the wait timed out or another
// workgroup reported a timeout.
__device__ __forceinline__ bool df_wait(const PoolRunArgs &a, const int64_t *tdone, int nx, int ny, int w, int rr,
                                        int tx, int rows, int tt, int64_t need) {
    __shared__ int df_ok;
    if (threadIdx.x < 64) {  // wavefront 0, all lanes active
        const int l = (int)threadIdx.x;
        const int idx = df_neighbour(l, nx, ny, w, rr, tx, rows, tt);
        bool ready = idx < 0 || __hip_atomic_load(tdone + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
        long long spins = 0;
        int good = 1;
        while (!__all(ready)) {
            const int err =
                __builtin_amdgcn_readfirstlane(__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (err != 0 || ++spins > a.spin_limit) {
                if (l == 0)
                    __hip_atomic_fetch_or(a.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                good = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
            if (!ready)
                ready = __hip_atomic_load(tdone + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
        }
        if (l == 0)
            df_ok = good;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return df_ok != 0;
}

// Slot of class tile t: the last j with tile_start[j] <= t.
__device__ __forceinline__ int df_slot(const PoolRunArgs &a, int t) {
    int lo = 0, hi = a.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.tile_start[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Grid: G <= resident workgroups of the pool's two-step block (1024 threads
// for FP32, one per compute unit by its LDS; 192 for FP64), the larger LDS
// need of the two tile forms; a.tile_start holds the two-step tile counts.  At
// least four wavefronts per SIMD: the registers the compiler chose otherwise
// (140) left fewer (batched workload, FP32 with 512-thread workgroups: 666
// against 622 solves/s, with 32 bytes of spills per lane; FP64, held to four
// workgroups of three wavefronts by its LDS, unchanged).
template <int DT, bool CORR, bool NT>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4))) void k_pool_df2(PoolRunArgs a) {
    using T = store_t<DT>;
    const int G = (int)gridDim.x;
    const int L = xcd_tile((int)blockIdx.x, G);
    const int ntiles = a.tile_start[a.n];
    int kmax = 0;  // most iterations among the owned tiles' slots
    for (int t = L; t < ntiles; t += G)
        kmax = max(kmax, (a.slots[df_slot(a, t)].run_steps + 1) / 2);
    for (int k = 0; k < kmax; ++k) {
        for (int t = L; t < ntiles; t += G) {
            const int j = df_slot(a, t);
            // descriptor fields into locals before any store (see pool_tile)
            const SlotDesc &dd = a.slots[j];
            const int steps = dd.run_steps;
            if (2 * k >= steps)  // this slot's run is over (uniform per workgroup)
                continue;
            const int nx = dd.nx, ny = dd.ny, w = dd.t2_w, sub = dd.t2_sub;
            const int64_t ps = dd.ps, rs = dd.rs;
            const Relax relax = dd.relax;
            int *flag = dd.flag;
            int64_t *tdone = dd.tdone;
            const int p = (dd.parity + k) & 1;
            void *src = dd.buf[p], *dst = dd.buf[p ^ 1];
            const int tt = t - a.tile_start[j];
            const int rr = sub * a.t2_R;  // rows of a whole-row tile
            if (k > 0 && !df_wait(a, tdone, nx, ny, w, rr, a.t2_tx, a.t2_rows, tt, a.base + k))
                return;
            if (2 * k + 2 <= steps) {
                Step2Args s{src, dst, nx, ny, a.t2_tx, a.t2_rows, (nx + a.t2_tx - 1) / a.t2_tx,
                            (ny + a.t2_rows - 1) / a.t2_rows, ps, rs, relax, flag};
                if (w > 0)
                    two_step_rows_tile<DT, CORR, kEqEntropic, NT>(s, tt, w, sub, a.t2_R);
                else
                    two_step_tile<DT, CORR, kEqEntropic, NT>(s, tt);
            } else {  // the odd last step: one step over the tile's own nodes
                int bx0 = 0, bnx = nx, by0, by1;
                if (w > 0) {
                    by0 = tt * rr;
                    by1 = min(by0 + rr, ny);
                } else {
                    const int tiles_x = (nx + a.t2_tx - 1) / a.t2_tx;
                    bx0 = (tt % tiles_x) * a.t2_tx;
                    bnx = min(a.t2_tx, nx - bx0);
                    by0 = (tt / tiles_x) * a.t2_rows;
                    by1 = min(by0 + a.t2_rows, ny);
                }
                const int cnt = bnx * (by1 - by0);
                for (int q = (int)threadIdx.x; q < cnt; q += (int)blockDim.x) {
                    const int yy = by0 + q / bnx, xx = bx0 + q % bnx;
                    step_node<2, DT, CORR>(static_cast<const T *>(src), static_cast<T *>(dst), nx, ny, 1, ps, rs,
                                           relax, flag, xx, yy, 0);
                }
            }
            // every wave's stores done before the next tile reuses the LDS ring (and
            // before the release below)
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
        // publish iteration k: one release at agent scope, then, by the same thread,
        // the counters of the tiles that took part
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            for (int t = L; t < ntiles; t += G) {
                const int j = df_slot(a, t);
                if (2 * k < a.slots[j].run_steps)
                    __hip_atomic_store(a.slots[j].tdone + (t - a.tile_start[j]), a.base + k + 1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// Gather the domain flags of n slots into one array (read at poll time).
__global__ void k_gather_flags(const int *const *flags, int n, int *out) {
    for (int k = (int)(blockIdx.x * blockDim.x + threadIdx.x); k < n; k += (int)(gridDim.x * blockDim.x))
        out[k] = *flags[k];
}

}  // namespace lbm
