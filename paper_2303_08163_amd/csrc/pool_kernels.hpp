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

namespace lbm {

struct SlotDesc {
    void *buf[2];
    int nx, ny, nz;
    int tiles_x, tiles_y;
    int parity;    // buffer holding the state at the start of the run
    int tw_shift;  // > 0: tiles are rows of 1 << tw_shift threads (row fit); 0: blockDim's shape
    int t2_w;      // two-step launches: > 0: whole-row sub-tiles of t2_w lanes, t2_sub per
    int t2_sub;    //   workgroup (two_step_rows_tile); 0: column tiles (two_step_tile)
    int pad_;
    int64_t ps, rs;
    Relax relax;
    int *flag;
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
__global__ __launch_bounds__(512) void k_pool_step2(PoolRunArgs a) {
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

// Gather the domain flags of n slots into one array (read at poll time).
__global__ void k_gather_flags(const int *const *flags, int n, int *out) {
    for (int k = (int)(blockIdx.x * blockDim.x + threadIdx.x); k < n; k += (int)(gridDim.x * blockDim.x))
        out[k] = *flags[k];
}

}  // namespace lbm
