// pool.hip -- host side of the pool C ABI (include/lbm.h): arena allocator,
// admission, run tables and launches of many domains together.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <vector>

#include "lbm.h"
#include "lbm_internal.hpp"
#include "pool_kernels.hpp"

namespace lbm {

constexpr int kClasses = 16;  // (D2Q9, D3Q27) x 4 dtypes x (correction off, on)
constexpr int kSpinLog2 = 26;  // default bound of a grid-barrier wait: 2^26 polls
constexpr int kStagingRing = 8;  // pinned run-table buffers in use in turn
constexpr int kEpochRing = 64;   // completion events of recent runs and admissions
constexpr int64_t kEpochStream = INT64_MAX;  // "all work on the pool's stream" (no event)

static size_t round256(size_t v) { return (v + 255) / 256 * 256; }

// Device table of one class: descriptors, running tile counts, remaining steps.
// (descriptors | one-step tile starts | remaining steps | two-step tile starts)
static size_t class_table_bytes(int max_slots) {
    return round256(sizeof(SlotDesc) * (size_t)max_slots) + round256(sizeof(int) * ((size_t)max_slots + 1)) +
           round256(sizeof(int64_t) * (size_t)max_slots) + round256(sizeof(int) * ((size_t)max_slots + 1));
}

static int resolve_tuning(const lbm_pool_tuning *t, lbm_pool_tuning *out) {
    lbm_pool_tuning r{};
    if (t)
        r = *t;
    if (r.time_block < 0 || r.time_block > 2) {
        set_error("pool tuning: time_block must be 0, 1 or 2");
        return LBM_EINVAL;
    }
    if (r.time_rows < 0 || r.time_rows > 4096) {
        set_error("pool tuning: time_rows must lie in 0 .. 4096");
        return LBM_EINVAL;
    }
    if (r.spin_log2 < 0 || r.spin_log2 > 40) {
        set_error("pool tuning: spin_log2 must lie in 0 .. 40");
        return LBM_EINVAL;
    }
    if (r.spin_log2 == 0)
        r.spin_log2 = kSpinLog2;
    if (r.tile_x == 0)
        r.tile_x = 64;
    if (r.tile_y == 0)
        r.tile_y = std::max(1, 256 / r.tile_x);
    if (r.tile_x < 1 || r.tile_y < 1 || r.tile_x * r.tile_y > 256 || (r.tile_x * r.tile_y) % 64 != 0) {
        set_error("pool tile: tile_x * tile_y must be a multiple of 64 and <= 256");
        return LBM_EINVAL;
    }
    if (r.persistent != 0 && r.persistent != 1) {
        set_error("pool tuning: persistent must be 0 or 1");
        return LBM_EINVAL;
    }
    if (r.workgroups < 0) {
        set_error("pool tuning: workgroups must be >= 0");
        return LBM_EINVAL;
    }
    if (r.flat != 0 && r.flat != 1) {
        set_error("pool tuning: flat must be 0 or 1");
        return LBM_EINVAL;
    }
    if (r.row_fit != 0 && r.row_fit != 1) {
        set_error("pool tuning: row_fit must be 0 or 1");
        return LBM_EINVAL;
    }
    if (r.row_fit && r.flat) {
        set_error("pool tuning: row_fit and flat exclude each other");
        return LBM_EINVAL;
    }
    if (r.layout == LBM_LAYOUT_DEFAULT)
        r.layout = LBM_LAYOUT_ROWS;
    if (r.layout != LBM_LAYOUT_ROWS && r.layout != LBM_LAYOUT_PLANES) {
        set_error("pool tuning: bad layout");
        return LBM_EINVAL;
    }
    *out = r;
    return LBM_OK;
}

// Layout of a slot: the single-domain layout with the pool's tile and one
// node per thread (the pool kernels are the one-node-per-thread kind).
static int slot_layout(const lbm_config *cfg, const lbm_pool_tuning &t, Layout *L) {
    if (cfg && cfg->equilibrium != LBM_EQ_ENTROPIC) {
        set_error("pool slots run the entropic equilibrium only");
        return LBM_EINVAL;
    }
    if (cfg && cfg->z_halo) {
        set_error("pool slots are periodic domains (z_halo = 0)");
        return LBM_EINVAL;
    }
    if (cfg && cfg->lattice != LBM_D2Q9 && cfg->lattice != LBM_D3Q27) {
        set_error("pool slots run D2Q9 or D3Q27");
        return LBM_EINVAL;
    }
    lbm_tuning st{};
    st.block_x = t.tile_x;
    st.block_y = t.tile_y;
    st.plane_pad = -1;
    st.nodes_per_thread = 1;
    st.flags = 0;
    st.layout = t.layout;
    return validate_config(cfg, &st, L);
}

// class = 8 * (D3Q27) + 2 * dtype + correction
static int class_of(const lbm_config *cfg) {
    return (cfg->lattice == LBM_D3Q27 ? 8 : 0) + 2 * cfg->dtype + (cfg->bulk_correction ? 1 : 0);
}

using PoolStepFn = void (*)(PoolRunArgs);
template <int DIM, int DT>
static PoolStepFn pool_kernel_dt(bool corr, bool persistent) {
    if (corr)
        return persistent ? k_pool_persistent<DIM, DT, true> : k_pool_step<DIM, DT, true>;
    return persistent ? k_pool_persistent<DIM, DT, false> : k_pool_step<DIM, DT, false>;
}
template <int DIM>
static PoolStepFn pool_kernel(int dtype, bool corr, bool persistent) {
    switch (dtype) {
    case kDevF64:
        return pool_kernel_dt<DIM, kDevF64>(corr, persistent);
    case kDevMixed:
        return pool_kernel_dt<DIM, kDevMixed>(corr, persistent);
    case kDevF32:
        return pool_kernel_dt<DIM, kDevF32>(corr, persistent);
    default:
        return pool_kernel_dt<DIM, kF64>(corr, persistent);
    }
}

// Two steps per launch in pools.  One launch has one workgroup shape.  FP32
// storage: 512 threads; a slot whose row, rounded up to 64, fits them runs as
// whole-row tiles (two_step_rows_tile: floor(512 / w) sub-tiles of w lanes,
// each sweeping its rows), wider slots as column tiles of 512.  Whole
// rows need no halo columns: with the earlier 128 x 16 column tiles the
// batched workload's narrow rows read 1.46x the algorithmic bytes (the column
// halos' cache lines and the 2 + 2 extra rows of every 16), with whole rows
// 1.10x.  FP64 storage: column tiles of 128 plus the halo wavefront (192
// threads) and 16 rows.  Whole-row tiles of up to 128 nodes in 128-thread
// workgroups (two wavefronts, four workgroups per compute unit) ran slower on
// the batched workload, 399 against 461 solves/s: FP64 rows need the loads
// in flight that only wider workgroups keep.
//
// The tile-ordered persistent form (persistent tunings) gives FP32 workgroups
// 1024 threads, one per compute unit: twice the sub-tiles per tile, half the
// tiles to wait for and publish (batched workload, FP32: 363 against 382 us per
// step; launches per two steps ran slower with them, 322 against 312).
static int t2_block(int dtype, bool persistent) { return dtype == kF64 ? 192 : (persistent ? 1024 : 512); }
static int t2_cols(int dtype, bool persistent) { return dtype == kF64 ? 128 : (persistent ? 1024 : 512); }
// Rows per sweep, measured on the batched workload: 16 with two-step launches (FP32: 16
// rows 830 solves/s, 12: 821, 24: 821, 32: 809, 48: 778; FP64: 8 to 16 within 1 %, 32:
// 452); in the tile-ordered persistent form 16 for FP32 in its 1024-thread workgroups
// (us per step: 8 rows 368, 12 352, 16 344, 20 345, 32 363, 48 379) and 64 for FP64,
// where longer sweeps mean fewer tiles to wait for (413 against 385 solves/s with 16).
static int t2_rows_default(int dtype, bool persistent) {
    if (!persistent)
        return 16;
    return dtype == kF64 ? 64 : 16;
}
static bool t2_whole_rows(int dtype) { return dtype != kF64; }
static int t2_rows(const lbm_pool_tuning &t, int dtype) {
    return t.time_rows > 0 ? t.time_rows : t2_rows_default(dtype, t.persistent != 0);
}

// Two-step tiling of a D2Q9 slot: whole-row tiles of sub sub-tiles of R rows
// each when the padded row fits the workgroup (w > 0, FP32 storage), else
// column tiles of t2_cols x R.
struct T2Geom {
    int w = 0, sub = 0;
    int64_t tiles = 0;
};
static T2Geom t2_geom(int64_t nx, int64_t ny, int dtype, int R, bool persistent) {
    T2Geom g;
    const int B = t2_block(dtype, persistent), TX = t2_cols(dtype, persistent);
    const int64_t w = (nx + 63) / 64 * 64;
    if (t2_whole_rows(dtype) && w <= B) {
        g.w = (int)w;
        g.sub = B / g.w;
        g.tiles = (ny + (int64_t)g.sub * R - 1) / ((int64_t)g.sub * R);
    } else {
        g.tiles = ((nx + TX - 1) / TX) * ((ny + R - 1) / R);
    }
    return g;
}

// Slots that the tile-ordered persistent form may advance (D2Q9, FP64 or FP32
// deviation storage, row-interleaved layout, persistent two-step tuning) carry
// one 8-byte completion counter per two-step tile after their buffers.
static bool t2_counters(const lbm_config *cfg, const lbm_pool_tuning &t) {
    return t.persistent && t.time_block == 2 && t.layout == LBM_LAYOUT_ROWS && cfg->lattice == LBM_D2Q9 &&
           (cfg->dtype == kF64 || cfg->dtype == kDevF64);
}
static size_t t2_counter_bytes(const lbm_config *cfg, const lbm_pool_tuning &t) {
    if (!t2_counters(cfg, t))
        return 0;
    return round256(sizeof(int64_t) *
                    (size_t)t2_geom(cfg->nx, cfg->ny, cfg->dtype, t2_rows(t, cfg->dtype), t.persistent != 0).tiles);
}

struct Slot {
    bool used = false;
    bool reported = false;
    DomainState d{};
    size_t off = 0, bytes = 0;
    int64_t remaining = 0;
    bool failed = false;      // retired: its state left the equilibrium's domain
    bool broken = false;      // retired: a persistent launch that advanced it timed out at a barrier
    bool unverified = false;  // admitted without a synchronisation: initial state not checked yet
    bool persistent = false;  // advanced by a persistent launch since the last poll
    int64_t last_epoch = 0;   // epoch whose completion covers all work enqueued for the slot (0: none)
    int tiles_x = 0, tiles_y = 0, tiles = 0;
    int tw_shift = 0;  // row_fit: tile rows of 1 << tw_shift threads; 0: the workgroup's own shape
    int cls = 0;
    int64_t *tdone = nullptr;  // two-step tile counters of the tile-ordered persistent form
};

}  // namespace lbm

using namespace lbm;

struct lbm_pool {
    hipStream_t stream = nullptr;
    hipStream_t aux = nullptr;  // reads of slots whose work has completed
    char *arena = nullptr;
    size_t arena_bytes = 0;
    lbm_pool_tuning tun{};
    int max_slots = 0;
    std::vector<Slot> slots;
    std::map<size_t, size_t> free_blocks;  // offset -> size, inside the slot region
    size_t table_bytes = 0, class_bytes = 0;
    unsigned *barrier = nullptr;
    int *error = nullptr;
    // pinned host copies of class tables, used in turn; each buffer's event marks the
    // end of its last upload
    char *staging[kStagingRing] = {};
    hipEvent_t staging_ev[kStagingRing] = {};
    bool staging_used[kStagingRing] = {};
    int staging_next = 0;
    // epochs: an event recorded on the stream after each run and each unsynchronised
    // admission; epoch e lives in ring entry e % kEpochRing while ep_seq says so
    hipEvent_t ep_ev[kEpochRing] = {};
    int64_t ep_seq[kEpochRing] = {};
    int64_t epoch = 0;
    std::vector<int64_t> run_epoch;  // epoch of run r at index r - 1
    char *gather_host = nullptr;  // pinned: flag pointers, then flag values
    char *gather_dev = nullptr;
    int cu_count = 0;
    int64_t runs = 0, launches = 0;
    int64_t df_base = 0;  // tile-ordered form: above every counter value stored so far
};

namespace {

bool pool_alloc(lbm_pool *p, size_t bytes, size_t *off) {
    for (auto it = p->free_blocks.begin(); it != p->free_blocks.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t roff = it->first + bytes;
            p->free_blocks.erase(it);
            if (rest)
                p->free_blocks[roff] = rest;
            return true;
        }
    }
    return false;
}

void pool_free(lbm_pool *p, size_t off, size_t bytes) {
    auto it = p->free_blocks.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != p->free_blocks.end() && it->first + it->second == next->first) {
        it->second += next->second;
        p->free_blocks.erase(next);
    }
    if (it != p->free_blocks.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            p->free_blocks.erase(it);
        }
    }
}

int check_slot(lbm_pool *p, int32_t slot) {
    if (!p || slot < 0 || slot >= p->max_slots || !p->slots[slot].used) {
        set_error("NULL pool or slot not in use");
        return LBM_EINVAL;
    }
    return LBM_OK;
}

// Record the next epoch on the pool's stream (after everything enqueued so far).
hipError_t record_epoch(lbm_pool *p, int64_t *out) {
    const int64_t e = p->epoch + 1;
    const int k = (int)(e % kEpochRing);
    hipError_t r = hipEventRecord(p->ep_ev[k], p->stream);
    if (r != hipSuccess)
        return r;
    p->epoch = e;
    p->ep_seq[k] = e;
    *out = e;
    return hipSuccess;
}

// The event whose completion implies that of epoch e: its own, or, once the
// ring has moved on, the newer epoch recorded in its entry (later in the stream).
hipEvent_t epoch_event(const lbm_pool *p, int64_t e) { return p->ep_ev[e % kEpochRing]; }

// hipSuccess when epoch e (<= 0: nothing; kEpochStream: everything enqueued on
// the stream) has completed, hipErrorNotReady when not.
hipError_t epoch_query(lbm_pool *p, int64_t e) {
    if (e <= 0)
        return hipSuccess;
    if (e == kEpochStream)
        return hipStreamQuery(p->stream);
    return hipEventQuery(epoch_event(p, e));
}

hipError_t epoch_wait(lbm_pool *p, int64_t e) {
    if (e <= 0)
        return hipSuccess;
    if (e == kEpochStream)
        return hipStreamSynchronize(p->stream);
    return hipEventSynchronize(epoch_event(p, e));
}

// Next pinned staging buffer: wait until its previous upload has left it.
hipError_t acquire_staging(lbm_pool *p, int *idx) {
    const int k = p->staging_next;
    p->staging_next = (k + 1) % kStagingRing;
    if (p->staging_used[k]) {
        hipError_t e = hipEventSynchronize(p->staging_ev[k]);
        if (e != hipSuccess)
            return e;
        p->staging_used[k] = false;
    }
    *idx = k;
    return hipSuccess;
}

// Domain flags of the listed slots into vals (pinned), on stream s, synchronised.
// The gather area is used by one call at a time: every caller synchronises
// before it returns.
hipError_t gather_flags(lbm_pool *p, const std::vector<int> &which, hipStream_t s, int **vals_out) {
    const int n = (int)which.size();
    int **ptrs = reinterpret_cast<int **>(p->gather_host);
    int *vals = reinterpret_cast<int *>(p->gather_host + round256(sizeof(int *) * (size_t)p->max_slots));
    int *dvals = reinterpret_cast<int *>(p->gather_dev + round256(sizeof(int *) * (size_t)p->max_slots));
    *vals_out = vals;
    if (n == 0)
        return hipSuccess;
    for (int j = 0; j < n; ++j)
        ptrs[j] = p->slots[which[j]].d.flag;
    hipError_t e = hipMemcpyAsync(p->gather_dev, ptrs, sizeof(int *) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_gather_flags, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           (const int *const *)p->gather_dev, n, dvals);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(vals, dvals, sizeof(int) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    return e;
}

// Release everything the pool holds on the host and in the runtime.
void pool_free_host(lbm_pool *p) {
    for (int k = 0; k < kStagingRing; ++k) {
        if (p->staging[k])
            (void)hipHostFree(p->staging[k]);
        if (p->staging_ev[k])
            (void)hipEventDestroy(p->staging_ev[k]);
    }
    for (int k = 0; k < kEpochRing; ++k)
        if (p->ep_ev[k])
            (void)hipEventDestroy(p->ep_ev[k]);
    if (p->gather_host)
        (void)hipHostFree(p->gather_host);
    if (p->aux)
        (void)hipStreamDestroy(p->aux);
    delete p;
}

}  // namespace

extern "C" {

// Gather area: flag pointers and flag values of up to max_slots slots.
static size_t gather_bytes(int max_slots) {
    return round256(sizeof(int *) * (size_t)max_slots) + round256(sizeof(int) * (size_t)max_slots);
}

size_t lbm_pool_table_bytes(int32_t max_slots) {
    if (max_slots < 1 || max_slots > 65536)
        return 0;
    return (size_t)kClasses * class_table_bytes(max_slots) + 512 + gather_bytes(max_slots);
}

size_t lbm_pool_slot_bytes(const lbm_config *cfg, const lbm_pool_tuning *tuning) {
    lbm_pool_tuning t;
    Layout L;
    if (resolve_tuning(tuning, &t) != LBM_OK || slot_layout(cfg, t, &L) != LBM_OK)
        return 0;
    return round256(L.ws_bytes) + t2_counter_bytes(cfg, t);
}

int lbm_pool_create(int32_t max_slots, const lbm_pool_tuning *tuning, void *arena, size_t arena_bytes,
                    void *stream, lbm_pool **out) {
    lbm_pool_tuning t;
    int rc = resolve_tuning(tuning, &t);
    if (rc != LBM_OK)
        return rc;
    const size_t tb = lbm_pool_table_bytes(max_slots);
    if (!arena || !out || tb == 0 || arena_bytes <= tb || reinterpret_cast<uintptr_t>(arena) % 256 != 0) {
        set_error("pool: NULL arena/out, max_slots outside 1..65536, arena too small or misaligned");
        return LBM_EINVAL;
    }
    lbm_pool *p = new (std::nothrow) lbm_pool();
    if (!p) {
        set_error("host allocation failed");
        return LBM_EINVAL;
    }
    p->stream = static_cast<hipStream_t>(stream);
    p->arena = static_cast<char *>(arena);
    p->arena_bytes = arena_bytes;
    p->tun = t;
    p->max_slots = max_slots;
    p->slots.resize(max_slots);
    p->class_bytes = class_table_bytes(max_slots);
    p->table_bytes = tb;
    p->barrier = reinterpret_cast<unsigned *>(p->arena + (size_t)kClasses * p->class_bytes);
    p->error = reinterpret_cast<int *>(p->arena + (size_t)kClasses * p->class_bytes + 256);
    const size_t slot_region = (arena_bytes - tb) / 256 * 256;
    if (slot_region > 0)
        p->free_blocks[tb] = slot_region;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&p->cu_count, hipDeviceAttributeMultiprocessorCount, dev);
    p->gather_dev = p->arena + (size_t)kClasses * p->class_bytes + 512;
    for (int k = 0; k < kStagingRing && e == hipSuccess; ++k) {
        e = hipHostMalloc(reinterpret_cast<void **>(&p->staging[k]), p->class_bytes, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&p->staging_ev[k], hipEventDisableTiming);
    }
    for (int k = 0; k < kEpochRing && e == hipSuccess; ++k)
        e = hipEventCreateWithFlags(&p->ep_ev[k], hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&p->gather_host), gather_bytes(max_slots), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking);
    if (e == hipSuccess) {
        // barrier counter and error word (and the words between them) start at zero
        hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, p->stream, reinterpret_cast<int *>(p->barrier), 128);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        pool_free_host(p);
        return hip_fail(e, "pool create");
    }
    *out = p;
    return LBM_OK;
}

// Admission: slot, arena block, tile counts, then f = f^eq(rho, u) enqueued.
// sync: wait for the initialisation and check the initial state now; else
// leave the check to the next poll or collect.
static int pool_admit_impl(lbm_pool *p, const lbm_config *cfg, const double *rho, const double *u,
                           int64_t nsteps, int32_t *slot, bool sync) {
    if (!p || !cfg || !rho || !u || !slot || nsteps < 0) {
        set_error("pool admit: NULL argument or negative step budget");
        return LBM_EINVAL;
    }
    Layout L;
    int rc = slot_layout(cfg, p->tun, &L);
    if (rc != LBM_OK)
        return rc;
    int k = -1;
    for (int i = 0; i < p->max_slots; ++i)
        if (!p->slots[i].used) {
            k = i;
            break;
        }
    if (k < 0) {
        set_error("pool admit: no free slot");
        return LBM_EBUSY;
    }
    const size_t counter_bytes = t2_counter_bytes(cfg, p->tun);
    const size_t bytes = round256(L.ws_bytes) + counter_bytes;
    // tile counts first, so that nothing is enqueued for a domain the pool refuses
    const int64_t block = (int64_t)L.block_x * L.block_y;
    int64_t tw = L.block_x, th = L.block_y;
    int tw_shift = 0;
    if (p->tun.row_fit) {
        // narrowest power-of-two row width from 64 that covers the padded row
        const int64_t pitch = L.layout == LBM_LAYOUT_ROWS ? L.ps : cfg->nx;
        int shift = 6;
        while ((int64_t)1 << shift < pitch && shift < 8 && block % ((int64_t)2 << shift) == 0)
            ++shift;
        tw_shift = shift;
        tw = (int64_t)1 << shift;
        th = block / tw;
    }
    const int64_t tiles_x = (cfg->nx + tw - 1) / tw, tiles_y = (cfg->ny + th - 1) / th;
    const int64_t tiles = p->tun.flat ? (L.n + block - 1) / block : tiles_x * tiles_y * cfg->nz;
    if (tiles > (int64_t)1 << 30 || counter_bytes > ((size_t)1 << 30)) {
        set_error("pool admit: domain has too many tiles");
        return LBM_EINVAL;
    }
    size_t off = 0;
    if (!pool_alloc(p, bytes, &off)) {
        set_error("pool admit: no free arena block large enough");
        return LBM_ENOMEM;
    }
    Slot &s = p->slots[k];
    s = Slot{};
    rc = domain_bind_and_init(s.d, cfg, L, p->arena + off, rho, u, p->stream);
    if (rc == LBM_OK && counter_bytes > 0) {
        // tile counters start at zero, below every value a launch waits for
        s.tdone = reinterpret_cast<int64_t *>(p->arena + off + round256(L.ws_bytes));
        hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(256), 0, p->stream, reinterpret_cast<int *>(s.tdone),
                           (int)(counter_bytes / sizeof(int)));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            rc = hip_fail(e, "pool counter clear");
    }
    int flag = 0;
    if (rc == LBM_OK && sync)
        rc = domain_read_flag(s.d, p->stream, &flag);
    if (rc == LBM_OK && flag) {
        set_error("initial state has a node with rho <= 0 or |u_alpha| >= 1");
        rc = LBM_EDOMAIN;
    }
    int64_t ep = 0;
    if (rc == LBM_OK && !sync) {
        hipError_t e = record_epoch(p, &ep);
        if (e != hipSuccess)
            rc = hip_fail(e, "pool admit event");
    }
    if (rc != LBM_OK) {
        // (an enqueued initialisation writes only this block, which stays free for
        // later admissions enqueued behind it)
        pool_free(p, off, bytes);
        s = Slot{};
        return rc;
    }
    s.used = true;
    s.off = off;
    s.bytes = bytes;
    s.remaining = nsteps;
    s.reported = false;
    s.unverified = !sync;
    s.last_epoch = ep;
    s.tw_shift = tw_shift;
    s.tiles_x = (int)tiles_x;
    s.tiles_y = (int)tiles_y;
    s.tiles = (int)tiles;
    s.cls = class_of(cfg);
    *slot = k;
    return LBM_OK;
}

int lbm_pool_admit(lbm_pool *p, const lbm_config *cfg, const double *rho, const double *u, int64_t nsteps,
                   int32_t *slot) {
    return pool_admit_impl(p, cfg, rho, u, nsteps, slot, true);
}

int lbm_pool_admit_async(lbm_pool *p, const lbm_config *cfg, const double *rho, const double *u, int64_t nsteps,
                         int32_t *slot) {
    return pool_admit_impl(p, cfg, rho, u, nsteps, slot, false);
}

// Enqueue the launches of every class with active slots; a slot that took part
// gets last_epoch = -1 (resolved by the caller).
//
// In a run of k steps slot j of a class takes s_j = min(k, remaining_j)
// steps.  One step per launch: launch s covers the slots with s_j > s, a
// prefix of the slots in order of decreasing remaining steps.  Two steps per
// launch (D2Q9): launch L covers the slots with s_j >= 2 L + 2 in two-step
// tiles, followed, when some slot has s_j = 2 L + 1, by a one-step launch over
// those; the slots are listed in two parts (whole-row, then column tiles),
// each in order of decreasing s_j, so that both sets are ranges of the list.
// A slot's buffer parity advances once per launch that covers it.
static int pool_run_classes(lbm_pool *p, int64_t k, bool &any) {
    for (int c = 0; c < kClasses; ++c) {
        std::vector<int> order;
        for (int i = 0; i < p->max_slots; ++i)
            if (p->slots[i].used && p->slots[i].remaining > 0 && p->slots[i].cls == c)
                order.push_back(i);
        if (order.empty())
            continue;
        any = true;
        auto steps_of = [&](int i) { return std::min<int64_t>(k, p->slots[i].remaining); };
        const int cdim = c >= 8 ? 3 : 2, cdtype = (c % 8) / 2;
        const bool corr = (c & 1) != 0;
        // two steps per launch: D2Q9 FP64 / FP32_DEV row-interleaved slots, when those
        // taking at least two steps hold as many nodes as a single domain needs for
        // two steps per launch to pay (2048^2 FP32, 1024^2 FP64; a workgroup sweeps its
        // rows one after another): with a few small slots the one-step form answers
        // sooner (served p50 latency 44 against 18 ms)
        bool two = p->tun.time_block == 2 && cdim == 2 && (cdtype == kF64 || cdtype == kDevF64) &&
                   p->tun.layout == LBM_LAYOUT_ROWS;
        size_t class_buf_bytes = 0;
        int64_t two_nodes = 0;
        for (int i : order) {
            class_buf_bytes += p->slots[i].d.L.buf_bytes;
            if (steps_of(i) >= 2)
                two_nodes += p->slots[i].d.L.n;
        }
        two = two && two_nodes >= (cdtype == kF64 ? (int64_t)1 << 20 : (int64_t)1 << 22);
        const bool pers = p->tun.persistent != 0;
        const int B = t2_block(cdtype, pers), TX = t2_cols(cdtype, pers);
        const int R = t2_rows(p->tun, cdtype);
        auto geom = [&](int i) { return t2_geom(p->slots[i].d.cfg.nx, p->slots[i].d.cfg.ny, cdtype, R, pers); };
        auto whole_w = [&](int i) { return geom(i).w; };  // whole-row sub-tile width, 0 for column tiles
        int nw = 0;  // slots in the whole-row part
        if (two) {
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                const bool wa = whole_w(a) > 0, wb = whole_w(b) > 0;
                if (wa != wb)
                    return wa;
                return p->slots[a].remaining > p->slots[b].remaining;
            });
            for (int i : order)
                nw += whole_w(i) > 0 ? 1 : 0;
        } else {
            std::stable_sort(order.begin(), order.end(),
                             [&](int a, int b) { return p->slots[a].remaining > p->slots[b].remaining; });
        }
        const int n = (int)order.size();
        int64_t smax = 0;
        for (int i : order)
            smax = std::max(smax, steps_of(i));
        // tile-ordered persistent form: all two-step iterations in one launch (runs
        // of up to 2^30 steps; longer ones take the launch-per-iteration form)
        const bool df = two && p->tun.persistent && smax <= ((int64_t)1 << 30);
        std::vector<int> tile_start(n + 1, 0), two_start(n + 1, 0);
        std::vector<int> sub(n, 0);
        for (int j = 0; j < n; ++j) {
            const Slot &sj = p->slots[order[j]];
            int64_t t2 = 0;
            if (two) {
                const T2Geom g = geom(order[j]);
                sub[j] = g.sub;
                t2 = g.tiles;
            }
            if ((int64_t)tile_start[j] + sj.tiles > INT32_MAX || (int64_t)two_start[j] + t2 > INT32_MAX) {
                set_error("pool run: more than 2^31 - 1 tiles in one class");
                return LBM_EINVAL;
            }
            tile_start[j + 1] = tile_start[j] + sj.tiles;
            two_start[j + 1] = two_start[j] + (int)t2;
        }
        // Host copy of the class table in the next pinned staging buffer (waiting
        // only if that buffer's previous upload has not left it yet).  The device
        // table is overwritten in stream order, after the previous run's kernels.
        int sb = 0;
        {
            hipError_t e = acquire_staging(p, &sb);
            if (e != hipSuccess)
                return hip_fail(e, "pool staging wait");
        }
        char *staging = p->staging[sb];
        const size_t off_desc = 0, off_start = round256(sizeof(SlotDesc) * p->max_slots),
                     off_rem = off_start + round256(sizeof(int) * (p->max_slots + 1)),
                     off_two = off_rem + round256(sizeof(int64_t) * p->max_slots);
        SlotDesc *desc = reinterpret_cast<SlotDesc *>(staging + off_desc);
        int *starts = reinterpret_cast<int *>(staging + off_start);
        int64_t *rem = reinterpret_cast<int64_t *>(staging + off_rem);
        int *starts2 = reinterpret_cast<int *>(staging + off_two);
        for (int j = 0; j < n; ++j) {
            const Slot &s = p->slots[order[j]];
            SlotDesc d{};
            d.buf[0] = s.d.buf[0];
            d.buf[1] = s.d.buf[1];
            d.nx = (int)s.d.cfg.nx;
            d.ny = (int)s.d.cfg.ny;
            d.nz = (int)s.d.cfg.nz;
            d.tiles_x = s.tiles_x;
            d.tiles_y = s.tiles_y;
            d.tw_shift = s.tw_shift;
            d.t2_w = two ? whole_w(order[j]) : 0;
            d.t2_sub = sub[j];
            d.run_steps = df ? (int)steps_of(order[j]) : 0;
            d.tdone = s.tdone;
            d.parity = s.d.cur;
            d.ps = s.d.L.ps;
            d.rs = s.d.L.rs;
            d.relax = s.d.relax;
            d.flag = s.d.flag;
            desc[j] = d;
            rem[j] = s.remaining;
        }
        std::memcpy(starts, tile_start.data(), sizeof(int) * (n + 1));
        std::memcpy(starts2, two_start.data(), sizeof(int) * (n + 1));
        // two-step launch parameters: block, dynamic LDS (the larger need of the two tile
        // forms: whole-row with the most sub-tiles, columns) and store kind
        const size_t elem = cdtype == kF64 ? 8 : 4;
        const bool nt = t2_nt_stores(class_buf_bytes);
        const size_t lds = nw > 0 ? std::max(t2_lds_bytes(TX, elem), t2_rows_lds_bytes(B / 64, 64, elem))
                                  : t2_lds_bytes(TX, elem);
        void (*fd)(PoolRunArgs) = nullptr;
        int64_t G = 0;
        if (df) {
            fd = cdtype == kF64 ? (corr ? (nt ? k_pool_df2<kF64, true, true> : k_pool_df2<kF64, true, false>)
                                        : (nt ? k_pool_df2<kF64, false, true> : k_pool_df2<kF64, false, false>))
                                : (corr ? (nt ? k_pool_df2<kDevF64, true, true> : k_pool_df2<kDevF64, true, false>)
                                        : (nt ? k_pool_df2<kDevF64, false, true> : k_pool_df2<kDevF64, false, false>));
            int per_cu = 0;
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fd), B, lds);
            if (e != hipSuccess)
                return hip_fail(e, "pool occupancy query");
            G = (int64_t)per_cu * p->cu_count;
            if (p->tun.workgroups > 0)
                G = std::min<int64_t>(G, p->tun.workgroups);
            // as few workgroups as give every one the same number of tiles, m or m - 1
            const int64_t T = two_start[n];
            G = std::max<int64_t>(1, std::min<int64_t>(G, T));
            const int64_t m = (T + G - 1) / G;
            G = (T + m - 1) / m;
        }
        char *table = p->arena + (size_t)c * p->class_bytes;
        hipError_t e = hipMemcpyAsync(table, staging, p->class_bytes, hipMemcpyHostToDevice, p->stream);
        if (e == hipSuccess)
            e = hipEventRecord(p->staging_ev[sb], p->stream);
        if (e != hipSuccess)
            return hip_fail(e, "pool table upload");
        p->staging_used[sb] = true;

        PoolRunArgs a{};
        a.slots = reinterpret_cast<const SlotDesc *>(table + off_desc);
        a.tile_start = reinterpret_cast<const int *>(table + off_start);
        a.remaining = reinterpret_cast<const int64_t *>(table + off_rem);
        a.n = n;
        a.barrier = p->barrier;
        a.error = p->error;
        a.spin_limit = 1ll << p->tun.spin_log2;
        a.flat = p->tun.flat;
        const int dim = cdim, dtype = cdtype;
        PoolStepFn fn = dim == 3 ? pool_kernel<3>(dtype, corr, p->tun.persistent)
                                 : pool_kernel<2>(dtype, corr, p->tun.persistent);
        dim3 block(p->tun.tile_x, p->tun.tile_y);
        if (two) {
            void (*fn2)(PoolRunArgs) =
                dtype == kF64 ? (corr ? (nt ? k_pool_step2<kF64, true, true> : k_pool_step2<kF64, true, false>)
                                      : (nt ? k_pool_step2<kF64, false, true> : k_pool_step2<kF64, false, false>))
                              : (corr ? (nt ? k_pool_step2<kDevF64, true, true> : k_pool_step2<kDevF64, true, false>)
                                      : (nt ? k_pool_step2<kDevF64, false, true> : k_pool_step2<kDevF64, false, false>));
            PoolStepFn fn1 = pool_kernel<2>(dtype, corr, false);
            // the larger LDS need of the two tile forms (whole-row: the most sub-tiles)
            PoolRunArgs a2 = a;
            a2.tile_start = reinterpret_cast<const int *>(table + off_two);
            a2.t2_tx = TX;
            a2.t2_rows = R;
            a2.t2_R = R;
            if (df) {
                a2.base = p->df_base;
                a2.step0 = 0;
                a2.nsteps = 0;
                void *args[] = {&a2};
                e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fd), dim3((unsigned)G), dim3((unsigned)B),
                                               args, (unsigned)lds, p->stream);
                if (e != hipSuccess)
                    return hip_fail(e, "pool tile-ordered launch");
                p->launches++;
                p->df_base += (smax + 1) / 2 + 1;
            }
            // s_j of the list, and the number of slots of each part with s_j >= m
            std::vector<int64_t> sj(n);
            for (int j = 0; j < n; ++j)
                sj[j] = steps_of(order[j]);
            auto count_ge = [&](int lo, int hi, int64_t m) {
                int q = lo;
                while (q < hi && sj[q] >= m)
                    ++q;
                return q;
            };
            auto launch = [&](void (*f)(PoolRunArgs), PoolRunArgs args, int t0, int t1, dim3 blk, size_t shm) {
                if (t1 <= t0)
                    return;
                args.tile_base = t0;
                hipLaunchKernelGGL(f, dim3((unsigned)(t1 - t0)), blk, (unsigned)shm, p->stream, args);
                p->launches++;
            };
            for (int64_t L = 0; !df && 2 * L + 1 <= smax; ++L) {
                a2.step0 = (int)L;
                a2.nsteps = 2;
                // two-step tiles of the slots with s_j >= 2 L + 2: a prefix of each part
                const int p1 = count_ge(0, nw, 2 * L + 2), p2 = count_ge(nw, n, 2 * L + 2);
                if (p1 == nw) {
                    launch(fn2, a2, 0, two_start[p2], dim3((unsigned)B), lds);
                } else {
                    launch(fn2, a2, 0, two_start[p1], dim3((unsigned)B), lds);
                    launch(fn2, a2, two_start[nw], two_start[p2], dim3((unsigned)B), lds);
                }
                // one-step tiles of the slots whose last step is 2 L + 1: a range of each part
                const int q1 = count_ge(0, nw, 2 * L + 1), q2 = count_ge(nw, n, 2 * L + 1);
                a.step0 = (int)L;
                a.nsteps = 1;
                if (q1 == nw && p2 == nw) {
                    launch(fn1, a, tile_start[p1], tile_start[q2], block, 0);
                } else {
                    launch(fn1, a, tile_start[p1], tile_start[q1], block, 0);
                    launch(fn1, a, tile_start[p2], tile_start[q2], block, 0);
                }
            }
            e = hipGetLastError();
            if (e != hipSuccess)
                return hip_fail(e, "pool two-step launch");
        } else if (p->tun.persistent) {
            const int64_t steps = steps_of(order[0]);
            int per_cu = 0;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, p->tun.tile_x * p->tun.tile_y, 0);
            if (e != hipSuccess)
                return hip_fail(e, "pool occupancy query");
            int64_t G = (int64_t)per_cu * p->cu_count;
            if (p->tun.workgroups > 0)
                G = std::min<int64_t>(G, p->tun.workgroups);
            G = std::max<int64_t>(1, std::min<int64_t>(G, tile_start[n]));
            // run in chunks so the barrier counter stays far from 2^32
            const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(1 << 20, (int64_t)0xF0000000u / G));
            for (int64_t s0 = 0; s0 < steps; s0 += chunk) {
                hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, p->stream, reinterpret_cast<int *>(p->barrier), 1);
                a.step0 = (int)s0;
                a.nsteps = (int)std::min<int64_t>(chunk, steps - s0);
                void *args[] = {&a};
                e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3((unsigned)G), block, args, 0,
                                               p->stream);
                if (e != hipSuccess)
                    return hip_fail(e, "pool persistent launch");
                p->launches++;
            }
        } else {
            const int64_t steps = steps_of(order[0]);
            for (int64_t s = 0; s < steps; ++s) {
                int cnt = 0;
                while (cnt < n && p->slots[order[cnt]].remaining > s)
                    ++cnt;
                const int P = tile_start[cnt];
                if (P == 0)
                    break;
                a.step0 = (int)s;
                a.nsteps = 1;
                a.tile_base = 0;
                hipLaunchKernelGGL(fn, dim3((unsigned)P), block, 0, p->stream, a);
                p->launches++;
            }
            e = hipGetLastError();
            if (e != hipSuccess)
                return hip_fail(e, "pool step launch");
        }
        for (int j = 0; j < n; ++j) {
            Slot &s = p->slots[order[j]];
            const int64_t done = std::min<int64_t>(k, s.remaining);
            s.d.cur ^= (int)((two ? done / 2 + done % 2 : done) & 1);  // one swap per launch
            s.d.steps += done;
            s.remaining -= done;
            s.persistent = s.persistent || (p->tun.persistent && (!two || df));
            s.last_epoch = -1;  // set by the caller, once the run's epoch is recorded
        }
    }
    return LBM_OK;
}

int lbm_pool_run(lbm_pool *p, int64_t k) {
    if (!p || k < 0) {
        set_error("pool run: NULL pool or negative step count");
        return LBM_EINVAL;
    }
    if (k == 0)
        return LBM_OK;
    bool any = false;
    int rc = pool_run_classes(p, k, any);
    if (!any)
        return rc;
    int64_t ep = kEpochStream;
    hipError_t e = record_epoch(p, &ep);
    if (e == hipSuccess) {
        p->runs++;
        p->run_epoch.push_back(ep);
    } else {
        ep = kEpochStream;  // no event: waits for these slots take the whole stream
    }
    for (Slot &s : p->slots)
        if (s.used && s.last_epoch == -1)
            s.last_epoch = ep;
    if (rc != LBM_OK)
        return rc;
    if (e != hipSuccess)
        return hip_fail(e, "pool run event");
    return LBM_OK;
}

int lbm_pool_poll(lbm_pool *p, int32_t *done, int32_t capacity, int32_t *count) {
    if (!p || !count || capacity < 0 || (capacity > 0 && !done)) {
        set_error("pool poll: bad arguments");
        return LBM_EINVAL;
    }
    int err = 0;
    hipError_t e = hipMemcpyAsync(&err, p->error, sizeof(int), hipMemcpyDeviceToHost, p->stream);
    // domain flags of the slots still running, and of those admitted without a check:
    // a slot whose state left the equilibrium's domain is retired (its remaining
    // steps are dropped)
    std::vector<int> check;
    for (int i = 0; i < p->max_slots; ++i) {
        const Slot &s = p->slots[i];
        if (s.used && !s.failed && !s.broken && (s.remaining > 0 || s.unverified))
            check.push_back(i);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(p->stream);  // every enqueued run and initialisation has completed
    int *vals = nullptr;
    if (e == hipSuccess)
        e = gather_flags(p, check, p->stream, &vals);
    if (e != hipSuccess)
        return hip_fail(e, "pool poll synchronise");
    for (int j = 0; j < (int)check.size(); ++j) {
        Slot &s = p->slots[check[j]];
        s.unverified = false;
        if (vals[j]) {
            s.failed = true;
            s.remaining = 0;
        }
    }
    if (err) {
        // a persistent launch stopped at a timed-out wait: the slots such
        // launches advanced hold the state of an unknown step; retire them, reset
        // the barrier words, and list them at the next poll
        for (Slot &s : p->slots)
            if (s.used && s.persistent) {
                s.broken = true;
                s.remaining = 0;
            }
        hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, p->stream, reinterpret_cast<int *>(p->barrier), 128);
        e = hipGetLastError();
        if (e == hipSuccess)
            e = hipStreamSynchronize(p->stream);
        for (Slot &s : p->slots)
            s.persistent = false;
        *count = 0;
        if (e != hipSuccess)
            return hip_fail(e, "pool barrier reset");
        set_error("pool: a persistent launch timed out at a grid barrier or a tile wait; the slots it "
                  "advanced are retired (device_error) and listed by the next poll");
        return LBM_EDEVICE;
    }
    for (Slot &s : p->slots)
        s.persistent = false;
    int32_t c = 0;
    for (int i = 0; i < p->max_slots && c < capacity; ++i) {
        Slot &s = p->slots[i];
        if (s.used && s.remaining == 0 && !s.reported) {
            s.reported = true;
            done[c++] = i;
        }
    }
    *count = c;
    return LBM_OK;
}

int lbm_pool_collect(lbm_pool *p, int64_t after_run, int32_t *done, int32_t capacity, int32_t *count) {
    if (!p || !count || capacity < 0 || (capacity > 0 && !done)) {
        set_error("pool collect: bad arguments");
        return LBM_EINVAL;
    }
    hipError_t e = hipSuccess;
    if (after_run >= 1 && after_run <= p->runs)
        e = epoch_wait(p, p->run_epoch[(size_t)(after_run - 1)]);
    // initial states of slots admitted without a check, where the initialisation is done
    std::vector<int> check;
    for (int i = 0; i < p->max_slots && e == hipSuccess; ++i) {
        const Slot &s = p->slots[i];
        if (s.used && s.unverified) {
            // the admission's own epoch precedes every later one, so last_epoch covers it
            const hipError_t q = epoch_query(p, s.last_epoch);
            if (q == hipSuccess)
                check.push_back(i);
            else if (q != hipErrorNotReady)
                e = q;
        }
    }
    int *vals = nullptr;
    if (e == hipSuccess)
        e = gather_flags(p, check, p->aux, &vals);
    if (e != hipSuccess)
        return hip_fail(e, "pool collect");
    for (int j = 0; j < (int)check.size(); ++j) {
        Slot &s = p->slots[check[j]];
        s.unverified = false;
        if (vals[j]) {
            s.failed = true;
            s.remaining = 0;  // its queued steps still run on its own block; nothing reads them
        }
    }
    int32_t c = 0;
    for (int i = 0; i < p->max_slots && c < capacity; ++i) {
        Slot &s = p->slots[i];
        if (!s.used || s.remaining != 0 || s.reported || s.unverified)
            continue;
        const hipError_t q = epoch_query(p, s.last_epoch);
        if (q == hipErrorNotReady)
            continue;
        if (q != hipSuccess)
            return hip_fail(q, "pool collect event");
        s.reported = true;
        done[c++] = i;
    }
    *count = c;
    return LBM_OK;
}

// Stream for a read of the slot: the second stream once the slot's work has
// completed (later runs keep going), else the pool's stream.
static int read_stream(lbm_pool *p, const Slot &s, hipStream_t *out) {
    const hipError_t q = epoch_query(p, s.last_epoch);
    if (q == hipSuccess) {
        *out = p->aux;
        return LBM_OK;
    }
    if (q != hipErrorNotReady)
        return hip_fail(q, "pool slot event");
    *out = p->stream;
    return LBM_OK;
}

int lbm_pool_moments(lbm_pool *p, int32_t slot, double *rho, double *u, lbm_diag *diag) {
    int rc = check_slot(p, slot);
    if (rc != LBM_OK)
        return rc;
    Slot &s = p->slots[slot];
    if (s.broken) {
        set_error("slot retired after a timed-out persistent launch: its state is not that of a known step");
        return LBM_EDEVICE;
    }
    hipStream_t st;
    rc = read_stream(p, s, &st);
    if (rc != LBM_OK)
        return rc;
    return domain_moments(s.d, st, rho, u, diag);
}

int lbm_pool_get_populations(lbm_pool *p, int32_t slot, double *out) {
    int rc = check_slot(p, slot);
    if (rc != LBM_OK)
        return rc;
    if (!out) {
        set_error("NULL output");
        return LBM_EINVAL;
    }
    Slot &s = p->slots[slot];
    if (s.broken) {
        set_error("slot retired after a timed-out persistent launch: its state is not that of a known step");
        return LBM_EDEVICE;
    }
    hipStream_t st;
    rc = read_stream(p, s, &st);
    if (rc != LBM_OK)
        return rc;
    return domain_export(s.d, st, out);
}

int lbm_pool_release(lbm_pool *p, int32_t slot) {
    int rc = check_slot(p, slot);
    if (rc != LBM_OK)
        return rc;
    Slot &s = p->slots[slot];
    // the block may be reused at once: the work enqueued for this slot must be done
    // (reads on the second stream are synchronous and already are)
    hipError_t e = epoch_wait(p, s.last_epoch);
    if (e != hipSuccess)
        return hip_fail(e, "pool release wait");
    pool_free(p, s.off, s.bytes);
    s = Slot{};
    return LBM_OK;
}

int lbm_pool_stats_get(lbm_pool *p, lbm_pool_stats *st) {
    if (!p || !st) {
        set_error("NULL pool or stats");
        return LBM_EINVAL;
    }
    st->max_slots = p->max_slots;
    st->used_slots = 0;
    for (const Slot &s : p->slots)
        st->used_slots += s.used ? 1 : 0;
    st->arena_bytes = (int64_t)p->arena_bytes;
    st->free_bytes = 0;
    st->largest_free_block = 0;
    for (const auto &b : p->free_blocks) {
        st->free_bytes += (int64_t)b.second;
        st->largest_free_block = std::max<int64_t>(st->largest_free_block, (int64_t)b.second);
    }
    st->runs = p->runs;
    st->launches = p->launches;
    return LBM_OK;
}

int lbm_pool_slot_info(lbm_pool *p, int32_t slot, lbm_slot_info *info) {
    if (!p || !info || slot < 0 || slot >= p->max_slots) {
        set_error("NULL pool/info or slot out of range");
        return LBM_EINVAL;
    }
    const Slot &s = p->slots[slot];
    info->used = s.used ? 1 : 0;
    info->finished = (s.used && s.remaining == 0) ? 1 : 0;
    info->steps_done = s.used ? s.d.steps : 0;
    info->steps_remaining = s.used ? s.remaining : 0;
    info->bytes = s.used ? (int64_t)s.bytes : 0;
    info->domain_error = (s.used && s.failed) ? 1 : 0;
    info->device_error = (s.used && s.broken) ? 1 : 0;
    return LBM_OK;
}

int lbm_pool_destroy(lbm_pool *p) {
    if (!p)
        return LBM_OK;
    hipError_t e = hipStreamSynchronize(p->stream);
    const hipError_t e2 = hipStreamSynchronize(p->aux);
    if (e == hipSuccess)
        e = e2;
    pool_free_host(p);
    if (e != hipSuccess)
        return hip_fail(e, "pool destroy synchronise");
    return LBM_OK;
}

}  // extern "C"
