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
constexpr long long kSpinLimit = 1ll << 26;

static size_t round256(size_t v) { return (v + 255) / 256 * 256; }

// Device table of one class: descriptors, running tile counts, remaining steps.
static size_t class_table_bytes(int max_slots) {
    return round256(sizeof(SlotDesc) * (size_t)max_slots) + round256(sizeof(int) * ((size_t)max_slots + 1)) +
           round256(sizeof(int64_t) * (size_t)max_slots);
}

static int resolve_tuning(const lbm_pool_tuning *t, lbm_pool_tuning *out) {
    lbm_pool_tuning r{};
    if (t)
        r = *t;
    if (r.time_block < 0 || r.time_block > 2) {
        set_error("pool tuning: time_block must be 0, 1 or 2");
        return LBM_EINVAL;
    }
    if (r.time_block == 2 && r.persistent) {
        set_error("pool tuning: time_block = 2 is not with persistent");
        return LBM_EINVAL;
    }
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

// Two-step pool tiles: 128 columns by 16 rows.  On the batched workload (rows
// 32..512 wide) 128 columns gave 730 solves/s FP32 and 461 FP64 against 708
// and 457 with 64: fewer re-read halo lines outweigh the idle lanes of the
// narrow slots.
constexpr int kPoolT2Tx = 128, kPoolT2Rows = 16;

struct Slot {
    bool used = false;
    bool reported = false;
    DomainState d{};
    size_t off = 0, bytes = 0;
    int64_t remaining = 0;
    bool failed = false;  // retired at poll: its state left the equilibrium's domain
    int tiles_x = 0, tiles_y = 0, tiles = 0;
    int tw_shift = 0;  // row_fit: tile rows of 1 << tw_shift threads; 0: the workgroup's own shape
    int cls = 0;
};

}  // namespace lbm

using namespace lbm;

struct lbm_pool {
    hipStream_t stream = nullptr;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    lbm_pool_tuning tun{};
    int max_slots = 0;
    std::vector<Slot> slots;
    std::map<size_t, size_t> free_blocks;  // offset -> size, inside the slot region
    size_t table_bytes = 0, class_bytes = 0;
    unsigned *barrier = nullptr;
    int *error = nullptr;
    char *staging = nullptr;  // pinned host copy of one class table
    char *gather_host = nullptr;  // pinned: flag pointers, then flag values
    char *gather_dev = nullptr;
    hipEvent_t staging_done = nullptr;
    bool staging_pending = false;
    int cu_count = 0;
    int64_t runs = 0, launches = 0;
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
    return round256(L.ws_bytes);
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
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&p->staging), p->class_bytes, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&p->gather_host), gather_bytes(max_slots), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&p->staging_done, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (p->staging)
            (void)hipHostFree(p->staging);
        if (p->gather_host)
            (void)hipHostFree(p->gather_host);
        delete p;
        return hip_fail(e, "pool create");
    }
    hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, p->stream, reinterpret_cast<int *>(p->barrier), 128);
    e = hipGetLastError();
    if (e != hipSuccess) {
        (void)hipHostFree(p->staging);
        (void)hipHostFree(p->gather_host);
        (void)hipEventDestroy(p->staging_done);
        delete p;
        return hip_fail(e, "pool create");
    }
    *out = p;
    return LBM_OK;
}

int lbm_pool_admit(lbm_pool *p, const lbm_config *cfg, const double *rho, const double *u, int64_t nsteps,
                   int32_t *slot) {
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
    const size_t bytes = round256(L.ws_bytes);
    size_t off = 0;
    if (!pool_alloc(p, bytes, &off)) {
        set_error("pool admit: no free arena block large enough");
        return LBM_ENOMEM;
    }
    Slot &s = p->slots[k];
    s = Slot{};
    rc = domain_bind_and_init(s.d, cfg, L, p->arena + off, rho, u, p->stream);
    int flag = 0;
    if (rc == LBM_OK)
        rc = domain_read_flag(s.d, p->stream, &flag);
    if (rc == LBM_OK && flag) {
        set_error("initial state has a node with rho <= 0 or |u_alpha| >= 1");
        rc = LBM_EDOMAIN;
    }
    if (rc != LBM_OK) {
        pool_free(p, off, bytes);
        return rc;
    }
    s.used = true;
    s.off = off;
    s.bytes = bytes;
    s.remaining = nsteps;
    s.reported = false;
    const int64_t block = (int64_t)L.block_x * L.block_y;
    int64_t tw = L.block_x, th = L.block_y;
    s.tw_shift = 0;
    if (p->tun.row_fit) {
        // narrowest power-of-two row width from 64 that covers the padded row
        const int64_t pitch = L.layout == LBM_LAYOUT_ROWS ? L.ps : cfg->nx;
        int shift = 6;
        while ((int64_t)1 << shift < pitch && shift < 8 && block % ((int64_t)2 << shift) == 0)
            ++shift;
        s.tw_shift = shift;
        tw = (int64_t)1 << shift;
        th = block / tw;
    }
    s.tiles_x = (int)((cfg->nx + tw - 1) / tw);
    s.tiles_y = (int)((cfg->ny + th - 1) / th);
    const int64_t tiles = p->tun.flat ? (L.n + block - 1) / block : (int64_t)s.tiles_x * s.tiles_y * cfg->nz;
    if (tiles > (int64_t)1 << 30) {
        pool_free(p, off, bytes);
        s = Slot{};
        set_error("pool admit: domain has too many tiles");
        return LBM_EINVAL;
    }
    s.tiles = (int)tiles;
    s.cls = class_of(cfg);
    *slot = k;
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
    for (int c = 0; c < kClasses; ++c) {
        std::vector<int> order;
        for (int i = 0; i < p->max_slots; ++i)
            if (p->slots[i].used && p->slots[i].remaining > 0 && p->slots[i].cls == c)
                order.push_back(i);
        if (order.empty())
            continue;
        any = true;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return p->slots[a].remaining > p->slots[b].remaining; });
        const int n = (int)order.size();
        const int64_t steps = std::min<int64_t>(k, p->slots[order[0]].remaining);
        const int cdim = c >= 8 ? 3 : 2, cdtype = (c % 8) / 2;
        // two steps per launch: D2Q9 FP64 / FP32_DEV row-interleaved slots that all take
        // the same even number of steps in this run, with as many nodes in the class as a
        // single domain needs for two steps per launch to pay (2048^2 FP32, 1024^2 FP64;
        // a workgroup sweeps its rows one after another): with a few small slots the
        // one-step form answers sooner (served p50 latency 44 against 18 ms)
        bool two = p->tun.time_block == 2 && cdim == 2 && (cdtype == kF64 || cdtype == kDevF64) &&
                   p->tun.layout == LBM_LAYOUT_ROWS && steps % 2 == 0;
        size_t class_buf_bytes = 0;
        int64_t class_nodes = 0;
        for (int j = 0; j < n && two; ++j) {
            two = std::min<int64_t>(k, p->slots[order[j]].remaining) == steps;
            class_buf_bytes += p->slots[order[j]].d.L.buf_bytes;
            class_nodes += p->slots[order[j]].d.L.n;
        }
        two = two && class_nodes >= (cdtype == kF64 ? (int64_t)1 << 20 : (int64_t)1 << 22);
        std::vector<int> tile_start(n + 1, 0);
        for (int j = 0; j < n; ++j) {
            const Slot &sj = p->slots[order[j]];
            const int64_t tiles = two ? ((sj.d.cfg.nx + kPoolT2Tx - 1) / kPoolT2Tx) *
                                            ((sj.d.cfg.ny + kPoolT2Rows - 1) / kPoolT2Rows)
                                      : (int64_t)sj.tiles;
            if ((int64_t)tile_start[j] + tiles > INT32_MAX) {
                set_error("pool run: more than 2^31 - 1 tiles in one class");
                return LBM_EINVAL;
            }
            tile_start[j + 1] = tile_start[j] + (int)tiles;
        }
        // Host copy of the class table in pinned memory; wait for the previous
        // upload from it to finish before overwriting.
        if (p->staging_pending) {
            hipError_t e = hipEventSynchronize(p->staging_done);
            if (e != hipSuccess)
                return hip_fail(e, "pool staging wait");
            p->staging_pending = false;
        }
        const size_t off_desc = 0, off_start = round256(sizeof(SlotDesc) * p->max_slots),
                     off_rem = off_start + round256(sizeof(int) * (p->max_slots + 1));
        SlotDesc *desc = reinterpret_cast<SlotDesc *>(p->staging + off_desc);
        int *starts = reinterpret_cast<int *>(p->staging + off_start);
        int64_t *rem = reinterpret_cast<int64_t *>(p->staging + off_rem);
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
            d.parity = s.d.cur;
            d.ps = s.d.L.ps;
            d.rs = s.d.L.rs;
            d.relax = s.d.relax;
            d.flag = s.d.flag;
            desc[j] = d;
            rem[j] = s.remaining;
        }
        std::memcpy(starts, tile_start.data(), sizeof(int) * (n + 1));
        char *table = p->arena + (size_t)c * p->class_bytes;
        hipError_t e = hipMemcpyAsync(table, p->staging, p->class_bytes, hipMemcpyHostToDevice, p->stream);
        if (e == hipSuccess)
            e = hipEventRecord(p->staging_done, p->stream);
        if (e != hipSuccess)
            return hip_fail(e, "pool table upload");
        p->staging_pending = true;

        PoolRunArgs a{};
        a.slots = reinterpret_cast<const SlotDesc *>(table + off_desc);
        a.tile_start = reinterpret_cast<const int *>(table + off_start);
        a.remaining = reinterpret_cast<const int64_t *>(table + off_rem);
        a.n = n;
        a.barrier = p->barrier;
        a.error = p->error;
        a.spin_limit = kSpinLimit;
        a.flat = p->tun.flat;
        const int dim = c >= 8 ? 3 : 2, dtype = (c % 8) / 2;
        const bool corr = (c & 1) != 0;
        PoolStepFn fn = dim == 3 ? pool_kernel<3>(dtype, corr, p->tun.persistent)
                                 : pool_kernel<2>(dtype, corr, p->tun.persistent);
        dim3 block(p->tun.tile_x, p->tun.tile_y);
        if (two) {
            // every slot takes `steps` (even) steps: steps / 2 two-step launches over all tiles
            const size_t elem = dtype == kF64 ? 8 : 4;
            const bool nt = t2_nt_stores(class_buf_bytes);
            void (*fn2)(PoolRunArgs) =
                dtype == kF64 ? (corr ? (nt ? k_pool_step2<kF64, true, true> : k_pool_step2<kF64, true, false>)
                                      : (nt ? k_pool_step2<kF64, false, true> : k_pool_step2<kF64, false, false>))
                              : (corr ? (nt ? k_pool_step2<kDevF64, true, true> : k_pool_step2<kDevF64, true, false>)
                                      : (nt ? k_pool_step2<kDevF64, false, true> : k_pool_step2<kDevF64, false, false>));
            a.t2_tx = kPoolT2Tx;
            a.t2_rows = kPoolT2Rows;
            for (int64_t L = 0; L < steps / 2; ++L) {
                a.step0 = (int)L;
                a.nsteps = 2;
                hipLaunchKernelGGL(fn2, dim3((unsigned)tile_start[n]), dim3((unsigned)t2_threads(kPoolT2Tx, elem)),
                                   (unsigned)t2_lds_bytes(kPoolT2Tx, elem), p->stream, a);
                p->launches++;
            }
            e = hipGetLastError();
            if (e != hipSuccess)
                return hip_fail(e, "pool two-step launch");
        } else if (p->tun.persistent) {
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
            for (int64_t s = 0; s < steps; ++s) {
                int cnt = 0;
                while (cnt < n && p->slots[order[cnt]].remaining > s)
                    ++cnt;
                const int P = tile_start[cnt];
                if (P == 0)
                    break;
                a.step0 = (int)s;
                a.nsteps = 1;
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
            s.d.cur ^= (int)((two ? done / 2 : done) & 1);  // one swap per launch
            s.d.steps += done;
            s.remaining -= done;
        }
    }
    if (any)
        p->runs++;
    return LBM_OK;
}

int lbm_pool_poll(lbm_pool *p, int32_t *done, int32_t capacity, int32_t *count) {
    if (!p || !count || capacity < 0 || (capacity > 0 && !done)) {
        set_error("pool poll: bad arguments");
        return LBM_EINVAL;
    }
    int err = 0;
    hipError_t e = hipMemcpyAsync(&err, p->error, sizeof(int), hipMemcpyDeviceToHost, p->stream);
    // domain flags of the slots still running: a slot whose state left the
    // equilibrium's domain is retired (its remaining steps are dropped)
    std::vector<int> running;
    for (int i = 0; i < p->max_slots; ++i)
        if (p->slots[i].used && p->slots[i].remaining > 0)
            running.push_back(i);
    const int nr = (int)running.size();
    int **ptrs = reinterpret_cast<int **>(p->gather_host);
    int *vals = reinterpret_cast<int *>(p->gather_host + round256(sizeof(int *) * (size_t)p->max_slots));
    int *dvals = reinterpret_cast<int *>(p->gather_dev + round256(sizeof(int *) * (size_t)p->max_slots));
    if (e == hipSuccess && nr > 0) {
        e = hipStreamSynchronize(p->stream);  // the pinned pointer list may still feed an earlier copy
        for (int j = 0; j < nr && e == hipSuccess; ++j)
            ptrs[j] = p->slots[running[j]].d.flag;
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->gather_dev, ptrs, sizeof(int *) * nr, hipMemcpyHostToDevice, p->stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_gather_flags, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, p->stream,
                               (const int *const *)p->gather_dev, nr, dvals);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(vals, dvals, sizeof(int) * nr, hipMemcpyDeviceToHost, p->stream);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess)
        return hip_fail(e, "pool poll synchronise");
    p->staging_pending = false;
    for (int j = 0; j < nr; ++j)
        if (vals[j]) {
            Slot &s = p->slots[running[j]];
            s.failed = true;
            s.remaining = 0;
        }
    int32_t c = 0;
    for (int i = 0; i < p->max_slots && c < capacity; ++i) {
        Slot &s = p->slots[i];
        if (s.used && s.remaining == 0 && !s.reported) {
            s.reported = true;
            done[c++] = i;
        }
    }
    *count = c;
    if (err) {
        set_error("pool: a persistent launch's grid barrier timed out");
        return LBM_EDEVICE;
    }
    return LBM_OK;
}

int lbm_pool_moments(lbm_pool *p, int32_t slot, double *rho, double *u, lbm_diag *diag) {
    int rc = check_slot(p, slot);
    if (rc != LBM_OK)
        return rc;
    return domain_moments(p->slots[slot].d, p->stream, rho, u, diag);
}

int lbm_pool_get_populations(lbm_pool *p, int32_t slot, double *out) {
    int rc = check_slot(p, slot);
    if (rc != LBM_OK)
        return rc;
    if (!out) {
        set_error("NULL output");
        return LBM_EINVAL;
    }
    return domain_export(p->slots[slot].d, p->stream, out);
}

int lbm_pool_release(lbm_pool *p, int32_t slot) {
    int rc = check_slot(p, slot);
    if (rc != LBM_OK)
        return rc;
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess)
        return hip_fail(e, "pool release synchronise");
    p->staging_pending = false;
    Slot &s = p->slots[slot];
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
    info->reserved = 0;
    return LBM_OK;
}

int lbm_pool_destroy(lbm_pool *p) {
    if (!p)
        return LBM_OK;
    hipError_t e = hipStreamSynchronize(p->stream);
    (void)hipHostFree(p->staging);
    (void)hipHostFree(p->gather_host);
    (void)hipEventDestroy(p->staging_done);
    delete p;
    if (e != hipSuccess)
        return hip_fail(e, "pool destroy synchronise");
    return LBM_OK;
}

}  // extern "C"
