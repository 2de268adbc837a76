// lbm_api.hip -- host side of the C ABI declared in include/lbm.h: argument
// validation, workspace layout, kernel selection and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "kernels.hpp"
#include "kernels_t2.hpp"
#include "lbm.h"
#include "lbm_internal.hpp"

namespace lbm {

thread_local char g_last_error[256] = "";

void set_error(const char *msg) { std::snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }

int hip_fail(hipError_t e, const char *what) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
    return LBM_EDEVICE;
}

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int validate_config(const lbm_config *cfg, const lbm_tuning *tun, Layout *out) {
    if (!cfg) {
        set_error("config is NULL");
        return LBM_EINVAL;
    }
    Layout L{};
    if (cfg->lattice == LBM_D1Q3) {
        L.dim = 1;
        L.q = 3;
    } else if (cfg->lattice == LBM_D2Q9) {
        L.dim = 2;
        L.q = 9;
    } else if (cfg->lattice == LBM_D3Q27) {
        L.dim = 3;
        L.q = 27;
    } else {
        set_error("lattice must be LBM_D1Q3, LBM_D2Q9 or LBM_D3Q27");
        return LBM_EINVAL;
    }
    if (cfg->dtype == LBM_FP64)
        L.elem = 8;
    else if (cfg->dtype == LBM_FP32_DEV || cfg->dtype == LBM_FP32_DEV_MIXED || cfg->dtype == LBM_FP32_DEV_F32)
        L.elem = 4;
    else {
        set_error("dtype must be LBM_FP64, LBM_FP32_DEV, LBM_FP32_DEV_MIXED or LBM_FP32_DEV_F32");
        return LBM_EINVAL;
    }
    if (cfg->equilibrium != LBM_EQ_ENTROPIC && cfg->equilibrium != LBM_EQ_POLY2 &&
        cfg->equilibrium != LBM_EQ_PRODUCT) {
        set_error("equilibrium must be LBM_EQ_ENTROPIC, LBM_EQ_POLY2 or LBM_EQ_PRODUCT");
        return LBM_EINVAL;
    }
    if (cfg->equilibrium != LBM_EQ_ENTROPIC && cfg->dtype != LBM_FP64 && cfg->dtype != LBM_FP32_DEV) {
        set_error("the polynomial equilibria run with LBM_FP64 or LBM_FP32_DEV storage only");
        return LBM_EINVAL;
    }
    L.eq = cfg->equilibrium;
    if (!(cfg->tau > 0.5) || !std::isfinite(cfg->tau)) {
        set_error("tau must be finite and > 1/2");
        return LBM_EINVAL;
    }
    if (cfg->bulk_correction != 0 && cfg->bulk_correction != 1) {
        set_error("bulk_correction must be 0 or 1");
        return LBM_EINVAL;
    }
    if (L.elem == 4 && (!(cfg->rho0 > 0.0) || !std::isfinite(cfg->rho0))) {
        set_error("rho0 must be finite and > 0 for FP32_DEV storage");
        return LBM_EINVAL;
    }
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) {
        set_error("grid extents must be >= 1");
        return LBM_EINVAL;
    }
    if (L.dim == 1 && (cfg->ny != 1 || cfg->nz != 1)) {
        set_error("ny and nz must be 1 for D1Q3");
        return LBM_EINVAL;
    }
    if (L.dim == 2 && cfg->nz != 1) {
        set_error("nz must be 1 for D2Q9");
        return LBM_EINVAL;
    }
    if (cfg->z_halo != 0 && cfg->z_halo != 1) {
        set_error("z_halo must be 0 or 1");
        return LBM_EINVAL;
    }
    if (cfg->reserved != 0) {
        set_error("lbm_config.reserved must be 0");
        return LBM_EINVAL;
    }
    if (cfg->z_halo && L.dim != 3) {
        set_error("z_halo needs LBM_D3Q27");
        return LBM_EINVAL;
    }
    if (cfg->z_halo && cfg->ny > (int64_t)INT32_MAX / 9) {
        set_error("z_halo needs 9 ny < 2^31 (one workgroup per packed run)");
        return LBM_EINVAL;
    }
    L.zhalo = cfg->z_halo != 0;
    if (cfg->nx > INT32_MAX || cfg->ny > INT32_MAX || cfg->nz > INT32_MAX) {
        set_error("grid extent beyond 2^31 - 1");
        return LBM_EINVAL;
    }
    L.n = cfg->nx * cfg->ny * cfg->nz;
    if (L.n > (int64_t)INT32_MAX - 4096) {
        set_error("more than 2^31 - 4096 nodes per population plane");
        return LBM_EINVAL;
    }
    // tuning
    int bx = 0, by = 0, pad = -1, npt = 0, flags = -1, layout = 0, tblock = 0, trows = 0;
    if (tun) {
        if (tun->reserved != 0) {
            set_error("lbm_tuning.reserved must be 0");
            return LBM_EINVAL;
        }
        bx = tun->block_x;
        by = tun->block_y;
        pad = tun->plane_pad;
        npt = tun->nodes_per_thread;
        flags = tun->flags;
        layout = tun->layout;
        tblock = tun->time_block;
        trows = tun->time_rows;
    }
    // the one-step kernel's shape left to the library (then the default may be two steps per launch)
    const bool shape_default = bx == 0 && by == 0 && npt == 0 && flags < 0 && layout == 0;
    if (layout == LBM_LAYOUT_DEFAULT)
        layout = LBM_LAYOUT_ROWS;
    if (layout != LBM_LAYOUT_ROWS && layout != LBM_LAYOUT_PLANES) {
        set_error("layout must be LBM_LAYOUT_ROWS or LBM_LAYOUT_PLANES");
        return LBM_EINVAL;
    }
    const bool fp32 = L.elem == 4;
    if (npt == 0) {
        // default: 16-byte vectors (4 floats or 2 doubles per thread) when rows tile evenly,
        // except for FP32 storage on D2Q9, where one node per thread in whole-row
        // workgroups measured faster (4096^2: 6.04 against 5.88 TB/s; on D1Q3 the vector
        // kernel is the faster one, 5.80 against 5.05)
        const int v = fp32 ? 4 : 2;
        npt = (cfg->nx % (64 * v) == 0 && !(fp32 && L.dim == 2)) ? v : 1;
    }
    if (npt != 1 && npt != 2 && npt != 4) {
        set_error("nodes_per_thread must be 1, 2 or 4");
        return LBM_EINVAL;
    }
    if (npt == 4 && !fp32) {
        set_error("nodes_per_thread = 4 needs FP32 storage");
        return LBM_EINVAL;
    }
    // measured best: non-temporal loads and stores for float runs, stores for double
    const int default_flags = fp32 ? LBM_TUNE_NT_STORE | LBM_TUNE_NT_LOAD : LBM_TUNE_NT_STORE;
    if (flags < 0)
        flags = npt > 1 ? default_flags : 0;
    if (flags > (LBM_TUNE_NT_STORE | LBM_TUNE_NT_LOAD) || (npt == 1 && flags != 0) ||
        flags == LBM_TUNE_NT_LOAD) {
        set_error("flags: NT_STORE, NT_STORE | NT_LOAD or 0, and only with nodes_per_thread > 1");
        return LBM_EINVAL;
    }
    if (L.eq != LBM_EQ_ENTROPIC && npt > 1 && (npt != (fp32 ? 4 : 2) || flags != default_flags)) {
        set_error("the polynomial equilibria take nodes_per_thread 1, or the default vector width "
                  "with the default flags");
        return LBM_EINVAL;
    }
    if (bx == 0) {
        if (npt > 1) {
            bx = 64;
        } else if (cfg->nx >= 64) {
            // a whole row per workgroup when it fits, else 256-wide tiles
            bx = (int)std::min<int64_t>(256, round_up(cfg->nx, 64));
        } else {
            bx = 64;
            while (bx > 1 && bx / 2 >= cfg->nx)
                bx /= 2;
        }
    }
    if (by == 0)
        by = L.dim == 1 && bx % 64 == 0 ? 1 : 256 / bx;  // a D1Q3 grid has one row
    if (bx < 1 || by < 1 || bx * by > 256 || (bx * by) % 64 != 0 ||
        (bx % 64 != 0 && (bx > 64 || (bx & (bx - 1)) != 0))) {
        set_error("block_x * block_y must be a multiple of 64 and <= 256; block_x a multiple "
                  "of 64 or a power of two <= 64");
        return LBM_EINVAL;
    }
    if (npt > 1 && (bx % 64 != 0 || cfg->nx % ((int64_t)bx * npt) != 0)) {
        set_error("nodes_per_thread > 1 needs block_x a multiple of 64 and nx % (block_x * "
                  "nodes_per_thread) == 0");
        return LBM_EINVAL;
    }
    {
        const int64_t tiles = ((cfg->nx + (int64_t)bx * npt - 1) / ((int64_t)bx * npt)) *
                              ((cfg->ny + by - 1) / by) * cfg->nz;
        if (tiles > (int64_t)INT32_MAX) {
            set_error("more than 2^31 - 1 workgroup tiles");
            return LBM_EINVAL;
        }
    }
    const bool t2_fits = L.dim == 2 && layout == LBM_LAYOUT_ROWS &&
                         (cfg->dtype == LBM_FP64 || cfg->dtype == LBM_FP32_DEV) && cfg->nx >= 64;
    // D1Q3, K steps per launch: owned nodes per workgroup (the LDS segment is 2 x 3 x
    // (tx + 2K) elements, 25 KB at K = 8), and nx >= tx + K for a single periodic wrap:
    // short rows take tx = nx - 8 (nx >= 16)
    const int t1_tx = (int)std::min<int64_t>(fp32 ? 1024 : 512, cfg->nx - 8);
    const bool t1_fits = L.dim == 1 && layout == LBM_LAYOUT_ROWS &&
                         (cfg->dtype == LBM_FP64 || cfg->dtype == LBM_FP32_DEV) && cfg->nx >= 16;
    if (tblock == 0) {
        // default: two steps per launch for large D2Q9 domains.  A workgroup sweeps its
        // rows one after another (about 1.4 us per row), so small grids lack the
        // parallelism; measured break-even near 2048^2 nodes for FP32 storage (1536^2:
        // 29.0 against 26.7 us per step; 2048^2: 39.0 against 49.0) and 1024^2 for FP64
        // (512^2: 12.1 against 8.9; 1024^2: 16.0 against 29.6)
        const int64_t big = fp32 ? (int64_t)2048 * 2048 : (int64_t)1024 * 1024;
        tblock = t2_fits && shape_default && trows == 0 && L.n >= big ? 2 : 1;
        // D1Q3: eight steps per launch whenever the row allows it (2^27 with the
        // correction: FP32 297 against 229 GLUPS, FP64 295 against 127; short rows are
        // bound by launches, and eight steps take one)
        if (t1_fits && shape_default && trows == 0)
            tblock = 8;
    }
    if (L.dim == 1 && tblock > 1) {
        if (tblock != 2 && tblock != 4 && tblock != 8) {
            set_error("time_block for D1Q3 must be 0, 1, 2, 4 or 8");
            return LBM_EINVAL;
        }
        if (!t1_fits || trows != 0) {
            set_error("time_block > 1 on D1Q3 needs the row-interleaved layout, LBM_FP64 or "
                      "LBM_FP32_DEV, nx >= 16, and time_rows = 0");
            return LBM_EINVAL;
        }
        L.tblock = tblock;
        L.t2_tx = t1_tx;
        L.t2_rows = 0;
        tblock = 1;  // the two-step D2Q9 checks below do not apply
    } else {
        L.tblock = 0;
    }
    if (tblock != 1 && tblock != 2) {
        set_error("time_block must be 0, 1 or 2 (D2Q9; 4 or 8 on D1Q3 only)");
        return LBM_EINVAL;
    }
    if (tblock == 1 && trows != 0) {
        set_error("time_rows needs time_block = 2");
        return LBM_EINVAL;
    }
    if (L.tblock == 0) {
        L.tblock = tblock;
        L.t2_tx = L.t2_rows = 0;
    }
    if (tblock == 2) {
        if (!t2_fits) {
            set_error("time_block = 2 needs D2Q9, the row-interleaved layout, LBM_FP64 or "
                      "LBM_FP32_DEV, and nx >= 64");
            return LBM_EINVAL;
        }
        if (trows < 0 || trows > cfg->ny) {
            set_error("time_rows must lie in 0 .. ny");
            return LBM_EINVAL;
        }
        // columns per tile: the widest of 1024 (FP32) or 128 (FP64), then 512, 256, 128, 64
        // that divides nx, or for other widths the widest not above nx (the last tile
        // partial).  FP32, us per step on one box, 512 against 1024 columns (76 KB of LDS and
        // two workgroups per compute unit, against 147 KB and one of 16 wavefronts): 2048^2
        // 35.0 / 34.4, 2500^2 57.6 / 57.6, 3072^2 81.8 / 76.7, 4000^2 122.7 / 116.0, 4096^2
        // 120.1 / 115.6, 6144^2 270.0 / 264.8 (256 columns: 126.9 at 4096^2 on another box,
        // 117.7 for 512 there).  FP64 takes 128 (37 KB, four workgroups of three wavefronts)
        int tx = fp32 ? 1024 : 128;
        if (cfg->nx % 64 == 0) {
            while (cfg->nx % tx != 0)
                tx /= 2;
        } else {
            while (tx > cfg->nx)
                tx /= 2;
        }
        const int64_t tiles_x = (cfg->nx + tx - 1) / tx;
        // workgroups resident at once: 256 compute units x those that fit 160 KB of LDS
        const int64_t per_cu = std::max<int64_t>(1, (int64_t)163840 / (int64_t)t2_lds_bytes(tx, L.elem));
        const int64_t round = 256 * std::min<int64_t>(per_cu, 8);
        if (trows == 0) {
            // A workgroup's time is about that of its rows + 2 sweep rows.  Take the row
            // count with the least (rounds of resident workgroups) x (rows + 2), so that
            // the last round is not mostly idle (3072^2 FP64, 1024 resident: 36 rows,
            // 2064 workgroups, 170.8 us per step; 16 rows: 139.9).
            int64_t best = -1;
            for (int cand : {16, 24, 32, 48, 64, 96, 128}) {
                const int64_t rws = std::min<int64_t>(cand, cfg->ny);
                const int64_t wgs = tiles_x * ((cfg->ny + rws - 1) / rws);
                const int64_t cost = (wgs + round - 1) / round * (rws + 2);
                if (best < 0 || cost < best) {
                    best = cost;
                    trows = (int)rws;
                }
            }
        }
        if (tiles_x * ((cfg->ny + trows - 1) / trows) > (int64_t)INT32_MAX) {
            set_error("more than 2^31 - 1 workgroup tiles");
            return LBM_EINVAL;
        }
        L.t2_tx = tx;
        L.t2_rows = trows;
    }
    L.block_x = bx;
    L.block_y = by;
    L.npt = npt;
    L.flags = flags;
    L.rowwave = npt > 1 && cfg->nx == (int64_t)64 * npt;
    if (pad < 0)
        pad = 0;
    if (pad > (1 << 20)) {
        set_error("plane_pad too large");
        return LBM_EINVAL;
    }
    L.layout = layout;
    if (L.zhalo && layout != LBM_LAYOUT_ROWS) {
        set_error("z_halo needs the row-interleaved layout");
        return LBM_EINVAL;
    }
    if (layout == LBM_LAYOUT_PLANES) {
        L.ps = round_up(L.n, 64) + round_up(pad, 64);
        L.rs = cfg->nx;
    } else {
        // runs padded to 16 elements (64 B FP32, 128 B FP64): measured faster on ragged
        // widths than 64 (the padding gaps between runs interrupt the streams)
        const int64_t pitch = cfg->nx < 16 ? cfg->nx : round_up(cfg->nx, 16);
        L.ps = pitch;
        L.rs = (int64_t)L.q * pitch;
    }
    L.plane = layout == LBM_LAYOUT_PLANES ? 0 : L.rs * cfg->ny;
    // a z-slab's buffers also hold the two halo planes, -1 below plane 0 and nz above nz - 1
    const int64_t elems =
        layout == LBM_LAYOUT_PLANES ? (int64_t)L.q * L.ps : L.rs * (L.n / cfg->nx) + (L.zhalo ? 2 * L.plane : 0);
    if (elems > ((int64_t)1 << 40)) {
        set_error("domain too large");
        return LBM_EINVAL;
    }
    L.buf_bytes = (size_t)elems * L.elem;
    L.red_blocks = (int)std::min<int64_t>(1024, (L.n + kReduceThreads - 1) / kReduceThreads);
    // workspace: buffer A | buffer B | flag block (256 B) | diag out (256 B) | partials
    L.off_buf[0] = 0;
    L.off_buf[1] = round_up(L.buf_bytes, 256);
    L.off_flag = L.off_buf[1] + round_up(L.buf_bytes, 256);
    L.off_diag = L.off_flag + 256;
    L.off_partials = L.off_diag + 256;
    L.ws_bytes = L.off_partials + round_up((size_t)L.red_blocks * kDiagFields * sizeof(double), 256);
    if (out)
        *out = L;
    return LBM_OK;
}

// Kernel selection.
using StepFn = void (*)(StepArgs);
template <int DIM, int DT, bool CORR, int NPT, bool RW>
static StepFn vec_kernel(int flags) {
    switch (flags) {
    case LBM_TUNE_NT_STORE:
        return k_stream_collide_vec<DIM, DT, CORR, NPT, RW, kNtStore>;
    case LBM_TUNE_NT_STORE | LBM_TUNE_NT_LOAD:
        return k_stream_collide_vec<DIM, DT, CORR, NPT, RW, kNtStore | kNtLoad>;
    default:
        return k_stream_collide_vec<DIM, DT, CORR, NPT, RW, 0>;
    }
}
template <int DIM, int DT, bool CORR>
static StepFn step_kernel_entropic(const Layout &L) {
    if (L.npt == 1)
        return k_stream_collide<DIM, DT, CORR>;
    if constexpr (DT != kF64) {
        if (L.npt == 4)
            return L.rowwave ? vec_kernel<DIM, DT, CORR, 4, true>(L.flags) : vec_kernel<DIM, DT, CORR, 4, false>(L.flags);
    }
    return L.rowwave ? vec_kernel<DIM, DT, CORR, 2, true>(L.flags) : vec_kernel<DIM, DT, CORR, 2, false>(L.flags);
}
// Polynomial equilibria: the scalar kernel, or the default vector width and
// flags (validate_config refuses other tunings for them).
template <int DIM, int DT, bool CORR, int EQ>
static StepFn step_kernel_poly(const Layout &L) {
    if (L.npt == 1)
        return k_stream_collide<DIM, DT, CORR, EQ>;
    constexpr int NPT = DT == kF64 ? 2 : 4;
    constexpr int FL = DT == kF64 ? kNtStore : kNtStore | kNtLoad;
    return L.rowwave ? k_stream_collide_vec<DIM, DT, CORR, NPT, true, FL, EQ>
                     : k_stream_collide_vec<DIM, DT, CORR, NPT, false, FL, EQ>;
}
template <int DIM, int DT, bool CORR>
static StepFn step_kernel_for(const Layout &L) {
    if constexpr (DT == kF64 || DT == kDevF64) {
        if (L.eq == LBM_EQ_POLY2)
            return step_kernel_poly<DIM, DT, CORR, kEqPoly2>(L);
        if (L.eq == LBM_EQ_PRODUCT)
            return step_kernel_poly<DIM, DT, CORR, kEqProduct>(L);
    }
    return step_kernel_entropic<DIM, DT, CORR>(L);
}
template <int DIM, int DT>
static StepFn step_kernel_dt(const Layout &L, bool corr) {
    return corr ? step_kernel_for<DIM, DT, true>(L) : step_kernel_for<DIM, DT, false>(L);
}
template <int DIM>
static StepFn step_kernel(const Layout &L, int dtype, bool corr) {
    switch (dtype) {
    case kDevMixed:
        return step_kernel_dt<DIM, kDevMixed>(L, corr);
    case kDevF64:
        return step_kernel_dt<DIM, kDevF64>(L, corr);
    case kDevF32:
        return step_kernel_dt<DIM, kDevF32>(L, corr);
    default:
        return step_kernel_dt<DIM, kF64>(L, corr);
    }
}

// Fused-halo z-slab steps (D3Q27): FP64 or FP32-deviation storage, one node
// per thread or the default vector width, with the default cache hints
// (results never depend on the hints).  lbm_step_halo refuses the rest.
static bool halo_supported(const Layout &L, int dtype) {
    if (L.dim != 3 || (dtype != kF64 && dtype != kDevF64))
        return false;
    return L.npt == 1 || L.npt == (dtype == kF64 ? 2 : 4);
}
using HaloStepFn = void (*)(StepArgs, HaloArgs);
template <int DT, bool CORR, int EQ>
static HaloStepFn halo_kernel_eq(const Layout &L) {
    constexpr int NPT = DT == kF64 ? 2 : 4;
    constexpr int FL = DT == kF64 ? kNtStore : kNtStore | kNtLoad;
    if (L.npt == 1)
        return k_stream_collide_halo<3, DT, CORR, EQ>;
    return L.rowwave ? k_stream_collide_vec_halo<3, DT, CORR, NPT, true, FL, EQ>
                     : k_stream_collide_vec_halo<3, DT, CORR, NPT, false, FL, EQ>;
}
template <int DT, bool CORR>
static HaloStepFn halo_kernel_for(const Layout &L) {
    if (L.eq == LBM_EQ_POLY2)
        return halo_kernel_eq<DT, CORR, kEqPoly2>(L);
    if (L.eq == LBM_EQ_PRODUCT)
        return halo_kernel_eq<DT, CORR, kEqProduct>(L);
    return halo_kernel_eq<DT, CORR, kEqEntropic>(L);
}
static HaloStepFn halo_kernel(const Layout &L, int dtype, bool corr) {
    if (dtype == kF64)
        return corr ? halo_kernel_for<kF64, true>(L) : halo_kernel_for<kF64, false>(L);
    return corr ? halo_kernel_for<kDevF64, true>(L) : halo_kernel_for<kDevF64, false>(L);
}

using InitFn = void (*)(InitArgs);
template <int DIM, bool DEV>
static InitFn init_kernel(int eq) {
    if (eq == LBM_EQ_POLY2)
        return k_init<DIM, DEV, kEqPoly2>;
    if (eq == LBM_EQ_PRODUCT)
        return k_init<DIM, DEV, kEqProduct>;
    return k_init<DIM, DEV, kEqEntropic>;
}

int launch_step(const Layout &L, const StepArgs &args, int dtype, bool corr, hipStream_t s, int nz,
                const HaloArgs *halo) {
    dim3 block(L.block_x, L.block_y, 1);
    dim3 grid((unsigned)(args.tiles_x * args.tiles_y * nz));
    if (halo) {
        hipLaunchKernelGGL(halo_kernel(L, dtype, corr), grid, block, 0, s, args, *halo);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return hip_fail(e, "stream-collide launch");
        return LBM_OK;
    }
    StepFn fn = L.dim == 1   ? step_kernel<1>(L, dtype, corr)
                : L.dim == 2 ? step_kernel<2>(L, dtype, corr)
                             : step_kernel<3>(L, dtype, corr);
    hipLaunchKernelGGL(fn, grid, block, 0, s, args);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, "stream-collide launch");
    return LBM_OK;
}

// Multi-step kernels by storage, correction, equilibrium and store hint.
template <int EQ, bool NT>
static void (*t1_kernel_nt(int dtype, bool corr))(StepKArgs) {
    return dtype == kF64 ? (corr ? k_stream_collide_t1<kF64, true, EQ, NT> : k_stream_collide_t1<kF64, false, EQ, NT>)
                         : (corr ? k_stream_collide_t1<kDevF64, true, EQ, NT>
                                 : k_stream_collide_t1<kDevF64, false, EQ, NT>);
}
template <int EQ>
static void (*t1_kernel(int dtype, bool corr, bool nt))(StepKArgs) {
    return nt ? t1_kernel_nt<EQ, true>(dtype, corr) : t1_kernel_nt<EQ, false>(dtype, corr);
}
template <int EQ, bool NT>
static void (*t2_kernel_nt(int dtype, bool corr))(Step2Args) {
    return dtype == kF64 ? (corr ? k_stream_collide2<kF64, true, EQ, NT> : k_stream_collide2<kF64, false, EQ, NT>)
                         : (corr ? k_stream_collide2<kDevF64, true, EQ, NT> : k_stream_collide2<kDevF64, false, EQ, NT>);
}
template <int EQ>
static void (*t2_kernel(int dtype, bool corr, bool nt))(Step2Args) {
    return nt ? t2_kernel_nt<EQ, true>(dtype, corr) : t2_kernel_nt<EQ, false>(dtype, corr);
}

// Several steps in one launch (time_block > 1): src -> dst = f*(t + time_block).
int launch_step2(const Layout &L, const StepArgs &args, int dtype, bool corr, hipStream_t s) {
    if (L.dim == 1) {
        StepKArgs a{args.src, args.dst, args.nx, L.t2_tx, L.tblock, L.ps, args.relax, args.flag};
        const bool nt = t2_nt_stores(L.buf_bytes);
        void (*fn)(StepKArgs) = L.eq == LBM_EQ_POLY2     ? t1_kernel<kEqPoly2>(dtype, corr, nt)
                                : L.eq == LBM_EQ_PRODUCT ? t1_kernel<kEqProduct>(dtype, corr, nt)
                                                         : t1_kernel<kEqEntropic>(dtype, corr, nt);
        hipLaunchKernelGGL(fn, dim3((unsigned)((args.nx + a.tx - 1) / a.tx)), dim3(256),
                           (unsigned)t1_lds_bytes(a.tx, a.K, L.elem), s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return hip_fail(e, "multi-step launch");
        return LBM_OK;
    }
    Step2Args a{args.src, args.dst, args.nx, args.ny, L.t2_tx, L.t2_rows, (args.nx + L.t2_tx - 1) / L.t2_tx,
                (args.ny + L.t2_rows - 1) / L.t2_rows, L.ps, L.rs, args.relax, args.flag};
    const bool nt = t2_nt_stores(L.buf_bytes);
    void (*fn)(Step2Args) = L.eq == LBM_EQ_POLY2     ? t2_kernel<kEqPoly2>(dtype, corr, nt)
                            : L.eq == LBM_EQ_PRODUCT ? t2_kernel<kEqProduct>(dtype, corr, nt)
                                                     : t2_kernel<kEqEntropic>(dtype, corr, nt);
    hipLaunchKernelGGL(fn, dim3((unsigned)(a.tiles_x * a.tiles_y)), dim3((unsigned)t2_threads(a.tx, L.elem)),
                       (unsigned)t2_lds_bytes(a.tx, L.elem), s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, "two-step launch");
    return LBM_OK;
}

int domain_bind_and_init(DomainState &d, const lbm_config *cfg, const Layout &L, void *workspace,
                         const double *rho, const double *u, hipStream_t s) {
    d.cfg = *cfg;
    d.L = L;
    d.ws = static_cast<char *>(workspace);
    // a z-slab's buffer pointers address plane 0, one halo plane into the buffer
    const size_t halo_bytes = L.zhalo ? (size_t)L.plane * L.elem : 0;
    d.buf[0] = d.ws + L.off_buf[0] + halo_bytes;
    d.buf[1] = d.ws + L.off_buf[1] + halo_bytes;
    d.cur = 0;
    if (L.zhalo) {
        // defined contents (zeros) in the halo planes until the first exchange fills them
        for (int k = 0; k < 2; ++k) {
            char *b = d.ws + L.off_buf[k];
            hipError_t e = hipMemsetAsync(b, 0, halo_bytes, s);
            if (e == hipSuccess)
                e = hipMemsetAsync(b + halo_bytes * (size_t)(cfg->nz + 1), 0, halo_bytes, s);
            if (e != hipSuccess)
                return hip_fail(e, "halo plane clear");
        }
    }
    d.flag = reinterpret_cast<int *>(d.ws + L.off_flag);
    d.diag_dev = reinterpret_cast<double *>(d.ws + L.off_diag);
    d.partials = reinterpret_cast<double *>(d.ws + L.off_partials);
    d.steps = 0;
    d.relax.omega = 1.0 / cfg->tau;
    d.relax.two_tau_m1 = 2.0 * cfg->tau - 1.0;
    d.relax.rho0 = cfg->dtype != LBM_FP64 ? cfg->rho0 : 0.0;

    hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, s, d.flag, 64);
    InitArgs ia{d.buf[0], rho, u, L.n, (int)cfg->nx, L.ps, L.rs, d.relax.rho0, d.flag};
    const bool dev = cfg->dtype != LBM_FP64;
    dim3 grid((unsigned)((L.n + 255) / 256)), block(256);
    InitFn init_fn = L.dim == 1   ? (dev ? init_kernel<1, true>(L.eq) : init_kernel<1, false>(L.eq))
                     : L.dim == 2 ? (dev ? init_kernel<2, true>(L.eq) : init_kernel<2, false>(L.eq))
                                  : (dev ? init_kernel<3, true>(L.eq) : init_kernel<3, false>(L.eq));
    hipLaunchKernelGGL(init_fn, grid, block, 0, s, ia);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, "init launch");
    return LBM_OK;
}

int domain_read_flag(const DomainState &d, hipStream_t s, int *flag) {
    int f = 0;
    hipError_t e = hipMemcpyAsync(&f, d.flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "domain flag read");
    *flag = f;
    return LBM_OK;
}

int domain_moments(DomainState &d, hipStream_t s, double *rho, double *u, lbm_diag *diag) {
    const Layout &L = d.L;
    const bool dev = d.cfg.dtype != LBM_FP64;
    MomentArgs ma{d.buf[d.cur], rho, u, L.n, (int)d.cfg.nx, L.ps, L.rs, d.relax.rho0, d.partials};
    dim3 grid((unsigned)L.red_blocks), block(kReduceThreads);
    void (*mom_fn)(MomentArgs) = L.dim == 1   ? (dev ? k_moments<1, true> : k_moments<1, false>)
                                 : L.dim == 2 ? (dev ? k_moments<2, true> : k_moments<2, false>)
                                              : (dev ? k_moments<3, true> : k_moments<3, false>);
    hipLaunchKernelGGL(mom_fn, grid, block, 0, s, ma);
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kReduceThreads), 0, s, (const double *)d.partials,
                       L.red_blocks, d.diag_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, "moments launch");
    double v[kDiagFields];
    int flag = 0;
    e = hipMemcpyAsync(v, d.diag_dev, sizeof(v), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&flag, d.flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "moments synchronise");
    if (diag) {
        diag->mass = v[0];
        diag->momentum[0] = v[1];
        diag->momentum[1] = v[2];
        diag->momentum[2] = v[3];
        diag->kinetic_energy = v[4];
        diag->max_abs_u = v[5];
        diag->min_rho = v[6];
        diag->steps = d.steps;
        diag->domain_error = flag ? 1 : 0;
        diag->reserved = 0;
    }
    if (flag) {
        set_error("a node left rho > 0, |u_alpha| < 1");
        return LBM_EDOMAIN;
    }
    return LBM_OK;
}

int domain_export(DomainState &d, hipStream_t s, double *out) {
    const Layout &L = d.L;
    const bool dev = d.cfg.dtype != LBM_FP64;
    ExportArgs ea{d.buf[d.cur], out, L.n, (int)d.cfg.nx, L.ps, L.rs, d.relax.rho0};
    dim3 grid((unsigned)((L.n + 255) / 256)), block(256);
    void (*exp_fn)(ExportArgs) = L.dim == 1   ? (dev ? k_export<1, true> : k_export<1, false>)
                                 : L.dim == 2 ? (dev ? k_export<2, true> : k_export<2, false>)
                                              : (dev ? k_export<3, true> : k_export<3, false>);
    hipLaunchKernelGGL(exp_fn, grid, block, 0, s, ea);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "population export");
    return LBM_OK;
}

int domain_energy(DomainState &d, hipStream_t s, const double *U, double rho_ref, double *out) {
    const Layout &L = d.L;
    const bool dev = d.cfg.dtype != LBM_FP64;
    EnergyArgs ea{d.buf[d.cur], L.n, (int)d.cfg.nx, L.ps, L.rs, d.relax.rho0, rho_ref, {0.0, 0.0, 0.0},
                  d.partials};
    for (int a = 0; a < L.dim; ++a)
        ea.U[a] = U ? U[a] : 0.0;
    void (*fn)(EnergyArgs) = L.dim == 1   ? (dev ? k_energy<1, true> : k_energy<1, false>)
                             : L.dim == 2 ? (dev ? k_energy<2, true> : k_energy<2, false>)
                                          : (dev ? k_energy<3, true> : k_energy<3, false>);
    hipLaunchKernelGGL(fn, dim3((unsigned)L.red_blocks), dim3(kReduceThreads), 0, s, ea);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kReduceThreads), 0, s, (const double *)d.partials,
                       L.red_blocks, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, "energy launch");
    return LBM_OK;
}

}  // namespace lbm

using namespace lbm;

// Steps of small domains are bound by the host's launch rate (about 3 us per
// launch), so long runs replay a captured HIP graph of kGraphSteps launches
// instead.  kGraphSteps is even: the population buffers are back in place
// after each replay, so one graph per starting buffer serves every call.  The
// graph holds the same kernels with the same arguments, so results are
// bitwise those of plain launches.
constexpr int kGraphSteps = 32;

struct lbm_handle {
    DomainState d;
    hipStream_t stream;
    hipStream_t capture = nullptr;            // private stream the graphs are captured on
    hipGraph_t graph[2] = {nullptr, nullptr};  // by the buffer holding the state at the start
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    bool graphs_off = false;                   // a graph call failed once: plain launches only
};

// Pack: plane 0's populations with c_z = -1 into `lower`, plane nz - 1's with
// c_z = +1 into `upper`.  Unpack: `lower` into the halo plane below plane 0
// (populations c_z = +1), `upper` into the halo plane above plane nz - 1
// (c_z = -1).  Populations are numbered i = (c_x + 1) + 3 (c_y + 1) +
// 9 (c_z + 1), so each row's 9 runs of one sign of c_z are adjacent.  Both
// faces go in one launch; a NULL buffer skips its face.
template <typename E>
static void launch_halo_copy(const DomainState &d, const void *lower, const void *upper, bool pack,
                             hipStream_t stream) {
    const int64_t nx = d.cfg.nx, ny = d.cfg.ny, nz = d.cfg.nz;
    HaloCopy<E> a{};
    a.nx = (int)nx;
    a.s_row = pack ? d.L.rs : 9 * nx;
    a.s_run = pack ? d.L.ps : nx;
    a.d_row = pack ? 9 * nx : d.L.rs;
    a.d_run = pack ? nx : d.L.ps;
    E *base = static_cast<E *>(d.buf[d.cur]);
    const void *ext[2] = {lower, upper};
    for (int f = 0; f < 2; ++f) {
        // plane of the slab and first population of the 9
        const int64_t plane = pack ? (f == 0 ? 0 : nz - 1) : (f == 0 ? -1 : nz);
        const int64_t first = pack ? (f == 0 ? 0 : 18) : (f == 0 ? 18 : 0);
        E *slab = base + (plane * ny) * d.L.rs + first * d.L.ps;  // elements from plane 0
        if (ext[f] == nullptr) {
            a.src[f] = nullptr;
            a.dst[f] = nullptr;
        } else if (pack) {
            a.src[f] = slab;
            a.dst[f] = static_cast<E *>(const_cast<void *>(ext[f]));
        } else {
            a.src[f] = static_cast<const E *>(ext[f]);
            a.dst[f] = slab;
        }
    }
    // one workgroup per run of nx elements: 9 ny runs per face (ny < 2^31 / 9
    // is checked at configuration)
    const unsigned threads = (unsigned)std::min<int64_t>(256, (nx + 63) / 64 * 64);
    hipLaunchKernelGGL(k_halo_copy<E>, dim3((unsigned)(9 * ny), 2), dim3(threads), 0, stream, a);
}

// Free streaming with the one-step kernel's launch: the kernel the handle's
// tuning selects, instantiated without the collision.
template <int DIM, int DT>
static StepFn stream_only_kernel(const Layout &L) {
    if (L.npt == 1)
        return k_stream_collide<DIM, DT, false, kEqStreamOnly>;
    constexpr int NPT = DT == kF64 ? 2 : 4;
    constexpr int FL = DT == kF64 ? kNtStore : kNtStore | kNtLoad;
    return L.rowwave ? k_stream_collide_vec<DIM, DT, false, NPT, true, FL, kEqStreamOnly>
                     : k_stream_collide_vec<DIM, DT, false, NPT, false, FL, kEqStreamOnly>;
}

// One float4 per thread, non-temporal loads and stores.
typedef float f32x4 __attribute__((ext_vector_type(4)));
static __global__ __launch_bounds__(256) void k_copy_nt(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst,
                                                        int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

extern "C" {

size_t lbm_workspace_bytes_tuned(const lbm_config *cfg, const lbm_tuning *tuning) {
    Layout L;
    if (validate_config(cfg, tuning, &L) != LBM_OK)
        return 0;
    return L.ws_bytes;
}

size_t lbm_workspace_bytes(const lbm_config *cfg) { return lbm_workspace_bytes_tuned(cfg, nullptr); }

static void prepare_step_graphs(lbm_handle *h);

int lbm_create_tuned(const lbm_config *cfg, const lbm_tuning *tuning, void *workspace, size_t ws_bytes,
                     const double *rho, const double *u, void *stream, lbm_handle **out) {
    Layout L;
    int rc = validate_config(cfg, tuning, &L);
    if (rc != LBM_OK)
        return rc;
    if (!workspace || !rho || !u || !out) {
        set_error("NULL workspace, rho, u or out");
        return LBM_EINVAL;
    }
    if (ws_bytes < L.ws_bytes) {
        set_error("workspace smaller than lbm_workspace_bytes()");
        return LBM_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) {
        set_error("workspace must be 256-byte aligned");
        return LBM_EINVAL;
    }
    lbm_handle *h = new (std::nothrow) lbm_handle();
    if (!h) {
        set_error("host allocation failed");
        return LBM_EINVAL;
    }
    h->stream = static_cast<hipStream_t>(stream);
    int flag = 0;
    rc = domain_bind_and_init(h->d, cfg, L, workspace, rho, u, h->stream);
    if (rc == LBM_OK)
        rc = domain_read_flag(h->d, h->stream, &flag);
    if (rc != LBM_OK) {
        delete h;
        return rc;
    }
    if (flag) {
        delete h;
        set_error("initial state has a node with rho <= 0 or |u_alpha| >= 1");
        return LBM_EDOMAIN;
    }
    // capture the step graphs now, so that no later call pays for it
    if (!L.zhalo) {
        prepare_step_graphs(h);
    }
    *out = h;
    return LBM_OK;
}

int lbm_create(const lbm_config *cfg, void *workspace, size_t ws_bytes, const double *rho, const double *u,
               void *stream, lbm_handle **out) {
    return lbm_create_tuned(cfg, nullptr, workspace, ws_bytes, rho, u, stream, out);
}

// Enqueue one plain step launch with the state in buffer `cur` on stream s.
static int enqueue_step(lbm_handle *h, int cur, hipStream_t s) {
    DomainState &d = h->d;
    const bool corr = d.cfg.bulk_correction != 0;
    const int tiles_x = (int)((d.cfg.nx + (int64_t)d.L.block_x * d.L.npt - 1) / ((int64_t)d.L.block_x * d.L.npt));
    const int tiles_y = (int)((d.cfg.ny + d.L.block_y - 1) / d.L.block_y);
    StepArgs a{d.buf[cur], d.buf[cur ^ 1], (int)d.cfg.nx, (int)d.cfg.ny, (int)d.cfg.nz, tiles_x, tiles_y,
               d.L.ps, d.L.rs, d.relax, d.flag, d.L.zhalo ? 1 : 0};
    return launch_step(d.L, a, d.cfg.dtype, corr, s, (int)d.cfg.nz, nullptr);
}

// Enqueue one launch of time_block steps (time_block > 1) from buffer `cur`.
static int enqueue_pair(lbm_handle *h, int cur, hipStream_t s) {
    DomainState &d = h->d;
    StepArgs a{d.buf[cur], d.buf[cur ^ 1], (int)d.cfg.nx, (int)d.cfg.ny, 1, 0, 0,
               d.L.ps, d.L.rs, d.relax, d.flag, 0};
    return launch_step2(d.L, a, d.cfg.dtype, d.cfg.bulk_correction != 0, s);
}

// The graph of kGraphSteps steps starting from buffer `cur` (captured when the
// handle is created; later calls find it).  Returns false (and turns graphs
// off for the handle) if any graph call fails; the caller then launches
// plainly.
static bool step_graph(lbm_handle *h, int cur) {
    if (h->graphs_off)
        return false;
    if (h->exec[cur])
        return true;
    hipError_t e = hipSuccess;
    if (!h->capture)
        e = hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        int rc = LBM_OK;
        // kGraphSteps steps: as many launches, or kGraphSteps / time_block launches of
        // time_block steps (2, 4 or 8); either way an even number of buffer swaps
        const int launches = kGraphSteps / h->d.L.tblock;
        for (int k = 0; k < launches && rc == LBM_OK; ++k)
            rc = h->d.L.tblock > 1 ? enqueue_pair(h, cur ^ (k & 1), h->capture)
                                   : enqueue_step(h, cur ^ (k & 1), h->capture);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(h->capture, &g);
        if (e == hipSuccess && rc == LBM_OK && g) {
            h->graph[cur] = g;
            e = hipGraphInstantiate(&h->exec[cur], g, nullptr, nullptr, 0);
        } else {
            if (g)
                (void)hipGraphDestroy(g);
            if (e == hipSuccess)
                e = hipErrorUnknown;
        }
    }
    if (e != hipSuccess || !h->exec[cur]) {
        (void)hipGetLastError();  // leave no sticky error behind for the next call
        if (h->exec[cur])
            (void)hipGraphExecDestroy(h->exec[cur]);
        h->exec[cur] = nullptr;
        h->graphs_off = true;
        return false;
    }
    return true;
}

// Both graphs (one per starting buffer), captured when the handle is created;
// the capture stream is released afterwards (a handle keeps no extra stream).
static void prepare_step_graphs(lbm_handle *h) {
    for (int cur = 0; cur < 2; ++cur)
        if (!step_graph(h, cur))
            break;
    if (h->capture) {
        // a failure here loses only the private capture stream; the graphs stay usable
        if (hipStreamDestroy(h->capture) != hipSuccess)
            (void)hipGetLastError();
        h->capture = nullptr;
    }
}

int lbm_step(lbm_handle *h, int64_t nsteps) {
    if (!h || nsteps < 0) {
        set_error("NULL handle or negative step count");
        return LBM_EINVAL;
    }
    DomainState &d = h->d;
    if (d.L.zhalo && nsteps > 1) {
        set_error("a z-slab takes one step between halo exchanges");
        return LBM_EINVAL;
    }
    int64_t s = 0;
    if (nsteps >= 2 * kGraphSteps && step_graph(h, d.cur)) {
        for (; s + kGraphSteps <= nsteps; s += kGraphSteps) {
            hipError_t e = hipGraphLaunch(h->exec[d.cur], h->stream);
            if (e != hipSuccess)
                return hip_fail(e, "step graph launch");
            d.steps += kGraphSteps;  // an even count of swaps: d.cur is unchanged
        }
    }
    if (d.L.tblock > 1) {
        for (; s + d.L.tblock <= nsteps; s += d.L.tblock) {
            int rc = enqueue_pair(h, d.cur, h->stream);
            if (rc != LBM_OK)
                return rc;
            d.cur ^= 1;
            d.steps += d.L.tblock;
        }
    }
    for (; s < nsteps; ++s) {
        int rc = enqueue_step(h, d.cur, h->stream);
        if (rc != LBM_OK)
            return rc;
        d.cur ^= 1;
        d.steps++;
    }
    return LBM_OK;
}

int lbm_step_halo(lbm_handle *h, const void *recv_lower, const void *recv_upper, void *send_lower,
                  void *send_upper) {
    if (!h || !recv_lower || !recv_upper || !send_lower || !send_upper) {
        set_error("NULL handle or halo buffer");
        return LBM_EINVAL;
    }
    DomainState &d = h->d;
    if (!d.L.zhalo) {
        set_error("the domain is not a z-slab (z_halo = 0)");
        return LBM_EINVAL;
    }
    if (!halo_supported(d.L, d.cfg.dtype)) {
        set_error("fused halo steps take FP64 or FP32_DEV storage and one node per thread or the default "
                  "vector width");
        return LBM_EINVAL;
    }
    const void *recv[2] = {recv_lower, recv_upper};
    const void *send[2] = {send_lower, send_upper};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            if (recv[a] == send[b]) {
                set_error("a receive buffer is also a send buffer");
                return LBM_EINVAL;
            }
    if (send_lower == send_upper) {
        set_error("the two send buffers are the same");
        return LBM_EINVAL;
    }
    const bool corr = d.cfg.bulk_correction != 0;
    const int tiles_x = (int)((d.cfg.nx + (int64_t)d.L.block_x * d.L.npt - 1) / ((int64_t)d.L.block_x * d.L.npt));
    const int tiles_y = (int)((d.cfg.ny + d.L.block_y - 1) / d.L.block_y);
    StepArgs a{d.buf[d.cur], d.buf[d.cur ^ 1], (int)d.cfg.nx, (int)d.cfg.ny, (int)d.cfg.nz, tiles_x, tiles_y,
               d.L.ps, d.L.rs, d.relax, d.flag, 1};
    const HaloArgs ha{{recv_lower, recv_upper}, {send_lower, send_upper}};
    int rc = launch_step(d.L, a, d.cfg.dtype, corr, h->stream, (int)d.cfg.nz, &ha);
    if (rc != LBM_OK)
        return rc;
    d.cur ^= 1;
    d.steps++;
    return LBM_OK;
}

size_t lbm_halo_bytes(const lbm_config *cfg) {
    Layout L;
    if (validate_config(cfg, nullptr, &L) != LBM_OK || !L.zhalo)
        return 0;
    return (size_t)9 * (size_t)cfg->nx * (size_t)cfg->ny * L.elem;
}

static int halo_copy(lbm_handle *h, const void *lower, const void *upper, bool pack) {
    if (!h || (!lower && !upper)) {
        set_error("NULL handle, or both buffers NULL");
        return LBM_EINVAL;
    }
    DomainState &d = h->d;
    if (!d.L.zhalo) {
        set_error("the domain is not a z-slab (z_halo = 0)");
        return LBM_EINVAL;
    }
    if (d.L.elem == 8)
        launch_halo_copy<uint64_t>(d, lower, upper, pack, h->stream);
    else
        launch_halo_copy<uint32_t>(d, lower, upper, pack, h->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, pack ? "halo pack launch" : "halo unpack launch");
    return LBM_OK;
}

int lbm_halo_pack(lbm_handle *h, void *lower, void *upper) { return halo_copy(h, lower, upper, true); }

int lbm_halo_unpack(lbm_handle *h, const void *lower, const void *upper) {
    return halo_copy(h, lower, upper, false);
}

int lbm_moments(lbm_handle *h, double *rho, double *u, lbm_diag *diag) {
    if (!h) {
        set_error("NULL handle");
        return LBM_EINVAL;
    }
    return domain_moments(h->d, h->stream, rho, u, diag);
}

int lbm_energy(lbm_handle *h, const double *U, double rho_ref, double *out) {
    if (!h || !out) {
        set_error("NULL handle or output");
        return LBM_EINVAL;
    }
    if (!(rho_ref > 0.0) || !std::isfinite(rho_ref)) {
        set_error("rho_ref must be finite and > 0");
        return LBM_EINVAL;
    }
    if (U)
        for (int a = 0; a < h->d.L.dim; ++a)
            if (!std::isfinite(U[a])) {
                set_error("U must be finite");
                return LBM_EINVAL;
            }
    return domain_energy(h->d, h->stream, U, rho_ref, out);
}

int lbm_energy_history(lbm_handle *h, int64_t steps, int64_t every, const double *U, double rho_ref, double *out) {
    if (!h || !out || every < 1 || steps < 0 || steps % every != 0) {
        set_error("NULL handle or output, every < 1, or steps not a non-negative multiple of every");
        return LBM_EINVAL;
    }
    if (h->d.L.zhalo) {
        set_error("a z-slab's steps need halo exchanges between them");
        return LBM_EINVAL;
    }
    int rc = lbm_energy(h, U, rho_ref, out);  // also checks U and rho_ref
    for (int64_t k = 1; rc == LBM_OK && k <= steps / every; ++k) {
        rc = lbm_step(h, every);
        if (rc == LBM_OK)
            rc = domain_energy(h->d, h->stream, U, rho_ref, out + k);
    }
    return rc;
}

// Checkpoint / restart: the stored population buffer holding the current
// state (whole, including row padding and a z-slab's halo planes), copied
// device to device on the handle's stream.
size_t lbm_state_bytes(const lbm_handle *h) { return h ? h->d.L.buf_bytes : 0; }

static char *state_base(const DomainState &d) {
    const size_t halo_bytes = d.L.zhalo ? (size_t)d.L.plane * d.L.elem : 0;
    return static_cast<char *>(d.buf[d.cur]) - halo_bytes;
}

int lbm_save_state(lbm_handle *h, void *dst, size_t bytes) {
    if (!h || !dst || bytes != h->d.L.buf_bytes) {
        set_error("NULL handle or buffer, or bytes != lbm_state_bytes()");
        return LBM_EINVAL;
    }
    hipError_t e = hipMemcpyAsync(dst, state_base(h->d), bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess)
        return hip_fail(e, "state save");
    return LBM_OK;
}

int lbm_load_state(lbm_handle *h, const void *src, size_t bytes, int64_t steps) {
    if (!h || !src || bytes != h->d.L.buf_bytes || steps < 0) {
        set_error("NULL handle or buffer, bytes != lbm_state_bytes(), or negative step count");
        return LBM_EINVAL;
    }
    hipError_t e = hipMemcpyAsync(state_base(h->d), src, bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, h->stream, h->d.flag, 64);
        e = hipGetLastError();
    }
    if (e != hipSuccess)
        return hip_fail(e, "state load");
    h->d.steps = steps;
    return LBM_OK;
}

int lbm_ceiling_stream(lbm_handle *h, int64_t nsteps) {
    if (!h || nsteps < 0) {
        set_error("NULL handle or negative step count");
        return LBM_EINVAL;
    }
    DomainState &d = h->d;
    const Layout &L = d.L;
    const int dt = d.cfg.dtype;
    const bool default_vec = L.npt == (dt == LBM_FP64 ? 2 : 4) &&
                             L.flags == (dt == LBM_FP64 ? LBM_TUNE_NT_STORE : LBM_TUNE_NT_STORE | LBM_TUNE_NT_LOAD);
    if (L.dim < 2 || L.zhalo || L.tblock != 1 || (dt != LBM_FP64 && dt != LBM_FP32_DEV) ||
        !(L.npt == 1 || default_vec)) {
        set_error("free streaming runs on D2Q9 / D3Q27 periodic domains with FP64 or FP32_DEV storage, one step "
                  "per launch, one node per thread or the default vector width and flags");
        return LBM_EINVAL;
    }
    StepFn fn = L.dim == 2 ? (dt == LBM_FP64 ? stream_only_kernel<2, kF64>(L) : stream_only_kernel<2, kDevF64>(L))
                           : (dt == LBM_FP64 ? stream_only_kernel<3, kF64>(L) : stream_only_kernel<3, kDevF64>(L));
    const int tiles_x = (int)((d.cfg.nx + (int64_t)L.block_x * L.npt - 1) / ((int64_t)L.block_x * L.npt));
    const int tiles_y = (int)((d.cfg.ny + L.block_y - 1) / L.block_y);
    for (int64_t s = 0; s < nsteps; ++s) {
        StepArgs a{d.buf[d.cur], d.buf[d.cur ^ 1], (int)d.cfg.nx, (int)d.cfg.ny, (int)d.cfg.nz, tiles_x, tiles_y,
                   L.ps, L.rs, d.relax, d.flag, 0};
        hipLaunchKernelGGL(fn, dim3((unsigned)(tiles_x * tiles_y * d.cfg.nz)), dim3(L.block_x, L.block_y, 1), 0,
                           h->stream, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return hip_fail(e, "free-streaming launch");
        d.cur ^= 1;
    }
    return LBM_OK;
}

int lbm_ceiling_copy(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(dst) % 16 != 0 || bytes > ((size_t)1 << 40)) {
        set_error("copy: NULL or misaligned buffer, or bytes not a multiple of 16");
        return LBM_EINVAL;
    }
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0)
        return LBM_OK;
    hipLaunchKernelGGL(k_copy_nt, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const f32x4 *>(src), static_cast<f32x4 *>(dst), n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, "copy launch");
    return LBM_OK;
}

int lbm_get_launch_info(const lbm_handle *h, lbm_launch_info *out) {
    if (!h || !out) {
        set_error("NULL handle or output");
        return LBM_EINVAL;
    }
    const Layout &L = h->d.L;
    lbm_launch_info r{};
    r.kernel = L.tblock > 1 ? (L.dim == 1 ? LBM_KERNEL_MULTI_STEP : LBM_KERNEL_TWO_STEP)
                            : (L.npt > 1 ? LBM_KERNEL_VECTOR : LBM_KERNEL_NODE);
    r.nodes_per_thread = L.npt;
    r.row_wave = L.rowwave ? 1 : 0;
    r.flags = L.flags;
    r.block_x = L.block_x;
    r.block_y = L.block_y;
    r.layout = L.layout;
    r.time_block = L.tblock;
    r.time_cols = L.tblock > 1 ? L.t2_tx : 0;
    r.time_rows = L.tblock == 2 && L.dim == 2 ? L.t2_rows : 0;
    r.graph_steps = (h->exec[0] || h->exec[1]) && !h->graphs_off ? kGraphSteps : 0;
    *out = r;
    return LBM_OK;
}

int lbm_get_populations(lbm_handle *h, double *out) {
    if (!h || !out) {
        set_error("NULL handle or output");
        return LBM_EINVAL;
    }
    return domain_export(h->d, h->stream, out);
}

int lbm_destroy(lbm_handle *h) {
    if (!h)
        return LBM_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    // release everything even after a failure; report the first one
    auto keep = [&e](hipError_t r) {
        if (e == hipSuccess)
            e = r;
    };
    for (int k = 0; k < 2; ++k) {
        if (h->exec[k])
            keep(hipGraphExecDestroy(h->exec[k]));
        if (h->graph[k])
            keep(hipGraphDestroy(h->graph[k]));
    }
    if (h->capture)
        keep(hipStreamDestroy(h->capture));
    delete h;
    if (e != hipSuccess)
        return hip_fail(e, "destroy synchronise");
    return LBM_OK;
}

const char *lbm_status_string(int status) {
    switch (status) {
    case LBM_OK:
        return "LBM_OK";
    case LBM_EINVAL:
        return "LBM_EINVAL: invalid argument";
    case LBM_EDOMAIN:
        return "LBM_EDOMAIN: a node left rho > 0, |u_alpha| < 1";
    case LBM_EDEVICE:
        return "LBM_EDEVICE: HIP runtime error";
    case LBM_ENOMEM:
        return "LBM_ENOMEM: does not fit the memory budget";
    case LBM_EBUSY:
        return "LBM_EBUSY: no free slot";
    default:
        return "unknown status";
    }
}

const char *lbm_last_error(void) { return g_last_error; }

const char *lbm_version(void) { return "lbm-entropic 0.4 (gfx950)"; }

}  // extern "C"
