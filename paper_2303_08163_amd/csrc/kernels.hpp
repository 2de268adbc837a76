// kernels.hpp -- gfx950 kernels of one periodic domain: initialisation, the
// fused pull-stream-and-collide step, moments with deterministic reductions,
// and population export.
//
// Data layout in HBM.  Nodes are grouped in rows along x: row = z ny + y.
// Population i of node (x, row) lives at buf[i * ps + row * rs + x], where
//   - row-interleaved layout (default): ps = pitch, rs = Q * pitch, i.e. each
//     row stores its Q population runs back to back ([z][y][i][x]); pitch is
//     nx rounded up to 16 elements (nx itself below 16);
//   - plane layout: ps = plane stride (>= N, a multiple of 64 plus optional
//     padding), rs = nx ([i][z][y][x], one plane per population).
// With the row-interleaved layout a row update reads 9 (D3Q27) or 3 (D2Q9)
// contiguous runs of 3 populations from the source rows (y - c_y, z - c_z) and
// writes one contiguous run of Q populations, so far fewer DRAM pages are open
// at once than with Q separate planes.  Two buffers alternate (read one,
// write the other).
//
// Streaming (Sec. "Basic concepts", left side of the LBGK equation) is done by
// pulling: the buffer holds post-collision values f*(r, t), and the step at r
// reads f*_i(r - c_i, t) = f_i(r, t + 1), collides, and writes f*_i(r, t + 1)
// back at r.  Every value is read once and written once per step: the
// algorithmic HBM traffic is 2 Q sizeof(storage) bytes per node update.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "node.hpp"

namespace lbm {

struct StepArgs {
    const void *src;
    void *dst;
    int nx, ny, nz;
    int tiles_x, tiles_y;  // workgroup tiles per row / per plane
    int64_t ps, rs;        // population and row strides (elements)
    Relax relax;
    int *flag;
    int zhalo;  // 1: z-slab, planes -1 and nz are halo planes (no periodic wrap in z)
};

// Fused halo exchange of a z-slab, the extra argument of the *_halo step
// kernels (a separate parameter, so that the plain kernels keep their
// argument layout).  recv[0] / recv[1]: packed [y][k][x] runs of the
// populations entering across the lower face (c_z = +1, i = 18..26) / upper
// face (c_z = -1, i = 0..8), read instead of the halo planes; send[0] /
// send[1]: the same packing of the populations leaving across the lower face
// (plane 0, i = 0..8) / upper face (plane nz - 1, i = 18..26), written besides
// the slab's own buffer.
struct HaloArgs {
    const void *recv[2];
    void *send[2];
};

// Row y' of the packed halo buffer: population k of the face's 9 starts at
// (y' * 9 + k) * nx.
__device__ __forceinline__ int64_t packed_run(int yrow, int k, int nx) { return ((int64_t)yrow * 9 + k) * nx; }

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup w runs on
// XCD w mod 8).  Give each XCD one contiguous range of tiles, walked in order,
// so that tiles adjacent in x (which share the cache lines at their boundary
// through the one-element shifted loads) run on the same XCD and its L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int w, int count) {
    const int per = count / kXcds, rem = count % kXcds;
    const int xcd = w % kXcds, k = w / kXcds;
    return xcd * per + (xcd < rem ? xcd : rem) + k;
}

// Record that some node of the calling wavefront left the equilibrium's
// domain: one store per wavefront (by its first active lane), not one atomic
// per node, so a domain that has blown up costs no more per step than a
// healthy one.  Every writer stores the same value, so the race is benign.
__device__ __forceinline__ void raise_flag(int *flag, bool bad) {
    const unsigned long long any = __ballot(bad);
    if (any != 0ull) {
        const unsigned long long active = __ballot(1);
        if ((int)__lane_id() == __ffsll((long long)active) - 1)
            __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Source rows r - c for c_y, c_z = -1, 0, +1 on the periodic grid, as element
// offsets of population 0.  In a z-slab (zhalo) the planes z - 1 and z + 1 are
// taken as they are: at the slab's faces they are the halo planes -1 and nz,
// which hold the neighbouring slabs' populations.
template <int DIM>
__device__ __forceinline__ void source_rows(int y, int z, int ny, int nz, int64_t rs, int64_t (&rowoff)[3][3],
                                            bool zhalo = false) {
    const int ys[3] = {y + 1 == ny ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
    int zs[3] = {z, z, z};
    if (DIM == 3) {
        zs[0] = z + 1 == nz && !zhalo ? 0 : z + 1;
        zs[2] = z == 0 && !zhalo ? nz - 1 : z - 1;
    }
#pragma unroll
    for (int cz = 0; cz < Lattice<DIM>::NZ; ++cz)
#pragma unroll
        for (int cy = 0; cy < Lattice<DIM>::NY; ++cy)
            rowoff[cz][cy] = (int64_t)(zs[cz] * ny + (DIM == 1 ? y : ys[cy])) * rs;
}

// One node's pull-stream, collision and store.  src/dst are population
// buffers of one domain; (x, y, z) must lie inside the grid, or, with pad set,
// in the row padding of the row-interleaved layout (nx <= x < ps).  A padding
// lane goes through the same instructions as the nodes of its wavefront --
// it reads the row's last node, and its result is discarded -- and stores
// zeros into the padding with the same store instructions, so that the lines
// at a ragged row end are written whole, by one instruction per population.
// (A separate branch for the padding lanes diverges: the wavefront then issues
// a second set of Q stores, each line at the row end is written in two parts,
// and a step on a ragged width took up to 1.6 times as long.)  The padding is
// never read.
// With HALO (a fused z-slab step, recv/send non-null) the populations
// entering across a face are read from the packed buffers and those leaving
// are also written to send.  Without it the halo arguments are ignored and
// the code is that of the plain step.
template <int DIM, int DT, bool CORR, int EQ = kEqEntropic, bool HALO = false>
__device__ __forceinline__ void step_node(const store_t<DT> *__restrict__ src, store_t<DT> *__restrict__ dst,
                                          int nx, int ny, int nz, int64_t ps, int64_t rs, const Relax &relax,
                                          int *flag, int x, int y, int z, bool pad = false, bool zhalo = false,
                                          const void *recv_lo = nullptr, const void *recv_hi = nullptr,
                                          void *send_lo = nullptr, void *send_hi = nullptr) {
    using T = store_t<DT>;
    constexpr int Q = Lattice<DIM>::Q;
    const int xn = pad ? nx - 1 : x;  // node whose sources are read
    const int xs[3] = {xn + 1 == nx ? 0 : xn + 1, xn, xn == 0 ? nx - 1 : xn - 1};  // x - c_x
    int64_t rowoff[3][3];
    source_rows<DIM>(y, z, ny, nz, rs, rowoff, zhalo);
    const int ys[3] = {y + 1 == ny ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};  // y - c_y
    const T *from_lo = HALO && DIM == 3 && z == 0 ? static_cast<const T *>(recv_lo) : nullptr;
    const T *from_hi = HALO && DIM == 3 && z == nz - 1 ? static_cast<const T *>(recv_hi) : nullptr;
    T f[Q];
#pragma unroll
    for (int cz = 0; cz < Lattice<DIM>::NZ; ++cz)
#pragma unroll
        for (int cy = 0; cy < Lattice<DIM>::NY; ++cy)
#pragma unroll
            for (int cx = 0; cx < 3; ++cx) {
                const int i = cx + 3 * cy + 9 * cz;
                if (HALO && cz == 2 && from_lo)
                    f[i] = from_lo[packed_run(ys[cy], i - 18, nx) + xs[cx]];
                else if (HALO && cz == 0 && from_hi)
                    f[i] = from_hi[packed_run(ys[cy], i, nx) + xs[cx]];
                else
                    f[i] = src[rowoff[cz][cy] + i * ps + xs[cx]];
            }

    const bool bad = collide_dt<DIM, DT, CORR, EQ>(f, relax);
    raise_flag(flag, bad && !pad);

    const int64_t self = (int64_t)(z * ny + y) * rs + x;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        dst[self + i * ps] = pad ? T(0) : f[i];
    if (HALO && DIM == 3 && !pad) {
        if (z == 0 && send_lo)
#pragma unroll
            for (int i = 0; i < 9; ++i)
                static_cast<T *>(send_lo)[packed_run(y, i, nx) + x] = f[i];
        if (z == nz - 1 && send_hi)
#pragma unroll
            for (int i = 18; i < Q; ++i)
                static_cast<T *>(send_hi)[packed_run(y, i - 18, nx) + x] = f[i];
    }
}

// Whether a lane at x >= nx has a padding position to fill (row-interleaved
// layout, x below the pitch); other lanes past the row end do nothing.
template <int DIM>
__device__ __forceinline__ bool in_padding(int64_t ps, int64_t rs, int x) {
    return rs == (int64_t)Lattice<DIM>::Q * ps && x < ps;
}

// One LBGK step over the whole domain.  1-D grid of tiles_x * tiles_y * nz
// workgroups of blockDim.x * blockDim.y threads, one node per thread.
// (The launch dimensions come from the kernel: read there, the workgroup size
// is known to be uniform, which spares a load per thread.)
//
// Plane of tile-plane p: in a fused z-slab step the two face planes, which
// also write the send buffers, go first (p = 0 -> plane 0, p = 1 -> plane
// nz - 1), so that their extra stores overlap the interior planes rather than
// trailing the grid, and the sends are complete early.
template <bool HALO>
__device__ __forceinline__ int plane_of(int p, int nz) {
    if (!HALO || nz < 2)
        return p;
    return p == 0 ? 0 : p == 1 ? nz - 1 : p - 1;
}
template <int DIM, int DT, bool CORR, int EQ, bool HALO>
__device__ __forceinline__ void stream_collide(const StepArgs &a, const HaloArgs &h, int bdx, int bdy, int gdx) {
    const int t = xcd_tile((int)blockIdx.x, gdx);
    const int tx = t % a.tiles_x;
    const int ty = (t / a.tiles_x) % a.tiles_y;
    const int z = plane_of<HALO>(t / (a.tiles_x * a.tiles_y), a.nz);
    const int x = tx * bdx + (int)threadIdx.x;
    const int y = ty * bdy + (int)threadIdx.y;
    const bool pad = x >= a.nx;
    if (y >= a.ny || (pad && !in_padding<DIM>(a.ps, a.rs, x)))
        return;
    step_node<DIM, DT, CORR, EQ, HALO>(static_cast<const store_t<DT> *>(a.src), static_cast<store_t<DT> *>(a.dst),
                                       a.nx, a.ny, a.nz, a.ps, a.rs, a.relax, a.flag, x, y, z, pad, a.zhalo != 0,
                                       h.recv[0], h.recv[1], h.send[0], h.send[1]);
}

template <int DIM, int DT, bool CORR, int EQ = kEqEntropic>
__global__ __launch_bounds__(256) void k_stream_collide(StepArgs a) {
    stream_collide<DIM, DT, CORR, EQ, false>(a, HaloArgs{}, (int)blockDim.x, (int)blockDim.y, (int)gridDim.x);
}

// A z-slab step with the halo exchange fused in.
template <int DIM, int DT, bool CORR, int EQ = kEqEntropic>
__global__ __launch_bounds__(256) void k_stream_collide_halo(StepArgs a, HaloArgs h) {
    stream_collide<DIM, DT, CORR, EQ, true>(a, h, (int)blockDim.x, (int)blockDim.y, (int)gridDim.x);
}

// ---------------------------------------------------------------------------
// Vectorised step: each thread owns NPT consecutive nodes of a row and moves
// every population run with one aligned NPT-wide load and store (16 bytes for
// float x 4 or double x 2).  The x-shifted populations need one element
// beyond the thread's run on one side; it comes from the neighbouring lane of
// the same wavefront by a lane rotation, and at the two ends of the
// wavefront's run from a single-lane load (or, when one wavefront spans the
// whole row, from the rotation itself, which then is the periodic wrap).
// Needs nx % (blockDim.x * NPT) == 0, blockDim.x a multiple of 64, and
// 16-byte aligned runs (ps and rs multiples of NPT).
template <typename T, int NPT>
struct VecT;
template <>
struct VecT<float, 4> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct VecT<float, 2> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct VecT<double, 2> {
    typedef double type __attribute__((ext_vector_type(2)));
};

// Kernel flags (results never depend on them).
constexpr int kNtStore = 1;  // non-temporal stores
constexpr int kNtLoad = 2;   // non-temporal loads

template <typename V, int FLAGS>
__device__ __forceinline__ V load_vec(const V *p) {
    if (FLAGS & kNtLoad)
        return __builtin_nontemporal_load(p);
    return *p;
}
template <typename V, int FLAGS>
__device__ __forceinline__ void store_vec(V v, V *p) {
    if (FLAGS & kNtStore)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// One population run of the vector step: an aligned NPT-wide load and, for the
// x-shifted populations (cx = 0: c_x = -1, cx = 2: c_x = +1), the element from
// the neighbouring lane or, at the wavefront's ends, a single-lane load.
template <typename T, typename V, int NPT, bool ROWWAVE, int FLAGS>
__device__ __forceinline__ void pull_run(const T *__restrict__ run, int x0, int lane, int x_left, int x_right, int cx,
                                         T (&gi)[NPT]) {
    const V v = load_vec<V, FLAGS>(reinterpret_cast<const V *>(run + x0));
    if (cx == 1) {
#pragma unroll
        for (int k = 0; k < NPT; ++k)
            gi[k] = v[k];
    } else if (cx == 2) {
        T left = __shfl(v[NPT - 1], (lane + 63) & 63, 64);
        if (!ROWWAVE && lane == 0)
            left = run[x_left];
        gi[0] = left;
#pragma unroll
        for (int k = 1; k < NPT; ++k)
            gi[k] = v[k - 1];
    } else {
        T right = __shfl(v[0], (lane + 1) & 63, 64);
        if (!ROWWAVE && lane == 63)
            right = run[x_right];
#pragma unroll
        for (int k = 0; k < NPT - 1; ++k)
            gi[k] = v[k + 1];
        gi[NPT - 1] = right;
    }
}

template <int DIM, int DT, bool CORR, int NPT, bool ROWWAVE, int FLAGS, int EQ, bool HALO>
__device__ __forceinline__ void stream_collide_vec(const StepArgs &a, const HaloArgs &h, int bdx, int bdy, int gdx) {
    using T = store_t<DT>;
    using V = typename VecT<T, NPT>::type;
    constexpr int Q = Lattice<DIM>::Q;
    const int t = xcd_tile((int)blockIdx.x, gdx);
    const int tx = t % a.tiles_x;
    const int ty = (t / a.tiles_x) % a.tiles_y;
    const int z = plane_of<HALO>(t / (a.tiles_x * a.tiles_y), a.nz);
    const int y = ty * bdy + (int)threadIdx.y;
    if (y >= a.ny)  // uniform per wavefront
        return;
    const int nx = a.nx;
    const int64_t ps = a.ps;
    const int lane = (int)threadIdx.x & 63;
    const int x0 = (tx * bdx + (int)threadIdx.x) * NPT;  // first node of this thread
    const T *__restrict__ src = static_cast<const T *>(a.src);
    T *__restrict__ dst = static_cast<T *>(a.dst);

    int64_t rowoff[3][3];
    source_rows<DIM>(y, z, a.ny, a.nz, a.rs, rowoff, a.zhalo != 0);
    // fused z-slab step: the face planes' entering runs come from the packed
    // buffers (wavefront-uniform choice)
    const int ys[3] = {y + 1 == a.ny ? 0 : y + 1, y, y == 0 ? a.ny - 1 : y - 1};  // y - c_y
    const T *from_lo = HALO && DIM == 3 && z == 0 ? static_cast<const T *>(h.recv[0]) : nullptr;
    const T *from_hi = HALO && DIM == 3 && z == a.nz - 1 ? static_cast<const T *>(h.recv[1]) : nullptr;
    // neighbours of the run at the wavefront's ends (periodic in x)
    const int x_left = x0 == 0 ? nx - 1 : x0 - 1;
    const int x_right = x0 + NPT == nx ? 0 : x0 + NPT;

    T g[Q][NPT];  // g[i][k]: value population i pulls into node x0 + k
    if constexpr (HALO) {
        // fused z-slab step: `face` selects, per wavefront, the variant that
        // reads the face planes' entering runs from the packed buffers, so
        // that rows inside the slab run the plain loads
        auto pull = [&](auto face) {
            constexpr bool F = decltype(face)::value;
#pragma unroll
            for (int cz = 0; cz < Lattice<DIM>::NZ; ++cz)
#pragma unroll
                for (int cy = 0; cy < Lattice<DIM>::NY; ++cy)
#pragma unroll
                    for (int cx = 0; cx < 3; ++cx) {
                        const int i = cx + 3 * cy + 9 * cz;
                        const T *__restrict__ run = F && cz == 2 && from_lo   ? from_lo + packed_run(ys[cy], i - 18, nx)
                                                    : F && cz == 0 && from_hi ? from_hi + packed_run(ys[cy], i, nx)
                                                                              : src + rowoff[cz][cy] + i * ps;
                        pull_run<T, V, NPT, ROWWAVE, FLAGS>(run, x0, lane, x_left, x_right, cx, g[i]);
                    }
        };
        if (from_lo || from_hi)  // uniform per wavefront
            pull(std::true_type{});
        else
            pull(std::false_type{});
    } else {
        // the plain step keeps its own loop (the generic lambda above compiles
        // to a longer instruction stream)
#pragma unroll
        for (int cz = 0; cz < Lattice<DIM>::NZ; ++cz)
#pragma unroll
            for (int cy = 0; cy < Lattice<DIM>::NY; ++cy)
#pragma unroll
                for (int cx = 0; cx < 3; ++cx) {
                    const int i = cx + 3 * cy + 9 * cz;
                    const T *__restrict__ run = src + rowoff[cz][cy] + i * ps;
                    const V v = load_vec<V, FLAGS>(reinterpret_cast<const V *>(run + x0));
                    if (cx == 1) {  // c_x = 0: aligned
#pragma unroll
                        for (int k = 0; k < NPT; ++k)
                            g[i][k] = v[k];
                    } else if (cx == 2) {  // c_x = +1 pulls from x - 1
                        T left = __shfl(v[NPT - 1], (lane + 63) & 63, 64);
                        if (!ROWWAVE && lane == 0)
                            left = run[x_left];
                        g[i][0] = left;
#pragma unroll
                        for (int k = 1; k < NPT; ++k)
                            g[i][k] = v[k - 1];
                    } else {  // c_x = -1 pulls from x + 1
                        T right = __shfl(v[0], (lane + 1) & 63, 64);
                        if (!ROWWAVE && lane == 63)
                            right = run[x_right];
#pragma unroll
                        for (int k = 0; k < NPT - 1; ++k)
                            g[i][k] = v[k + 1];
                        g[i][NPT - 1] = right;
                    }
                }
    }

    bool bad = false;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        T f[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i)
            f[i] = g[i][k];
        bad |= collide_dt<DIM, DT, CORR, EQ>(f, a.relax);
#pragma unroll
        for (int i = 0; i < Q; ++i)
            g[i][k] = f[i];
    }
    raise_flag(a.flag, bad);

    const int64_t self = (int64_t)(z * a.ny + y) * a.rs + x0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        V v;
#pragma unroll
        for (int k = 0; k < NPT; ++k)
            v[k] = g[i][k];
        store_vec<V, FLAGS>(v, reinterpret_cast<V *>(dst + self + i * ps));
    }
    if (HALO && DIM == 3 && z == 0 && h.send[0]) {  // leaving across the lower face: i = 0..8
        T *out = static_cast<T *>(h.send[0]);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            V v;
#pragma unroll
            for (int k = 0; k < NPT; ++k)
                v[k] = g[i][k];
            store_vec<V, FLAGS>(v, reinterpret_cast<V *>(out + packed_run(y, i, nx) + x0));
        }
    }
    if (HALO && DIM == 3 && z == a.nz - 1 && h.send[1]) {  // leaving across the upper face: i = 18..26
        T *out = static_cast<T *>(h.send[1]);
#pragma unroll
        for (int i = 18; i < Q; ++i) {
            V v;
#pragma unroll
            for (int k = 0; k < NPT; ++k)
                v[k] = g[i][k];
            store_vec<V, FLAGS>(v, reinterpret_cast<V *>(out + packed_run(y, i - 18, nx) + x0));
        }
    }
}

template <int DIM, int DT, bool CORR, int NPT, bool ROWWAVE, int FLAGS, int EQ = kEqEntropic>
__global__ __launch_bounds__(256) void k_stream_collide_vec(StepArgs a) {
    stream_collide_vec<DIM, DT, CORR, NPT, ROWWAVE, FLAGS, EQ, false>(a, HaloArgs{}, (int)blockDim.x, (int)blockDim.y,
                                                                      (int)gridDim.x);
}

// A z-slab step with the halo exchange fused in.
template <int DIM, int DT, bool CORR, int NPT, bool ROWWAVE, int FLAGS, int EQ = kEqEntropic>
__global__ __launch_bounds__(256) void k_stream_collide_vec_halo(StepArgs a, HaloArgs h) {
    stream_collide_vec<DIM, DT, CORR, NPT, ROWWAVE, FLAGS, EQ, true>(a, h, (int)blockDim.x, (int)blockDim.y,
                                                                     (int)gridDim.x);
}

// Zero `count` 32-bit words (a kernel rather than a memset, so that the call
// sequence stays valid inside captured HIP graphs).
static __global__ void k_clear_words(int *p, int count) {
    for (int k = threadIdx.x; k < count; k += blockDim.x)
        p[k] = 0;
}

// Halo exchange of a z-slab: copy the 9 population runs with one sign of c_z
// of every row of one plane between the slab's buffer and a packed buffer
// [y][k][x] (k = 0..8 in population order, nx elements per run).  Element
// (y, k, x) is at src[y * s_row + k * s_run + x] and dst[y * d_row + k * d_run + x].
// A bit copy (E = element width), so the stored values move unchanged.  Up to
// two faces per launch (blockIdx.y); a face with a null dst is skipped.  One
// workgroup per run (blockIdx.x = y * 9 + k), threads along x: no per-element
// index division.
template <typename E>
struct HaloCopy {
    const E *src[2];
    E *dst[2];
    int nx;
    int64_t s_row, s_run, d_row, d_run;
};

template <typename E>
__global__ __launch_bounds__(256) void k_halo_copy(HaloCopy<E> a) {
    const int f = (int)blockIdx.y;
    const E *__restrict__ src = a.src[f];
    E *__restrict__ dst = a.dst[f];
    if (dst == nullptr)
        return;
    const int64_t y = blockIdx.x / 9, k = blockIdx.x - y * 9;
    const E *__restrict__ s = src + y * a.s_row + k * a.s_run;
    E *__restrict__ d = dst + y * a.d_row + k * a.d_run;
    for (int x = (int)threadIdx.x; x < a.nx; x += (int)blockDim.x)
        d[x] = s[x];
}

// Element offset of population 0 of node n (x fastest) in a buffer.
__device__ __forceinline__ int64_t node_offset(int64_t n, int nx, int64_t rs) {
    const int64_t row = n / nx;
    return row * rs + (n - row * nx);
}

struct InitArgs {
    void *dst;
    const double *rho;
    const double *u;  // D planes of N
    int64_t n;
    int nx;
    int64_t ps, rs;
    double rho0;
    int *flag;
};

// f = f^eq(rho, u) at every node.
template <int DIM, bool DEV, int EQ = kEqEntropic>
__global__ __launch_bounds__(256) void k_init(InitArgs a) {
    using T = store_t<DEV>;
    constexpr int Q = Lattice<DIM>::Q;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.n)
        return;
    double u[3] = {a.u[n], DIM >= 2 ? a.u[a.n + n] : 0.0, DIM == 3 ? a.u[2 * a.n + n] : 0.0};
    double f[Q];
    const bool bad = equilibrium_stored<DIM, DEV, EQ>(a.rho[n], u, a.rho0, f);
    raise_flag(a.flag, bad);
    T *dst = static_cast<T *>(a.dst) + node_offset(n, a.nx, a.rs);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        dst[i * a.ps] = (T)f[i];
}

// Diagnostics partials per workgroup: mass, momentum x/y/z, kinetic energy,
// max |u_a|, min rho.
constexpr int kDiagFields = 7;
constexpr int kReduceThreads = 256;

struct MomentArgs {
    const void *src;
    double *rho;  // may be null
    double *u;    // may be null
    int64_t n;
    int nx;
    int64_t ps, rs;
    double rho0;
    double *partials;  // gridDim.x * kDiagFields
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

// Reduce kDiagFields values across a 256-thread workgroup in a fixed order
// (wavefront butterflies, then the 4 wave results in index order).
__device__ __forceinline__ void block_reduce_diag(double (&acc)[kDiagFields], double *out) {
    __shared__ double lds[kReduceThreads / 64][kDiagFields];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 5; ++k)
        acc[k] = wave_sum(acc[k]);
    acc[5] = wave_max(acc[5]);
    acc[6] = wave_min(acc[6]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < kDiagFields; ++k)
            lds[wave][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        double r[kDiagFields];
#pragma unroll
        for (int k = 0; k < kDiagFields; ++k)
            r[k] = lds[0][k];
        for (int w = 1; w < kReduceThreads / 64; ++w) {
#pragma unroll
            for (int k = 0; k < 5; ++k)
                r[k] += lds[w][k];
            r[5] = fmax(r[5], lds[w][5]);
            r[6] = fmin(r[6], lds[w][6]);
        }
#pragma unroll
        for (int k = 0; k < kDiagFields; ++k)
            out[k] = r[k];
    }
}

template <int DIM, bool DEV>
__global__ __launch_bounds__(kReduceThreads) void k_moments(MomentArgs a) {
    using T = store_t<DEV>;
    constexpr int Q = Lattice<DIM>::Q;
    const T *src = static_cast<const T *>(a.src);
    double acc[kDiagFields] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, INFINITY};
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < a.n;
         n += (int64_t)gridDim.x * blockDim.x) {
        const T *p = src + node_offset(n, a.nx, a.rs);
        double f[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i)
            f[i] = (double)p[i * a.ps];
        double rho, j[3];
        node_moments<DIM>(f, DEV ? a.rho0 : 0.0, rho, j);
        const double inv = 1.0 / rho;
        const double u[3] = {j[0] * inv, j[1] * inv, j[2] * inv};
        if (a.rho)
            a.rho[n] = rho;
        if (a.u) {
#pragma unroll
            for (int d = 0; d < DIM; ++d)
                a.u[d * a.n + n] = u[d];
        }
        acc[0] += rho;
        acc[1] += j[0];
        acc[2] += j[1];
        acc[3] += j[2];
        acc[4] += 0.5 * ((j[0] * u[0] + j[1] * u[1]) + j[2] * u[2]);
        acc[5] = fmax(acc[5], fmax(fabs(u[0]), fmax(fabs(u[1]), fabs(u[2]))));
        acc[6] = fmin(acc[6], rho);
    }
    block_reduce_diag(acc, a.partials + (int64_t)blockIdx.x * kDiagFields);
}

// Second pass: one workgroup folds the per-workgroup partials in a fixed order.
static __global__ __launch_bounds__(kReduceThreads) void k_reduce_partials(const double *partials, int count,
                                                                    double *out) {
    double acc[kDiagFields] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, INFINITY};
    for (int b = threadIdx.x; b < count; b += blockDim.x) {
        const double *p = partials + (int64_t)b * kDiagFields;
#pragma unroll
        for (int k = 0; k < 5; ++k)
            acc[k] += p[k];
        acc[5] = fmax(acc[5], p[5]);
        acc[6] = fmin(acc[6], p[6]);
    }
    block_reduce_diag(acc, out);
}

// Quadratic acoustic energy about a reference state (rho_ref, U), summed over
// the grid: e = rho_ref |u - U|^2 / 2 + c_s^2 (rho - rho_ref)^2 / (2 rho_ref),
// c_s^2 = 1/3.  Per-workgroup partial sums, then one fixed-order fold.
struct EnergyArgs {
    const void *src;
    int64_t n;
    int nx;
    int64_t ps, rs;
    double rho0;  // deviation reference of the storage (0 for FP64 storage)
    double rho_ref;
    double U[3];
    double *partials;  // gridDim.x values
};

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double lds[kReduceThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0)
        lds[wave] = v;
    __syncthreads();
    double r = lds[0];
    for (int w = 1; w < kReduceThreads / 64; ++w)
        r += lds[w];
    return r;
}

template <int DIM, bool DEV>
__global__ __launch_bounds__(kReduceThreads) void k_energy(EnergyArgs a) {
    using T = store_t<DEV>;
    constexpr int Q = Lattice<DIM>::Q;
    const T *src = static_cast<const T *>(a.src);
    const double half_cs2_over_rho = (1.0 / 6.0) / a.rho_ref;
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < a.n;
         n += (int64_t)gridDim.x * blockDim.x) {
        const T *p = src + node_offset(n, a.nx, a.rs);
        double f[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i)
            f[i] = (double)p[i * a.ps];
        double rho, j[3];
        node_moments<DIM>(f, DEV ? a.rho0 : 0.0, rho, j);
        const double inv = 1.0 / rho;
        double du2 = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const double du = j[d] * inv - a.U[d];
            du2 = fma(du, du, du2);
        }
        const double dr = rho - a.rho_ref;
        acc += fma(0.5 * a.rho_ref, du2, (dr * dr) * half_cs2_over_rho);
    }
    const double r = block_sum(acc);
    if (threadIdx.x == 0)
        a.partials[blockIdx.x] = r;
}

static __global__ __launch_bounds__(kReduceThreads) void k_sum_partials(const double *partials, int count,
                                                                        double *out) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < count; b += blockDim.x)
        acc += partials[b];
    const double r = block_sum(acc);
    if (threadIdx.x == 0)
        *out = r;
}

struct ExportArgs {
    const void *src;
    double *out;
    int64_t n;
    int nx;
    int64_t ps, rs;
    double rho0;
};

template <int DIM, bool DEV>
__global__ __launch_bounds__(256) void k_export(ExportArgs a) {
    using T = store_t<DEV>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.n)
        return;
    const T *p = static_cast<const T *>(a.src) + node_offset(n, a.nx, a.rs);
#pragma unroll
    for (int i = 0; i < Lattice<DIM>::Q; ++i) {
        double v = (double)p[i * a.ps];
        if (DEV)
            v = fma(Lattice<DIM>::weight(i), a.rho0, v);
        a.out[i * a.n + n] = v;
    }
}

}  // namespace lbm
