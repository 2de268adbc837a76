// vn.hip -- von Neumann spectra on the GPU: one amplification matrix per
// thread (see vn.hpp), batched over cases, and the largest spectral radius
// over a grid of wave vectors for many states at once (the inner loop of the
// linear-stability-domain search of Sec. "Linear stability domain").
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "lbm.h"
#include "lbm_internal.hpp"
#include "vn.hpp"

namespace lbm {

constexpr int kVnThreads = 64;  // one wavefront per workgroup

// Largest v over the wavefront (all 64 lanes take part): the device
// library's reduction, by lane moves within and across rows of 16 lanes and
// two lane reads, with none of the round trips through LDS that a shuffle
// takes (the QR loop waits on this value after every step).
__device__ __forceinline__ int wave_max_int(int v) { return __ockl_wfred_max_i32(v); }

struct VnSpectraArgs {
    const double *cases;  // count x 5: tau, u_x, u_y, k_x, k_y
    int64_t count;
    double *radius;  // count, or null
    double *eig;     // count x N x 2, or null
    int *info;       // count, or null: QR steps taken, -1 if the limit was reached
    double *flops;   // count, or null: FP64 operations spent on the case
};

template <int DIM, int EQ, bool CORR>
__global__ __launch_bounds__(kVnThreads) void k_vn_spectra(VnSpectraArgs a) {
    constexpr int N = DIM == 1 ? 3 : 9;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // lanes past the end repeat the last case (every lane must reach the
    // wavefront-wide reductions of the eigensolver) and write nothing
    const bool live = t0 < a.count;
    const int64_t t = live ? t0 : a.count - 1;
    const double *p = a.cases + 5 * t;
    const double tau = p[0];
    const double u[2] = {p[1], DIM == 2 ? p[2] : 0.0};
    const double k[2] = {p[3], DIM == 2 ? p[4] : 0.0};
    cplx H[N][N];
    vn_matrix<DIM, EQ, CORR>(tau, u, k, H);
    hessenberg<N>(H);
    double work = vn_build_flops<DIM, EQ, CORR>() + vn_reduce_flops<N>();
    const int steps = hessenberg_eigenvalues<N>(H, wave_max_int, &work);
    if (!live)
        return;
    double r2 = 0.0;  // largest |eigenvalue|^2 (O(1) values: no rescaling)
#pragma unroll
    for (int i = 0; i < N; ++i) {
        r2 = fmax(r2, fma(H[i][i].re, H[i][i].re, H[i][i].im * H[i][i].im));
        if (a.eig) {
            a.eig[(t * N + i) * 2 + 0] = H[i][i].re;
            a.eig[(t * N + i) * 2 + 1] = H[i][i].im;
        }
    }
    if (a.radius)
        a.radius[t] = sqrt(r2);
    if (a.info)
        a.info[t] = steps;
    if (a.flops)
        a.flops[t] = work;
}

struct VnMaxArgs {
    const double *states;  // n_states x 3: tau, u_x, u_y
    int64_t n_states;
    int nk;                    // wave-vector points per axis on [0, pi]
    int64_t per_state;         // nk^DIM
    unsigned long long *rmax;  // n_states: bit pattern of the largest radius (non-negative doubles order as integers)
    int *unconverged;          // one counter
};

template <int DIM, int EQ, bool CORR>
__global__ __launch_bounds__(kVnThreads) void k_vn_max_radius(VnMaxArgs a) {
    constexpr int N = DIM == 1 ? 3 : 9;
    const int64_t total = a.n_states * a.per_state;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = t0 < total;  // lanes past the end repeat the last matrix, write nothing
    const int64_t t = live ? t0 : total - 1;
    const int64_t s = t / a.per_state;
    const int64_t q = t - s * a.per_state;
    const double dk = a.nk > 1 ? 3.141592653589793 / (double)(a.nk - 1) : 0.0;
    const int ix = (int)(q % a.nk), iy = DIM == 2 ? (int)(q / a.nk) : 0;
    const double *p = a.states + 3 * s;
    const double tau = p[0];
    const double u[2] = {p[1], DIM == 2 ? p[2] : 0.0};
    const double k[2] = {ix * dk, iy * dk};
    cplx H[N][N];
    vn_matrix<DIM, EQ, CORR>(tau, u, k, H);
    hessenberg<N>(H);
    const int steps = hessenberg_eigenvalues<N>(H, wave_max_int);
    if (!live)
        return;
    double r2 = 0.0;  // largest |eigenvalue|^2 (O(1) values: no rescaling)
#pragma unroll
    for (int i = 0; i < N; ++i)
        r2 = fmax(r2, fma(H[i][i].re, H[i][i].re, H[i][i].im * H[i][i].im));
    const double r = sqrt(r2);
    if (steps < 0)
        atomicAdd(a.unconverged, 1);
    atomicMax(a.rmax + s, (unsigned long long)__double_as_longlong(r));
}

static __global__ void k_vn_clear(unsigned long long *p, int64_t n, int *counter) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n)
        p[t] = 0ull;
    if (t == 0)
        *counter = 0;
}

static __global__ void k_vn_bits_to_double(const unsigned long long *bits, int64_t n, double *out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n)
        out[t] = __longlong_as_double((long long)bits[t]);
}

using SpectraFn = void (*)(VnSpectraArgs);
using MaxFn = void (*)(VnMaxArgs);

template <int DIM, int EQ>
static void pick(bool corr, SpectraFn &sf, MaxFn &mf) {
    sf = corr ? k_vn_spectra<DIM, EQ, true> : k_vn_spectra<DIM, EQ, false>;
    mf = corr ? k_vn_max_radius<DIM, EQ, true> : k_vn_max_radius<DIM, EQ, false>;
}

template <int DIM>
static void pick_eq(int eq, bool corr, SpectraFn &sf, MaxFn &mf) {
    if (eq == LBM_EQ_POLY2)
        pick<DIM, kEqPoly2>(corr, sf, mf);
    else if (eq == LBM_EQ_PRODUCT)
        pick<DIM, kEqProduct>(corr, sf, mf);
    else
        pick<DIM, kEqEntropic>(corr, sf, mf);
}

static int vn_select(int32_t lattice, int32_t equilibrium, int32_t corr, SpectraFn &sf, MaxFn &mf, int &dim) {
    if (lattice != LBM_D1Q3 && lattice != LBM_D2Q9) {
        set_error("von Neumann spectra: lattice must be LBM_D1Q3 or LBM_D2Q9");
        return LBM_EINVAL;
    }
    if (equilibrium != LBM_EQ_ENTROPIC && equilibrium != LBM_EQ_POLY2 && equilibrium != LBM_EQ_PRODUCT) {
        set_error("von Neumann spectra: bad equilibrium");
        return LBM_EINVAL;
    }
    if (corr != 0 && corr != 1) {
        set_error("von Neumann spectra: bulk_correction must be 0 or 1");
        return LBM_EINVAL;
    }
    dim = lattice == LBM_D1Q3 ? 1 : 2;
    if (dim == 1)
        pick_eq<1>(equilibrium, corr != 0, sf, mf);
    else
        pick_eq<2>(equilibrium, corr != 0, sf, mf);
    return LBM_OK;
}

// Scratch of the allocation-free form of lbm_vn_max_radius: the per-state
// running maxima (bit patterns) of kVnStaticStates states.  In host code the
// name is only a stand-in; kernels get the device address that
// hipGetSymbolAddress returns for the current device (each GPU holds its own
// copy).
constexpr int64_t kVnStaticStates = 65536;
static __device__ __align__(256) unsigned long long scratch[kVnStaticStates];

constexpr int kVnMaxDevices = 64;
static std::mutex g_scratch_mutex;
static unsigned long long *g_scratch_ptr[kVnMaxDevices];

// Device address of `scratch` on the current device, looked up once per device.
static int static_scratch(unsigned long long **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "device query");
    if (dev < 0 || dev >= kVnMaxDevices) {
        set_error("device index beyond the static scratch table");
        return LBM_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_fail(e, "scratch symbol address");
        g_scratch_ptr[dev] = static_cast<unsigned long long *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

// The three launches of a max-radius call on `bits` (n_states entries, 8-byte
// aligned): clear, per-matrix radii into the maxima, maxima to doubles.
static int launch_max_radius(MaxFn mf, int dim, const double *states, int64_t n_states, int32_t nk,
                             double *max_radius, unsigned long long *bits, int32_t *unconverged, hipStream_t s) {
    const int64_t per = dim == 1 ? (int64_t)nk : (int64_t)nk * nk;
    const int64_t total = n_states * per;
    if (total > ((int64_t)INT32_MAX - 1) * kVnThreads) {
        set_error("von Neumann max radius: too many matrices per call");
        return LBM_EINVAL;
    }
    const int64_t nclear = n_states > 0 ? n_states : 1;
    hipLaunchKernelGGL(k_vn_clear, dim3((unsigned)((nclear + 255) / 256)), dim3(256), 0, s, bits, n_states,
                       unconverged);
    if (total > 0) {
        VnMaxArgs a{states, n_states, nk, per, bits, unconverged};
        hipLaunchKernelGGL(mf, dim3((unsigned)((total + kVnThreads - 1) / kVnThreads)), dim3(kVnThreads), 0, s, a);
        hipLaunchKernelGGL(k_vn_bits_to_double, dim3((unsigned)((n_states + 255) / 256)), dim3(256), 0, s,
                           (const unsigned long long *)bits, n_states, max_radius);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, "von Neumann max radius launch");
    return LBM_OK;
}

}  // namespace lbm

using namespace lbm;

extern "C" {

int lbm_vn_spectra(int32_t lattice, int32_t equilibrium, int32_t bulk_correction, const double *cases,
                   int64_t count, double *radius, double *eig, int32_t *info, double *flops, void *stream) {
    SpectraFn sf;
    MaxFn mf;
    int dim;
    int rc = vn_select(lattice, equilibrium, bulk_correction, sf, mf, dim);
    if (rc != LBM_OK)
        return rc;
    if (count < 0 || (count > 0 && !cases) || count > ((int64_t)1 << 40)) {
        set_error("von Neumann spectra: NULL cases or bad count");
        return LBM_EINVAL;
    }
    if (count == 0)
        return LBM_OK;
    VnSpectraArgs a{cases, count, radius, eig, info, flops};
    const int64_t blocks = (count + kVnThreads - 1) / kVnThreads;
    if (blocks > INT32_MAX) {
        set_error("von Neumann spectra: too many cases");
        return LBM_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(sf, dim3((unsigned)blocks), dim3(kVnThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, "von Neumann spectra launch");
    return LBM_OK;
}

int lbm_vn_max_radius(int32_t lattice, int32_t equilibrium, int32_t bulk_correction, const double *states,
                      int64_t n_states, int32_t nk, double *max_radius, void *scratch, int32_t *unconverged,
                      void *stream) {
    SpectraFn sf;
    MaxFn mf;
    int dim;
    int rc = vn_select(lattice, equilibrium, bulk_correction, sf, mf, dim);
    if (rc != LBM_OK)
        return rc;
    if (n_states < 0 || nk < 1 || nk > 65536 || (n_states > 0 && (!states || !max_radius || !scratch)) ||
        !unconverged) {
        set_error("von Neumann max radius: NULL pointer or bad sizes");
        return LBM_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(scratch) & 7u) != 0) {
        set_error("von Neumann max radius: scratch must be 8-byte aligned");
        return LBM_EINVAL;
    }
    return launch_max_radius(mf, dim, states, n_states, nk, max_radius, static_cast<unsigned long long *>(scratch),
                             unconverged, static_cast<hipStream_t>(stream));
}

int lbm_vn_max_radius_noalloc(int32_t lattice, int32_t equilibrium, int32_t bulk_correction, const double *states,
                              int64_t n_states, int32_t nk, double *max_radius, int32_t *unconverged, void *stream) {
    SpectraFn sf;
    MaxFn mf;
    int dim;
    int rc = vn_select(lattice, equilibrium, bulk_correction, sf, mf, dim);
    if (rc != LBM_OK)
        return rc;
    if (n_states < 0 || nk < 1 || nk > 65536 || (n_states > 0 && (!states || !max_radius)) || !unconverged) {
        set_error("von Neumann max radius: NULL pointer or bad sizes");
        return LBM_EINVAL;
    }
    if (n_states > kVnStaticStates) {
        set_error("von Neumann max radius (no allocation): more than 65536 states per call");
        return LBM_EINVAL;
    }
    unsigned long long *bits = nullptr;
    rc = static_scratch(&bits);
    if (rc != LBM_OK)
        return rc;
    return launch_max_radius(mf, dim, states, n_states, nk, max_radius, bits, unconverged,
                             static_cast<hipStream_t>(stream));
}

}  // extern "C"
