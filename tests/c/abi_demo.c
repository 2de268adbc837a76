/* abi_demo.c -- a plain C99 caller of the library's C ABI (include/lbm.h).
 *
 * Uses only the header and the HIP runtime API for device memory; no C++ and
 * no Python.  Checks, on the GPU:
 *   1. a D3Q27 FP32 domain: create, 50 steps, moments (mass conserved to
 *      rounding, step count), populations, destroy;
 *   2. argument errors (LBM_EINVAL) on the paths a C caller can take;
 *   3. a pool of two D2Q9 domains of different sizes run to completion;
 *   4. a z-slab that is its own neighbour equals the periodic domain of the
 *      same planes, bitwise, with the halo exchange through pack/unpack and
 *      with it fused into the step (lbm_step_halo).
 * Prints "abi_demo ok" and returns 0 on success; prints the failed check and
 * returns 1 otherwise. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm.h"

static int failures = 0;
#define CHECK(cond, what)                                      \
    do {                                                       \
        if (!(cond)) {                                         \
            printf("FAILED: %s (line %d)\n", what, __LINE__); \
            fflush(stdout);                                    \
            failures++;                                        \
        }                                                      \
    } while (0)
#define HIPCHECK(x)                                                              \
    do {                                                                         \
        hipError_t e_ = (x);                                                     \
        if (e_ != hipSuccess) {                                                  \
            printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                            \
        }                                                                        \
    } while (0)

/* Smooth initial fields on an nx x ny x nz grid (x fastest): rho and D planes of u. */
static void fields(int64_t nx, int64_t ny, int64_t nz, int dim, double *rho, double *u) {
    const int64_t n = nx * ny * nz;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t k = (z * ny + y) * nx + x;
                const double a = 6.283185307179586 * (double)x / (double)nx;
                const double b = 6.283185307179586 * (double)y / (double)ny;
                const double c = 6.283185307179586 * (double)z / (double)nz;
                rho[k] = 1.0 + 0.01 * cos(a) * cos(c);
                u[k] = 0.05 * sin(b) * cos(c);
                u[n + k] = 0.03 * sin(a);
                if (dim == 3)
                    u[2 * n + k] = 0.02 * cos(a + b);
            }
}

static lbm_config config(int lattice, int64_t nx, int64_t ny, int64_t nz, int dtype, int z_halo) {
    lbm_config c;
    memset(&c, 0, sizeof c);
    c.lattice = lattice;
    c.dtype = dtype;
    c.nx = nx;
    c.ny = ny;
    c.nz = nz;
    c.tau = 0.6;
    c.bulk_correction = 1;
    c.equilibrium = LBM_EQ_ENTROPIC;
    c.rho0 = 1.0;
    c.z_halo = z_halo;
    return c;
}

/* Device copies of the initial fields of a grid. */
static int upload(int64_t nx, int64_t ny, int64_t nz, int dim, double **rho_d, double **u_d, double *mass) {
    const int64_t n = nx * ny * nz;
    double *rho = (double *)malloc(sizeof(double) * (size_t)n);
    double *u = (double *)calloc((size_t)(dim * n), sizeof(double));
    if (!rho || !u)
        return 1;
    fields(nx, ny, nz, dim, rho, u);
    *mass = 0.0;
    for (int64_t k = 0; k < n; ++k)
        *mass += rho[k];
    HIPCHECK(hipMalloc((void **)rho_d, sizeof(double) * (size_t)n));
    HIPCHECK(hipMalloc((void **)u_d, sizeof(double) * (size_t)(dim * n)));
    HIPCHECK(hipMemcpy(*rho_d, rho, sizeof(double) * (size_t)n, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(*u_d, u, sizeof(double) * (size_t)(dim * n), hipMemcpyHostToDevice));
    free(rho);
    free(u);
    return 0;
}

static int single_domain(void) {
    const int64_t nx = 40, ny = 24, nz = 18, n = nx * ny * nz;
    double *rho_d, *u_d, mass0;
    if (upload(nx, ny, nz, 3, &rho_d, &u_d, &mass0))
        return 1;
    lbm_config cfg = config(LBM_D3Q27, nx, ny, nz, LBM_FP32_DEV, 0);
    const size_t ws_bytes = lbm_workspace_bytes(&cfg);
    CHECK(ws_bytes > 0, "workspace size");
    void *ws;
    HIPCHECK(hipMalloc(&ws, ws_bytes));
    lbm_handle *h = NULL;
    CHECK(lbm_create(&cfg, ws, ws_bytes, rho_d, u_d, NULL, &h) == LBM_OK, "create");
    if (!h)
        return 1;
    CHECK(lbm_step(h, 50) == LBM_OK, "step");
    lbm_diag d;
    CHECK(lbm_moments(h, rho_d, u_d, &d) == LBM_OK, "moments");
    CHECK(d.steps == 50 && d.domain_error == 0, "step count");
    CHECK(fabs(d.mass - mass0) < 1e-9 * mass0, "mass conservation");
    double *f_d;
    HIPCHECK(hipMalloc((void **)&f_d, sizeof(double) * 27 * (size_t)n));
    CHECK(lbm_get_populations(h, f_d) == LBM_OK, "populations");
    double f0;
    HIPCHECK(hipMemcpy(&f0, f_d, sizeof(double), hipMemcpyDeviceToHost));
    CHECK(f0 > 0.0 && f0 < 1.0, "population value");
    /* checkpoint at step 50, run on, restart from it: the same bits again */
    const size_t st_bytes = lbm_state_bytes(h);
    void *st;
    HIPCHECK(hipMalloc(&st, st_bytes));
    CHECK(lbm_save_state(h, st, st_bytes) == LBM_OK, "save state");
    lbm_diag d1, d2;
    CHECK(lbm_step(h, 7) == LBM_OK && lbm_moments(h, NULL, NULL, &d1) == LBM_OK, "run on");
    CHECK(lbm_load_state(h, st, st_bytes, 50) == LBM_OK, "load state");
    CHECK(lbm_step(h, 7) == LBM_OK && lbm_moments(h, NULL, NULL, &d2) == LBM_OK, "run on again");
    CHECK(d1.steps == 57 && d2.steps == 57 && d1.kinetic_energy == d2.kinetic_energy && d1.mass == d2.mass,
          "restart is bit-exact");
    CHECK(lbm_load_state(h, st, st_bytes - 1, 50) == LBM_EINVAL, "load refuses a wrong size");
    HIPCHECK(hipFree(st));
    /* argument errors */
    CHECK(lbm_step(h, -1) == LBM_EINVAL, "negative step count");
    CHECK(lbm_step(NULL, 1) == LBM_EINVAL, "NULL handle");
    CHECK(lbm_halo_pack(h, f_d, NULL) == LBM_EINVAL, "halo pack on a periodic domain");
    lbm_config bad = cfg;
    bad.tau = 0.5;
    CHECK(lbm_workspace_bytes(&bad) == 0, "tau = 1/2 rejected");
    lbm_handle *h2 = NULL;
    CHECK(lbm_create(&bad, ws, ws_bytes, rho_d, u_d, NULL, &h2) == LBM_EINVAL && h2 == NULL, "create rejects tau");
    CHECK(lbm_create(&cfg, ws, 16, rho_d, u_d, NULL, &h2) == LBM_EINVAL, "create rejects a small workspace");
    CHECK(lbm_status_string(LBM_EINVAL) != NULL && strlen(lbm_last_error()) > 0, "error strings");
    CHECK(lbm_destroy(h) == LBM_OK && lbm_destroy(NULL) == LBM_OK, "destroy");
    HIPCHECK(hipFree(f_d));
    HIPCHECK(hipFree(ws));
    HIPCHECK(hipFree(rho_d));
    HIPCHECK(hipFree(u_d));
    return 0;
}

static int pool(void) {
    const int64_t dims[2][2] = {{70, 33}, {128, 96}};
    const int64_t steps[2] = {40, 25};
    double *rho_d[2], *u_d[2], mass0[2];
    size_t arena_bytes = lbm_pool_table_bytes(4);
    lbm_config cfg[2];
    for (int k = 0; k < 2; ++k) {
        if (upload(dims[k][0], dims[k][1], 1, 2, &rho_d[k], &u_d[k], &mass0[k]))
            return 1;
        cfg[k] = config(LBM_D2Q9, dims[k][0], dims[k][1], 1, k == 0 ? LBM_FP64 : LBM_FP32_DEV, 0);
        const size_t b = lbm_pool_slot_bytes(&cfg[k], NULL);
        CHECK(b > 0, "slot size");
        arena_bytes += b;
    }
    void *arena;
    HIPCHECK(hipMalloc(&arena, arena_bytes));
    lbm_pool *p = NULL;
    CHECK(lbm_pool_create(4, NULL, arena, arena_bytes, NULL, &p) == LBM_OK, "pool create");
    if (!p)
        return 1;
    int32_t slot[2];
    for (int k = 0; k < 2; ++k)
        CHECK(lbm_pool_admit(p, &cfg[k], rho_d[k], u_d[k], steps[k], &slot[k]) == LBM_OK, "admit");
    CHECK(lbm_pool_run(p, 100) == LBM_OK, "pool run");
    int32_t done[4], count = 0;
    CHECK(lbm_pool_poll(p, done, 4, &count) == LBM_OK && count == 2, "poll: both done");
    for (int k = 0; k < 2; ++k) {
        lbm_diag d;
        CHECK(lbm_pool_moments(p, slot[k], NULL, NULL, &d) == LBM_OK, "pool moments");
        CHECK(d.steps == steps[k], "pool step budget");
        CHECK(fabs(d.mass - mass0[k]) < 1e-9 * mass0[k], "pool mass conservation");
        CHECK(lbm_pool_release(p, slot[k]) == LBM_OK, "release");
    }
    CHECK(lbm_pool_destroy(p) == LBM_OK, "pool destroy");
    HIPCHECK(hipFree(arena));
    for (int k = 0; k < 2; ++k) {
        HIPCHECK(hipFree(rho_d[k]));
        HIPCHECK(hipFree(u_d[k]));
    }
    return 0;
}

static int slab_self_ring(void) {
    const int64_t nx = 36, ny = 20, nz = 9, n = nx * ny * nz;
    double *rho_d, *u_d, mass0;
    if (upload(nx, ny, nz, 3, &rho_d, &u_d, &mass0))
        return 1;
    lbm_config per = config(LBM_D3Q27, nx, ny, nz, LBM_FP64, 0);
    lbm_config slab = config(LBM_D3Q27, nx, ny, nz, LBM_FP64, 1);
    const size_t wp = lbm_workspace_bytes(&per), wsl = lbm_workspace_bytes(&slab), hb = lbm_halo_bytes(&slab);
    CHECK(wp > 0 && wsl > wp && hb == (size_t)(9 * nx * ny * 8), "slab sizes");
    void *ws1, *ws2, *lo, *hi;
    HIPCHECK(hipMalloc(&ws1, wp));
    HIPCHECK(hipMalloc(&ws2, wsl));
    HIPCHECK(hipMalloc(&lo, hb));
    HIPCHECK(hipMalloc(&hi, hb));
    lbm_handle *a = NULL, *b = NULL;
    CHECK(lbm_create(&per, ws1, wp, rho_d, u_d, NULL, &a) == LBM_OK, "create periodic");
    CHECK(lbm_create(&slab, ws2, wsl, rho_d, u_d, NULL, &b) == LBM_OK, "create slab");
    if (!a || !b)
        return 1;
    CHECK(lbm_step(b, 2) == LBM_EINVAL, "slab refuses two steps");
    CHECK(lbm_halo_pack(b, lo, hi) == LBM_OK && lbm_halo_unpack(b, hi, lo) == LBM_OK, "initial exchange");
    for (int s = 0; s < 6; ++s) {
        CHECK(lbm_step(b, 1) == LBM_OK, "slab step");
        CHECK(lbm_halo_pack(b, lo, hi) == LBM_OK && lbm_halo_unpack(b, hi, lo) == LBM_OK, "exchange");
    }
    CHECK(lbm_step(a, 6) == LBM_OK, "periodic steps");
    /* a second slab stepped with the exchange fused in: two send sets, each
       step reads the set the previous step wrote */
    void *ws3, *fs[2][2];
    HIPCHECK(hipMalloc(&ws3, wsl));
    for (int p = 0; p < 2; ++p)
        for (int f = 0; f < 2; ++f)
            HIPCHECK(hipMalloc(&fs[p][f], hb));
    lbm_handle *c = NULL;
    CHECK(lbm_create(&slab, ws3, wsl, rho_d, u_d, NULL, &c) == LBM_OK, "create fused slab");
    if (!c)
        return 1;
    CHECK(lbm_halo_pack(c, fs[1][0], fs[1][1]) == LBM_OK, "seed the fused exchange");
    for (int s = 0; s < 6; ++s) {
        const int p = s % 2;
        CHECK(lbm_step_halo(c, fs[1 - p][1], fs[1 - p][0], fs[p][0], fs[p][1]) == LBM_OK, "fused step");
    }
    CHECK(lbm_step_halo(c, fs[0][1], fs[0][0], fs[0][1], fs[1][1]) == LBM_EINVAL, "fused step rejects aliasing");
    double *fa, *fb;
    HIPCHECK(hipMalloc((void **)&fa, sizeof(double) * 27 * (size_t)n));
    HIPCHECK(hipMalloc((void **)&fb, sizeof(double) * 27 * (size_t)n));
    CHECK(lbm_get_populations(a, fa) == LBM_OK && lbm_get_populations(b, fb) == LBM_OK, "populations");
    double *ha = (double *)malloc(sizeof(double) * 27 * (size_t)n), *hb_ = (double *)malloc(sizeof(double) * 27 * (size_t)n);
    if (!ha || !hb_)
        return 1;
    HIPCHECK(hipMemcpy(ha, fa, sizeof(double) * 27 * (size_t)n, hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(hb_, fb, sizeof(double) * 27 * (size_t)n, hipMemcpyDeviceToHost));
    CHECK(memcmp(ha, hb_, sizeof(double) * 27 * (size_t)n) == 0, "slab self-ring equals periodic domain bitwise");
    CHECK(lbm_get_populations(c, fb) == LBM_OK, "fused populations");
    HIPCHECK(hipMemcpy(hb_, fb, sizeof(double) * 27 * (size_t)n, hipMemcpyDeviceToHost));
    CHECK(memcmp(ha, hb_, sizeof(double) * 27 * (size_t)n) == 0, "fused self-ring equals periodic domain bitwise");
    CHECK(lbm_destroy(c) == LBM_OK, "destroy fused slab");
    HIPCHECK(hipFree(ws3));
    for (int p = 0; p < 2; ++p)
        for (int f = 0; f < 2; ++f)
            HIPCHECK(hipFree(fs[p][f]));
    free(ha);
    free(hb_);
    CHECK(lbm_destroy(a) == LBM_OK && lbm_destroy(b) == LBM_OK, "destroy");
    HIPCHECK(hipFree(fa));
    HIPCHECK(hipFree(fb));
    HIPCHECK(hipFree(ws1));
    HIPCHECK(hipFree(ws2));
    HIPCHECK(hipFree(lo));
    HIPCHECK(hipFree(hi));
    HIPCHECK(hipFree(rho_d));
    HIPCHECK(hipFree(u_d));
    return 0;
}

int main(void) {
    printf("abi_demo: %s\n", lbm_version());
    fflush(stdout);
    if (single_domain() || pool() || slab_self_ring()) {
        printf("abi_demo: setup failed\n");
        return 1;
    }
    if (failures) {
        printf("abi_demo: %d checks failed\n", failures);
        return 1;
    }
    printf("abi_demo ok\n");
    return 0;
}
