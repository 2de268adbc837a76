// lbm_internal.hpp -- host-side layout of a domain's workspace and shared
// helpers of the C-ABI implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kernels.hpp"
#include "lbm.h"

namespace lbm {

// Workspace layout of one domain (all offsets in bytes, 256-byte aligned).
struct Layout {
    int dim, q;
    size_t elem;       // bytes per stored population
    int64_t n;         // nodes
    int layout;        // LBM_LAYOUT_ROWS or LBM_LAYOUT_PLANES
    int eq;            // LBM_EQ_* (kEq* in the device code)
    int64_t ps, rs;    // population and row strides (elements)
    int block_x, block_y;
    int npt;           // nodes per thread along x
    int flags;         // LBM_TUNE_* bits
    bool rowwave;      // one wavefront spans a whole row (vector kernels)
    int tblock;        // LBGK steps per launch (1; 2 on D2Q9; 2, 4 or 8 on D1Q3)
    int t2_tx, t2_rows;  // multi-step kernels: owned columns (nodes) and rows per workgroup
    bool zhalo;        // z-slab: each buffer holds halo planes -1 and nz around the nz planes
    int64_t plane;     // elements of one plane (rows layout: ny * rs)
    int red_blocks;    // workgroups of the moments reduction
    size_t buf_bytes;  // one population buffer
    size_t off_buf[2], off_flag, off_diag, off_partials, ws_bytes;
};

// One domain's state inside a workspace (owned by a handle or a pool slot).
struct DomainState {
    lbm_config cfg;
    Layout L;
    char *ws;
    void *buf[2];
    int cur;  // buffer holding the current state
    int *flag;
    double *diag_dev;
    double *partials;
    int64_t steps;
    Relax relax;
};

void set_error(const char *msg);
int hip_fail(hipError_t e, const char *what);
int validate_config(const lbm_config *cfg, const lbm_tuning *tun, Layout *out);
int launch_step(const Layout &L, const StepArgs &args, int dtype, bool corr, hipStream_t s, int nz,
                const HaloArgs *halo);
int launch_step2(const Layout &L, const StepArgs &args, int dtype, bool corr, hipStream_t s);

// Bind a domain to its workspace and enqueue f = f^eq(rho, u) plus the flag
// clear; the caller synchronises and reads the flag (domain_read_flag).
int domain_bind_and_init(DomainState &d, const lbm_config *cfg, const Layout &L, void *workspace,
                         const double *rho, const double *u, hipStream_t s);
// Synchronise the stream and return the domain flag (0/1) in *flag.
int domain_read_flag(const DomainState &d, hipStream_t s, int *flag);
int domain_moments(DomainState &d, hipStream_t s, double *rho, double *u, lbm_diag *diag);
int domain_export(DomainState &d, hipStream_t s, double *out);
// Enqueue the acoustic energy about (rho_ref, U) into the device double *out.
int domain_energy(DomainState &d, hipStream_t s, const double *U, double rho_ref, double *out);

}  // namespace lbm
