/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for lattice-BGK with the
 * entropic equilibrium.
 *
 * Method: S. A. Hosseini and I. V. Karlin, "Entropic equilibrium for the lattice
 * Boltzmann method: Hydrodynamics and numerical properties", arXiv:2303.08163.
 * One time step of a domain is the LBGK evolution equation of Sec. "Basic
 * concepts",
 *     f_i(r + c_i, t + 1) = f_i(r, t) + 2 beta (f_i^eq(rho, u) - f_i(r, t)),
 * on a periodic D1Q3, D2Q9 or D3Q27 first-neighbour lattice (Sec. "Basic
 * concepts": 1-D weights {1/6, 2/3, 1/6} and their tensor products), in lattice units
 * (dr = dt = 1, varsigma^2 = 1/3), with
 *   - f^eq the entropic equilibrium, eq. (Entropic_isothermal_EDF);
 *   - beta from eq. (relaxation_frequency) with nu = (tau - 1/2) / 3, i.e.
 *     2 beta = 1 / tau; or, with the bulk-viscosity correction of Sec.
 *     "Correction of leading-order bulk viscosity error", beta from
 *     eq. (redefined_relaxation rate) with the entropic A of eq.
 *     (entropic_bulk) evaluated at the node's own pre-collision velocity.  The
 *     paper derives A on a 1-D lattice; a multi-dimensional node uses
 *     A = min over axes of A(u_alpha).
 *
 * Conventions shared by every entry point:
 *   - Fields are node-major planes with x fastest: node n = x + nx (y + ny z).
 *     A density field is N = nx ny nz doubles; a velocity field is D planes of
 *     N doubles (u_x plane, then u_y, then u_z for D3Q27; D = 1, 2, 3).
 *   - "device pointer" means memory allocated on the GPU the library runs on
 *     (hipMalloc or a torch CUDA tensor); "host pointer" means CPU memory.
 *   - Every call returns an lbm_status (0 = LBM_OK, negative = error) unless
 *     stated otherwise; no exception crosses the ABI.  Arguments are validated
 *     before any GPU work is enqueued; on error nothing is written to outputs.
 *   - A handle is not thread-safe.  Distinct handles are independent.  Work is
 *     enqueued on the handle's HIP stream; calls that return data to the host
 *     synchronise that stream.
 *   - The equilibrium is defined only for rho > 0 and |u_alpha| < 1 (Sec.
 *     "Discrete entropic equilibrium construction"); the library does not
 *     clamp.  A node that reaches a state outside that domain sets the
 *     handle's domain flag, reported as LBM_EDOMAIN.
 */
#ifndef LBM_ENTROPIC_H
#define LBM_ENTROPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum lbm_status {
    LBM_OK = 0,
    LBM_EINVAL = -1,  /* invalid argument or configuration */
    LBM_EDOMAIN = -2, /* some node left rho > 0, |u_alpha| < 1 (results still written) */
    LBM_EDEVICE = -3, /* a HIP runtime call failed */
    LBM_ENOMEM = -4,  /* a request does not fit the memory budget */
    LBM_EBUSY = -5    /* no free slot */
};

/* Lattices: the value is Q.  D1Q3 domains have ny = nz = 1 and run on the
 * single-domain entry points only. */
enum { LBM_D1Q3 = 3, LBM_D2Q9 = 9, LBM_D3Q27 = 27 };

/* Population storage and arithmetic.
 *   LBM_FP64:           populations stored and computed in IEEE double.
 *   LBM_FP32_DEV:       populations stored in IEEE single as deviations
 *                       f_i - w_i rho0 from the rest equilibrium at density rho0;
 *                       every step widens them to double, computes moments,
 *                       equilibrium and relaxation in double, and rounds the
 *                       result to nearest-even single on store.
 *   LBM_FP32_DEV_MIXED: the same storage; moment sums, square roots and the
 *                       per-axis equilibrium factors in double, the
 *                       per-population equilibrium and relaxation in single on
 *                       deviation-sized quantities (precision ablation).
 *   LBM_FP32_DEV_F32:   the same storage with every operation in single
 *                       (precision ablation).
 * The two ablation modes are not held to the FP32 error budget. */
enum { LBM_FP64 = 0, LBM_FP32_DEV = 1, LBM_FP32_DEV_MIXED = 2, LBM_FP32_DEV_F32 = 3 };

/* Equilibrium.
 *   LBM_EQ_ENTROPIC: eq. (Entropic_isothermal_EDF), the product form of the
 *                    exact entropic equilibrium (every storage mode).
 *   LBM_EQ_POLY2:    eq. (Poly2_isothermal_EDF), the second-order polynomial
 *                    equilibrium (LBM_FP64 and LBM_FP32_DEV only).
 *   LBM_EQ_PRODUCT:  eq. (Product_isothermal_EDF), the product-form polynomial
 *                    equilibrium (LBM_FP64 and LBM_FP32_DEV only).
 * With bulk_correction = 1 the two polynomial kinds use A = 1 - (3/2) u^2 / varsigma^2
 * (eq. LBGK_bulk) in eq. (redefined_relaxation rate_poly), A taken at the node's
 * largest |u_alpha|; A is not clamped.  The polynomial kinds run on the
 * single-domain entry points only (lbm_pool_admit returns LBM_EINVAL) and, with
 * nodes_per_thread > 1, only with the default vector width and flags. */
enum { LBM_EQ_ENTROPIC = 0, LBM_EQ_POLY2 = 1, LBM_EQ_PRODUCT = 2 };

/* Problem statement of one periodic domain (plain data, caller-owned). */
typedef struct lbm_config {
    int32_t lattice;         /* LBM_D1Q3, LBM_D2Q9 or LBM_D3Q27 */
    int32_t dtype;           /* LBM_FP64, LBM_FP32_DEV, LBM_FP32_DEV_MIXED or LBM_FP32_DEV_F32 */
    int64_t nx, ny, nz;      /* grid extent; nz must be 1 for D2Q9; each >= 1 */
    double tau;              /* relaxation time, tau > 1/2 and finite; 2 beta = 1/tau */
    int32_t bulk_correction; /* 0 = off, 1 = eq. (redefined_relaxation rate) */
    int32_t equilibrium;     /* LBM_EQ_ENTROPIC, LBM_EQ_POLY2 or LBM_EQ_PRODUCT */
    double rho0;             /* reference density of the FP32 deviation storage (> 0); ignored for FP64 */
    int32_t z_halo;          /* 0: periodic in every direction.  1: a z-slab, nz planes of a larger
                                domain that is split along z (D3Q27, row-interleaved layout only):
                                no wrap in z; the planes below plane 0 and above plane nz - 1 are
                                halo planes that lbm_halo_unpack fills (see there) */
    int32_t reserved;        /* must be 0 */
} lbm_config;

/* Launch tuning (optional).  Zero fields take the library default.  Results do
 * not depend on the tuning: every node's arithmetic is the same. */
typedef struct lbm_tuning {
    int32_t block_x;          /* threads along x per workgroup: a multiple of 64, or (one node
                                 per thread only) a power of two below 64 */
    int32_t block_y;          /* rows along y per workgroup; block_x * block_y a multiple of 64,
                                 <= 256 */
    int32_t plane_pad;        /* LBM_LAYOUT_PLANES only: extra elements between population
                                 planes (>= 0; < 0 selects the default, 0) */
    int32_t nodes_per_thread; /* consecutive x nodes per thread: 1, 2 or 4 (4 for FP32 storage
                                 only); > 1 needs nx % (block_x * nodes_per_thread) == 0.
                                 0 = default: 4 floats or 2 doubles when nx allows, except
                                 1 for FP32 storage on D2Q9 */
    int32_t flags;            /* LBM_TUNE_* bits for the vector kernels; < 0 selects the default */
    int32_t layout;           /* LBM_LAYOUT_*; 0 = default (row-interleaved) */
    int32_t time_block;       /* LBGK steps per launch, the intermediate states kept in LDS
                                 (LBM_FP64 or LBM_FP32_DEV, any equilibrium, row-interleaved
                                 layout): 1 = one; 2 on D2Q9 with nx >= 64; 2, 4 or 8 on
                                 D1Q3 with nx >= 16.  Step counts that are not a multiple
                                 end with one-step launches of the kernel the other fields
                                 select.
                                 0 = default: 2 for D2Q9 domains of >= 2048^2 nodes (FP32) or
                                 1024^2 (FP64), 8 for D1Q3 where allowed, else 1 -- when
                                 block_x, block_y, nodes_per_thread, flags and layout are
                                 left at their defaults */
    int32_t time_rows;        /* time_block = 2: rows swept per workgroup (>= 1; 0 = default);
                                 must be 0 otherwise */
    int32_t reserved;         /* must be 0 */
} lbm_tuning;

/* lbm_tuning.flags bits. */
enum { LBM_TUNE_NT_STORE = 1, LBM_TUNE_NT_LOAD = 2 };

/* Population layouts in device memory (the library's private format; results
 * do not depend on it).  Rows run along x; row = z ny + y.
 *   LBM_LAYOUT_ROWS:   each row holds its Q population runs back to back,
 *                      each run padded to a multiple of 16 elements (rows
 *                      narrower than 16 are not padded) ([z][y][i][x]).
 *   LBM_LAYOUT_PLANES: one plane of N nodes per population ([i][z][y][x]),
 *                      planes padded to 64 elements plus plane_pad. */
enum { LBM_LAYOUT_DEFAULT = 0, LBM_LAYOUT_ROWS = 1, LBM_LAYOUT_PLANES = 2 };

/* Whole-domain diagnostics, all from the current populations. */
typedef struct lbm_diag {
    double mass;           /* sum_r rho */
    double momentum[3];    /* sum_r rho u_alpha (unused components 0) */
    double kinetic_energy; /* sum_r rho |u|^2 / 2 */
    double max_abs_u;      /* max over nodes and axes of |u_alpha| */
    double min_rho;        /* min over nodes of rho */
    int64_t steps;         /* steps taken since lbm_create */
    int32_t domain_error;  /* 1 if any node left the domain since lbm_create */
    int32_t reserved;
} lbm_diag;

typedef struct lbm_handle lbm_handle;

/* Bytes of device workspace a domain needs: two population buffers
 * (Q planes each, padded), the domain flag and the reduction scratch.
 * Returns 0 for an invalid configuration.  Host-only; no GPU call. */
size_t lbm_workspace_bytes(const lbm_config *cfg);

/* Same with explicit tuning (tuning may be NULL = defaults). */
size_t lbm_workspace_bytes_tuned(const lbm_config *cfg, const lbm_tuning *tuning);

/* Create a domain and initialise f = f^eq(rho, u) (the state the paper's
 * experiments start from).
 *   cfg        host pointer, copied.
 *   workspace  device pointer to ws_bytes >= lbm_workspace_bytes(cfg) bytes,
 *              256-byte aligned, owned by the caller and borrowed by the handle
 *              until lbm_destroy (the library never frees it).
 *   rho, u     device pointers to the initial density (N doubles) and velocity
 *              (D * N doubles); read before the call returns.
 *   stream     hipStream_t to enqueue on (NULL = the null stream).
 *   out        receives the handle; untouched on error.
 * Synchronises the stream.  Errors: LBM_EINVAL (NULL pointer, tau <= 1/2 or
 * not finite, an extent < 1, nz != 1 for D2Q9, ny or nz != 1 for D1Q3, more than 2^31 - 4096 nodes,
 * bad lattice/dtype/equilibrium/tuning, rho0 <= 0 for FP32_DEV, workspace too
 * small or misaligned); LBM_EDOMAIN (an initial node has rho <= 0 or |u_alpha| >= 1;
 * no handle is created); LBM_EDEVICE. */
int lbm_create(const lbm_config *cfg, void *workspace, size_t ws_bytes, const double *rho,
               const double *u, void *stream, lbm_handle **out);

/* lbm_create with explicit tuning (tuning may be NULL = defaults). */
int lbm_create_tuned(const lbm_config *cfg, const lbm_tuning *tuning, void *workspace,
                     size_t ws_bytes, const double *rho, const double *u, void *stream,
                     lbm_handle **out);

/* Enqueue nsteps time steps (one fused stream-and-collide kernel launch each)
 * on the handle's stream and return without synchronising.  Runs of 64 steps
 * or more replay a captured HIP graph of 32 launches (the same kernels and
 * arguments, so bitwise the same results) to relieve the host's launch rate;
 * the graphs are captured by lbm_create.  nsteps = 0 is a no-op.  Errors: LBM_EINVAL (h NULL, nsteps < 0, nsteps > 1 on a z-slab,
 * which needs a halo exchange between steps); LBM_EDEVICE (launch failure). */
int lbm_step(lbm_handle *h, int64_t nsteps);

/* Halo exchange of a z-slab (lbm_config.z_halo = 1).  A periodic domain split
 * along z into slabs advances exactly as the whole domain when, between two
 * steps, each slab receives the populations that stream into it across its
 * two faces (the streaming of the lattice BGK equation, Sec. "Basic concepts":
 * f_i at r comes from r - c_i; only populations with c_z = +1 cross a face
 * upwards and c_z = -1 downwards).  With populations numbered
 * i = (c_x + 1) + 3 (c_y + 1) + 9 (c_z + 1), the 9 with c_z = -1 are i = 0..8
 * and the 9 with c_z = +1 are i = 18..26.
 *
 * A packed buffer holds one face: 9 nx ny stored values (FP64 or FP32
 * deviations, the domain's storage type; lbm_halo_bytes bytes) in the order
 * [y][k][x], k = 0..8 the 9 populations in increasing i.  Its contents are the
 * library's stored values, meant to be moved unchanged (RCCL send/recv, peer
 * copy) to the slab that unpacks them.
 *
 *   lbm_halo_pack(h, lower, upper): plane 0's populations with c_z = -1 into
 *       `lower` (for the slab below), plane nz - 1's with c_z = +1 into
 *       `upper` (for the slab above).
 *   lbm_halo_unpack(h, lower, upper): `lower` (the slab below's `upper` pack)
 *       into the halo plane below plane 0, `upper` (the slab above's `lower`
 *       pack) into the halo plane above plane nz - 1.
 * Each call moves both faces in one kernel launch; a NULL buffer skips its
 * face (not both).
 *
 * Sequence per step for every slab: lbm_step(h, 1); pack; move the buffers;
 * unpack.  Before the first step the halo planes must be filled the same way
 * (they start as zeros).  A slab that is its own neighbour on both sides
 * (lbm_halo_pack(h, a, b); lbm_halo_unpack(h, b, a)) advances as the periodic
 * domain of its nz planes.  The buffers are device pointers owned by the
 * caller; the copies are enqueued on the handle's stream without
 * synchronising.  Errors: LBM_EINVAL (h NULL, both buffers NULL, the domain is
 * not a z-slab); LBM_EDEVICE. */
size_t lbm_halo_bytes(const lbm_config *cfg); /* 0 for a config that is not a valid z-slab */

/* One step of a z-slab with the halo exchange fused into the stream-collide
 * kernel (no pack or unpack launch): the populations entering across the two
 * faces are read from recv_lower (the slab below's outgoing upper face) and
 * recv_upper (the slab above's outgoing lower face) instead of the halo
 * planes, and the populations leaving are written to send_lower (plane 0,
 * c_z = -1) and send_upper (plane nz - 1, c_z = +1) while the step stores the
 * slab's own state.  All four buffers are packed as for lbm_halo_pack (the
 * two forms interoperate: a first step can read buffers lbm_halo_pack
 * filled), lbm_halo_bytes each, device pointers owned by the caller; a
 * receive buffer must not overlap a send buffer of the same call, so
 * neighbours on one device alternate two sets of send buffers.  The halo
 * planes are neither read nor written.  Enqueued without synchronising.
 * Runs with LBM_FP64 or LBM_FP32_DEV storage and one node per thread or the
 * default vector width (with the default cache hints).  Errors: LBM_EINVAL (h
 * or a buffer NULL, a receive buffer equal to a send buffer, equal send
 * buffers, the domain is not a z-slab, another storage type or tuning);
 * LBM_EDEVICE. */
int lbm_step_halo(lbm_handle *h, const void *recv_lower, const void *recv_upper, void *send_lower,
                  void *send_upper);
int lbm_halo_pack(lbm_handle *h, void *lower, void *upper);
int lbm_halo_unpack(lbm_handle *h, const void *lower, const void *upper);

/* Moments of the current state: rho (N doubles) and u (D * N doubles) into
 * device pointers, and diagnostics into a host struct.  Any of rho, u, diag may
 * be NULL.  Synchronises the stream.  Returns LBM_EDOMAIN when any node left
 * the domain since lbm_create (the outputs are still written), LBM_EINVAL for
 * h NULL, LBM_EDEVICE on a HIP failure. */
int lbm_moments(lbm_handle *h, double *rho, double *u, lbm_diag *diag);

/* Copy the current populations out as doubles in the library's canonical
 * order, population-major: out[i * N + n] for population i, node n, where
 * i = (c_x + 1) + 3 (c_y + 1) + 9 (c_z + 1) (D1Q3: i = c_x + 1) and the stored state is the
 * post-collision f*(r, t) (its moments equal those of the pre-collision state).
 * FP32_DEV storage is widened and rho0 w_i added back.  out is a device
 * pointer to Q * N doubles.  Synchronises the stream. */
int lbm_get_populations(lbm_handle *h, double *out);

/* The launch the library chose for a domain's steps (from its configuration
 * and tuning), so that callers and tests can state which kernel ran. */
enum {
    LBM_KERNEL_NODE = 1,      /* one node per thread (any nx) */
    LBM_KERNEL_VECTOR = 2,    /* nodes_per_thread consecutive x nodes per thread, one 16-byte
                                 load and store per population run, x shifts by lane rotation */
    LBM_KERNEL_TWO_STEP = 3,  /* D2Q9, two steps per launch, the intermediate state in LDS */
    LBM_KERNEL_MULTI_STEP = 4 /* D1Q3, time_block steps per launch in LDS segments */
};
typedef struct lbm_launch_info {
    int32_t kernel;           /* LBM_KERNEL_* of full launches (step counts that are not a multiple
                                 of time_block end with launches of the one-step kernel that
                                 block_x .. layout describe) */
    int32_t nodes_per_thread; /* of the one-step kernel */
    int32_t row_wave;         /* 1: one wavefront spans a whole row, so the lane rotation is
                                 itself the periodic wrap (nx = 64 nodes_per_thread) */
    int32_t flags;            /* LBM_TUNE_* cache hints of the one-step kernel */
    int32_t block_x, block_y; /* one-step workgroup shape (threads) */
    int32_t layout;           /* LBM_LAYOUT_ROWS or LBM_LAYOUT_PLANES */
    int32_t time_block;       /* steps per launch of `kernel` (1, 2, 4 or 8) */
    int32_t time_cols;        /* multi-step kernels: owned columns (nodes) per workgroup, else 0 */
    int32_t time_rows;        /* two-step kernel: rows swept per workgroup, else 0 */
    int32_t graph_steps;      /* steps per replay of the captured step graph (0: no graph) */
    int32_t reserved;
} lbm_launch_info;

/* Fill *out for handle h (host-only; no GPU call).  Errors: LBM_EINVAL (h or
 * out NULL). */
int lbm_get_launch_info(const lbm_handle *h, lbm_launch_info *out);

/* Checkpoint and restart: the current state as the library stores it (its
 * private format: the storage type, layout and padding of the handle's
 * configuration and tuning), so that a restart is bit-exact for every storage
 * type.  lbm_state_bytes: the size of a saved state (0 for h NULL).
 * lbm_save_state copies the state into dst; lbm_load_state replaces the
 * handle's state with src, sets its step count to `steps` and clears the
 * domain flag (save a state only while lbm_moments reports no domain error).
 * dst / src are device pointers owned by the caller, of exactly
 * lbm_state_bytes(h) bytes; a state is valid only for a handle with the same
 * configuration and tuning.  Enqueued on the handle's stream without
 * synchronising.  Errors: LBM_EINVAL (h or the buffer NULL, bytes not
 * lbm_state_bytes(h), steps < 0); LBM_EDEVICE.  (lbm_get_populations gives
 * the portable, canonical FP64 form.) */
size_t lbm_state_bytes(const lbm_handle *h);
int lbm_save_state(lbm_handle *h, void *dst, size_t bytes);
int lbm_load_state(lbm_handle *h, const void *src, size_t bytes, int64_t steps);

/* Quadratic acoustic energy of the current state about a reference state
 * (rho_ref, U), summed over the nodes:
 *     E = sum_r [ rho_ref |u - U|^2 / 2 + c_s^2 (rho - rho_ref)^2 / (2 rho_ref) ],
 * c_s^2 = 1/3 (Sec. "Validation via dissipation of isothermal pressure waves":
 * the energy whose decay rate gives the effective viscosity; the paper's
 * printed integrand is linear in rho - rho0 and sums to a constant on a
 * periodic grid, so the quadratic form of linear acoustics is used).
 *   U        host pointer to D doubles (NULL = zero velocity).
 *   rho_ref  > 0 and finite.
 *   out      device pointer to one double, written when the stream reaches
 *            the call.
 * Enqueues two kernels and returns without synchronising, so that an energy
 * history E(t) can be recorded step by step into a device array and read
 * once.  The sum is taken in a fixed order (bitwise reproducible).  Errors:
 * LBM_EINVAL (h or out NULL, rho_ref <= 0 or not finite, U not finite);
 * LBM_EDEVICE. */
int lbm_energy(lbm_handle *h, const double *U, double rho_ref, double *out);

/* An energy history over a run (Sec. "Validation via dissipation of isothermal
 * pressure waves": the decay of E(t) gives the effective viscosity): the
 * energy of lbm_energy before the first step and after every `every` steps of
 * lbm_step, over `steps` steps, all enqueued by this one call.
 *   steps  >= 0, a multiple of every;  every >= 1.
 *   U, rho_ref  as for lbm_energy.
 *   out    device pointer to steps / every + 1 doubles: out[k] is the energy
 *          after k * every steps, written when the stream reaches it.
 * The same kernels run in the same order as the calls made one by one, so the
 * values and the final state are bitwise theirs.  Returns without
 * synchronising.  Errors: LBM_EINVAL (those of lbm_energy; every < 1, steps
 * < 0 or not a multiple of every; a z-slab domain), checked before anything is
 * enqueued; LBM_EDEVICE (the work enqueued before the failing launch stays
 * enqueued). */
int lbm_energy_history(lbm_handle *h, int64_t steps, int64_t every, const double *U, double rho_ref, double *out);

/* Measurement aids (not part of the method): the speed of the access pattern
 * alone, as the ceiling against which the stream-collide kernel is read.
 *
 * lbm_ceiling_stream: nsteps steps of free streaming, f_i(r, t + 1) =
 * f_i(r - c_i, t), with no collision: the launch, loads and stores of the
 * handle's one-step kernel (the streaming half of the LBGK evolution equation
 * of Sec. "Basic concepts") with the arithmetic left out.  It replaces the
 * handle's state by the freely streamed one and leaves its step count alone:
 * use a domain made for the measurement.  D2Q9 / D3Q27 periodic domains with
 * LBM_FP64 or LBM_FP32_DEV storage, one step per launch, one node per thread
 * or the default vector width and flags.  Enqueued without synchronising.
 * Errors: LBM_EINVAL (h NULL, nsteps < 0, another configuration); LBM_EDEVICE.
 *
 * lbm_ceiling_copy: copies `bytes` (a multiple of 16) from src to dst (device
 * pointers, 16-byte aligned, not overlapping), one 16-byte non-temporal load
 * and store per thread; enqueued on `stream` without synchronising.  Errors:
 * LBM_EINVAL; LBM_EDEVICE. */
int lbm_ceiling_stream(lbm_handle *h, int64_t nsteps);
int lbm_ceiling_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Release the handle (host state only; the caller's workspace is untouched).
 * Synchronises the stream first.  lbm_destroy(NULL) returns LBM_OK. */
int lbm_destroy(lbm_handle *h);

/* Static, human-readable name of a status code. */
const char *lbm_status_string(int status);

/* ---------------------------------------------------------------------------
 * Pools: many independent domains advanced together (batching and serving).
 *
 * A pool owns no memory: the caller hands it one device arena, which the pool
 * divides into a table region and slot workspaces (first-fit, coalescing free
 * list).  A slot is one periodic domain (any lattice and dtype; its own tau,
 * correction and step budget).  lbm_pool_run advances every active slot; one
 * step of all slots of a (lattice, dtype) class is one kernel launch (the
 * default), or all steps of a run are one persistent cooperative launch.  In
 * that launch one-step classes wait at a device-side grid barrier between
 * steps (on MI355X the barrier costs more than a kernel boundary, 0.2-0.3 ms
 * per step at full occupancy).  D2Q9 two-step classes (persistent with
 * time_block = 2) have no grid barrier: each two-step tile keeps a completion
 * counter, and a tile's next two steps wait only for the tiles within two
 * nodes of it.  A slot's populations are bitwise the same as
 * those of a single domain (lbm_create) with the same configuration and
 * layout: every kernel uses the same per-node arithmetic.  Pools are not
 * thread-safe; slots of one pool share its stream.
 * ------------------------------------------------------------------------- */
typedef struct lbm_pool lbm_pool;

/* Pool tuning.  Zero fields take the defaults. */
typedef struct lbm_pool_tuning {
    int32_t tile_x;     /* threads (one node each) per workgroup along x (default 64) */
    int32_t tile_y;     /* rows per workgroup (default 256 / tile_x); tile_x * tile_y a
                           multiple of 64, <= 256 */
    int32_t persistent; /* 1: one cooperative launch per run and class; 0: one launch per step */
    int32_t workgroups; /* persistent grid size (0 = as many as are co-resident) */
    int32_t layout;     /* LBM_LAYOUT_* of the slots (0 = row-interleaved) */
    int32_t flat;       /* 0: a workgroup covers tile_x nodes of tile_y rows; 1: it covers
                           tile_x * tile_y consecutive nodes of its slot in x-fastest order,
                           across rows and planes (no idle lanes at ragged row ends) */
    int32_t row_fit;    /* 1: each slot maps the workgroup's tile_x * tile_y threads onto rows
                           of w threads, w the narrowest of 64, 128, 256 (dividing the
                           workgroup) that covers the slot's padded row, or the widest such w
                           when none does, with tile_x * tile_y / w rows per workgroup; a
                           wavefront always stays within one row.  0: every slot uses
                           tile_x x tile_y.  Not with flat; other values are LBM_EINVAL */
    int32_t time_block; /* 2: D2Q9 classes (LBM_FP64 or LBM_FP32_DEV, row-interleaved slots)
                           advance two steps per launch, the intermediate state in LDS, in
                           runs where the class's slots that take at least two steps hold
                           >= 2^22 nodes (FP32) or 2^20 (FP64); a slot whose step count in
                           the run is odd takes its last step in a one-step launch.  FP32:
                           slots whose row, rounded up to 64, is at most 512 nodes (1024
                           with persistent = 1) run as whole-row tiles (no halo columns),
                           wider ones as column tiles of 512 (1024); FP64: column tiles of
                           128.  Other runs take one step per
                           launch.  Results are bitwise those of one step per launch.
                           With persistent = 1 such a class takes every iteration of a
                           run (two steps each, and a last single step for slots with
                           an odd count) in one cooperative launch ordered by per-tile
                           counters, for runs of at most 2^30 steps; its slots then hold
                           8 bytes per two-step tile more (lbm_pool_slot_bytes).  Other
                           classes of such a pool run persistent as with time_block 0.
                           0 or 1: one step per launch */
    int32_t time_rows;  /* time_block = 2: rows swept by each whole-row sub-tile and each column
                           tile (0 = default: 16; in the tile-ordered persistent form 16
                           for FP32, 64 for FP64; at most 4096) */
    int32_t spin_log2;  /* persistent form: a workgroup waits at most 2^spin_log2 polls of the
                           grid barrier's counter, or of its tile's neighbours' counters,
                           before it reports a timeout (1..40; 0 = the
                           default, 26, seconds of waiting).  Small values exist to exercise
                           the timeout path: every workgroup still leaves normally */
} lbm_pool_tuning;

typedef struct lbm_pool_stats {
    int32_t max_slots, used_slots;
    int64_t arena_bytes, free_bytes, largest_free_block;
    int64_t runs, launches;
} lbm_pool_stats;

typedef struct lbm_slot_info {
    int32_t used;         /* 1 if the slot holds a domain */
    int32_t finished;     /* 1 if its step budget is spent (or it was retired) */
    int64_t steps_done, steps_remaining;
    int64_t bytes;        /* arena bytes held */
    int32_t domain_error; /* 1 if it was retired because its state left the domain */
    int32_t device_error; /* 1 if a persistent launch that advanced it stopped at a timed-out
                             wait: its state is that of an unknown step, and
                             lbm_pool_moments / lbm_pool_get_populations return LBM_EDEVICE */
} lbm_slot_info;

/* Arena bytes the pool keeps for its tables (the rest holds slots). */
size_t lbm_pool_table_bytes(int32_t max_slots);

/* Arena bytes one slot of this configuration occupies (0 if invalid). */
size_t lbm_pool_slot_bytes(const lbm_config *cfg, const lbm_pool_tuning *tuning);

/* Create a pool of at most max_slots (1..65536) slots on `arena` (device
 * pointer, 256-byte aligned, arena_bytes > lbm_pool_table_bytes(max_slots)),
 * enqueuing on `stream`.  tuning may be NULL.  The pool keeps a second,
 * non-blocking stream of its own for reads of finished slots, pinned host
 * staging for its run tables (8 x the table of one class) and a ring of HIP
 * events.  Errors: LBM_EINVAL, LBM_EDEVICE (pinned staging allocation, stream
 * or event creation, device query). */
int lbm_pool_create(int32_t max_slots, const lbm_pool_tuning *tuning, void *arena, size_t arena_bytes,
                    void *stream, lbm_pool **out);

/* Admit a domain: initialise f = f^eq(rho, u) (device pointers as in
 * lbm_create) in a free slot with a budget of nsteps steps.  Synchronises the
 * stream.  Returns the slot index in *slot.  Errors: LBM_EBUSY (no free slot),
 * LBM_ENOMEM (no free arena block large enough), LBM_EINVAL, LBM_EDOMAIN (the
 * initial state; the slot is not taken), LBM_EDEVICE. */
int lbm_pool_admit(lbm_pool *pool, const lbm_config *cfg, const double *rho, const double *u, int64_t nsteps,
                   int32_t *slot);

/* lbm_pool_admit without the synchronisation, for callers that keep work in
 * flight (a serving loop): the initialisation is enqueued on the pool's stream
 * behind the work already there, and the call returns at once.  rho and u
 * must stay valid until the stream has run the initialisation (memory that
 * the caller allocated in stream order on the same stream, e.g. torch's
 * caching allocator on that stream, may be freed right after the call).  The
 * initial state is checked on the device: a slot whose initial state has a
 * node with rho <= 0 or |u_alpha| >= 1 is retired by the next lbm_pool_poll or
 * lbm_pool_collect that finds its initialisation done (listed as done,
 * domain_error = 1, lbm_pool_moments returns LBM_EDOMAIN).  Errors:
 * LBM_EBUSY, LBM_ENOMEM, LBM_EINVAL, LBM_EDEVICE; nothing is enqueued then. */
int lbm_pool_admit_async(lbm_pool *pool, const lbm_config *cfg, const double *rho, const double *u,
                         int64_t nsteps, int32_t *slot);

/* Advance every slot with steps remaining by min(k, remaining) steps.
 * Enqueues and returns without synchronising.  k = 0 is a no-op.  Runs are
 * numbered from 1 in lbm_pool_stats.runs (a run that enqueues nothing gets
 * no number).  Errors: LBM_EINVAL; LBM_EDEVICE (a launch failed: the slots of
 * the failing class keep their step counts and state of before the run). */
int lbm_pool_run(lbm_pool *pool, int64_t k);

/* Synchronise, then list (up to capacity) slots whose budget is spent and that
 * were not listed before; *count receives how many were written.  A slot whose
 * domain flag is set (some node left rho > 0, |u_alpha| < 1) is retired here:
 * its remaining steps are dropped, it is listed as done, its slot info shows
 * domain_error = 1 and lbm_pool_moments returns LBM_EDOMAIN for it.
 * If a persistent launch's wait timed out since the last poll, every
 * slot that such a launch advanced is retired with device_error = 1 (listed
 * as done by this or a later poll; lbm_pool_moments returns LBM_EDEVICE for
 * it), the barrier state is reset so that the pool stays usable, and the call
 * returns LBM_EDEVICE after writing the list. */
int lbm_pool_poll(lbm_pool *pool, int32_t *done, int32_t capacity, int32_t *count);

/* Non-blocking completion, for callers that enqueue run n + 1 before they
 * collect the results of run n.  First waits until the device has finished
 * run number after_run (lbm_pool_stats.runs numbering; <= 0 or a run not yet
 * enqueued: no wait), while later work keeps running.  Then lists, without
 * synchronising the stream, up to capacity slots whose budget is spent, whose
 * enqueued work has all completed on the device, and that were not listed
 * before.  The initial states of slots admitted by lbm_pool_admit_async whose
 * initialisation has completed are checked here too (retired as in
 * lbm_pool_poll).  Domain flags raised later are reported by lbm_pool_moments
 * (LBM_EDOMAIN) and by lbm_pool_poll, which also retires running slots early.
 * Errors: LBM_EINVAL, LBM_EDEVICE. */
int lbm_pool_collect(lbm_pool *pool, int64_t after_run, int32_t *done, int32_t capacity, int32_t *count);

/* Moments / populations of one slot, as lbm_moments / lbm_get_populations.
 * LBM_EDOMAIN concerns this slot only; LBM_EDEVICE for a slot retired after a
 * timed-out persistent launch (outputs not written).  When the slot's enqueued
 * work has completed on the device (a slot listed by lbm_pool_collect) the
 * read runs on the pool's second stream and does not wait for later runs;
 * otherwise it synchronises the pool's stream. */
int lbm_pool_moments(lbm_pool *pool, int32_t slot, double *rho, double *u, lbm_diag *diag);
int lbm_pool_get_populations(lbm_pool *pool, int32_t slot, double *out);

/* Free a slot and its arena block.  Waits until the device has finished the
 * work enqueued for this slot (not the later work of other slots). */
int lbm_pool_release(lbm_pool *pool, int32_t slot);

int lbm_pool_stats_get(lbm_pool *pool, lbm_pool_stats *stats);
int lbm_pool_slot_info(lbm_pool *pool, int32_t slot, lbm_slot_info *info);

/* Synchronise and free the pool's host state (the arena is the caller's).
 * lbm_pool_destroy(NULL) returns LBM_OK. */
int lbm_pool_destroy(lbm_pool *pool);

/* ---------------------------------------------------------------------------
 * Linear (von Neumann) stability: Sec. "Linear stability analysis".
 *
 * A plane-wave perturbation f'_i = F_i exp(i (k . r - omega t)) of the uniform
 * equilibrium state (rho = 1, u) evolves by eq. (PerturbedDiscreteLBE); its
 * amplification matrix is M = E (I + J) (eq. VN_eigen), E_ii = exp(-i c_i . k),
 * J the Jacobian of the collision operator at that state, and every
 * eigenvalue is lambda = exp(-i omega): a mode grows when |lambda| > 1.
 * With the bulk correction the node's relaxation rate is taken at u (its
 * derivative does not enter J, because f^eq - f = 0 at the reference state).
 * Lattices: LBM_D1Q3 and LBM_D2Q9 (the paper's analysis is 2-D).  All
 * arithmetic is FP64; eigenvalues come from a Householder reduction to
 * Hessenberg form and shifted QR steps, one matrix per GPU thread.
 * -------------------------------------------------------------------------*/

/* Spectra of `count` independent cases.
 *   cases   device pointer, count records of 5 doubles: tau, u_x, u_y, k_x, k_y
 *           (u_y and k_y are ignored for D1Q3).  tau > 1/2 is not checked
 *           per case; a non-finite record gives non-finite results.
 *   radius  device pointer to count doubles: max |lambda| (NULL: not written).
 *   eig     device pointer to count * Q * 2 doubles: the Q eigenvalues of
 *           each case as (re, im), in no particular order (NULL: not written).
 *   info    device pointer to count int32: QR steps taken, or -1 when the
 *           iteration limit (30 Q steps) was reached first (NULL: not written).
 *   flops   device pointer to count doubles: FP64 operations the solver spent
 *           on the case, counting its own active block at every QR step
 *           (additions, multiplications, divisions, square roots, sines and
 *           cosines 1, a fused multiply-add 2, the refined reciprocal square
 *           root 2; absolute values, maxima and comparisons 0) (NULL: not
 *           written).
 *   stream  hipStream_t (NULL = the null stream).
 * Enqueues one kernel and returns without synchronising.  Errors: LBM_EINVAL
 * (lattice other than D1Q3/D2Q9, bad equilibrium or bulk_correction, count < 0,
 * cases NULL with count > 0); LBM_EDEVICE. */
int lbm_vn_spectra(int32_t lattice, int32_t equilibrium, int32_t bulk_correction, const double *cases,
                   int64_t count, double *radius, double *eig, int32_t *info, double *flops, void *stream);

/* Largest spectral radius over a wave-vector grid, for n_states states: for
 * state s = (tau, u_x, u_y) (device array of n_states * 3 doubles) the
 * maximum of max |lambda| over k = (pi a / (nk - 1), pi b / (nk - 1)),
 * a, b = 0..nk-1 (k_x only for D1Q3; k = 0 when nk = 1), the grid over
 * [0, pi]^2 of Sec. "Linear stability domain".
 *   max_radius   device pointer to n_states doubles (written).
 *   scratch      device pointer to n_states * 8 bytes, 8-byte aligned
 *                (caller-owned; overwritten).
 *   unconverged  device pointer to one int32: number of matrices whose QR
 *                iteration hit the limit (written).
 * Enqueues three kernels and returns without synchronising.  The maximum does
 * not depend on the order of evaluation.  Errors: LBM_EINVAL (as for
 * lbm_vn_spectra; nk < 1 or > 65536; NULL pointers; n_states * nk^D above
 * 2^31 * 64); LBM_EDEVICE. */
int lbm_vn_max_radius(int32_t lattice, int32_t equilibrium, int32_t bulk_correction, const double *states,
                      int64_t n_states, int32_t nk, double *max_radius, void *scratch, int32_t *unconverged,
                      void *stream);

/* lbm_vn_max_radius for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation and results, with the scratch held by the library in a
 * static device array of 65536 entries (512 KiB on each GPU the library runs
 * on, kept until the process ends) instead of a caller's buffer.  No memory is
 * allocated; the clear, the spectra and the conversion are three kernel
 * launches on `stream` (the first call on a device also looks up the array's
 * device address).  Calls on one GPU share the array: calls that overlap on
 * the device (on different streams, or from several threads) race; calls in
 * one stream are ordered.  Errors: as lbm_vn_max_radius, and LBM_EINVAL for
 * n_states > 65536. */
int lbm_vn_max_radius_noalloc(int32_t lattice, int32_t equilibrium, int32_t bulk_correction, const double *states,
                              int64_t n_states, int32_t nk, double *max_radius, int32_t *unconverged, void *stream);

/* Message of the last error raised on the calling thread (static storage,
 * empty if none). */
const char *lbm_last_error(void);

/* Library version string (static). */
const char *lbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_ENTROPIC_H */
