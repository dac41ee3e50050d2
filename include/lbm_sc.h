/*
 * lbm_sc.h - C ABI of the MI355X (gfx950) Shan-Chen D3Q19 lattice Boltzmann library.
 *
 * The library relaxes hydrostatic droplets, bubbles and flat slabs of a Shan-Chen non-ideal fluid
 * (Lulli, Biferale, Falcucci, Sbragaglia, Shan, "A Mesoscale Perspective on the Tolman Length",
 * arXiv:2105.08772) on one GPU. One time step is the lattice transport of Sec. 2, Eq. (lbm),
 * with the BGK collision Eq. (sm:omega_i), the Guo forcing term, the second-order equilibrium and
 * the Guo equilibrium velocity that follow it, and the Shan-Chen force Eq. (SCForce). The
 * observables are those of Sec. 3 and Sec. 4: mass, momentum, centre of mass, the lattice
 * pressure tensor Eq. (sm:pt) along a line or averaged over planes, P_in, P_out, the generalized
 * surface tension Eq. (gen_sigma) and its minimum R_s, the equimolar radius R_e, the flat-interface
 * sigma_0 and the velocity-change convergence measure.
 *
 * Conventions shared by every entry point:
 *   - Every function returns an lbm_sc_status (0 on success, a negative code otherwise) unless
 *     stated otherwise; lbm_sc_last_error() then describes the failure. No C++ exception crosses
 *     this boundary.
 *   - The handle owns all device memory it allocates and frees it in lbm_sc_destroy. The caller
 *     owns every pointer it passes; the library keeps none of them after the call returns, except
 *     the stream in lbm_sc_config.
 *   - A handle is used from one host thread at a time.
 *   - Host arrays of populations use the canonical layout f[i][z][y][x] (x fastest, no padding,
 *     FP64) and hold the pre-collision populations f_i(x, t) of the current time t. The D3Q19
 *     order is: i = 0 rest; 1..6 = +x, -x, +y, -y, +z, -z; 7..18 = (1,1,0), (-1,-1,0), (1,-1,0),
 *     (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).
 *     Every moving velocity is followed by its opposite.
 *   - Boxes are periodic along all three axes.
 */
#ifndef LBM_SC_H
#define LBM_SC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_sc lbm_sc; /* opaque handle */

typedef enum {
    LBM_SC_OK = 0,
    LBM_SC_EINVAL = -1,    /* invalid argument or configuration */
    LBM_SC_ENOMEM = -2,    /* device or host allocation failed */
    LBM_SC_EDEVICE = -3,   /* a HIP runtime call or a kernel launch failed */
    LBM_SC_EUNSTABLE = -4  /* a non-finite value or n <= 0 was seen by lbm_sc_observables */
} lbm_sc_status;

/* Pseudopotentials of Sec. 4. */
enum { LBM_SC_PSI_EXP = 0 /* psi = exp(-1/n) */, LBM_SC_PSI_ONEMINUS = 1 /* psi = 1 - exp(-n) */ };

/* Initial geometry (Sec. 4 tanh profile). FROM_HOST leaves the state undefined until
 * lbm_sc_set_populations is called. */
enum { LBM_SC_DROPLET = 0, LBM_SC_BUBBLE = 1, LBM_SC_SLAB = 2, LBM_SC_FROM_HOST = 3 };

/* Population storage. FP64 stores f_i in double precision and computes in double precision.
 * FP32_SHIFTED stores g_i = f_i - w_i rho_ref in single precision and computes the step in
 * single precision. FP32_SHIFTED_MATH64 stores the same single-precision g_i (same memory and
 * HBM traffic) but does the step's arithmetic (psi, force, velocity, equilibrium, collision) in
 * double precision, rounding only the stored populations. Observables are always computed in
 * double precision. */
enum { LBM_SC_FP64 = 0, LBM_SC_FP32_SHIFTED = 1, LBM_SC_FP32_SHIFTED_MATH64 = 2 };

typedef struct {
    int32_t nx, ny, nz;      /* periodic box, each >= 1; x is the fastest axis */
    int32_t psi;             /* LBM_SC_PSI_* */
    int32_t geom;            /* LBM_SC_DROPLET / BUBBLE / SLAB / FROM_HOST */
    int32_t prec;            /* LBM_SC_FP64 / LBM_SC_FP32_SHIFTED / LBM_SC_FP32_SHIFTED_MATH64 */
    int32_t slab_axis;       /* slab normal: 0 = x, 1 = y, 2 = z */
    int32_t packed_rows;     /* 0: rows of the stored populations padded to whole 128-byte lines
                                (for the default x-y tiles); 1: rows packed at pitch nx, for
                                full-row tiles (lbm_sc_launch / lbm_sc_group_launch tile_x 0),
                                which then leave no lanes idle over padding. Results are the same */
    double tau;              /* BGK relaxation time, > 0.5 */
    double g_over_gc;        /* coupling G = g_over_gc * G_c(psi); G_c < 0, so > 1 separates phases */
    double radius;           /* droplet/bubble radius R of the tanh profile (Sec. 4), > 0 */
    double width;            /* tanh width w: n = (n_in+n_out)/2 - (n_in-n_out)/2 tanh((r-R)/w), > 0 */
    double slab_thickness;   /* slab: thickness of the liquid layer centred at floor(L/2) */
    double n_in, n_out;      /* densities inside/outside; both 0 => flat coexistence densities from
                                lbm_sc_coexistence (liquid inside for DROPLET and SLAB, gas inside for
                                BUBBLE) */
    double noise_amp;        /* additive uniform noise in [-noise_amp, noise_amp) on the initial n */
    uint64_t seed;           /* noise of node k = SplitMix64(seed ^ k), k = (z*ny + y)*nx + x */
    double rho_ref;          /* shifted FP32 reference density; 0 => (n_in + n_out)/2 */
    void* stream;            /* hipStream_t to enqueue on, or NULL for a stream the handle owns */
} lbm_sc_config;

typedef struct {
    int64_t step;            /* time steps taken since creation or the last set_populations */
    double mass, mass0;      /* sum_x n now and at creation / last set_populations */
    double mom[3];           /* sum_x n u, u = (sum_i xi_i f_i + F/2)/n (Sec. 2) */
    double com[3];           /* centre of mass: c + sum n d / M, d the minimum-image offset from
                                c = floor(L/2); for even L the node at offset L/2 counts 0 */
    double n_center, n_far;  /* n at c and at the far probe ((c + floor(L/2)) mod L per axis) */
    double P_in, P_out, dP;  /* P^xx of Eq. (sm:pt) at the two probes (Sec. 4), dP = P_in - P_out */
    double C;                /* int_0^{R_out} r^2 (P_out - P^yy(c + r e_x)) dr, trapezoid on nodes */
    double R_s, sigma_s;     /* minimum of sigma[R] = dP R/3 + C/R^2 (Eq. gen_sigma): (6C/dP)^(1/3),
                                dP R_s/2; NaN unless dP > 0 and C > 0 (droplet/bubble only) */
    double R_e;              /* equimolar radius (Sec. 4) from mass, n_center, n_far */
    double sigma0_flat;      /* slab: sum over the half box [L/2, L) along the normal of P_N - P_T */
    double pn_spread;        /* slab: max - min over planes of the plane-averaged P_N */
    double du_l1;            /* L^-3 sum_x sum_a |u_a - u_a(previous observables call)| (Sec. 4) */
    double du_max;           /* max_x max_a of the same difference */
    double n_min, n_max;     /* extrema of n over the box */
    int32_t finite;          /* 1 if every n is finite and > 0 and every u finite, else 0 */
    int32_t has_du;          /* 1 if du_l1/du_max compare against an earlier call */
} lbm_sc_obs;

typedef struct {
    double G;                /* coupling used */
    double Gc;               /* critical coupling of the pseudopotential */
    double n_in, n_out;      /* densities used for the initial profile */
    double rho_ref;          /* shifted FP32 reference density (0 for FP64) */
    int64_t nodes;           /* nx*ny*nz */
    int64_t device_bytes;    /* device memory held by the handle */
    int64_t bytes_per_step;  /* algorithmic HBM bytes of one step: 2 * 19 * sizeof(storage) * nodes */
    int32_t block_x, block_y, z_chunk; /* tile and chunk of the fused step kernel's launch shape */
    int32_t reserved;
} lbm_sc_info;

/* Create a box. Validates cfg (LBM_SC_EINVAL on any out-of-range field: sizes < 1, tau <= 0.5,
 * unknown enums, radius/width <= 0 for DROPLET/BUBBLE/SLAB, g_over_gc <= 1 when the densities must
 * come from lbm_sc_coexistence; also for boxes of more than 2^31 nodes or whose z-planes are so
 * large that the 19 populations of one plane exceed 4 GiB, i.e. beyond about 53 M (FP32 storage)
 * or 26 M (FP64) nodes per plane), allocates two population buffers and the box's small
 * observation buffers (among them the last observed velocity, 24 bytes per node) on the current
 * HIP device (LBM_SC_ENOMEM), and builds the initial state on the device: the tanh
 * profile plus noise, psi, the force of Eq. (SCForce), and f = f_eq(n, u = -F/(2n)) so that the
 * physical velocity (sum xi f + F/2)/n is zero. Returns after the work is enqueued and *out set.
 * On failure *out is NULL and nothing is leaked. */
int lbm_sc_create(const lbm_sc_config* cfg, lbm_sc** out);

/* Like lbm_sc_create, but the two population buffers (the ping-pong state, the bulk of a box's
 * memory) are supplied by the caller, e.g. from a tensor allocator: a and b are device memory of
 * the current device, 256-byte aligned, not overlapping, each with at least
 * lbm_sc_population_bytes(cfg) bytes (`bytes`) inside its allocation. The library uses them in
 * place, never frees them, and does not keep them beyond lbm_sc_destroy; the caller keeps them
 * alive until then. The observation buffers are still allocated by the library (device_bytes of
 * lbm_sc_get_info counts only those). Work of other streams on a or b must have finished before
 * this call (the initial state is written on the box's stream, unordered with other streams).
 * LBM_SC_EINVAL, with nothing allocated, if a buffer is NULL, misaligned, too small, not device
 * memory of the current device, or the two overlap. */
int lbm_sc_create_with_buffers(const lbm_sc_config* cfg, void* a, void* b, size_t bytes,
                               lbm_sc** out);

/* Bytes of one population buffer of a box with this configuration (for
 * lbm_sc_create_with_buffers); a negative lbm_sc_status if cfg is invalid. Host only. */
int64_t lbm_sc_population_bytes(const lbm_sc_config* cfg);

/* Enqueue nsteps (>= 0) time steps of Eq. (lbm) on the handle's stream: fused pull streaming,
 * density and psi, Shan-Chen force, Guo equilibrium velocity, BGK collision with the Guo term.
 * With two steps per pass (lbm_sc_launch.steps_per_pass, the default for FP32 storage and
 * arithmetic at tau = 1) pairs of steps run as one launch and an odd last step as a single one;
 * the results are bitwise those of single steps. Runs of graph_steps steps are replayed from a
 * hipGraph the handle captures on first use. While the caller is capturing the stream the call
 * records plain launches into the caller's graph: nsteps must then be even (LBM_SC_EINVAL
 * otherwise, nothing recorded; with two steps per pass a count that is not a multiple of 4 is
 * recorded as single steps), every replay advances the box by nsteps, and the host step counter
 * advances once, at the capture (lbm_sc_set_step corrects it after replays). Returns after
 * enqueueing (asynchronous); LBM_SC_EDEVICE if a launch fails. */
int lbm_sc_step(lbm_sc* h, int64_t nsteps);

/* Wait until all work enqueued on the handle's stream has finished. This call, and every other
 * call documented as synchronising or uploading, returns LBM_SC_EINVAL without touching the
 * stream while the caller is capturing it (a capture can hold neither). */
int lbm_sc_sync(lbm_sc* h);

/* Compute the observables of the current state in FP64 (listed in lbm_sc_obs) and synchronise.
 * prof may be NULL; otherwise prof_len must be 4*L where L is nx (droplet/bubble/from-host: the line
 * y = floor(ny/2), z = floor(nz/2), x = 0..nx-1) or the box length along slab_axis (slab: averages
 * over planes normal to the axis); it receives [n, P^xx, P^yy, P^zz] each of length L. The
 * velocity field of this call becomes the reference of the next call's du_l1/du_max. Returns
 * LBM_SC_EUNSTABLE (with *out filled) if out->finite is 0. Not for use inside a stream capture. */
int lbm_sc_observables(lbm_sc* h, lbm_sc_obs* out, double* prof, size_t prof_len);

/* Copy the current pre-collision populations f_i(x, t) to the host array f (canonical layout,
 * len must be 19*nx*ny*nz). Shifted FP32 states are widened to FP64 and the shift w_i rho_ref
 * added back. Synchronises. Not for use inside a stream capture. */
int lbm_sc_get_populations(lbm_sc* h, double* f, size_t len);

/* Replace the state by the host array f (canonical layout, pre-collision populations at the
 * current time, len 19*nx*ny*nz). Shifted FP32 storage holds them rounded after subtracting w_i rho_ref.
 * Resets the step counter (which also seeds the rounding dither of the FP32 rest population, so
 * the same state stepped the same number of times gives the same result), mass0 and the du
 * reference. Synchronises. Not for use inside a stream capture. */
int lbm_sc_set_populations(lbm_sc* h, const double* f, size_t len);

/* Set the step counter (>= 0; LBM_SC_EINVAL otherwise) together with the step count that seeds
 * the FP32 rest-population dither, e.g. after lbm_sc_set_populations when resuming a saved
 * state: a state saved with lbm_sc_get_populations at step n and restored with
 * lbm_sc_set_populations + lbm_sc_set_step(n) continues bitwise as the uninterrupted run would
 * (FP64 and FP32 storage alike). Synchronises. Not for use inside a stream capture. */
int lbm_sc_set_step(lbm_sc* h, int64_t step);

/* Launch shape of the fused step kernel. The workgroup is 64*waves threads (waves wave64s) and
 * owns an x-y tile tile_x nodes wide and waves*rows*(64/tile_x) rows high (at tile_x = 32 each
 * wave row covers two rows of 32 nodes), and a run of z_chunk planes along z. Supported shapes:
 * waves 4 with rows 1, 2 or 4 (rows 1 or 2 at tile_x 32) and either prefetch setting; waves 8
 * with rows 1 or 2 and prefetch 0. tile_x = 0 selects full-row tiles for boxes with short rows:
 * the workgroup (prefetch 0) owns whole rows, `rows` is the number of nodes each thread holds per
 * plane (waves 8: 2, 4, or 8 with FP32 arithmetic; waves 4: 4), and a tile has
 * rows*64*waves/px - 2 rows, px being the row pitch (less up to 31 slots that align packed rows
 * with the line grid; LBM_SC_EINVAL if that is below 1). steps_per_pass = 2 selects the
 * two-steps-per-pass kernel instead (FP32 storage and arithmetic, tau = 1), whose shapes are
 * tile_x 64 with rows 1 and waves 8 (64 x 8 tiles, either prefetch setting), tile_x 32 with rows
 * 2 and waves 8 (32 x 16 tiles, either prefetch setting), tile_x 32 with rows 2 and waves 4
 * (32 x 16 tiles, two nodes per thread, prefetch 0) or tile_x 64 with rows 2 and waves 16
 * (64 x 16 tiles, prefetch 0); it is the default for those boxes (32 x 16 tiles of 4 waves from
 * 2.3 M nodes, 64 x 8 with prefetch below), and lbm_sc_get_launch reports the shape of the kernel
 * in use. */
typedef struct {
    int32_t rows;       /* tile rows per wave: 1, 2 or 4 (full-row tiles: nodes per thread, 2, 4, 8) */
    int32_t z_chunk;    /* planes per workgroup, >= 1 (clamped to nz) */
    int32_t xcd_remap;  /* 1: hand neighbouring tiles to the same XCD (shared L2); 0: identity */
    int32_t prefetch;   /* 1: issue the next plane's loads before the collision of the current one */
    int32_t waves;      /* wave64s per workgroup: 4 or 8 */
    int32_t tile_x;     /* tile width: 64 or 32; 0 for full-row tiles */
    int32_t graph_steps;/* lbm_sc_step replays a hipGraph of this many steps (even, <= 4096;
                           0: plain launches; default 64; plain launches inside a caller's
                           stream capture) */
    int32_t steps_per_pass; /* 1, or 2: two time steps per kernel pass (FP32 storage and
                           arithmetic, tau = 1 only; the fields above then give its shape, and
                           an odd last step runs in the last single-step shape set, or the
                           default one). The box streams through HBM once per two steps; the
                           results are bitwise those of single steps */
} lbm_sc_launch;

/* Set / read the launch shape. The shape changes only the schedule: every node's arithmetic and
 * result are identical for every shape (bitwise). Used by the autotuner. LBM_SC_EINVAL for values
 * out of range. */
int lbm_sc_set_launch(lbm_sc* h, const lbm_sc_launch* launch);
int lbm_sc_get_launch(lbm_sc* h, lbm_sc_launch* out);

/* ------------------------------------------------------------------------------------------
 * Groups: many boxes advanced by one fused launch per time step.
 *
 * A group steps a set of existing boxes (handles made by lbm_sc_create) together: every step is
 * one launch of the multi-box step kernel over the flattened list of (box, x-y tile, z chunk)
 * work items, so boxes of different sizes, pseudopotentials, couplings and relaxation times share
 * the GPU in a single launch. The per-node arithmetic is the same as lbm_sc_step, so a box
 * stepped in a group ends bitwise equal to the same box stepped alone. All boxes of a group must
 * have the same precision (any of the three) and must have been created on the group's stream. Boxes stay
 * owned by the caller; the group keeps their handles until the next lbm_sc_group_set or
 * lbm_sc_group_destroy, and they must not be destroyed in between.
 * ------------------------------------------------------------------------------------------ */
typedef struct lbm_sc_group lbm_sc_group;

typedef struct {
    int32_t rows;        /* tile rows per wave (supported tile shapes as for lbm_sc_launch) */
    int32_t z_chunk;     /* planes per work item, >= 1 (clamped to each box's nz); 0: each box is
                            cut into z chunks of about equal work, items_per_cu items per CU */
    int32_t xcd_remap;   /* non-persistent launch: hand neighbouring items to the same XCD */
    int32_t prefetch;    /* issue the next plane's loads before the current collision */
    int32_t persistent;  /* 1: fixed grid of `workers` workgroups drawing items from 8 per-XCD
                            work queues; 0: one workgroup per item */
    int32_t workers;     /* persistent grid size, a multiple of 8 (0 = 256) */
    int32_t graph_steps; /* steps captured per hipGraph and replayed (even, 0 = no graph) */
    int32_t waves;       /* wave64s per workgroup: 4 or 8 */
    int32_t tile_x;      /* tile width: 64 or 32; 0 for full-row tiles (FP32 boxes for rows 8) */
    int32_t items_per_cu;/* z_chunk 0: work items per CU in total (0 = 8, at most 4096) */
    int32_t steps_per_pass; /* 0 or 1: one time step per launch; 2: two time steps per launch by
                            the two-steps-per-pass kernel (every box with FP32 storage and
                            arithmetic at tau = 1; the tile shapes of lbm_sc_launch with
                            steps_per_pass 2; persistent 0). The group then reads and writes each
                            box once per two steps; a graph holds graph_steps / 2 launches when
                            graph_steps is a multiple of 4 (plain launches otherwise), and an odd
                            last step runs as one single-step launch per box, in the box's own
                            single-step shape. Results are bitwise those of single steps */
} lbm_sc_group_launch;

/* Create an empty group that enqueues on `stream` (a hipStream_t, required: the boxes of the
 * group must have been created with this same stream). */
int lbm_sc_group_create(void* stream, lbm_sc_group** out);

/* Set the boxes stepped by the group (nbox >= 0; an empty group steps nothing). Validates that
 * every box has the group's stream and that all share one precision (LBM_SC_EINVAL otherwise),
 * builds the work list for the current launch shape and uploads it (stream-ordered). Not for use
 * inside a stream capture. */
int lbm_sc_group_set(lbm_sc_group* g, lbm_sc* const* boxes, int32_t nbox);

/* Enqueue nsteps (>= 0) time steps of every box of the group: one multi-box launch per step (per
 * two steps with steps_per_pass 2), replayed from a captured hipGraph in chunks of graph_steps.
 * Each box's step counter advances by nsteps. Asynchronous. LBM_SC_EINVAL, with nothing enqueued, while the group's stream is being
 * captured by the caller. */
int lbm_sc_group_step(lbm_sc_group* g, int64_t nsteps);

/* Set / read the group's launch shape (the work list is rebuilt; results are unchanged). Setting
 * it is not for use inside a stream capture. */
int lbm_sc_group_set_launch(lbm_sc_group* g, const lbm_sc_group_launch* launch);
int lbm_sc_group_get_launch(lbm_sc_group* g, lbm_sc_group_launch* out);

/* Number of boxes, work items, nodes and algorithmic HBM bytes of one group step. */
int lbm_sc_group_info(lbm_sc_group* g, int32_t* nbox, int64_t* items, int64_t* nodes,
                      int64_t* bytes_per_step);

/* Release the group (after waiting for its stream); the boxes are untouched. NULL is ignored.
 * Not for use inside a stream capture (it waits and frees device memory). */
void lbm_sc_group_destroy(lbm_sc_group* g);

/* Most boxes one call of lbm_sc_step_boxes_noalloc takes. */
#define LBM_SC_NOALLOC_MAX_BOXES 1024

/* For callers that cannot allocate device memory: code recording into a HIP graph of its own,
 * serving loops that must not call hipMalloc/hipFree, harnesses that forbid it. Enqueues nsteps
 * (>= 0) time steps of the nbox boxes with one multi-box launch per step, like a group holding
 * these boxes under `launch` (same kernels, so the result is bitwise that of lbm_sc_group_step
 * and of lbm_sc_step), but without a group object: the work list and the persistent kernel's
 * queue state are written, by small kernels on the boxes' stream, into a fixed device array that
 * the library holds once per GPU (122,952 bytes, kept until the process ends). Nothing is
 * allocated on the device or freed, and no host buffer is staged. Limit: at most
 * LBM_SC_NOALLOC_MAX_BOXES boxes per call (LBM_SC_EINVAL beyond, nothing enqueued).
 * The boxes stay owned by the caller; every box must be non-NULL, appear once, share one
 * precision and have been created on one stream, where the work is enqueued; launch follows the
 * rules of lbm_sc_group_set_launch and must fit every box (LBM_SC_EINVAL otherwise, nothing
 * enqueued). With steps_per_pass 2 the two-step kernel takes the work items in list order (a
 * group also spreads them over the XCDs by cost) and an odd last step runs as one single-step
 * launch per box; inside a caller's capture a count of 4k + 2 records its last pair of steps that
 * way too, so that every replay leaves each box in the buffer the next one expects. Each box's step counter advances by nsteps. Asynchronous. Calls that overlap in time
 * on one GPU (enqueued on different streams) race on the shared array; calls on one stream are
 * ordered. While the caller is capturing the stream the launches are recorded into the caller's
 * graph: nsteps must then be even, every replay advances the boxes by nsteps, and the host step
 * counters advance once, at the capture. LBM_SC_EDEVICE if a launch fails (the counters then
 * advance by the steps enqueued before it). */
int lbm_sc_step_boxes_noalloc(lbm_sc* const* boxes, int32_t nbox, int64_t nsteps,
                              const lbm_sc_group_launch* launch);

/* Measurement helper, not part of the method: copy `bytes` (a multiple of 16; src and dst
 * 16-byte aligned device pointers that do not overlap) with a plain streaming kernel on `stream`
 * (hipStream_t or NULL for the null stream), each lane moving lane_bytes (4, 8 or 16) per access.
 * Asynchronous. It measures the achievable HBM bandwidth that the step kernel is compared with;
 * the 4-byte form has the access width of the FP32 step. LBM_SC_EINVAL, with nothing launched, on
 * bad sizes, alignment or lane_bytes, or unless each of the two ranges lies inside one device
 * allocation of the current device. */
int lbm_sc_stream_copy(const void* src, void* dst, size_t bytes, int32_t lane_bytes, void* stream);

/* Describe the handle (coupling, densities, sizes, launch shape). */
int lbm_sc_get_info(lbm_sc* h, lbm_sc_info* out);

/* Release everything the handle owns (after waiting for its stream). NULL is ignored. Not for
 * use inside a stream capture (it waits and frees device memory), nor while a graph that the
 * caller recorded from this handle's steps may still be replayed. A box that groups still list
 * leaves them: each rebuilds its work list without it before its next launch. */
void lbm_sc_destroy(lbm_sc* h);

/* Message of the last failure on the calling thread; valid until the next call on that thread.
 * Never NULL. */
const char* lbm_sc_last_error(void);

/* Critical coupling G_c of the bulk pressure P(n) = n c_s^2 + (G c_s^2/2) psi(n)^2 (Eq. bulkp):
 * dP/dn = d^2P/dn^2 = 0, i.e. -e^2 for LBM_SC_PSI_EXP and -4 for LBM_SC_PSI_ONEMINUS. Returns NaN
 * for an unknown psi. Host only. */
double lbm_sc_gc(int32_t psi);

/* Bytes per node of the observation workspace shared by the boxes of one device (below). */
#define LBM_SC_OBS_WORKSPACE_BYTES_PER_NODE 40

/* Device memory a box with this configuration will hold (populations, the last observed velocity
 * and small buffers), in bytes, without allocating anything; used to admit work by free HBM.
 * Not counted: the observation workspace that the boxes of one device share (density, psi and
 * momentum of every node, LBM_SC_OBS_WORKSPACE_BYTES_PER_NODE per node of the largest box
 * observed, created with the first
 * box, get or set that needs it and freed with the device's last box); calls that use it
 * (create, observables, get and set populations) on boxes of one device take turns, each holding
 * it until its own stream has drained. Returns a negative lbm_sc_status if cfg is invalid. Host
 * only. */
int64_t lbm_sc_device_bytes(const lbm_sc_config* cfg);

/* Flat-interface coexistence densities and pressure for G = g_over_gc * G_c (the "equilibrium
 * values of n_g, n_l for a flat interface" of Sec. 4), from the leading-order lattice rule
 * P(n_g) = P(n_l) = p0 and int_{n_g}^{n_l} (p0 - P(n)) psi'(n)/psi(n) dn = 0, which follows from
 * the flat-interface constancy of P_N stated after Eq. (sm:pt). Host only; any output pointer may
 * be NULL. LBM_SC_EINVAL if g_over_gc <= 1 or no coexistence exists. */
int lbm_sc_coexistence(int32_t psi, double g_over_gc, double* n_gas, double* n_liquid, double* p0);

#ifdef __cplusplus
}
#endif

#endif /* LBM_SC_H */
