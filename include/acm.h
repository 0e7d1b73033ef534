/*
 * acm.h - C ABI of the MI355X SMAME library (libacm.so).
 *
 * The library advances the simplified artificial-compressibility equations
 * of Huang, arXiv 2012.03525 ("SMAME"):
 *   continuity  (Eq. 2.10)  rho^{n+1} = rho^n - dt d_a(rho u_a)^n
 *                                       + 1/2 cs^2 dt^2 d_aa rho^n
 *   momentum    (Eq. 2.11)  (rho u_a)^{n+1} = (rho u_a)^n
 *                             - dt d_b(rho u_a u_b + rho cs^2 delta_ab)^n
 *                             + nu dt d_bb (rho u_a)^n
 *                             - (nu + 1/2 cs^2 dt)(d_a rho^{n+1} - d_a rho^n)
 *                             + dt rho^{n+1} g_a            (body force, Sec. 2)
 *                             - dt phi d_a mu               (two-phase, Sec. 2)
 * with centred second-order differences (Eqs. 2.12-2.13) on a collocated
 * grid, and, for two-phase flow, the Cahn-Hilliard equation (Eq. 2.14)
 * with mu = 4 a phi (phi^2 - 1) - kappa d_aa phi, a = 3 sigma/(4W),
 * kappa = 3 sigma W/8, isotropic stencils and Heun's second-order
 * Runge-Kutta step.
 *
 * Conventions shared by every entry point
 * - Fields are caller-owned DEVICE arrays, structure of arrays, x fastest:
 *   element (i, j, k) of an nx*ny*nz grid lives at (k*ny + j)*nx + i.
 *   Density is stored as the deviation drho = rho - rho0 (rho0 = 1 in the
 *   paper, Sec. 2 last paragraph), so FP32 storage keeps its O(Ma^2) signal.
 * - Element type is double for ACM_F64 and float for ACM_F32.
 * - Every call that launches work is asynchronous on the stream given at
 *   initialisation (a hipStream_t passed as void*; NULL = the null stream),
 *   except the calls documented as synchronising.
 * - Errors are returned as acm_status; no exception crosses the ABI.
 *   acm_last_error() returns a thread-local message for the last failure.
 * - A handle is not thread-safe; use one handle per stream.
 */
#ifndef ACM_H
#define ACM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ACM_OK = 0,
    ACM_EINVAL = -1,      /* bad size, pointer, boundary pairing or parameter   */
    ACM_EUNSTABLE = -2,   /* linear stability check failed (see acm_stability)  */
    ACM_EHIP = -3,        /* a HIP runtime call failed                          */
    ACM_ENONFINITE = -4,  /* diagnostics found a NaN/Inf (fields still returned)*/
    ACM_ESTATE = -5       /* call not valid in the handle's current state       */
} acm_status;

/* Boundary type of a face.  Faces are ordered -x, +x, -y, +y, -z, +z.
 * PERIODIC must be paired with PERIODIC on the opposite face.
 * WALL is a no-slip (optionally moving) wall halfway between the last node
 * and its ghost: ghost drho = mirror drho, ghost u = 2 u_wall - mirror u.
 * SYMMETRY is a mirror plane halfway between nodes: every field mirrored,
 * normal velocity negated.  For two-phase runs phi and mu are mirrored at
 * both (contact angle 90 degrees, Sec. 2 wetting condition with cos = 0).
 * The paper states the physical conditions (Sec. 3.2-3.6) but not their
 * discretisation; the halfway placement is this library's reading. */
typedef enum { ACM_BC_PERIODIC = 0, ACM_BC_WALL = 1, ACM_BC_SYMMETRY = 2 } acm_bc;

typedef enum { ACM_F64 = 0, ACM_F32 = 1 } acm_precision;

/* Problem statement (Sec. 2; Sec. 3 opening: dx = L/N_L, dt = T_c/N_t). */
typedef struct acm_config {
    int32_t dim;            /* 2 or 3                                         */
    int32_t nx, ny, nz;     /* nodes per axis (nz ignored in 2D); each >= 4;
                               at most 4e9 nodes; 3D: nx*ny values of one
                               plane below 2 GiB                              */
    double dx, dt;          /* grid spacing and time step                     */
    double nu;              /* kinematic viscosity                            */
    double cs;              /* sound speed; <= 0 selects dx/(dt sqrt 3)       */
    double rho0;            /* reference density (1 in the paper)             */
    double sat_rho;         /* multiplier of the continuity SAT (paper: 1)    */
    double sat_mom;         /* multiplier of the momentum SAT (paper: 1)      */
    double g[3];            /* uniform body force per unit mass               */
    int32_t bc[6];          /* acm_bc per face                                */
    double wall_u[6][3];    /* wall velocity per face (normal part must be 0) */
    int32_t two_phase;      /* 1: Cahn-Hilliard coupling (2D or 3D)           */
    double sigma;           /* surface tension                                */
    double width;           /* interface width W                              */
    double mobility;        /* mobility M                                     */
    int32_t precision;      /* acm_precision                                  */
    int32_t allow_unstable; /* 1: skip the stability check                    */
    int32_t graph_chunk;    /* steps per captured HIP graph (even); 0 = 64    */
    int32_t tile;           /* kernel tile variant; 0 = default.  2D single-
                               phase: 1 32x8, 2 64x8, 3 16x16, 4 128x4,
                               5 32x16 (0: 64x4).  2D axisymmetric: 1
                               32x8, 2 64x8, 4 64x4 (0: 32x16).  2D two-phase: 1 32x8,
                               2 64x8, 3 16x16 (0: 32x16).  3D: low byte
                               1 32x8, 2 64x8, 3 32x4, 4 64x4, 5 64x16,
                               7 32x16, 9 128x4, 12 128x8, 13 64x8 with two
                               rows per thread on fully periodic grids
                               (else as 2); 14 (FP32) 64x8, 15 32x8: two
                               steps per launch on fully periodic grids with
                               rho0 = 1 (acm_run; each run ends with one
                               one-step launch), else the default; 16, 17,
                               19: whole x rows per wave in bands of 4, 6, 2
                               rows (FP32 fully periodic grids with rho0 = 1,
                               nx 64, 128 or 256, ny >= band + 4; else the
                               default); 0: the whole-row kernel with 4-row
                               bands where it applies (chunk chosen for the
                               CU count), else 13 with 64-plane chunks,
                               or a smaller shape and chunk (down to 32x8
                               with 4-plane chunks) when that gives fewer
                               than two workgroups per CU (FP64 accepts 3,
                               4, else 32x8); bits 8+ = z chunk / 16 (0:
                               64 planes).  Results do not depend on the
                               tile. */
    double wet_cos[6];      /* two-phase: cos(contact angle) of each wall face
                               for the wetting condition of Sec. 2,
                               d_n phi = -(2/W) cos(theta) (1 - phi_w^2),
                               in [-1, 1]; 0 (90 degrees) mirrors phi       */
    int32_t axisym;         /* 1: axisymmetric 2D run, x axial, y radial,
                               the -y face the axis (must be
                               ACM_BC_SYMMETRY), row j at r = (j + 1/2) dx;
                               Eqs. (2.10)-(2.11) with the cylindrical
                               divergence and Laplacian in flux form, the
                               hoop term -cs^2 drho / r and -m_r / r^2 in the
                               radial momentum; two-phase runs add
                               (1/r) G_iso,r to L_iso in mu and in (2.14).
                               The stability guard uses the planar symbol;
                               diagnostics are volume integrals and volume
                               averages (cell volume 2 pi r dx^2) with the
                               cylindrical divergence.  0: planar           */
} acm_config;

/* Device pointers of one complete state.  w is used in 3D only, phi in
 * two-phase runs only; unused members may be NULL. */
typedef struct acm_fields {
    void* drho;
    void* u;
    void* v;
    void* w;
    void* phi;
} acm_fields;

/* Diagnostics of the newest state (all FP64, deterministic reductions).
 * Sums over nodes use the cell volume dx^D where stated; in axisymmetric
 * runs the cell volume is 2 pi r dx^2, phi_sum is weighted the same way, the
 * means over S are volume averages and the divergence is the cylindrical
 * one of the continuity update. */
typedef struct acm_diag {
    double mass;        /* sum(drho) dx^D                                      */
    double mom[3];      /* sum(rho u_a) dx^D                                   */
    double ke;          /* E_k = 1/2 sum |u|^2 dx^D (Sec. 3.1, not rho-weighted)*/
    double dumax;       /* max | |u|^{n+1} - |u|^n | (steady test, Sec. 3.2)   */
    double umax;        /* max |u|                                             */
    double enstrophy;   /* (1/2S) sum |omega|^2 dS, centred vorticity (Eq. 3.4)*/
    double energy;      /* (1/2S) sum |u|^2 dS (Eq. 3.4)                       */
    double div_rms;     /* rms of the centred divergence of u                  */
    double div_max;     /* max |centred divergence of u|                       */
    double phi_sum;     /* sum(phi) (two-phase)                                */
    int64_t step;       /* steps taken since init                              */
    int32_t nonfinite;  /* 1 if any stored value is NaN or Inf                 */
    int32_t which;      /* 0: set a holds the newest state, 1: set b           */
} acm_diag;

typedef struct acm_handle acm_handle;

/* Largest modulus of the amplification factor of the step linearised about
 * rest (Eqs. 2.10-2.13 in Fourier space, over all wavenumbers), and for
 * two-phase runs the Heun stability number dt M lambda (8a + kappa lambda)
 * of the bulk Cahn-Hilliard mode (stable when <= 2).  Pure host call. */
acm_status acm_stability(const acm_config* cfg, double* max_amplification, double* che_number);

/* Bytes of device scratch that acm_init needs for cfg: the FP64 partial and
 * final sums of the diagnostics reductions (about 14 doubles per 256 nodes,
 * at most 229 KiB) and, for 3D two-phase runs, four fields of nx*ny*nz
 * values of the precision type (phi* of Heun's first stage and the surface-
 * tension force phi G_iso mu per axis, Sec. 2).  Returns 0 and sets
 * acm_last_error for an invalid cfg.  Pure host call. */
size_t acm_scratch_bytes(const acm_config* cfg);

/* Validate cfg, check stability (unless allow_unstable), bind the two
 * caller-owned state sets a and b (each sized for the grid and precision)
 * and the caller-owned scratch buffer, and capture the HIP graphs of one
 * chunk of steps from either set.  The initial state must already be in a.
 * force_x: NULL or a device array of ny elements (precision type) added to
 * g[0] on row j (e.g. Kolmogorov forcing).  scratch: device memory of at
 * least acm_scratch_bytes(cfg) bytes (scratch_bytes), 256-byte aligned; it
 * must stay allocated, and must not be used by anything else, until
 * acm_destroy.  stream: hipStream_t or NULL.  The handle allocates no device
 * memory: it owns host data, a capture stream and the graph executables.
 * ACM_EINVAL for a NULL, misaligned or short scratch buffer. */
acm_status acm_init(const acm_config* cfg, const acm_fields* a, const acm_fields* b, const void* force_x,
                    void* scratch, size_t scratch_bytes, void* stream, acm_handle** out);

/* One step: the newest state moves from one set to the other.  Async. */
acm_status acm_step(acm_handle* h);

/* nsteps steps, launched as captured HIP graphs of graph_chunk steps plus
 * single launches for the remainder (tile codes 14 and 15: two steps per
 * launch, the last step of the run on its own, so the other set always
 * holds the state one step back).  Async. */
acm_status acm_run(acm_handle* h, int64_t nsteps);

/* Diagnostics of the newest state (dumax compares with the other set, so it
 * is meaningful once at least one step has run).  SYNCHRONISES the stream.
 * Returns ACM_ENONFINITE (with *out filled) if a stored value is not finite. */
acm_status acm_diagnostics(acm_handle* h, acm_diag* out);

/* Which set holds the newest state (0 = a, 1 = b) and the step counter. */
acm_status acm_current(const acm_handle* h, int32_t* which, int64_t* step);

/* Resume bookkeeping after the caller restored a checkpoint into set
 * `which`: the scheme is one-step, so a state plus its step count is a
 * complete checkpoint. */
acm_status acm_set_current(acm_handle* h, int32_t which, int64_t step);

/* Adjoint of one step (for training through the solver; not part of the
 * paper's method): with s = S(q) the step (2.10)-(2.13) with the body force
 * and the handle's forcing row, taken from state q, writes the
 * vector-Jacobian product adj_q = (dS/dq)^T adj_s.  q, s, adj_s, adj_q: device
 * fields drho, u, v of the handle's grid and precision, caller-owned; s must
 * hold S(q) (its density and velocity enter the derivative of u' = m'/rho').
 * adj_q must not alias the other three (ACM_EINVAL).  Covers planar 2D
 * single-phase handles with any mix of periodic, wall (moving or not) and
 * symmetry faces, whose ghost rules enter the derivative (ACM_EINVAL for 3D,
 * two-phase or axisymmetric handles).  Asynchronous on the handle's stream;
 * the handle's own sets are not touched. */
acm_status acm_step_adjoint(acm_handle* h, const acm_fields* q, const acm_fields* s, const acm_fields* adj_s,
                            const acm_fields* adj_q);

/* Release the handle (not the caller's fields).  Synchronises the stream. */
void acm_destroy(acm_handle* h);

/* Message of the last failing call on this thread ("" if none). */
const char* acm_last_error(void);

/* ------------------------------------------------------------------------ */
/* Batched independent 2D cases (serving-style sweeps)                       */
/* ------------------------------------------------------------------------ */
/* Hundreds of independent single-phase 2D cases of uneven size advance
 * together: each step is ONE launch over the active (case, tile) items,
 * either persistent workgroups claiming them from atomic work queues or one
 * workgroup per item (acm_batch_opts.mode), applying the same per-node
 * arithmetic as acm_step (results are bitwise equal to running each case
 * alone).  Steps are captured in HIP graphs of `chunk` steps; after every
 * chunk a health check retires cases that finished or diverged. */
typedef struct acm_batch acm_batch;

typedef struct acm_batch_case {
    acm_config cfg;        /* dim 2, single-phase; one precision per batch   */
    acm_fields a, b;       /* caller-owned state sets; initial state in a    */
    const void* force_x;   /* NULL or ny values added to g[0] on row j       */
    int64_t nsteps;        /* steps to run (rounded up to whole chunks)      */
    int32_t tile;          /* 2D tile variant 0..5, or -1: the tile recorded
                              for this (nx, ny, precision, launch mode) by
                              acm_batch_autotune / acm_batch_set_tuned_tile  */
} acm_batch_case;

typedef struct acm_batch_opts {
    int32_t chunk;         /* steps per captured graph, even; 0 = 500        */
    int32_t blocks;        /* mode 1: persistent workgroups; 0 = CUs x
                              occupancy                                      */
    int32_t grab;          /* mode 1: items per claim on the work queue once
                              a workgroup's fixed share is done; 0 = 2       */
    double umax_limit;     /* max |u| above this marks divergence; 0 = 0.3   */
    int32_t mode;          /* 0: one workgroup per (case, tile) item,
                              launched over the item capacity; 1: persistent
                              workgroups (blocks) in eight XCD groups, each
                              group over a contiguous range of the items:
                              fixed shares over half the range, then claims
                              of `grab` items from the group's counter.
                              Results do not depend on the mode.             */
} acm_batch_opts;

typedef struct acm_batch_case_status {
    int64_t steps_done;
    int32_t state;         /* 0 running, 1 finished, 2 diverged              */
    int32_t which;         /* set holding the newest state (always 0: chunks are even) */
    double done_ms;        /* batch start to the end of its last chunk; -1 while running */
    double umax;           /* max |u| at the last health check               */
} acm_batch_case_status;

/* Bytes of device scratch acm_batch_init needs for these cases and options:
 * the case records, the item table (for a case with tile -1 sized for the
 * variant with the most tiles), the item count, the queue counters (eight
 * group counters 128 bytes apart and a done counter: 1028 bytes), the
 * active list and the health pairs, each part 256-byte aligned.  Returns 0
 * and sets acm_last_error when a case or option is invalid.  Pure host call. */
size_t acm_batch_scratch_bytes(const acm_batch_case* cases, int32_t ncases, const acm_batch_opts* opts);

/* Validate every case (2D, single-phase, common precision, stability unless
 * allow_unstable), upload the case table into the caller's scratch (at least
 * acm_batch_scratch_bytes bytes, 256-byte aligned, kept allocated and unused
 * by anything else until acm_batch_destroy), size the persistent grid and
 * capture the chunk graph.  A case with tile -1 takes the tile that
 * acm_batch_autotune (or acm_batch_set_tuned_tile) recorded for its grid
 * shape, precision and launch mode in this process: ACM_ESTATE if there is
 * none.  The batch allocates no device memory.  Synchronises the stream
 * once (the case table upload). */
acm_status acm_batch_init(const acm_batch_case* cases, int32_t ncases, const acm_batch_opts* opts, void* scratch,
                          size_t scratch_bytes, void* stream, acm_batch** out);

/* Run up to max_chunks chunks (-1: until every case finished or diverged).
 * Synchronises the stream once per chunk (health read-back).
 * *active_left (may be NULL) receives the number of cases still running. */
acm_status acm_batch_run(acm_batch* b, int32_t max_chunks, int32_t* active_left);

/* Per-case progress, outcome and completion time. */
acm_status acm_batch_status(const acm_batch* b, int32_t i, acm_batch_case_status* out);

/* Wall time (GPU events) since the first run call and lattice-node updates done. */
acm_status acm_batch_timing(const acm_batch* b, double* total_ms, int64_t* lattice_updates);

void acm_batch_destroy(acm_batch* b);

/* Tile autotuner: time `copies` periodic nx x ny cases for `steps` steps
 * (even) with every 2D tile variant (0..5) through the batched kernel in the
 * given launch mode; ms_per_tile[6] receives ms per step, *best the fastest
 * variant, which is also recorded for (nx, ny, precision, mode) for the
 * life of the process (the choice changes only speed, never results).
 * scratch: device memory of acm_batch_autotune_scratch_bytes bytes,
 * 256-byte aligned, for the copies' fields and the tuning batches' tables;
 * free again when the call returns.  Synchronises the stream. */
size_t acm_batch_autotune_scratch_bytes(int32_t nx, int32_t ny, int32_t precision, int32_t copies);
acm_status acm_batch_autotune(int32_t nx, int32_t ny, int32_t precision, int32_t mode, int32_t copies, int32_t steps,
                              void* scratch, size_t scratch_bytes, void* stream, double* ms_per_tile, int32_t* best);

/* The tile recorded for (nx, ny, precision, mode) in this process
 * (ACM_ESTATE if none), and a way to record one measured earlier, e.g. in a
 * previous process on the same kind of GPU.  Pure host calls. */
acm_status acm_batch_tuned_tile(int32_t nx, int32_t ny, int32_t precision, int32_t mode, int32_t* tile);
acm_status acm_batch_set_tuned_tile(int32_t nx, int32_t ny, int32_t precision, int32_t mode, int32_t tile);

/* ------------------------------------------------------------------------ */
/* Learned closure: a CNN correcting a 4x-coarser SMAME step                 */
/* ------------------------------------------------------------------------ */
/* Network: ACM_CNN_LAYERS 3x3 convolutions with circular padding, channels
 * 3 -> 32 -> 32 -> 32 -> 32 -> 3 (the 3-channel input and output are padded
 * to 16 channels in memory), ReLU after every layer but the last.  It is not
 * part of the paper's method; it corrects the coarse step toward box-filtered
 * fine-grid states: q <- S_c(q) + D f(N S_c(q)), N and D per-channel scales.
 * Layouts: activations bf16 [ny][nx][C] (channel fastest); weights bf16
 * [9][C_out][C_in] with tap t = (dy+1)*3 + (dx+1); biases, gradients, master
 * weights and Adam moments fp32.  Grids need nx % 64 == 0 and ny % 8 == 0.
 * All calls are asynchronous on `stream`; buffers are caller-owned. */
#define ACM_CNN_LAYERS 5
enum { ACM_CONV_RELU = 0, ACM_CONV_RAW = 1, ACM_CONV_MASK = 2 };

/* Padded (C_in, C_out) of a layer: (16,32), (32,32) x3, (32,16). */
acm_status acm_cnn_layer_shape(int32_t layer, int32_t* cin, int32_t* cout);

/* y = conv3x3(x, w) on the bf16 matrix cores (FP32 accumulation):
 * ACM_CONV_RELU: y bf16 = relu(conv + bias); ACM_CONV_RAW: y fp32 = conv + bias;
 * ACM_CONV_MASK: y bf16 = conv * (mask > 0) (data gradient through a ReLU,
 * with w the weights from acm_cnn_transpose; bias unused).
 * Supported (cin, cout): (16,32), (32,32), (32,16) as the modes require. */
acm_status acm_cnn_conv(int32_t nx, int32_t ny, int32_t cin, int32_t cout, int32_t mode, const void* x,
                        const void* w, const float* bias, const void* mask, void* y, void* stream);

/* Weights of the transposed convolution: wt[t][i][o] = w[8-t][o][i]. */
acm_status acm_cnn_transpose(int32_t cin, int32_t cout, const void* w, void* wt, void* stream);

/* Weight and bias gradients of sum(g * conv(x)): dw[9][cout][cin], db[cout]
 * (fp32, overwritten), by per-workgroup MFMA partial sums in `workspace`
 * (acm_cnn_wgrad_workspace bytes) reduced in a fixed order. */
size_t acm_cnn_wgrad_workspace(int32_t nx, int32_t ny, int32_t cin, int32_t cout);
acm_status acm_cnn_wgrad(int32_t nx, int32_t ny, int32_t cin, int32_t cout, const void* x, const void* g,
                         float* workspace, float* dw, float* db, void* stream);

/* As acm_cnn_wgrad, but adds the gradients to dw and db (for sums over the
 * steps of an unrolled trajectory). */
acm_status acm_cnn_wgrad_add(int32_t nx, int32_t ny, int32_t cin, int32_t cout, const void* x, const void* g,
                             float* workspace, float* dw, float* db, void* stream);

/* Network input a0 (bf16, 16 channels) = in_scale[c] * (drho, u, v)[c]. */
acm_status acm_cnn_pack(int32_t nx, int32_t ny, const float* drho, const float* u, const float* v,
                        const float* in_scale, void* a0, void* stream);

/* In-place correction: (drho, u, v)[c] += out_scale[c] * raw[p][c]. */
acm_status acm_cnn_apply(int32_t nx, int32_t ny, const float* raw, const float* out_scale, float* drho,
                         float* u, float* v, void* stream);

/* Mean squared error of raw (fp32, 16 channels) against the target
 * residual (target[c] - base[c]) / out_scale[c] over pixels and the active
 * channels; grad (bf16, 16 channels) = d loss / d raw; *loss (device double)
 * is set.  A channel with out_scale[c] == 0 is excluded (zero error and
 * gradient; the closure then leaves that field uncorrected).  ACM_EINVAL for
 * a negative or non-finite scale or when all three are zero. */
size_t acm_cnn_loss_workspace(int32_t nx, int32_t ny);
acm_status acm_cnn_loss(int32_t nx, int32_t ny, const float* raw, const float* const* base,
                        const float* const* target, const float* out_scale, void* grad, double* workspace,
                        double* loss, void* stream);

/* acm_cnn_loss without the workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training or
 * serving loops, harnesses that forbid allocation): the per-workgroup
 * partial sums go to a static device array of ACM_LOSS_SCRATCH_DOUBLES
 * doubles that the library holds on each GPU it runs on until the process
 * ends, so grids are limited to ACM_LOSS_SCRATCH_DOUBLES * 256 pixels
 * (ACM_EINVAL beyond).  The array belongs to the device current at the call,
 * which must be the stream's device.  The call allocates nothing; results
 * equal acm_cnn_loss's bit for bit.  Every call on one GPU shares that
 * GPU's array (each call writes every partial it reads, so nothing needs
 * clearing): calls that overlap on one GPU, e.g. on two streams, race. */
#define ACM_LOSS_SCRATCH_DOUBLES 8192
acm_status acm_cnn_loss_noalloc(int32_t nx, int32_t ny, const float* raw, const float* const* base,
                                const float* const* target, const float* out_scale, void* grad, double* loss,
                                void* stream);

/* Loss of a state against a target for training through several steps:
 * e_c = (q[c] - target[c]) / out_scale[c] on the channels with
 * out_scale[c] > 0; *loss (device double) += weight * mean(e^2) over pixels
 * and those channels; adj[c] (fp32, in place) += weight * d mean(e^2) / d q[c].
 * workspace: acm_cnn_loss_workspace bytes.  ACM_EINVAL for NULL pointers, a
 * negative or non-finite scale, all scales zero, or a non-finite weight. */
acm_status acm_cnn_state_loss(int32_t nx, int32_t ny, const float* const* q, const float* const* target,
                              const float* out_scale, float weight, float* const* adj, double* workspace,
                              double* loss, void* stream);

/* Divergence penalty of a correction: d = G.(a - b), the centred divergence
 * (Eq. 2.12, grid units, periodic) of the velocity difference a - b (a, b:
 * fp32 u and v fields); *loss += weight * mean(d^2); adj_a[c] += its gradient
 * with respect to a; adj_b (optional) -= the same.  workspace:
 * acm_cnn_loss_workspace bytes.  Needs nx, ny >= 3; ACM_EINVAL for NULL
 * pointers or a non-finite weight. */
acm_status acm_cnn_div_penalty(int32_t nx, int32_t ny, const float* const* a, const float* const* b, float weight,
                               float* const* adj_a, float* const* adj_b, double* workspace, double* loss,
                               void* stream);

/* Adam update of n fp32 parameters (bias-corrected, step t >= 1); p16
 * (optional) receives the bf16 copy used by the convolutions. */
acm_status acm_cnn_adam(int64_t n, float* p, const float* g, float* m, float* v, void* p16, float lr, float b1,
                        float b2, float eps, int64_t t, void* stream);

acm_status acm_cnn_to_bf16(size_t n, const float* src, void* dst, void* stream);

/* Coarse (I, J) = mean of fine nodes (fI..fI+f-1, fJ..fJ+f-1) for drho, u, v. */
acm_status acm_filter_box(int32_t nxf, int32_t nyf, int32_t factor, int32_t precision, const acm_fields* fine,
                          const acm_fields* coarse, void* stream);

/* Periodic bilinear interpolation coarse -> fine (coarse node I at fine
 * coordinate f I + (f-1)/2); used to continue on the fine grid. */
acm_status acm_prolong_bilinear(int32_t nxc, int32_t nyc, int32_t factor, int32_t precision,
                                const acm_fields* coarse, const acm_fields* fine, void* stream);

/* Whole-network inference in one launch:
 *   out[c] = in[c] + out_scale[c] * f(in_scale * in)[c],  c = drho, u, v,
 * f the five layers above with the same bf16 rounding of every activation
 * (only the order of the FP32 sums differs from acm_cnn_conv); a channel
 * with out_scale[c] == 0 is copied unchanged.  Each 16x16
 * tile evaluates layer l on the tile grown by 4 - l nodes, entirely in LDS.
 * weights/biases: ACM_CNN_LAYERS device pointers (bf16 [9][C_out][C_in] /
 * fp32).  Needs nx, ny multiples of 16; in and out fields must be distinct
 * (ACM_EINVAL otherwise). */
acm_status acm_cnn_correct(int32_t nx, int32_t ny, const acm_fields* in, const acm_fields* out,
                           const void* const* weights, const float* const* biases, const float* in_scale,
                           const float* out_scale, void* stream);

/* Closure inference: every coarse step is the SMAME step followed by the
 * network correction into the other buffer set, captured in HIP graphs of
 * `chunk` steps (even; 0 = 100).  On fully periodic grids both run in one
 * launch (the correction kernel performs the step on its tiles); otherwise
 * the step writes the workspace and acm_cnn_correct follows.  weights/biases
 * as for acm_cnn_correct.  workspace: acm_closure_workspace bytes of device
 * memory (the uncorrected state).  Grids need nx, ny multiples of 16. */
typedef struct acm_closure acm_closure;
size_t acm_closure_workspace(int32_t nx, int32_t ny);
acm_status acm_closure_init(const acm_config* cfg, const acm_fields* a, const acm_fields* b, const void* force_x,
                            const void* const* weights, const float* const* biases, const float* in_scale,
                            const float* out_scale, void* workspace, int32_t chunk, void* stream,
                            acm_closure** out);
/* 0: plain coarse steps (the network is skipped), 1: corrected steps,
 * 2: corrected steps with the SMAME step always launched on its own
 * (identical results; for checking and timing).  Other values: ACM_EINVAL. */
acm_status acm_closure_set_network(acm_closure* h, int32_t enabled);
acm_status acm_closure_run(acm_closure* h, int64_t nsteps);
acm_status acm_closure_current(const acm_closure* h, int32_t* which, int64_t* step);
void acm_closure_destroy(acm_closure* h);

/* Plain device-to-device copy of `bytes` bytes (both pointers 16-byte
 * aligned), asynchronous on `stream`.  Used to measure the practical copy
 * bandwidth that the stencil kernels are compared with, and to calibrate
 * hardware byte counters.  Returns ACM_EINVAL for NULL or misaligned
 * pointers. */
acm_status acm_stream_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Library version string. */
const char* acm_version(void);

#ifdef __cplusplus
}
#endif
#endif
