/*
 * ugks.h - C ABI of the MI355X (gfx950) UGKS phase-space step.
 *
 * The library advances the discrete-velocity BGK-Shakhov model with the
 * unified gas-kinetic scheme on an unstructured mesh held by one GPU: the
 * sweep over all discrete velocities of microscopic least-squares
 * reconstruction, time-integrated interface flux (equilibrium part plus
 * upwind free-transport part), velocity-moment reduction to the conservative
 * variables, and the two-stage trapezoidal collision update (paper Sec. 2.1,
 * Eqs. fv_micro_update ... f_final; one step = the one-step algorithm of
 * Sec. 2.2 with a single physical subdomain that owns every velocity block).
 *
 * Conventions shared by every call
 *   - Every call returns an int status: UGKS_OK (0) or a negative UGKS_E*
 *     code.  No C++ exception crosses this boundary.  After a failure,
 *     ugks_last_error() on the same context (or with NULL for failures of
 *     ugks_create) returns a human-readable reason.
 *   - Host arrays passed in are read during the call and copied; the caller
 *     keeps ownership.  Output buffers belong to the caller.  A pointer
 *     documented "on_device" is a device address in the library's current
 *     HIP device (for example a PyTorch CUDA tensor's data_ptr()).
 *   - All device memory is allocated by ugks_create / ugks_batch_create and
 *     freed by ugks_destroy / ugks_batch_destroy.
 *   - A context is used by one host thread at a time.  The library keeps no
 *     global mutable state; calls on different contexts are independent.
 *   - Units are the caller's; the workloads of this project use rho0 = 1,
 *     T0 = 1, length 1, speed sqrt(2 R T0) (so R = 1/2).
 *   - A gas has K >= 0 internal degrees of freedom; K_xi = K + 3 - D
 *     (Eq. Kxi_def).  For a monatomic gas in 3-D, K_xi = 0 and b = B = B+ = 0,
 *     so only h is stored; otherwise h and b are.  For K > 0 the Shakhov
 *     correction of Eq. shakhov_fp takes (2 lambda (c^2 + xi^2) - (K + 5)) and
 *     the factor 4 (1 - Pr) lambda^2 / ((K + 5) rho), which conserve momentum
 *     and give the heat flux (1 - Pr) q; reduced, H+ = A c.q (2 lambda c^2 -
 *     D - 2) H and B+ = A c.q (K_xi / 2 lambda)(2 lambda c^2 - D) H (for K = 0
 *     these are Eqs. H_plus, B_plus; the printed B_plus holds for K = 0 only).
 */
#ifndef UGKS_H
#define UGKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------- */
#define UGKS_OK 0
#define UGKS_EINVAL (-1)        /* invalid argument, mesh or velocity set   */
#define UGKS_ENOMEM (-2)        /* device allocation failed                  */
#define UGKS_EHIP (-3)          /* a HIP runtime call failed                 */
#define UGKS_ENUMERIC (-4)      /* non-positive density or temperature      */
#define UGKS_EUNSUPPORTED (-5)  /* valid request outside the built features */

/* ---- boundary kinds (ugks_mesh.face_bc, ugks_bc.kind) ------------------ */
#define UGKS_BC_INTERIOR 0 /* two cells; periodic faces are interior + shift */
#define UGKS_BC_WALL 1     /* diffuse Maxwell wall (Eqs. wall_bc .. wall_density_condition) */
#define UGKS_BC_FARFIELD 2 /* ghost cell: W_inf when U_inf.n < 0, else the interior state */
#define UGKS_BC_OUTFLOW 3  /* ghost cell: the interior state */

/* ---- precision forms (ugks_options.precision) -------------------------- */
/* most rows one ugks_mlp_forward_noalloc call takes (its static staging array) */
#define UGKS_NOALLOC_MAX_ROWS 65536

#define UGKS_FP64 64 /* h, b, their gradients and fluxes in FP64 */
#define UGKS_FP32 32 /* h, b stored and fluxed in FP32; moments, the
                        macroscopic update and the interface equilibrium in FP64 */

typedef struct ugks_ctx ugks_ctx;

/*
 * Unstructured mesh as a face list (Sec. 2.1: control volumes Omega_i,
 * interfaces S_ij with unit normal n_ij, neighbour sets N(i)).
 *   cell_volume[n_cells]            |Omega_i| > 0
 *   cell_centroid[n_cells*dim]      row-major (x, y[, z]) per cell
 *   face_cells[2*n_faces]           (L, R) per face; R = -1 on a physical boundary
 *   face_area[n_faces]              S_ij > 0
 *   face_normal[n_faces*dim]        unit normal pointing from L to R (outward on boundaries)
 *   face_centroid[n_faces*dim]      face centroid as seen from L
 *   face_shift[n_faces*dim] or NULL periodic translation: R's image is centroid[R] + shift
 *   face_bc[n_faces]                UGKS_BC_* kind (INTERIOR for periodic faces)
 *   face_bc_id[n_faces]             row of the ugks_bc table for boundary faces
 * Every cell must be closed (sum_j sigma_ij S_j n_j = 0) and have at most 8
 * faces.  Validation failures return UGKS_EINVAL.
 */
typedef struct {
  int32_t dim; /* 2 or 3 */
  int64_t n_cells, n_faces;
  const double* cell_volume;
  const double* cell_centroid;
  const int64_t* face_cells;
  const double* face_area;
  const double* face_normal;
  const double* face_centroid;
  const double* face_shift;
  const int32_t* face_bc;
  const int32_t* face_bc_id;
} ugks_mesh;

/*
 * Discrete velocity set {u_k, omega_k} (Eqs. velocity_quadrature, omega_k):
 *   u[nv*dim] row-major points, w[nv] ordinary quadrature weights (> 0).
 * The library pads the set to a multiple of its velocity block with
 * zero-weight points (Eq. padded_velocity_number), which leaves every moment
 * unchanged.
 */
typedef struct {
  int64_t nv;
  const double* u;
  const double* w;
} ugks_velocity;

/*
 * Gas model (Eqs. bgk_shakhov, shakhov_fp, lambda_def):
 *   K internal degrees of freedom (>= 0; 0 = monatomic), Pr Prandtl number, R gas
 *   constant, mu = mu_ref (T / T_ref)^omega, tau = mu / p.
 *   dt > 0 fixes the time step; dt = 0 takes
 *     dt = cfl * min_i 2 |Omega_i| / max_k sum_{j in faces(i)} S_j |u_k . n_j|.
 */
typedef struct {
  int32_t K;
  double Pr, R, T_ref, mu_ref, omega;
  double cfl, dt;
} ugks_gas;

/*
 * One boundary-table row.  Walls use T (wall temperature) and U (wall
 * velocity; must be tangential, U . n = 0).  Far field uses rho, U, T of
 * the free stream.  Outflow uses nothing.
 */
typedef struct {
  int32_t kind;
  double rho;
  double U[3];
  double T;
} ugks_bc;

/*
 * Options.
 *   precision  UGKS_FP64 (default when 0) or UGKS_FP32.
 *   block_v    velocity-block size B_v of the fused sweep: velocities per
 *              work item (a multiple of 64; 0 = 4096), the
 *              paper's B_v (Eq. velocity_block_partition) as a scheduling unit.
 *   tile_cells cells per tile of the fused sweep's schedule (0 = 32); each
 *              XCD runs one tile through one velocity block at a time.
 *   flags      bit 0: skip the density residual (saves one small reduction).
 *              bit 1: use the staged sweep even where the fused one applies.
 *              bit 2: keep the caller's cell order internally (by default
 *                     cells are renumbered along a Z-order curve of their
 *                     centroids; inputs and outputs always use the caller's order).
 *              bit 4: first-order reconstruction: every least-squares gradient
 *                     (Sec. 2.2 steps 4 and 5) is zero, so each face sees the
 *                     piecewise-constant states of its two cells; robust where
 *                     unlimited second-order slopes overshoot (strong shocks).
 *              bit 6: track the boundary flux (ugks_boundary_flux).
 *              bit 7: local time steps for steady problems (steady-state
 *                     acceleration, which the paper's conclusion names as
 *                     future work; this library's reading): cell i advances
 *                     by dt_i = dt b_i / min_j b_j, b_i = 2 V_i / max_k sum_j
 *                     S_j |u_k . n_j| its own bound (the most restrictive cell
 *                     keeps dt).  Every face still integrates its fluxes
 *                     (Eqs. micro_flux, macro_flux) over the global dt; cell i
 *                     applies them scaled by dt_i / dt and relaxes (Eqs.
 *                     f_tilde, f_final) over dt_i.  Not time-accurate, but a
 *                     steady state of the global step is one of this step
 *                     and vice versa.  Excludes bit 6 (UGKS_EINVAL); the
 *                     batched form refuses it (UGKS_EUNSUPPORTED).  ugks_info's
 *                     dt stays the global dt.
 *              bit 5: replay each step from a HIP graph of its kernels
 *                     (captured at the first step that can use it; not on the
 *                     null stream, nor while profiling).  Same results as
 *                     kernel-by-kernel launches.
 *   The fused sweep (one pass for reconstruction, interface flux, moment
 *   sums and the first stage) applies when every velocity point lies on the
 *   tensor product of one 1-D node set symmetric about zero of at most 64
 *   nodes (the full product listed with the first axis slowest, or any
 *   subset of it, such as a locally refined set whose levels are lattices;
 *   a point whose mirror is absent is paired with a weight-0 pad slot), and
 *   every cell has at most 4 faces (far-field and outflow faces read
 *   per-step ghost rows holding the ghost Maxwellian).  Otherwise
 *   the staged sweep keeps the microscopic gradients and fluxes of the whole
 *   velocity space in device memory.
 *   stream     hipStream_t to enqueue on, or NULL for a library-owned stream.
 *              A caller stream is borrowed, never destroyed.
 *   limiter    1 limits every least-squares gradient the step reconstructs
 *              with (Sec. 2.1, Eq. initial_reconstruction; each conservative
 *              component of W and each (cell, velocity) of h and b) by
 *              Venkatakrishnan's smooth limiter (J. Comput. Phys. 118, 1995):
 *              with v_max, v_min over the cell and its stencil values, at each
 *              face d- = g.(x_f - x_i), d+ = v_max - v_i (d- > 0) or
 *              v_min - v_i (d- < 0), psi = (d+^2 + eps^2 + 2 d- d+) /
 *              (d+^2 + 2 d-^2 + d- d+ + eps^2), and g is scaled by
 *              min(1, min_faces psi), on either sweep.  limiter_k sets eps
 *              (0: strictly within the stencil bounds).  UGKS_EINVAL for another limiter or a negative or
 *              non-finite K; the batched form refuses it (UGKS_EUNSUPPORTED).
 */
typedef struct {
  int32_t precision;
  int32_t block_v;
  int32_t flags;
  int32_t tile_cells;
  void* stream;
  int32_t limiter;   /* 0: none; 1: Venkatakrishnan's limiter (see below) */
  double limiter_k;  /* its constant K >= 0: eps^2 = (K V_i^(1/D))^3 */
} ugks_options;

/* Read-only facts about a context. */
typedef struct {
  int32_t dim, n_r;          /* n_r = 2 in 2-D (h and b), 1 in 3-D (h only) */
  int32_t precision, block_v;
  int64_t n_cells, n_faces, nv, nv_padded;
  double dt;
  int64_t steps_done;
  int64_t device_bytes;      /* device memory held by the context */
  int32_t fused;             /* 1: the fused sweep runs; 0: the staged sweep */
  int32_t tile_cells;        /* fused sweep: cells per tile */
} ugks_info_t;

/*
 * ugks_create - build a context for one mesh, velocity set and gas, with the
 * initial state h = H(W0), b = B(W0) (Eqs. H_def, B_def).
 *   bcs[n_bc]   boundary table indexed by mesh.face_bc_id
 *   W0[n_cells*(dim+2)]  conservative variables (rho, rho U, rho E) per cell
 *   opt         may be NULL (all defaults)
 *   out         receives the new context; unchanged on failure
 * Errors: UGKS_EINVAL (bad mesh, velocity set, table or state),
 *         UGKS_ENOMEM, UGKS_EHIP.
 */
int ugks_create(const ugks_mesh* mesh, const ugks_velocity* vel, const ugks_gas* gas,
                const ugks_bc* bcs, int32_t n_bc, const double* W0, const ugks_options* opt,
                ugks_ctx** out);

/*
 * ugks_step - advance n_steps >= 0 time steps (the one-step algorithm of
 * Sec. 2.2): heat flux, macroscopic reconstruction, interface equilibrium,
 * wall densities, the velocity sweep (microscopic reconstruction, interface
 * flux, moment reduction, first stage, Eq. f_tilde), the conservative update
 * (Eq. macro_update) and the second stage (Eq. f_final).
 *   residual_out  NULL, or two doubles receiving, for the last step, the
 *                 density residual ||rho^n - rho^{n-1}||_{2,V} normalised by
 *                 the first non-zero such change, and the same change
 *                 normalised by ||rho^{n-1}||_{2,V}.
 * The work is enqueued on the context's stream; the call returns after the
 * stream has completed (it synchronises once per call, not per step).
 * Errors: UGKS_ENUMERIC (a cell or face density or temperature became
 * non-positive: the state is left at the last completed step),
 * UGKS_EHIP, UGKS_EINVAL (n_steps < 0).
 */
int ugks_step(ugks_ctx* ctx, int32_t n_steps, double* residual_out);

/*
 * ugks_moments - macroscopic output (Eq. macro_W).
 *   which = 0: the conservative state W (the master state), n_cells*(dim+2)
 *   which = 1: the discrete moments sum_k omega_k psi_k (h, b), n_cells*(dim+2)
 *   which = 2: the heat flux q of the current distributions (Eq.
 *              reduced_heat_flux), n_cells*dim
 *   out           caller buffer in the caller's cell order
 *   out_on_device 0: host pointer; 1: device pointer
 */
int ugks_moments(ugks_ctx* ctx, int32_t which, double* out, int32_t out_on_device);

/*
 * ugks_boundary_flux - the boundary flux accumulated over the steps since
 * create (or the last ugks_set_state), for balance checks (Eq. macro_update
 * summed over the cells: sum_i V_i W_i^n - sum_i V_i W_i^0 + A = 0 up to
 * rounding, A = sum over steps and boundary faces of S_f F_f, F_f the face's
 * time-integrated flux of mass, momentum and energy, Eq. macro_flux).
 * Needs options.flags bit 6 (boundary-flux tracking) at create: the wall
 * pass then also keeps each wall face's flux (fused sweep) or the staged
 * sweep's face fluxes are summed, one small reduction per step.
 * out: host, dim+2 doubles, written.  complete: optional host int32, set to
 * 1 if A covers every boundary face, 0 on the fused sweep with far-field or
 * outflow faces (there only the wall faces are summed).
 * Errors: UGKS_EINVAL (null context or out, tracking off), UGKS_EHIP.
 */
int ugks_boundary_flux(ugks_ctx* ctx, double* out, int32_t* complete);

/*
 * ugks_get_state / ugks_set_state - checkpoint, restart and warm start.
 *   W[n_cells*(dim+2)], h[n_cells*nv], b[n_cells*nv] in the caller's cell
 *   order and the caller's velocity order (padding excluded), FP64 on the
 *   host.  Any of the three may be NULL (b is ignored in 3-D).  set_state
 *   rounds h, b to FP32 in the FP32 form.
 */
int ugks_get_state(ugks_ctx* ctx, double* W, double* h, double* b);
int ugks_set_state(ugks_ctx* ctx, const double* W, const double* h, const double* b);

/*
 * ugks_face_data - diagnostics of the last step, caller face order:
 *   F[n_faces*(dim+2)] macroscopic time-integrated face fluxes (Eq. macro_flux)
 *   rho_w[n_faces]     wall densities (Eq. wall_density_condition), 0 off walls
 * Either pointer may be NULL.  Host buffers.
 */
int ugks_face_data(ugks_ctx* ctx, double* F, double* rho_w);

int ugks_info(const ugks_ctx* ctx, ugks_info_t* out);

/*
 * Kernel timing with HIP events recorded on the context's stream around
 * every kernel a step enqueues (measurement support, not part of the method).
 *   ugks_profile_enable(ctx, 1) starts recording, 0 stops; either call
 *     discards what was recorded.
 *   ugks_profile_read fills out[0..max-1] with one row per kernel kind
 *     (launch count, summed duration) and sets *n_out to the number of kinds;
 *     it synchronises the stream.  Recording costs two event records per launch.
 */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
} ugks_kernel_time;

int ugks_profile_enable(ugks_ctx* ctx, int32_t on);
int ugks_profile_read(ugks_ctx* ctx, ugks_kernel_time* out, int32_t max, int32_t* n_out);

/* Releases every device buffer; accepts NULL. */
void ugks_destroy(ugks_ctx* ctx);

/*
 * Batched form: many independent cases (each its own mesh, velocity set, gas
 * and boundary table, one dimension and one precision for all) advanced
 * together, one launch per phase of the step for the whole batch.  Scheduling
 * follows the paper's velocity-block work decomposition (Eq.
 * velocity_block_partition, Sec. 3): the velocity sweep is one persistent
 * launch walking a list of (case, cell, velocity block) work items, the
 * other phases flatten the cells, faces or wall faces of every case behind
 * case-offset tables, and the whole step is captured once into a HIP graph
 * and replayed.  Every case must qualify for the fused sweep (a tensor
 * product of one symmetric 1-D node set; any face kinds;
 * at most four faces per cell).
 *
 * The velocity-block size and the cell-tile size of each case, and the
 * lanes per work-group of the sweep, are chosen by an autotuner that times
 * the sweep on the device at create (options.block_v = 0 and tile_cells = 0)
 * unless the process-wide tuning cache already holds the case's shape; a
 * nonzero block_v / tile_cells fixes them for every case instead.
 * options.flags bit 3 runs the step eagerly (no graph); the other bits act
 * as for ugks_create.  options.stream as for ugks_create.
 */
typedef struct ugks_batch ugks_batch;

typedef struct {
  const ugks_mesh* mesh;
  const ugks_velocity* vel;
  const ugks_gas* gas;
  const ugks_bc* bcs;
  int32_t n_bc;
  const double* W0;          /* [n_cells*(dim+2)] */
} ugks_case;

typedef struct {
  int32_t n_cases;
  int32_t dim;
  int32_t precision;
  int32_t threads;           /* lanes per work-group of the batched sweep */
  int64_t work_items;        /* (case, cell, velocity block) items of one sweep */
  int64_t grid;              /* persistent work-groups of the sweep */
  int32_t graph;             /* 1: steps replay a captured HIP graph */
  int32_t tuned;             /* 1: schedule from the autotuner (timed or cached) */
  int64_t tune_timings;      /* sweep launches the autotuner timed at create (0 on a cache hit) */
  int64_t steps_done;
} ugks_batch_info_t;

/*
 * ugks_batch_create - cases[0..n_cases-1] are copied; the caller keeps its
 * arrays.  Errors: UGKS_EINVAL (any case invalid, mixed dim, n_cases < 1),
 * UGKS_EUNSUPPORTED (a case does not qualify for the fused sweep, or its gas
 * has K > 0; options with the limiter or local time steps), UGKS_ENOMEM,
 * UGKS_EHIP.  The failing case is named in ugks_batch_last_error(NULL).
 */
int ugks_batch_create(const ugks_case* cases, int32_t n_cases, const ugks_options* opt,
                      ugks_batch** out);

/*
 * ugks_batch_step - advance every case n_steps >= 0 steps.  residual_out is
 * NULL or 2*n_cases doubles: per case the two residuals of ugks_step.  On a
 * non-positive density or temperature in any case: UGKS_ENUMERIC, with the
 * failing case named in ugks_batch_last_error.
 */
int ugks_batch_step(ugks_batch* batch, int32_t n_steps, double* residual_out);

/* Per-case access, as ugks_moments / ugks_get_state / ugks_info for case i. */
int ugks_batch_moments(ugks_batch* batch, int32_t i, int32_t which, double* out, int32_t on_device);
int ugks_batch_get_state(ugks_batch* batch, int32_t i, double* W, double* h, double* b);
int ugks_batch_case_info(ugks_batch* batch, int32_t i, ugks_info_t* out);
int ugks_batch_info(const ugks_batch* batch, ugks_batch_info_t* out);
void ugks_batch_destroy(ugks_batch* batch);
const char* ugks_batch_last_error(const ugks_batch* batch);

/*
 * Process-wide autotuner cache (thread-safe).  Entries are keyed by the
 * case shape (dim, precision, lanes, cells, velocities) and by the batch's
 * list of shapes.  save writes a plain text file; load merges a file written
 * by save (UGKS_EINVAL on a malformed file, nothing merged); clear empties it.
 */
int ugks_autotune_save(const char* path);
int ugks_autotune_load(const char* path);
void ugks_autotune_clear(void);

/*
 * Learned warm start.  A 9-64-64-9 tanh network maps per-cell features of
 * the macroscopic state to the nonequilibrium stress and heat flux, and the
 * initial f of a cell is Grad's 13-moment form about the Maxwellian of W
 * built from them; this is a Chapman-Enskog-type closure of the BGK-Shakhov
 * model of Sec. 2.1 learned from the method's own solutions, used to start
 * the steady-state iteration of Sec. 2.2 closer to its answer.
 *
 * Features (9, dimensionless, from W, its least-squares gradient as in the
 * macroscopic reconstruction, and tau = mu/p):
 *   tau S_xx, tau S_yy, tau S_xy, tau S_xz, tau S_yz   (S: traceless strain rate)
 *   L dT/dx / T, L dT/dy / T, L dT/dz / T               (L = tau sqrt(2RT))
 *   L |grad rho| / rho                                  (local Knudsen number)
 * Targets / outputs (9): sigma/p for xx yy zz xy xz yz (sigma_ab = int c_a c_b f
 * - p d_ab; in 2-D the zz entry comes from b) and q/(p sqrt(2RT)) for x y z
 * (Eq. reduced_heat_flux).  Rows of 9 floats, one row per cell or sample.
 *
 * The network: y = out_scale * N(in_scale * x), tanh hidden layers, linear
 * output; parameters as 5385 floats W1[64][9] b1[64] W2[64][64] b2[64]
 * W3[9][64] b3[9] (rows are output units).  Inference rounds weights and
 * layer inputs to bfloat16 and accumulates in FP32 on the matrix cores;
 * training is FP32 (forward, backward, Adam with beta = 0.9, 0.999,
 * eps = 1e-8) on the mean over samples of sum_j (N_j - t_j/out_scale_j)^2.
 *
 * Ownership as for contexts: the network copies its inputs and owns its
 * device memory; `stream` is borrowed (NULL: the network makes its own).
 * on_device = 1: x, t, y are device pointers (e.g. a tensor's data_ptr()).
 */
typedef struct ugks_mlp ugks_mlp;

int ugks_mlp_create(const float* params, const float* in_scale, const float* out_scale,
                    void* stream, ugks_mlp** out);
/* FP32 parameters, 5385 floats, to host memory */
int ugks_mlp_get_params(ugks_mlp* net, float* params);
/* training box: a cell whose features leave [lo, hi] (9 each) keeps the Maxwellian */
int ugks_mlp_set_box(ugks_mlp* net, const float* lo, const float* hi);
/* y[rows*9] = network(x[rows*9]) in physical units (bf16 matrix-core inference) */
int ugks_mlp_forward(ugks_mlp* net, const float* x, int64_t rows, float* y, int32_t on_device);
/*
 * ugks_mlp_forward_noalloc - the inference of ugks_mlp_forward for callers
 * that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc).
 *
 * x: device pointer, rows x 9 floats (row-major features); y: device
 * pointer, rows x 9 floats (outputs, physical units), written.  The caller
 * owns both.  The call only enqueues work on the network's stream and
 * returns: y is ready once that stream has reached this point.  It allocates
 * nothing: its staging rows live in a static device array of
 * UGKS_NOALLOC_MAX_ROWS rows (8 MiB per GPU, held until the process ends),
 * looked up once per device.  Every call on one GPU shares that array, so
 * calls that overlap on one GPU (other streams, other threads) race; calls
 * ordered on one stream do not.  Nothing in the array has to start at zero.
 * The network's device must be current.
 * Errors: UGKS_EINVAL for rows < 0 or rows > UGKS_NOALLOC_MAX_ROWS, null
 * pointers, or another current device (nothing is enqueued); UGKS_EHIP if a
 * launch fails.
 */
int ugks_mlp_forward_noalloc(ugks_mlp* net, const float* x, int64_t rows, float* y);
/* loss and its gradient (5385 floats, host) over all rows; the parameters are unchanged */
int ugks_mlp_loss_grad(ugks_mlp* net, const float* x, const float* t, int64_t rows, float* grad,
                       double* loss, int32_t on_device);
/* `steps` Adam steps over consecutive slices of `batch` rows (wrapping to the
 * start when a slice would run past the end); loss_out NULL or steps doubles */
int ugks_mlp_train(ugks_mlp* net, const float* x, const float* t, int64_t rows, int64_t batch,
                   int32_t steps, float lr, int32_t on_device, double* loss_out);
void ugks_mlp_destroy(ugks_mlp* net);
const char* ugks_mlp_last_error(const ugks_mlp* net);

/*
 * ugks_snapshot - features and targets of every cell of the current state
 * (host arrays of n_cells*9 floats, caller's cell order; either may be NULL).
 * Monatomic gases only (K > 0: UGKS_EUNSUPPORTED), as ugks_warm_start.
 */
int ugks_snapshot(ugks_ctx* ctx, float* features, float* targets);

/*
 * ugks_warm_start - optionally set W (caller order, as ugks_set_state), then
 * replace h and b of every cell by the Grad-type distribution from the
 * network's prediction for its features, or by the Maxwellian of W where the
 * features leave the training box.  *n_fallback (may be NULL) receives the
 * number of Maxwellian cells.  The residual normalisation restarts.  The
 * closure is defined for monatomic gases: K > 0 returns UGKS_EUNSUPPORTED.
 */
int ugks_warm_start(ugks_ctx* ctx, const ugks_mlp* net, const double* W, int64_t* n_fallback);

/* Reason for the last failure on ctx (NULL: the last failed ugks_create of this thread). */
const char* ugks_last_error(const ugks_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* UGKS_H */
