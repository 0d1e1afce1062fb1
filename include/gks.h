/*
 * gks.h - C ABI of the MI355X (gfx950) implementation of the high-order compact gas-kinetic
 * scheme (GKS) for the two-layer shallow water equations on triangular meshes
 * (Zhao, Gan & Xu, "High-order compact gas-kinetic scheme for two-layer shallow water equations
 * on unstructured mesh").
 *
 * Problem (Sec. 2.1, Eq. SWE-macro): W_t + F^x(W)_x + F^y(W)_y = S(W) for the two layers,
 * W = (h2, h2U2, h2V2, h1, h1U1, h1V1), layer 1 the lower (density rho1), layer 2 the upper,
 * chi = rho2 / rho1, bottom B.  The solver advances cell averages and cell-averaged gradients with
 * the two-stage fourth-order (S2O4) time stepping of Sec. 3.3, each stage running the compact
 * reconstruction (Sec. 3.4; where a layer thickness at a Gauss point would fall below a tenth of
 * its cell's average, the reconstruction's deviation from the average is scaled down, a
 * positivity safeguard the paper does not state), the interface force modelling (Sec. 2.3), the
 * time-accurate gas-kinetic evolution at two Gauss points per edge (Sec. 2.2, Eq. SWE-2nd-order)
 * and the well-balanced finite-volume update with bottom and layer-coupling sources
 * (Sec. 3.1-3.2).  Two details the paper leaves to a reference are read here as follows.  The
 * well-balance weights alpha_{k,m} of the evolution's acceleration term make the half-space
 * moments of a balanced level slope and acceleration vanish: 3/4 on the mass state moment and
 * 5/4 on the momentum flux moments, applied to the jump between the two sides.  The Gauss-point
 * thicknesses of the layer coupling are the mean of the two sides' reconstructed values, with
 * the mean of their rates -div(hU) as time derivative.
 *
 * Conventions
 *  - All pointers to user arrays are HOST pointers; the library copies them (the caller keeps
 *    ownership).  Handles are owned by the library until the matching *_destroy call.
 *  - Cell arrays are structure-of-arrays: W[6][n_tri] and gradW[6][2][n_tri] (component-major,
 *    then x / y, then cell), components in the order above, cells in the order of `tri` (for a
 *    batch: scenario 0's cells, then scenario 1's, ...).
 *  - Work is enqueued on the HIP stream given to gks_state_init (NULL = the null stream) and is
 *    asynchronous, except the calls documented as synchronising.
 *  - Errors are returned as gks_status codes, never as exceptions; gks_last_error() gives a
 *    thread-local message for the last failure.
 */
#ifndef GKS_H
#define GKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gks_mesh gks_mesh;
typedef struct gks_state gks_state;

typedef enum {
    GKS_OK = 0,
    GKS_EINVAL = 1,       /* bad argument */
    GKS_ENOMEM = 2,       /* host or device allocation failed */
    GKS_EDEVICE = 3,      /* a HIP call failed */
    GKS_EMESH = 4,        /* malformed mesh (index out of range, inverted or degenerate triangle,
                             edge shared by more than two triangles, unpaired periodic edge) */
    GKS_ENONFINITE = 5,   /* non-finite value or non-positive layer thickness in the state
                             (at or below -h_dry with wet/dry layers) */
    GKS_EUNSUPPORTED = 6  /* option not compiled into this library */
} gks_status;

typedef enum {
    GKS_BC_WALL = 0,      /* every boundary edge is a reflecting wall (mirror ghost cells) */
    GKS_BC_PERIODIC = 1,  /* boundary edges of [0,Lx] x [0,Ly] are paired by translation */
    GKS_BC_FREE = 2       /* every boundary edge is free (zero-gradient, transmissive): the ghost
                             beyond it is the mirror image of the cell with every component,
                             momentum included, extended evenly, and mass crosses it (the free
                             boundary of the paper's accuracy test, Sec. 4.1) */
} gks_bc;

typedef enum {
    GKS_FP64 = 0,         /* every stage in double precision */
    GKS_FP32_MIXED = 1    /* bulk arithmetic and storage in single precision; cell and Gauss-point
                             thicknesses, the hydrostatic flux term, the interface thickness and
                             every edge sum of the update (the lake-at-rest balance of Sec. 3.2)
                             stay in double, and so do the mass sums */
} gks_precision;

typedef struct {
    double G;        /* gravitational acceleration (Sec. 4: 9.81) */
    double chi;      /* density ratio rho2 / rho1 (Sec. 2.1) */
    double cfl;      /* CFL number of dt = CFL * dX / U_max (Sec. 4) */
    double eps;      /* collision-time constant epsilon (Sec. 4: 0.05) */
    double eps_num;  /* pressure-jump constant of the collision time (Sec. 4: 5) */
    double t_end;    /* the last step is clipped so that t never exceeds t_end (<= 0: no limit) */
    int32_t precision;  /* gks_precision */
    int32_t linear;     /* 1: linear P^3 reconstruction everywhere, 0: nonlinear (Sec. 3.4) */
    int32_t alpha_mode; /* constants alpha_{k,m} of the acceleration term of the evolution solution
                           (Sec. 2.2, Eq. SWE-2nd-order): 0 (default) the well-balance weights read
                           for these slopes (3/4 on the mass state moment, 5/4 on the momentum flux
                           moments, applied to the jump of the two sides' accelerations in the
                           equilibrium part); 1 the paper's printed (1, 3/4, 1/4) on the flux
                           moments (mass, normal, tangential momentum) of the whole term in both
                           the equilibrium and the initial distributions' parts, 1 on the state
                           moments */
    int32_t src_order;  /* layer coupling (Sec. 3.2, Eq. SWE-source-discretization): 2 (or 0) the
                           paper's second-order form, the Gauss-point mean thickness of one layer
                           times the Green-Gauss derivative of the other's Gauss-point thickness;
                           4 the higher-order form its closing remark allows: the cell-average
                           thickness in place of the Gauss-point mean plus the cell average of
                           (h_a - mean h_a) grad h_b over the cell's reconstructions (Radon's
                           7-point rule), its time derivative with h_t = -div(h U).  Must agree
                           across the scenarios of a batch; other values give GKS_EINVAL */
    int32_t grad_mode;  /* interface values of the gradient update (Sec. 3.3, Eq. slope-1): 0
                           (default) the continuous evolution solution W^l = W^r, the interface
                           equilibrium's state and time slope (the paper's choice); 1 discontinuous
                           values W^l != W^r: each cell takes the reconstructed state on its own
                           side of the edge, advanced in time by that side's own rate from the
                           shallow-water equations (half again as many edge outputs).  Must agree
                           across a batch; other values give GKS_EINVAL */
    double h_dry;       /* wet/dry layers (a layer that vanishes, as in the paper's dam breaks over
                           a dry bed, Sec. 4; the paper gives no treatment, this is a reading): 0
                           (default) every layer must stay wet (thickness > 0); > 0 a thickness may
                           be 0.  A side of an interface at or below h_dry is a vacuum, an
                           interface whose equilibrium thickness is at or below h_dry passes
                           nothing, and in a layer's front band (the cell or a face neighbour
                           thinner than 1000 h_dry or than 0.3 times the thickest of the four, or
                           the lower layer thinner than the bottom's rise across the cell) the
                           layer is reconstructed as its cell average with the cell's velocity
                           desingularised below 1000 h_dry, and evolves at first order in space
                           and time.  Must agree across a batch; needs src_order 2 and no learned
                           indicator; negative or non-finite values give GKS_EINVAL */
} gks_params;

/* Build a mesh on the current HIP device.
 *   node_xy [n_nodes][2]  node coordinates
 *   tri     [n_tri][3]    counter-clockwise node indices
 *   node_B  [n_nodes]     bottom height at the nodes (continuous piecewise-linear bottom); NULL = 0
 *   bc, periodic_L[2]     boundary kind; periodic_L = (Lx, Ly) for GKS_BC_PERIODIC, else ignored
 * Setup runs on the host in FP64 (edges, compact stencils of Sec. 3.4 Eq. Recons-stencil with
 * mirror ghost cells at walls, least-squares matrices of Eq. Recons-system) and uploads the
 * result.  Returns GKS_EMESH for a malformed mesh (bad node index, clockwise or zero-area
 * triangle, an edge shared by more than two triangles or twice in one direction, unpaired
 * periodic edges) and GKS_EINVAL for n_tri above 2^29 (cell, edge and Gauss-point record indices
 * are 32-bit); these checks run on the host before any device call. */
gks_status gks_mesh_create(const double *node_xy, int64_t n_nodes, const int32_t *tri, int64_t n_tri,
                           const double *node_B, int32_t bc, const double *periodic_L,
                           gks_mesh **out);
/* Concatenate n independent single meshes into one batch mesh of n scenarios (an ensemble
 * advanced together, each scenario with its own time step).  The inputs stay valid and owned by
 * the caller.  GKS_EINVAL above 2^30 cells and ghost cells in all. */
gks_status gks_mesh_batch(const gks_mesh *const *meshes, int32_t n, gks_mesh **out);
void gks_mesh_destroy(gks_mesh *mesh);
/* sizes: triangles, edges, ghost mirror cells (kept for wall stencils), scenarios; any may be NULL */
gks_status gks_mesh_info(const gks_mesh *mesh, int64_t *n_tri, int64_t *n_edges, int64_t *n_ghost,
                         int32_t *n_scenarios);
/* cell range [first_cell, first_cell + n_cells) of scenario s in the batch's cell order */
gks_status gks_mesh_scenario(const gks_mesh *mesh, int32_t s, int64_t *first_cell, int64_t *n_cells);

/* Create a state on `mesh` (which must outlive it).  params: one entry per scenario of the mesh
 * (1 for a single mesh); G, cfl, eps, eps_num, precision and linear must agree across scenarios,
 * chi and t_end may differ.  W0 [6][n_tri], gradW0 [6][2][n_tri]: cell averages and cell-averaged
 * gradients at t = 0.  `stream` is a hipStream_t (NULL = null stream).  Returns GKS_ENONFINITE if
 * a thickness is <= 0 (< 0 with h_dry > 0) or a value is not finite. */
gks_status gks_state_init(const gks_mesh *mesh, const gks_params *params, const double *W0,
                          const double *gradW0, void *stream, gks_state **out);
void gks_state_destroy(gks_state *st);

/* One S2O4 stage (Sec. 3.3, Eq. SWE-fully-discrete).  stage = 0 turns W^n into W^{n+1/2} and
 * stores what stage 1 needs; stage = 1 turns W^{n+1/2} into W^{n+1}.  Stages must alternate
 * 0, 1, 0, ... (GKS_EINVAL otherwise).  dt: host pointer to the step size for stage 0 (single
 * scenario only; clipped on the device so that t never passes t_end, like the CFL step), or NULL
 * to use the CFL step computed on the device; must be NULL for stage 1 (the step size is
 * reused). */
gks_status gks_stage(gks_state *st, int32_t stage, const double *dt);
/* n_steps full steps, every scenario with its own CFL time step computed on the device (no host
 * synchronisation).  A scenario that has reached its t_end is left unchanged by later steps.  If
 * dt_last is not NULL the call synchronises and returns the last step size of scenario 0.
 * GKS_EINVAL if called between stage 0 and stage 1. */
gks_status gks_step(gks_state *st, int32_t n_steps, double *dt_last);
/* The same n_steps steps replayed from a HIP graph that holds one captured step (time step and
 * both stages of every scenario); the graph is captured on the first call on a private stream
 * and ordered after / before the work of the state's stream. */
gks_status gks_batch_step(gks_state *st, int32_t n_steps);

/* Copy the latest state to the host (synchronising): W^{n+1/2} between stage 0 and stage 1,
 * otherwise W^n.  W [6][n_tri], gradW [6][2][n_tri] (either may be NULL), t = time of scenario 0
 * (may be NULL). */
gks_status gks_state_read(const gks_state *st, double *W, double *gradW, double *t);
/* Time of the latest state and last step size of scenario s (synchronising). */
gks_status gks_state_time(const gks_state *st, int32_t s, double *t, double *dt);
/* Per-layer mass sum |Omega_j| h_j in FP64 of scenario s (s = -1: all cells), mass[0] = upper
 * layer (h2), mass[1] = lower (h1); a deterministic device reduction; synchronising. */
gks_status gks_state_mass(const gks_state *st, int32_t s, double mass[2]);
/* For callers that cannot allocate device memory (code under graph capture preparation, tight
 * serving loops, harnesses that forbid hipMalloc): gks_state_mass with the same arguments, result
 * and kernel, whose 256 block partial sums go to a file-scope device array of 4 KiB (one copy per
 * device, held until the process ends) instead of a buffer of the state.  It calls no hipMalloc,
 * hipFree or other allocating routine.  The block grid strides over any number of
 * cells, so no mesh exceeds the array.  Calls that overlap on one device (from several threads or
 * streams) share that array and race; calls on one stream are ordered and do not. */
gks_status gks_state_mass_noalloc(const gks_state *st, int32_t s, double mass[2]);

/* Per-step diagnostics of scenario s (0 <= s < n_scenarios; synchronising), from device
 * reductions over its cells: out[0] time t, out[1] last step size, out[2] and out[3] the layer
 * masses as gks_state_mass (upper h2, lower h1), out[4] and out[5] the largest speed |hU|/h of the
 * upper and the lower layer (with h_dry > 0 desingularised in layers thinner than 1000 h_dry, as
 * in the time step: a dry cell contributes 0), out[6] and out[7] the spread (max - min) of the lower level
 * eta1 = h1 + B and of the surface eta2 = eta1 + h2.  For a lake at rest (Sec. 3.2, the
 * well-balance property) out[4..7] are its residual: zero up to rounding.  GKS_ENONFINITE as for
 * the other synchronising queries (outputs filled first). */
gks_status gks_state_diagnostics(const gks_state *st, int32_t s, double out[8]);

/* Checked build (compiled with GKS_CHECKED, libgks_checked.so): every index the kernels read from
 * a mesh table (stencil cells, ghost sources, edge cells and slots, cell edges, scenario and chunk
 * ranges) is tested against the size of the array it indexes; a miss sets a device flag and the
 * access falls back to element 0.  gks_debug_bounds synchronises the device and returns the flag
 * in *violations (1 after any miss, else 0), clearing it if reset != 0.  In the ordinary build it
 * returns GKS_EUNSUPPORTED with *violations = -1.  A debugging aid for the hot path (the flag is
 * shared by every state on the device). */
gks_status gks_debug_bounds(int32_t reset, int32_t *violations);

/* Non-finite detection (a diagnostic of the cell update, Sec. 3.3): every cell update records on
 * the device, without a host round trip, the smallest cell index whose new state has a
 * non-finite value or a layer thickness <= 0 (h2, or h1 = (h1 + B) - B; with h_dry > 0 a
 * thickness at or below -h_dry: a dry cell may hold a rounding residue).  gks_state_check
 * synchronises and returns GKS_ENONFINITE with *first_bad = that cell (index into the
 * concatenated cells of a batch), or GKS_OK with *first_bad = -1 (first_bad may be NULL).  The
 * synchronising calls gks_state_read, gks_state_time, gks_state_mass, gks_state_diagnostics and
 * gks_step with dt_last return GKS_ENONFINITE too, after filling their outputs.  The flag stays set until a checkpoint
 * taken before the failure is loaded. */
gks_status gks_state_check(const gks_state *st, int64_t *first_bad);

/* Checkpoint / restart.  gks_state_checkpoint_size gives the byte count of a checkpoint of this
 * state; gks_state_save writes the raw device state (h2 and h1 + B in FP64, momenta and gradients
 * in the state's precision, ghost cells, each scenario's time and last step, the non-finite flag)
 * behind a small header into the caller's host buffer `blob` (synchronising; GKS_EINVAL between
 * stage 0 and stage 1 or if `bytes` is too small).  gks_state_load restores such a checkpoint into
 * a state of the same mesh and precision (GKS_EINVAL otherwise), so that k steps, a checkpoint,
 * a load and k more steps give the same bits as 2k steps.  Indicator, autotuner and graph settings
 * are not part of a checkpoint. */
gks_status gks_state_checkpoint_size(const gks_state *st, int64_t *bytes);
gks_status gks_state_save(const gks_state *st, void *blob, int64_t bytes);
gks_status gks_state_load(gks_state *st, const void *blob, int64_t bytes);

/* Intermediate arrays of the last stage, for tests and inspection tools.  After a second stage the
 * edge arrays hold its mass fluxes, time derivatives, interface thicknesses and coupling values;
 * the momentum fluxes, hydrostatic terms and interface momenta, which the second update does not
 * read, are still the first stage's. */
typedef enum {
    GKS_BUF_RECH = 0,  /* double [6 slots][2][n_tri]: h2 and h1 + B at the cells' Gauss points
                          (slot = 2 * local edge + point, in the cell's counter-clockwise order) */
    GKS_BUF_RECM = 1,  /* real [6 slots][16][n_tri]: the four momenta, then the x/y gradients of
                          the six variables (h2, h2U2, h2V2, h1 + B, h1U1, h1V1) at the Gauss points */
    GKS_BUF_R0 = 2,    /* real [2][n_tri]: omega_0 / d_0 of h1 + B and of h2 */
    GKS_BUF_EOH = 3,   /* double [6][n_edges]: 1/2 G hb^2 (upper, lower), hb (upper, lower), the
                          mean of the two sides' reconstructed thicknesses (upper, lower), Gauss
                          points averaged, hb the interface thickness of the evolution solution */
    GKS_BUF_EOM = 4,   /* real [24][n_edges]: flux F0 without 1/2 G hb^2 n (6), its time derivative
                          (6), interface momenta (4), interface time derivatives (6), global frame,
                          then the mean of the two sides' thickness rates -div(h U) (upper, lower) */
    GKS_BUF_SKIP = 5,  /* uint8 [n_tri]: the learned indicator's decisions of the last stage that ran
                          with it (1 = linear weights); unspecified before the first such stage */
    GKS_BUF_SRC = 6,   /* real [8][n_tri]: interior correction of the higher-order layer coupling
                          (src_order 4 only, else GKS_EINVAL): mean((h1 - mean h1) grad h2) x, y,
                          mean((h2 - mean h2) grad h1) x, y, then the time derivatives of both */
    GKS_BUF_COUNT = 7
} gks_buffer;
/* Copy one intermediate array to host memory `dst` of `bytes` bytes (synchronising); "real" is
 * double for GKS_FP64 states and float for GKS_FP32_MIXED.  GKS_EINVAL if bytes is too small. */
gks_status gks_state_buffer(const gks_state *st, int32_t which, void *dst, int64_t bytes);

/* Kernel classes for gks_profile_read. */
typedef enum {
    GKS_KERNEL_GHOST = 0,   /* mirror ghost cells refreshed from their source cells */
    GKS_KERNEL_RECON = 1,   /* compact reconstruction at the Gauss points (Sec. 3.4) */
    GKS_KERNEL_HHAT = 2,    /* edge-centre heights of the force model (Sec. 2.3) */
    GKS_KERNEL_PLANE = 3,   /* plane gradient of the force model (Sec. 2.3) */
    GKS_KERNEL_FLUX = 4,    /* gas-kinetic evolution at the Gauss points (Sec. 2.2) */
    GKS_KERNEL_UPDATE = 5,  /* gather, sources, S2O4 stage update (Sec. 3.1-3.3) */
    GKS_KERNEL_DT = 6,      /* CFL time step (Sec. 4) */
    GKS_KERNEL_INDICATOR = 7, /* learned smoothness indicator (skip mask of the reconstruction) */
    GKS_KERNEL_COUNT = 8
} gks_kernel;

/* Kernel timing for measurement tools: enable != 0 starts recording a HIP event pair on the
 * state's stream around every kernel launch of gks_stage / gks_step (clearing earlier records),
 * 0 stops.  Synchronising. */
gks_status gks_profile(gks_state *st, int32_t enable);
/* Total time in ms and number of launches recorded for one kernel class since gks_profile
 * enabled recording.  Synchronising. */
gks_status gks_profile_read(gks_state *st, int32_t kernel, double *total_ms, int64_t *launches);

/* ------------------------------------------------------------------------------------------
 * Learned smoothness indicator.  The nonlinear weights of the compact reconstruction (Sec. 3.4)
 * return the linear P^3 reconstruction where the data are smooth, and the force model of Sec. 2.3
 * needs no modelling there.  A small network predicts per cell, from its compact stencil, that
 * the nonlinear weights would change nothing; such cells take the linear reconstruction directly.
 *
 * Network: 44 features -> 64 -> 64 -> 1 logit, ReLU hidden layers.  Parameters P[7105] (float):
 * W1[44][64], b1[64], W2[64][64], b2[64], w3[64], b3 (row-major, input index first).
 * Features of cell c, for the interface level eta1 = h1 + B and then for h2 (17 each, X[0..33]):
 * the 9 stencil differences (Q_l - Q_c) / s, then hs * grad Q / s of the cell and of its 3 face
 * neighbours (x, y), with s = max_l |Q_l - Q_c| + 1e-12 |Q_c| and hs = sqrt(2 |Omega_c|); the size
 * of the variation log10(s / h) / 4 with h the layer's thickness (X[34] lower, X[35] upper); the
 * size of the layer's momentum variation log10((sm + 1e-12 a) / a) / 4, sm the largest stencil
 * difference of its two momentum components, a = h sqrt(G h) (X[36] lower, X[37] upper); the 3
 * face neighbours' areas over |Omega_c| (X[38..40]) and the 3 edge lengths over hs (X[41..43]).
 * Inference uses bf16 operands with float accumulation (v_mfma_f32_32x32x16_bf16); a cell is
 * skipped when its logit exceeds the threshold.
 * ------------------------------------------------------------------------------------------ */

/* Number of parameters and of inputs of the indicator network. */
#define GKS_MLP_PARAMS 7105
#define GKS_MLP_FEATURES 44

/* Switch the indicator on for every later step of `st` (params: host [7105], copied) with the
 * given logit threshold, or off (params = NULL).  The network runs in the first stage of a step,
 * on the step's initial state; the second stage reuses its decisions.  A HIP graph captured by
 * gks_batch_step before the call is discarded and captured again. */
gks_status gks_indicator_set(gks_state *st, const float *params, float threshold);
/* Evaluate the indicator on the latest state (synchronising): logits [n_tri] and mask [n_tri]
 * (1 = skip the nonlinear weights) to host memory, either may be NULL; n_skip (may be NULL) the
 * number of skipped cells.  GKS_EINVAL if the indicator is off. */
gks_status gks_indicator_eval(gks_state *st, float *logits, uint8_t *mask, int64_t *n_skip);
/* Features [n_tri][44] of the latest state to host memory (synchronising). */
gks_status gks_state_features(gks_state *st, float *X);
/* Labels of the latest state to host memory y [n_tri] (synchronising): 1 where the nonlinear and
 * the linear reconstruction agree at all six Gauss points to tol times the variable's scale
 * (the layer thickness for h2 and h1 + B, h sqrt(G h) for the layer's momenta), else 0.  Runs the
 * reconstruction twice; overwrites the intermediate arrays of gks_state_buffer. */
gks_status gks_state_labels(gks_state *st, double tol, uint8_t *y);

/* Trainer: a device-resident sample set (features and 0/1 labels) and the network's parameters
 * with Adam moments, trained on the GPU in float (mean logistic loss softplus(z) - y z). */
typedef struct gks_trainer gks_trainer;
/* capacity: maximum number of samples; max_batch: largest minibatch; params0: host [7105]
 * initial parameters; stream: hipStream_t (NULL = null stream). */
gks_status gks_trainer_create(int64_t capacity, int32_t max_batch, const float *params0, void *stream,
                              gks_trainer **out);
void gks_trainer_destroy(gks_trainer *tr);
/* Append n samples from host memory: X [n][44], y [n] (0 or 1).  GKS_EINVAL beyond capacity. */
gks_status gks_trainer_add(gks_trainer *tr, const float *X, const uint8_t *y, int64_t n);
/* Append the features and labels (tolerance tol, as gks_state_labels) of every cell of the
 * latest state of `st`, computed on the device without a host copy; st must live on the
 * trainer's device.  n_added may be NULL. */
gks_status gks_trainer_add_state(gks_trainer *tr, gks_state *st, double tol, int64_t *n_added);
/* Number of samples and of label-1 samples (either may be NULL). */
gks_status gks_trainer_info(const gks_trainer *tr, int64_t *n_samples, int64_t *n_positive);
/* Mean loss and its gradient [7105] at the current parameters over the samples idx [B] (host),
 * 1 <= B <= max_batch (synchronising).  Sums over the batch run in sample order. */
gks_status gks_trainer_grad(gks_trainer *tr, const int32_t *idx, int32_t B, float *loss, float *grad);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) over `epochs` passes of minibatches
 * of `batch` samples, the order of each pass a Fisher-Yates shuffle drawn from splitmix64 seeded
 * with `seed`.  epoch_loss [epochs] (may be NULL): mean minibatch loss of each pass
 * (synchronising). */
gks_status gks_trainer_fit(gks_trainer *tr, int32_t epochs, int32_t batch, float lr, uint64_t seed,
                           float *epoch_loss);
/* Current parameters to host memory [7105] (synchronising). */
gks_status gks_trainer_params(const gks_trainer *tr, float *params);
/* Logits of every sample with the inference arithmetic (bf16 operands) to host memory [n]
 * (synchronising). */
gks_status gks_trainer_logits(gks_trainer *tr, float *logits);
/* Threshold for gks_indicator_set: the smallest logit threshold at which at most
 * max_false_skip * n samples of label 0 would be skipped, with the inference arithmetic. */
gks_status gks_trainer_threshold(gks_trainer *tr, double max_false_skip, float *threshold);

/* Launch-shape autotuner (for batches and single meshes alike): for the ghost, force-model, flux
 * and update kernels it times `reps` full steps of this state with 64, 128 and 256 threads per
 * block, one kernel class after the other, and keeps the fastest; the state's values, time and
 * step size are restored afterwards (results are independent of the launch shape).  chosen (may be
 * NULL): host [GKS_KERNEL_COUNT] threads per block of each kernel class after tuning.  A captured
 * graph is discarded.  Synchronising; allocates a copy of the state while it runs. */
gks_status gks_autotune(gks_state *st, int32_t reps, int32_t *chosen);

const char *gks_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
