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
 * reconstruction (Sec. 3.4), the interface force modelling (Sec. 2.3), the time-accurate
 * gas-kinetic evolution at two Gauss points per edge (Sec. 2.2, Eq. SWE-2nd-order) and the
 * well-balanced finite-volume update with bottom and layer-coupling sources (Sec. 3.1-3.2).
 *
 * Conventions
 *  - All pointers to user arrays are HOST pointers; the library copies them (the caller keeps
 *    ownership).  Handles are owned by the library until the matching *_destroy call.
 *  - Cell arrays are structure-of-arrays: W[6][n_tri] and gradW[6][2][n_tri] (component-major,
 *    then x / y, then cell), components in the order above, cells in the order of `tri`.
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
    GKS_ENONFINITE = 5,   /* non-finite value or non-positive layer thickness in the state */
    GKS_EUNSUPPORTED = 6  /* option not available in this build */
} gks_status;

typedef enum {
    GKS_BC_WALL = 0,      /* every boundary edge is a reflecting wall (mirror ghost cells) */
    GKS_BC_PERIODIC = 1   /* boundary edges of [0,Lx] x [0,Ly] are paired by translation */
} gks_bc;

typedef enum {
    GKS_FP64 = 0          /* every stage in double precision */
} gks_precision;

typedef struct {
    double G;        /* gravitational acceleration (Sec. 4: 9.81) */
    double chi;      /* density ratio rho2 / rho1 (Sec. 2.1) */
    double cfl;      /* CFL number of dt = CFL * dX / U_max (Sec. 4) */
    double eps;      /* collision-time constant epsilon (Sec. 4: 0.05) */
    double eps_num;  /* pressure-jump constant of the collision time (Sec. 4: 5) */
    double t_end;    /* the last step is clipped so that t never exceeds t_end */
    int32_t precision;  /* gks_precision */
    int32_t linear;     /* 1: linear P^3 reconstruction everywhere, 0: nonlinear (Sec. 3.4) */
} gks_params;

/* Build a mesh on the current HIP device.
 *   node_xy [n_nodes][2]  node coordinates
 *   tri     [n_tri][3]    counter-clockwise node indices
 *   node_B  [n_nodes]     bottom height at the nodes (continuous piecewise-linear bottom); NULL = 0
 *   bc, periodic_L[2]     boundary kind; periodic_L = (Lx, Ly) for GKS_BC_PERIODIC, else ignored
 * Setup runs on the host in FP64 (edges, compact stencils of Sec. 3.4 Eq. Recons-stencil with
 * mirror ghost cells at walls, least-squares matrices of Eq. Recons-system) and uploads the
 * result.  Returns GKS_EMESH for a malformed mesh. */
gks_status gks_mesh_create(const double *node_xy, int64_t n_nodes, const int32_t *tri, int64_t n_tri,
                           const double *node_B, int32_t bc, const double *periodic_L,
                           gks_mesh **out);
void gks_mesh_destroy(gks_mesh *mesh);
/* sizes: n_tri, n_edges, n_ghost (mirror cells kept for wall stencils) */
gks_status gks_mesh_info(const gks_mesh *mesh, int64_t *n_tri, int64_t *n_edges, int64_t *n_ghost);

/* Create a state on `mesh` (which must outlive it) from host arrays W0 [6][n_tri] and
 * gradW0 [6][2][n_tri] (cell averages and cell-averaged gradients at t = 0).  `stream` is a
 * hipStream_t (NULL = null stream).  Returns GKS_ENONFINITE if a thickness is <= 0 or a value is
 * not finite. */
gks_status gks_state_init(const gks_mesh *mesh, const gks_params *params, const double *W0,
                          const double *gradW0, void *stream, gks_state **out);
void gks_state_destroy(gks_state *st);

/* One S2O4 stage (Sec. 3.3, Eq. SWE-fully-discrete).  stage = 0 turns W^n into W^{n+1/2} and
 * stores what stage 1 needs; stage = 1 turns W^{n+1/2} into W^{n+1}.  Stages must alternate
 * 0, 1, 0, ... (GKS_EINVAL otherwise).  dt: host pointer to the step size for stage 0, or NULL to
 * use the CFL step computed on the device; must be NULL for stage 1 (the step size is reused). */
gks_status gks_stage(gks_state *st, int32_t stage, const double *dt);
/* n_steps full steps with the CFL time step computed on the device (no host synchronisation).
 * If dt_last is not NULL the call synchronises and returns the last step size.  GKS_EINVAL if
 * called between stage 0 and stage 1. */
gks_status gks_step(gks_state *st, int32_t n_steps, double *dt_last);

/* Copy the latest state to the host (synchronising): W^{n+1/2} between stage 0 and stage 1,
 * otherwise W^n.  W [6][n_tri], gradW [6][2][n_tri] (either may be NULL), t = its time (may be
 * NULL). */
gks_status gks_state_read(const gks_state *st, double *W, double *gradW, double *t);
/* Per-layer mass sum |Omega_j| h_j in FP64, mass[0] = upper layer (h2), mass[1] = lower (h1);
 * a deterministic device reduction; synchronising. */
gks_status gks_state_mass(const gks_state *st, double mass[2]);

/* Kernel classes for gks_profile_read. */
typedef enum {
    GKS_KERNEL_GHOST = 0,   /* mirror ghost cells refreshed from their source cells */
    GKS_KERNEL_RECON = 1,   /* compact reconstruction at the Gauss points (Sec. 3.4) */
    GKS_KERNEL_HHAT = 2,    /* edge-centre heights of the force model (Sec. 2.3) */
    GKS_KERNEL_PLANE = 3,   /* plane gradient of the force model (Sec. 2.3) */
    GKS_KERNEL_FLUX = 4,    /* gas-kinetic evolution at the Gauss points (Sec. 2.2) */
    GKS_KERNEL_UPDATE = 5,  /* gather, sources, S2O4 stage update (Sec. 3.1-3.3) */
    GKS_KERNEL_DT = 6,      /* CFL time step (Sec. 4) */
    GKS_KERNEL_COUNT = 7
} gks_kernel;

/* Kernel timing for measurement tools: enable != 0 starts recording a HIP event pair on the
 * state's stream around every kernel launch (clearing earlier records), 0 stops.  Synchronising. */
gks_status gks_profile(gks_state *st, int32_t enable);
/* Total time in ms and number of launches recorded for one kernel class since gks_profile
 * enabled recording.  Synchronising. */
gks_status gks_profile_read(gks_state *st, int32_t kernel, double *total_ms, int64_t *launches);

const char *gks_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
