/*
 * Oracle for the compact gas-kinetic scheme (GKS) for the two-layer shallow water equations on
 * triangular meshes (Zhao, Gan & Xu, "High-order compact gas-kinetic scheme for two-layer shallow
 * water equations on unstructured mesh").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow FP64 CPU implementation written
 * from the paper's equations, used to check the HIP implementation.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product never calls it.  It
 * shares no source with the HIP library.
 *
 * State layout used by every function: W[6][T] cell averages and gW[6][2][T] cell-averaged
 * gradients, components in the order of the conservative system (Sec. 2.1, Eq. SWE-macro):
 *   0 h2, 1 h2*U2, 2 h2*V2, 3 h1, 4 h1*U1, 5 h1*V1      (layer 1 = lower, layer 2 = upper).
 */
#ifndef GKS_ORACLE_H
#define GKS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct om_mesh om_mesh;

typedef struct {
    double G;        /* gravitational acceleration */
    double chi;      /* density ratio rho2 / rho1 */
    double cfl;      /* CFL number of the time step rule (Sec. 4) */
    double eps;      /* relaxation constant epsilon of the collision time (Sec. 4), 0.05 */
    double eps_num;  /* pressure-jump constant of the collision time (Sec. 4), 5 */
    int linear;      /* 1: linear P^3 reconstruction everywhere (all weights at their linear
                        values), 0: the nonlinear compact reconstruction */
    int per_side_gb; /* test only: 1 gives each side of an interface its own cell's bottom slope
                        in the evolution instead of the single-valued mean (shows what the
                        single-valued slope is for); 0 in every real use */
    int alpha_mode;  /* the constants alpha_{k,m} of the evolution solution (Sec. 2.2): 0 the
                        well-balance weights read here (3/4 on the state moment of mass, 5/4 on
                        the momentum flux moments, on the jump of the sides' accelerations in the
                        equilibrium part), 1 the paper's printed (1, 3/4, 1/4) on the flux moments
                        of the acceleration term in both the equilibrium and the initial parts,
                        1 on the state moments */
    int src_order;   /* layer coupling (Sec. 3.2, Eq. SWE-source-discretization): 2 (or 0) the
                        paper's second-order form, Gauss-point mean thickness times the
                        Green-Gauss derivative of the other layer; 4 the higher-order form its
                        closing remark allows: the cell average in place of the Gauss-point mean
                        plus the interior integral of (h_a - mean h_a) grad h_b over the cell's
                        reconstructions */
    int grad_mode;   /* interface values of the gradient update (Sec. 3.3, Eq. slope-1): 0 the
                        continuous evolution solution W^l = W^r (the interface equilibrium's state
                        and time slope, the paper's choice); 1 discontinuous values W^l != W^r:
                        each cell takes the state on its own side of the interface, advanced by
                        that side's own time derivative (om_side_rate) */
    double h_dry;    /* wet/dry layers (a vanishing layer, Sec. 4's dam breaks over a dry bed; the
                        paper gives no treatment, this is a reading): 0 (off) the scheme as above;
                        > 0 a layer thickness at or below h_dry is dry.  A dry side of an interface
                        carries no particles (vacuum), an interface whose equilibrium thickness is
                        at or below h_dry passes nothing, and in a layer's front band (the cell or
                        a face neighbour thinner than OM_THIN h_dry or than OM_FRONT times the
                        thickest of the four, or the lower layer thinner than the bottom's rise
                        across the cell) the layer is reconstructed as its constant cell average
                        with the cell's desingularised velocity (om_cell_velocity) and evolves at
                        first order in space and time */
} om_params;

/* The two-stage fourth-order time stepping (S2O4, Sec. 3.3, Eq. SWE-fully-discrete) on n values:
 * stage  out = W + dt/2 L + dt^2/8 Lt               (the state at t + dt/2)
 * final  out = W + dt L + dt^2/6 Lt + dt^2/3 Lt2     (Lt2 = time derivative at the stage state) */
void om_s2o4_stage(int n, double dt, const double *W, const double *L, const double *Lt, double *out);
void om_s2o4_final(int n, double dt, const double *W, const double *L, const double *Lt, const double *Lt2,
                   double *out);

/* Threads used by the per-cell and per-edge loops (OpenMP); results do not depend on it. */
void om_set_threads(int n);
int om_max_threads(void);

/* Mesh: node coordinates [nn][2], counter-clockwise triangles [nt][3], bottom at the nodes
 * (piecewise linear).  bc (passed as `periodic`): 1 pairs the boundary edges of [0,Lx]x[0,Ly] by
 * translation, 2 makes every boundary edge free (zero-gradient), 0 a reflecting wall.  Returns
 * NULL on a malformed mesh. */
om_mesh *om_mesh_new(const double *node_xy, int nn, const int *tri, int nt, const double *node_B,
                     int periodic, double Lx, double Ly);
void om_mesh_free(om_mesh *m);
int om_mesh_n_edges(const om_mesh *m);

/* Force model pieces (Sec. 2.3).  om_edge_height: interface height xi zl + (1 - xi) zr of the two
 * sides' heights zl, zr, with xi = 1/2 erfc(-sqrt(lambda) (unl + unr) / 2), lambda = 2 / (G (hl + hr))
 * from the layer thicknesses hl, hr and normal velocities unl, unr (normal from left to right).
 * om_plane_gradient: gradient out[2] of the plane through the values hk[3] at the centres of cell c's
 * local edges (edge k joins vertices k and k + 1 of the triangle as given to om_mesh_new). */
double om_edge_height(double zl, double zr, double hl, double hr, double unl, double unr, double G);
void om_plane_gradient(const om_mesh *m, int c, const double *hk, double *out);

/* Stencil of cell c: 10 (cell, map) images; cells[10], maps[10][6] = (R00 R01 R10 R11 t0 t1). */
void om_stencil(const om_mesh *m, int c, int *cells, double *maps);
/* Least-squares solution matrix of cell c, [9][17] row-major (Sec. 3.4, Eq. Recons-system). */
void om_lsq_matrix(const om_mesh *m, int c, double *M);
/* Smallest sine of the angle between the two centroid offsets of a plane candidate of the
 * nonlinear reconstruction (a sub-stencil {0, i, j}); flatter sub-stencils are not candidates. */
#define OM_PLANE_SINE_MIN 0.2
/* the front band of a layer (h_dry > 0): the cell or a face neighbour thinner than OM_THIN h_dry
 * or than OM_FRONT times the thickest of the four (see h_dry) */
#define OM_THIN 1000.0
#define OM_FRONT 0.3

/* Reconstruction of all six variables in cell c (with eta1 = h1 + B in place of h1) at the cell's
 * six Gauss points (local edge k, point g -> index 2k+g):
 *   val[6 gp][6 comp], grad[6 gp][6 comp][2], r0[6 comp] = omega_0 / d_0.
 * linear != 0 returns the linear P^3 reconstruction (all weights at their linear values).  G enters
 * the floor of the smoothness indicators of the momenta (scale 1e-8 h sqrt(G h)). */
void om_reconstruct_cell(const om_mesh *m, int c, const double *W, const double *gW, int linear, double G,
                         double *val, double *grad, double *r0);

/* One Gauss point, one layer, local frame (u along the normal).  side = {h, U, V, dh_n, dh_t,
 * d(hU)_n, d(hU)_t, d(hV)_n, d(hV)_t, Phi_n, Phi_t}.  Outputs in the local frame.  The
 * acceleration term of the interface equilibrium carries the well-balance weights alpha_{k,m}
 * (Sec. 2.2, Eq. SWE-2nd-order) as read here: on the jump between the two sides' accelerations,
 * 3/4 on the mass state moment and 5/4 on the momentum flux moments. */
void om_gks_point(const double *sideL, const double *sideR, double G, double dt, double eps,
                  double eps_num, double *F0, double *Ft, double *Wb, double *Wbt);
/* Same with the choice of the constants alpha_{k,m} (alpha_mode as in om_params). */
void om_gks_point_mode(const double *sideL, const double *sideR, double G, double dt, double eps,
                       double eps_num, int alpha_mode, double *F0, double *Ft, double *Wb, double *Wbt);
/* Same, returning the time-integrated flux F(delta) for one delta (for the closed-form pins). */
void om_gks_point_integrated(const double *sideL, const double *sideR, double G, double delta,
                             double tau, double *F);
/* Velocity of a layer with cell-average thickness h and momentum component m: m / h where h is at
 * least hs = OM_THIN h_dry (or h_dry is 0); below it the desingularised form
 * sqrt(2) h m / sqrt(h^4 + hs^4) (Kurganov and Petrova 2007), which tends to zero with h. */
double om_cell_velocity(double h, double m, double h_dry);
/* The evolution at one Gauss point with wet/dry sides (h_dry as in om_params): a side whose
 * thickness is at or below zero is a vacuum (the caller zeroes a dry side's record), and an
 * interface whose equilibrium thickness is at or below h_dry gives zero fluxes and interface values.
 * order1 != 0: first order in time, F0 the step's mean flux F(dt) / dt and Ft = 0 (the caller
 * zeroes the sides' slopes and accelerations for first order in space). */
void om_gks_point_wd(const double *sideL, const double *sideR, double G, double dt, double eps,
                     double eps_num, int alpha_mode, double h_dry, int order1, double *F0, double *Ft,
                     double *Wb, double *Wbt);
/* Time derivative (h, hU_n, hU_t)_t of one side's own state (side as in om_gks_point, local
 * frame) from the compatibility condition on that side's Maxwellian: minus the full-space moments
 * of its slope and acceleration polynomial (Sec. 2.2).  The inner-side value of the discontinuous
 * reading of the gradient update (grad_mode 1) evolves with it. */
void om_side_rate(const double *side, double G, double *Wt);
/* Normalised moments <u^k>, k = 0..K-1, of the Gaussian with mean U and variance 1/(2 lambda):
 * half = 0 full space, +1 over u > 0, -1 over u < 0. */
void om_moments(double U, double lam, int half, int K, double *out);
/* Time integrals of the coefficients C1..C5 of the evolution solution over [0, delta]. */
void om_time_integrals(double delta, double tau, double *g5);

/* Time step from the CFL rule (Sec. 4) for the state W. */
double om_dt(const om_mesh *m, const om_params *p, const double *W);

/* Spatial operator of one stage: for the stage state (W, gW) and the step's dt, returns
 * L[6][T], Lt[6][T] (right-hand side and its time derivative) and the Green-Gauss gradients of
 * the interface values GW[6][2][T], GWt[6][2][T] (Sec. 3.1-3.3).  The layer coupling takes its
 * Gauss-point thicknesses as the mean of the two sides' reconstructed values (Sec. 3.2). */
int om_operator(const om_mesh *m, const om_params *p, double dt, const double *W, const double *gW,
                double *L, double *Lt, double *GW, double *GWt);
/* Same, also returning the layer-coupling part of L and Lt (S[4][T], St[4][T]: lower layer x, y,
 * upper layer x, y; NULL to skip). */
int om_operator_src(const om_mesh *m, const om_params *p, double dt, const double *W, const double *gW,
                    double *L, double *Lt, double *GW, double *GWt, double *S, double *St);
/* The interior correction of the higher-order layer coupling in cell c (corr[8], see src_order):
 * mean((h1 - mean h1) grad h2), mean((h2 - mean h2) grad h1), then their time derivatives. */
void om_coupling_correction(const om_mesh *m, int c, const double *W, const double *gW, int linear, double G,
                            double *corr);

/* One S2O4 step (Sec. 3.3, Eq. SWE-fully-discrete and the two-stage interface update).
 * nstages = 1 stops after the first stage and returns W^{n+1/2}. */
int om_step(const om_mesh *m, const om_params *p, double dt, int nstages, const double *W,
            const double *gW, double *Wout, double *gWout);

/* Per-layer mass sum_j |Omega_j| h_j, mass[0] = upper (h2), mass[1] = lower (h1). */
void om_mass(const om_mesh *m, const double *W, double *mass);
void om_cell_geometry(const om_mesh *m, double *area, double *cx, double *cy);

/* Learned smoothness indicator (reference for the GPU kernels).
 * Features X[T][44] of each cell: for the interface level eta1 = h1 + B, then h2: the 9 stencil
 * differences (Q_l - Q_0)/s and the 8 scaled gradients h grad Q_l / s of the cell and its face
 * neighbours, s = max_l |Q_l - Q_0| + 1e-12 |Q_0| (17 each, X[0..33]); then log10(s / h)/4 with h
 * the layer's thickness in the cell (eta1: h1, then h2; X[34], X[35]); then for the lower and the
 * upper layer log10((sm + 1e-12 c) / c)/4 with sm the largest stencil difference of the layer's two
 * momentum components and c = h sqrt(G h) (X[36], X[37]); then the face neighbours' area ratios
 * (X[38..40]) and the cell's edge lengths over h = sqrt(2 |Omega|) (X[41..43]).
 * MLP 44 -> 64 -> 64 -> 1 with ReLU hidden layers; parameters P[7105] = W1[44][64], b1[64],
 * W2[64][64], b2[64], w3[64], b3.  Loss: mean over the batch of softplus(z) - y z (logistic loss
 * on the logit z). */
void om_features(const om_mesh *m, double G, const double *W, const double *gW, double *X);
void om_mlp_forward(const double *P, const double *X, int B, double *z);
double om_mlp_grad(const double *P, const double *X, const double *y, int B, double *grad);
/* The forward pass with the operand rounding of a bfloat16 matrix-core evaluation: the inputs,
 * W1, the first hidden layer's activations and W2 rounded to single precision and then to 8
 * significant bits (ties to even) before their products; sums, biases and the output layer in
 * double.  Used where a decision (logit > threshold) must be taken in the kernel's precision. */
void om_mlp_forward_bf16(const double *P, const double *X, int B, double *z);

#ifdef __cplusplus
}
#endif
#endif
