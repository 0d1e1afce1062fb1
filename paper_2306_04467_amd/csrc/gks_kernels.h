// Device kernels of one S2O4 stage of the compact gas-kinetic scheme (gfx950, wave64).
//
// Every kernel is a template on R, the precision of the bulk arithmetic and storage: double for
// the FP64 path, float for the mixed path.  Whatever decides the lake-at-rest balance stays in
// double in both: cell thicknesses (h2 and the interface level eta1 = h1 + B), Gauss-point
// thicknesses, the hydrostatic part 1/2 G h^2 of the normal momentum flux, the interface
// thickness, and every edge sum of the cell update (flux divergence, Green-Gauss derivatives,
// sources).  What is computed in R there vanishes exactly at rest by left/right symmetry.
//
// Data layout:
//   state  structure of arrays, index = component * stride + cell: Wh[2][TG] (double: h2, eta1),
//          Wm[4][TG] (R: h2U2, h2V2, h1U1, h1V1), gW[12][TG] (R: x/y gradients of h2, h2U2, h2V2,
//          eta1, h1U1, h1V1), TG = T + NG ghosts
//   rec    GpHead[6 T] and GpTail[6 T], cell-major: the reconstruction at each cell's six Gauss
//          points, read by the edge kernels as 16-byte words (one cache line per record)
//   eoh    [6][E] double: per edge, Gauss points averaged: 1/2 G hb^2 (upper, lower), hb (upper,
//          lower), hb the interface thickness of the evolution, then the mean of the two sides'
//          reconstructed thicknesses (upper, lower) for the layer coupling
//   eom    [24][E] R: F0 (6, hydrostatic part removed), Ft (6), interface momenta (4), interface
//          time derivatives (6), global frame, then the mean of the two sides' thickness rates
//          (upper, lower); read by the cell update's gather
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gks_mlp.h"

namespace gks {

struct MeshDev {
    int64_t T, E, NG;
    int32_t S;                      // number of scenarios (independent meshes) in this mesh
    // FP64 tables
    const double *area, *Bbar, *gB, *fl, *gg, *eBgp, *gR, *sdxmin;
    // tables in the bulk precision (double or float copies); M, the least-squares operators, is
    // block-major [ceil(T / RECON_CELLS)][153][RECON_CELLS]
    const void *M, *hs, *vtx, *nbc, *en, *egB;
    const float *igeo;              // [6][T] indicator geometry
    const uint8_t *cand;            // [T] plane candidates of the nonlinear reconstruction (bits 0..2)
    const int32_t *cedge, *sten, *eL, *eR, *eslot, *gsrc;
    const int32_t *cscen, *escen;   // scenario of each cell / edge, nullptr when S == 1
    // batches: the cells cut into chunks that never straddle two scenarios, chunk c covering
    // [cb[c], cb[c + 1]); scenario s owns chunks [sc0[s], sc0[s + 1])
    const int64_t *cb;
    const int32_t *sc0;
    int32_t NCH;
    const int64_t *scell;           // [S + 1] first cell of each scenario
};

struct Phys {
    double G, eps, eps_num, cfl;
    double h_dry;         // wet/dry threshold (0: every layer is wet everywhere)
    int linear;
    int alpha_mode;       // 0: the well-balance weights read here, 1: the paper's printed constants
    const double *chi;    // [S] density ratio
    const double *t_end;  // [S]
    double *scal;         // [2S] per scenario: dt of the current step, time at its end
    unsigned long long *bad;  // smallest cell whose updated state is non-finite or has a layer
                              // thickness <= 0 (all ones: none), kept until the state is reloaded
};

// the force model's weight w is taken as 1 when it is within 1e-12 of 1: the blend would then
// change the acceleration by less than its own FP64 rounding
constexpr double W_ONE = 1.0 - 1e-12;

// Wet/dry layers (Phys::h_dry > 0; the paper's dam breaks over a dry bed, with no treatment given
// there): a side of an interface whose thickness is at or below h_dry is a vacuum, an interface
// whose equilibrium thickness is at or below h_dry passes nothing, and the front band of a layer --
// the cells where the layer, in the cell or in one of its face neighbours, is thinner than
// WD_THIN h_dry or than WD_FRONT times the thickest of the four, and the cells where the lower
// layer is thinner than the bottom's rise across the cell -- is reconstructed at first order and
// evolves at first order in space and time.  Below WD_THIN h_dry a cell's velocity is
// desingularised (Kurganov and Petrova 2007).
constexpr double WD_THIN = 1000.0, WD_FRONT = 0.3;

__host__ __device__ inline double wd_velocity(double h, double m, double h_dry)
{
    const double hs = WD_THIN * h_dry;
    if (!(h_dry > 0) || h >= hs) return m / h;
    const double h2 = h * h, d2 = hs * hs;
    return 1.4142135623730950488 * h * m / sqrt(h2 * h2 + d2 * d2);
}


// relative floor of the smoothness indicators of the nonlinear reconstruction, above the
// rounding of the bulk precision: the weights leave their linear values once a variable varies
// by about 1e-9 of its scale (FP64), 1e-5 in the mixed path, whose reconstruction runs in FP32
template <typename R>
__device__ constexpr R eps_rel()
{
    return sizeof(R) == 8 ? R(1e-18) : R(1e-10);
}

template <typename R>
__device__ inline const R *tab(const void *p)
{
    return static_cast<const R *>(p);
}

// Checked build (GKS_CHECKED): every index read from a mesh table is tested against the size of
// the array it indexes before it is used; a miss sets oob_flag and the access falls back to
// element 0, so the kernel itself stays in bounds.  Other builds take the index as it is.
#ifdef GKS_CHECKED
__device__ unsigned int oob_flag;
__device__ inline int64_t checked_index(int64_t i, int64_t n)
{
    if (i < 0 || i >= n) {
        atomicOr(&oob_flag, 1u);
        return 0;
    }
    return i;
}
#define GKS_IX(i, n) ::gks::checked_index((int64_t)(i), (int64_t)(n))
#else
#define GKS_IX(i, n) (i)
#endif

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.  Cells and edges
// are numbered with spatial locality, so give each XCD one contiguous range of blocks: neighbour
// gathers then hit the same L2 instead of being fetched from HBM by several XCDs.
constexpr int N_XCD = 8;

__device__ inline int64_t xcd_block()
{
    const int64_t b = blockIdx.x, nb = gridDim.x;
    const int64_t q = nb / N_XCD, r = nb % N_XCD, x = b % N_XCD, j = b / N_XCD;
    return x * q + (x < r ? x : r) + j;
}

// the four momentum components in paper order 1, 2, 4, 5 -> slots 0..3 of Wm
__device__ inline int mom_slot(int v) { return v < 3 ? v - 1 : v - 2; }

// a / b in the bulk precision: in FP32 the product with the hardware reciprocal (one instruction,
// within about an ulp, where the correctly rounded quotient costs about ten; FP32 results are
// held to FP32 tolerances), in FP64 the correctly rounded quotient
__device__ inline float div_(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ inline double div_(double a, double b) { return a / b; }

// Gauss-point records of one cell at one of its six Gauss points (slot = 2 * local edge + point),
// written by the reconstruction and read by the edge kernels.  Records are stored cell-major,
// index 6 c + slot, in two arrays: the head (thicknesses and momenta, all that the force model's
// edge kernel reads) and the tail (gradients), so that each is read as a few 16-byte words.
//   head.h[0] h2, head.h[1] eta1 = h1 + B (double in both precisions)
//   head.q[0..3]  momenta h2U2, h2V2, h1U1, h1V1
//   tail.g[2 v], tail.g[2 v + 1]  x / y derivative of paper component v (v = 0..5, eta1 for h1)
template <typename R>
struct alignas(16) GpHead {
    double h[2];
    R q[4];
};

template <typename R>
struct alignas(16) GpTail {
    R g[12];
};

template <typename R>
struct GpRecs {
    GpHead<R> *head;
    GpTail<R> *tail;
};


// --------------------------------------------------------------------------------------------
// ghost mirror cells: state of the source cell seen through an orthogonal map

template <typename R>
__global__ void k_ghost_fill(MeshDev m, double *__restrict__ Wh, R *__restrict__ Wm, R *__restrict__ gW)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= m.NG) return;
    const int64_t TG = m.T + m.NG, s = GKS_IX(m.gsrc[g], m.T), d = m.T + g, NG = m.NG;
    // R (a b; c e) maps gradient directions, V (va vb; vc ve) momentum vectors: V = R across a
    // wall, V = I across a free boundary (each component extended evenly)
    const double a = m.gR[g], b = m.gR[NG + g], c = m.gR[2 * NG + g], e = m.gR[3 * NG + g];
    const double va = m.gR[4 * NG + g], vb = m.gR[5 * NG + g], vc = m.gR[6 * NG + g], ve = m.gR[7 * NG + g];
#pragma unroll
    for (int l = 0; l < 2; l++) {  // l = 0 upper (paper components 0..2), 1 lower (3..5)
        const int o = 3 * l;
        Wh[l * TG + d] = Wh[l * TG + s];
        const double mx = Wm[(2 * l) * TG + s], my = Wm[(2 * l + 1) * TG + s];
        Wm[(2 * l) * TG + d] = (R)(va * mx + vb * my);
        Wm[(2 * l + 1) * TG + d] = (R)(vc * mx + ve * my);
        const double hx = gW[(2 * o) * TG + s], hy = gW[(2 * o + 1) * TG + s];
        gW[(2 * o) * TG + d] = (R)(a * hx + b * hy);
        gW[(2 * o + 1) * TG + d] = (R)(c * hx + e * hy);
        // momentum gradient G[i][j] = d m_i / d x_j  ->  V G R^T
        const double g00 = gW[(2 * o + 2) * TG + s], g01 = gW[(2 * o + 3) * TG + s];
        const double g10 = gW[(2 * o + 4) * TG + s], g11 = gW[(2 * o + 5) * TG + s];
        const double r00 = va * g00 + vb * g10, r01 = va * g01 + vb * g11;
        const double r10 = vc * g00 + ve * g10, r11 = vc * g01 + ve * g11;
        gW[(2 * o + 2) * TG + d] = (R)(r00 * a + r01 * b);
        gW[(2 * o + 3) * TG + d] = (R)(r00 * c + r01 * e);
        gW[(2 * o + 4) * TG + d] = (R)(r10 * a + r11 * b);
        gW[(2 * o + 5) * TG + d] = (R)(r10 * c + r11 * e);
    }
}

// --------------------------------------------------------------------------------------------
// compact reconstruction (Sec. 3.4): one thread per (cell, variable); 192 threads = 32 cells x 6.
// Wave 0 holds the two thicknesses (h2, eta1), waves 1 and 2 the momenta of each layer, so a
// wave never splits between the FP64 thickness path and the momentum path.

constexpr int RECON_CELLS = 32;

// values of one variable at a cell's six Gauss points and its gradient there
template <typename R>
struct ReconOut {
    // Gauss-point values: a thickness (h2, eta1) in double, a momentum in the bulk precision widened
    // to double (exact); one array for both keeps every access at a constant index (registers)
    double v[6];
    R gx[6], gy[6];
};

// right-hand side of the least-squares system of variable v of cell c
template <typename R>
struct ReconRhs {
    R rhs[17];  // average differences, then scaled gradients of the cell and its face neighbours
    R hs, Q0;
    double Q0h;  // cell average of a thickness in double
    double hl;   // momenta: thickness of the variable's layer (scale of the smoothness floor)
};

template <typename R>
__device__ inline void recon_rhs(const MeshDev &m, const double *__restrict__ Wh, const R *__restrict__ Wm,
                                 const R *__restrict__ gW, int v, bool thick, int64_t c, ReconRhs<R> &q)
{
    const int64_t T = m.T, TG = m.T + m.NG;
    const R hs = tab<R>(m.hs)[c];
    // differences of thicknesses are taken in FP64 before rounding
    double Q0h = 0;
    R Q0 = 0;
    R *rhs = q.rhs;
    int32_t nb[9];
#pragma unroll
    for (int s = 0; s < 9; s++) nb[s] = GKS_IX(m.sten[s * T + c], T + m.NG);
    // the level of the variable's layer (h2, or eta1 for the lower layer), loaded outside the
    // branch so that a wave holding a thickness and a momentum issues it once: a thickness
    // differences it, a momentum takes its layer's thickness from it
    const double hq = Wh[(v < 3 ? 0 : TG) + c], bq = m.Bbar[c];
    if (thick) {
        const double *Q = Wh + (v == 3 ? TG : 0);
        Q0h = hq;
        Q0 = (R)Q0h;
#pragma unroll
        for (int s = 0; s < 9; s++) rhs[s] = (R)(Q[nb[s]] - Q0h);
    } else {
        const R *Q = Wm + mom_slot(v) * TG;
        Q0 = Q[c];
#pragma unroll
        for (int s = 0; s < 9; s++) rhs[s] = Q[nb[s]] - Q0;
    }
    q.hl = v < 3 ? hq : hq - bq;
    rhs[9] = hs * gW[(2 * v) * TG + c];
    rhs[10] = hs * gW[(2 * v + 1) * TG + c];
#pragma unroll
    for (int l = 0; l < 3; l++) {
        rhs[11 + 2 * l] = hs * gW[(2 * v) * TG + nb[l]];
        rhs[12 + 2 * l] = hs * gW[(2 * v + 1) * TG + nb[l]];
    }
    q.hs = hs;
    q.Q0 = Q0;
    q.Q0h = Q0h;
}

// reconstruction of variable v of cell c: P^3 coefficients from its right-hand side (Ms points
// at the cell's least-squares operator in LDS, entry j at Ms[32 j]), then the weights and the
// Gauss-point values
// coefficients k0 <= k < k1 of the P^3 fit; Ms holds the operator rows from row 17 k0 on
template <int k0, int k1, typename R>
__device__ inline void recon_coeffs(const ReconRhs<R> &q, const R *Ms, R a[9])
{
#pragma unroll
    for (int k = k0; k < k1; k++) {
        R s = 0;
#pragma unroll
        for (int r = 0; r < 17; r++) s = fma(Ms[((k - k0) * 17 + r) * RECON_CELLS], q.rhs[r], s);
        a[k] = s;
    }
}

// the reconstruction from the P^3 coefficients a; lin: take the linear weights (no smoothness
// indicators)
// the combination that recon_cell settled on, for evaluations away from the Gauss points:
// R(x) = Q0 + theta (ratio P(x) + sbx x + sby y) in scaled coordinates (P the zero-mean P^3 part)
template <typename R>
struct ReconComb {
    R ratio, sbx, sby, theta;
};

template <typename R>
__device__ inline void recon_cell(const MeshDev &m, const Phys &p, bool lin, R *__restrict__ r0, int v, bool thick,
                                  int64_t c, const ReconRhs<R> &q, const R a[9], ReconOut<R> &out,
                                  ReconComb<R> &comb)
{
    const int64_t T = m.T;
    const R *rhs = q.rhs;
    const R hs = q.hs, Q0 = q.Q0;
    const double Q0h = q.Q0h;
    // scaled vertices (centroid at the origin) and the cell means of the basis
    const R *vt = tab<R>(m.vtx);
    R vx[3], vy[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        vx[k] = vt[(2 * k) * T + c];
        vy[k] = vt[(2 * k + 1) * T + c];
    }
    R mxx = 0, mxy = 0, myy = 0, mx3 = 0, mx2y = 0, mxy2 = 0, my3 = 0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        mxx += vx[k] * vx[k];
        mxy += vx[k] * vy[k];
        myy += vy[k] * vy[k];
        mx3 += vx[k] * vx[k] * vx[k];
        mx2y += vx[k] * vx[k] * vy[k];
        mxy2 += vx[k] * vy[k] * vy[k];
        my3 += vy[k] * vy[k] * vy[k];
    }
    const R c12 = R(1) / R(12), c30 = R(1) / R(30);
    const R mean_const = a[2] * mxx * c12 + a[3] * mxy * c12 + a[4] * myy * c12 + a[5] * mx3 * c30 +
                         a[6] * mx2y * c30 + a[7] * mxy2 * c30 + a[8] * my3 * c30;
    // lower-order candidates (reading of the nonlinear compact reconstruction): planes through
    // the averages of {0, f0, f1}, {0, f1, f2}, {0, f2, f0} and the cell's own gradient.  A
    // sub-stencil whose centroid offsets are nearly parallel is not a candidate (bit clear in
    // m.cand, decided at setup in FP64): its plane would carry a huge slope into the combination
    // below; its linear weight goes to P^3.
    const R *nbc = tab<R>(m.nbc);
    const unsigned cmask = m.cand[c] | 8u;  // the own-gradient plane is always a candidate
    R bx[4], by[4];
#pragma unroll
    for (int s = 0; s < 3; s++) {
        const int sa = s, sb = (s + 1) % 3;
        const R ax_ = nbc[(2 * sa) * T + c], ay_ = nbc[(2 * sa + 1) * T + c];
        const R bx_ = nbc[(2 * sb) * T + c], by_ = nbc[(2 * sb + 1) * T + c];
        const R ra = rhs[sa], rb = rhs[sb];
        const R invd = R(1) / (ax_ * by_ - ay_ * bx_);
        const R inv = ((cmask >> s) & 1u) ? invd : R(0);  // excluded planes: slope 0, weight 0
        bx[s] = (ra * by_ - ay_ * rb) * inv;
        by[s] = (ax_ * rb - ra * bx_) * inv;
    }
    bx[3] = rhs[9];
    by[3] = rhs[10];
    const int ncand = __builtin_popcount(cmask);
    const R d0 = ncand == 4 ? R(0.8) : ncand == 3 ? R(0.85) : ncand == 2 ? R(0.9) : R(0.95), dm = R(0.05);
    R w0 = d0, wm[4];
#pragma unroll
    for (int s = 0; s < 4; s++) wm[s] = ((cmask >> s) & 1u) ? dm : R(0);
    const bool nonlinear = !p.linear && !lin;
    if (nonlinear) {
        // smoothness indicator of P^3 in scaled coordinates: the cell has area 1/2 there, so the
        // |Omega|^(|alpha|-1) weights become (1/2)^(|alpha|-1) and integrals are averages / 2.
        // First derivatives (quadratics): 6-point degree-4 rule; second (linear): edge midpoints.
        const R qa[2] = {R(0.445948490915964886), R(0.091576213509770743)};
        const R qw[2] = {R(0.223381589678011466), R(1.0 / 3.0 - 0.223381589678011466)};
        R s1 = 0;
#pragma unroll
        for (int r = 0; r < 2; r++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const R l0 = (j == 0) ? 1 - 2 * qa[r] : qa[r];
                const R l1 = (j == 1) ? 1 - 2 * qa[r] : qa[r];
                const R l2 = (j == 2) ? 1 - 2 * qa[r] : qa[r];
                const R x = l0 * vx[0] + l1 * vx[1] + l2 * vx[2];
                const R y = l0 * vy[0] + l1 * vy[1] + l2 * vy[2];
                const R px = a[0] + 2 * a[2] * x + a[3] * y + 3 * a[5] * x * x + 2 * a[6] * x * y + a[7] * y * y;
                const R py = a[1] + a[3] * x + 2 * a[4] * y + a[6] * x * x + 2 * a[7] * x * y + 3 * a[8] * y * y;
                s1 += qw[r] * (px * px + py * py);
            }
        R s2 = 0;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const R x = R(0.5) * (vx[j] + vx[(j + 1) % 3]), y = R(0.5) * (vy[j] + vy[(j + 1) % 3]);
            const R pxx = 2 * a[2] + 6 * a[5] * x + 2 * a[6] * y;
            const R pxy = a[3] + 2 * a[6] * x + 2 * a[7] * y;
            const R pyy = 2 * a[4] + 2 * a[7] * x + 6 * a[8] * y;
            s2 += (pxx * pxx + pxy * pxy + pyy * pyy) * (R(1) / R(3));
        }
        const R s3 = 36 * a[5] * a[5] + 4 * a[6] * a[6] + 4 * a[7] * a[7] + 36 * a[8] * a[8];
        const R beta0 = R(0.5) * s1 + R(0.25) * s2 + R(0.125) * s3;
        R tz = 0, bm[4];
#pragma unroll
        for (int s = 0; s < 4; s++) {
            bm[s] = R(0.5) * (bx[s] * bx[s] + by[s] * by[s]);
            tz += ((cmask >> s) & 1u) ? fabs(beta0 - bm[s]) : R(0);
        }
        tz = ncand == 4 ? tz * R(0.25) : div_(tz, R(ncand));
        // floor of the smoothness indicators with the variable's scale: the level of a thickness,
        // 1e-8 h sqrt(G h) of the layer for a momentum
        const R S2 = thick ? R(1e-20) : (R)(1e-16 * p.G * q.hl * q.hl * q.hl);
        const R epsw = eps_rel<R>() * fmax(Q0 * Q0, S2);
        const R t0 = d0 * (1 + div_(tz, beta0 + epsw));
        R sum = t0, tm[4];
#pragma unroll
        for (int s = 0; s < 4; s++) {
            tm[s] = ((cmask >> s) & 1u) ? dm * (1 + div_(tz, bm[s] + epsw)) : R(0);
            sum += tm[s];
        }
        // where every unnormalised weight equals its linear weight (tau = 0, or tau / (beta + eps)
        // below the rounding of 1), the weights are the linear ones, which sum to one: take them
        // exactly instead of dividing by their rounded sum
        bool lin = t0 == d0;
#pragma unroll
        for (int s = 0; s < 4; s++) lin = lin && tm[s] == wm[s];
        const R isum = lin ? R(1) : div_(R(1), sum);
        w0 = t0 * isum;
#pragma unroll
        for (int s = 0; s < 4; s++) wm[s] = tm[s] * isum;
    }
    const R ratio = w0 / d0;
    if (v == 3) r0[c] = ratio;
    if (v == 0) r0[T + c] = ratio;
    // combined polynomial R = ratio (P0 - sum dm Pm) + sum wm Pm, Pm = Q0 + b . x
    R sbx = 0, sby = 0;
#pragma unroll
    for (int s = 0; s < 4; s++) {
        const R cm = wm[s] - ratio * (((cmask >> s) & 1u) ? dm : R(0));
        sbx += cm * bx[s];
        sby += cm * by[s];
    }
    const R ihs = div_(R(1), hs);
    const R gs[2] = {R(0.5 - 0.28867513459481288225), R(0.5 + 0.28867513459481288225)};
    // positivity safeguard (not in the paper): where a layer thickness at a Gauss point would fall
    // below a tenth of the cell's average, the deviation from the average is scaled down
    // (Zhang-Shu scaling) until it does not; the lower layer's thickness is eta1 minus the
    // piecewise-linear bottom.  The factor is 1 at rest and in ordinary flows; it is formed in the
    // bulk precision (it only decides how far to pull the values back).
    const R hbar = (R)(v == 0 ? Q0h : Q0h - m.Bbar[c]), floor_h = R(0.1) * hbar;
    const R gBx = v == 3 ? (R)m.gB[c] : R(0), gBy = v == 3 ? (R)m.gB[T + c] : R(0);
    R theta = 1;
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
        for (int g = 0; g < 2; g++) {
            const int k1 = (k + 1) % 3;
            const R x = vx[k] + gs[g] * (vx[k1] - vx[k]);
            const R y = vy[k] + gs[g] * (vy[k1] - vy[k]);
            const R P = a[0] * x + a[1] * y + a[2] * x * x + a[3] * x * y + a[4] * y * y + a[5] * x * x * x +
                        a[6] * x * x * y + a[7] * x * y * y + a[8] * y * y * y - mean_const;
            const R Px = a[0] + 2 * a[2] * x + a[3] * y + 3 * a[5] * x * x + 2 * a[6] * x * y + a[7] * y * y;
            const R Py = a[1] + a[3] * x + 2 * a[4] * y + a[6] * x * x + 2 * a[7] * x * y + 3 * a[8] * y * y;
            // all candidates share the cell average Q0 (ratio + sum cm = 1)
            const R dev = ratio * P + sbx * x + sby * y;
            const int slot = 2 * k + g;
            out.v[slot] = thick ? Q0h + (double)dev : (double)(Q0 + dev);
            out.gx[slot] = (ratio * Px + sbx) * ihs;
            out.gy[slot] = (ratio * Py + sby) * ihs;
            if (thick && dev < 0) {
                const R bdev = hs * (gBx * x + gBy * y);
                theta = fmin(theta, fmax(R(0), div_(hbar - bdev - floor_h, -dev)));
            }
        }
    if (theta < R(1)) {
#pragma unroll
        for (int slot = 0; slot < 6; slot++) {
            out.v[slot] = Q0h + (double)theta * (out.v[slot] - Q0h);
            out.gx[slot] *= theta;
            out.gy[slot] *= theta;
        }
    }
    comb.ratio = ratio;
    comb.sbx = sbx;
    comb.sby = sby;
    comb.theta = theta;
}

// Higher-order layer coupling (Sec. 3.2, Eq. SWE-source-discretization, and its remark that more
// integration points raise the order): the part of the cell average of h_a grad h_b that the
// product of averages misses, mean((h_a - mean h_a) grad h_b), and its time derivative with the
// thickness rate h_t = -div(h U), from the cell's own reconstructions.  Each variable thread
// evaluates three numbers per interior point: a thickness its deviation from the cell average and
// its gradient (the lower layer's thickness is eta1 minus the linear bottom), a momentum its
// derivative along its own direction and that derivative's gradient (so the two momentum threads
// of a layer sum to div(h U)).  Radon's 7-point rule is exact for these degree-5 products.
// cell geometry for the interior evaluations: scaled vertices and the cell mean of P^3's
// non-constant part (as in recon_cell)
template <typename R>
struct SrcGeo {
    R vx[3], vy[3], mean_const, ihs;
};

template <typename R>
__device__ inline void src_geo(const MeshDev &m, int64_t c, const R a[9], R hs, SrcGeo<R> &g)
{
    const R *vt = tab<R>(m.vtx);
    R mxx = 0, mxy = 0, myy = 0, mx3 = 0, mx2y = 0, mxy2 = 0, my3 = 0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const R vx = vt[(2 * k) * m.T + c], vy = vt[(2 * k + 1) * m.T + c];
        g.vx[k] = vx;
        g.vy[k] = vy;
        mxx += vx * vx;
        mxy += vx * vy;
        myy += vy * vy;
        mx3 += vx * vx * vx;
        mx2y += vx * vx * vy;
        mxy2 += vx * vy * vy;
        my3 += vy * vy * vy;
    }
    const R c12 = R(1) / R(12), c30 = R(1) / R(30);
    g.mean_const = a[2] * mxx * c12 + a[3] * mxy * c12 + a[4] * myy * c12 + a[5] * mx3 * c30 +
                   a[6] * mx2y * c30 + a[7] * mxy2 * c30 + a[8] * my3 * c30;
    g.ihs = div_(R(1), hs);
}

// three numbers of variable v at the scaled point (x, y), see the block comment above
template <typename R>
__device__ inline void src_point(const MeshDev &m, int v, bool thick, int64_t c, const R a[9],
                                 const ReconComb<R> &cb, const SrcGeo<R> &g, R hs, R x, R y, R o[3])
{
    const R ihs = g.ihs;
    const R Px = a[0] + 2 * a[2] * x + a[3] * y + 3 * a[5] * x * x + 2 * a[6] * x * y + a[7] * y * y;
    const R Py = a[1] + a[3] * x + 2 * a[4] * y + a[6] * x * x + 2 * a[7] * x * y + 3 * a[8] * y * y;
    if (thick) {
        const R P = a[0] * x + a[1] * y + a[2] * x * x + a[3] * x * y + a[4] * y * y + a[5] * x * x * x +
                    a[6] * x * x * y + a[7] * x * y * y + a[8] * y * y * y - g.mean_const;
        o[0] = cb.theta * (cb.ratio * P + cb.sbx * x + cb.sby * y);
        o[1] = cb.theta * (cb.ratio * Px + cb.sbx) * ihs;
        o[2] = cb.theta * (cb.ratio * Py + cb.sby) * ihs;
        if (v == 3) {  // h1 = eta1 - B: remove the linear bottom's deviation and slope
            const R gBx = (R)m.gB[c], gBy = (R)m.gB[m.T + c];
            o[0] -= hs * (gBx * x + gBy * y);
            o[1] -= gBx;
            o[2] -= gBy;
        }
    } else {
        const R Pxx = 2 * a[2] + 6 * a[5] * x + 2 * a[6] * y;
        const R Pxy = a[3] + 2 * a[6] * x + 2 * a[7] * y;
        const R Pyy = 2 * a[4] + 2 * a[7] * x + 6 * a[8] * y;
        const bool dx = (v == 1 || v == 4);  // x-momentum: d/dx; y-momentum: d/dy
        const R i2 = ihs * ihs;
        o[0] = dx ? (cb.ratio * Px + cb.sbx) * ihs : (cb.ratio * Py + cb.sby) * ihs;
        o[1] = cb.ratio * (dx ? Pxx : Pxy) * i2;
        o[2] = cb.ratio * (dx ? Pxy : Pyy) * i2;
    }
}

// the learned indicator inside the reconstruction: bf16 weight matrices, FP32 parameters, logit
// threshold, and where to leave the decisions (1 = linear weights) for inspection
struct IndArgs {
    const short *W1b, *W2b;
    const float *P;
    float thr;
    uint8_t *mask;
};

// IND: the learned indicator decides per cell whether the smoothness indicators are computed.
// IND = 1: its 44 features come from the right-hand sides the block has gathered anyway; one wave
// evaluates the network for the block's 32 cells on the matrix cores and the decisions go to
// ind.mask.  IND = 2: the decisions are read from ind.mask (the network ran on the step's first
// stage, the second reuses them).
// SRC = 1: the block then also forms the interior correction of the higher-order layer coupling
// (src[8][T], see src_point) in the LDS space the records used.
// whether cell c lies in the front band of the layer of variable v (h2 for v < 3, the lower layer
// eta1 - B for v >= 3); a wall ghost holds its cell's mirrored state and bottom
__device__ inline bool wd_band(const MeshDev &m, const Phys &p, const double *__restrict__ Wh, int v, int64_t c)
{
    const int64_t T = m.T, TG = m.T + m.NG;
    const bool lower = v >= 3;
    const double *H = Wh + (lower ? TG : 0);
    double hk[4];
#pragma unroll
    for (int l = 0; l < 4; l++) {
        const int64_t i = l == 0 ? c : (int64_t)GKS_IX(m.sten[(l - 1) * T + c], TG);
        double h = H[i];
        if (lower) h -= m.Bbar[i < T ? i : (int64_t)GKS_IX(m.gsrc[i - T], T)];
        hk[l] = h;
    }
    const double hmax = fmax(fmax(hk[0], hk[1]), fmax(hk[2], hk[3])), thin = WD_THIN * p.h_dry;
    bool band = false;
#pragma unroll
    for (int l = 0; l < 4; l++) band = band || hk[l] < thin || hk[l] < WD_FRONT * hmax;
    // the lower layer thinner than the bottom's rise across the cell (scale sqrt(2 area)): its
    // shoreline lies inside the cell (a partially flooded cell)
    if (lower) {
        const double gx = m.gB[c], gy = m.gB[T + c];
        band = band || hk[0] < sqrt(2.0 * m.area[c]) * sqrt(gx * gx + gy * gy);
    }
    return band;
}

template <typename R, int IND, int SRC = 0>
__global__ void __launch_bounds__(192) k_recon(MeshDev m, Phys p, const double *__restrict__ Wh,
                                               const R *__restrict__ Wm, const R *__restrict__ gW, IndArgs ind,
                                               GpRecs<R> rec, R *__restrict__ r0, R *__restrict__ src)
{
    // LDS: first the block's 32 least-squares operators, loaded once with coalesced reads and
    // shared by the six variable threads of each cell; then, in the same space, the indicator's
    // features and hidden activations (with IND); then the block's 32 x 6 Gauss-point records
    // (heads, then tails), each array written out as one contiguous span
    constexpr int NR = RECON_CELLS * 6;
    // the operator is staged in two parts (rows of coefficients 0..4, then the other 153 - ROWS1
    // rows of 5..8), both loaded at once into registers, so that the LDS holds only the larger part
    constexpr int ROWS1 = 5 * 17;
    constexpr int MBYTES = ROWS1 * RECON_CELLS * (int)sizeof(R);
    constexpr int OBYTES = NR * (int)(sizeof(GpHead<R>) + sizeof(GpTail<R>));
    constexpr int IBYTES = IND == 1 ? RECON_CELLS * (FB + HB) * 2 + 4 * RECON_CELLS * 8 + RECON_CELLS : 0;
    constexpr int B1 = MBYTES > OBYTES ? MBYTES : OBYTES, LBYTES = B1 > IBYTES ? B1 : IBYTES;
    __shared__ uint4 lds[(LBYTES + 15) / 16];
    R *Ms = reinterpret_cast<R *>(lds);
    GpHead<R> *th = reinterpret_cast<GpHead<R> *>(lds);
    GpTail<R> *tt = reinterpret_cast<GpTail<R> *>(th + NR);
    const int lane = threadIdx.x & 31, wv = threadIdx.x >> 5;
    const int v = (wv == 0) ? 0 : (wv == 1) ? 3 : (wv == 2) ? 1 : (wv == 3) ? 2 : (wv == 4) ? 4 : 5;
    const bool thick = (v == 0 || v == 3);
    const int64_t c0 = xcd_block() * RECON_CELLS, c = c0 + lane;
    const int64_t T = m.T;
    const int ncell = T - c0 < RECON_CELLS ? (int)(T - c0) : RECON_CELLS;
    const bool valid = lane < ncell;
    // the cell's own gathers are issued first, so that they overlap the operator staging
    ReconRhs<R> q;
    if (valid) recon_rhs<R>(m, Wh, Wm, gW, v, thick, c, q);
    R a[9];
    {
        // every load of the staging is issued before the first LDS write
        constexpr int NM = 153 * RECON_CELLS, NM1 = ROWS1 * RECON_CELLS, IT = (NM + 191) / 192;
        const R *M = tab<R>(m.M);
        R buf[IT];
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int i = (int)threadIdx.x + 192 * it, l = i % RECON_CELLS;
            buf[it] = (i < NM && l < ncell) ? M[c0 * 153 + i] : R(0);  // block-major operators
        }
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int i = (int)threadIdx.x + 192 * it;
            if (i < NM1) Ms[i] = buf[it];
        }
        __syncthreads();
        if (valid) recon_coeffs<0, 5, R>(q, Ms + lane, a);
        __syncthreads();
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int i = (int)threadIdx.x + 192 * it;
            if (i >= NM1 && i < NM) Ms[i - NM1] = buf[it];
        }
        __syncthreads();
        if (valid) recon_coeffs<5, 9, R>(q, Ms + lane, a);
    }
    bool lin = false;
    if constexpr (IND == 2) lin = valid && ind.mask[c] != 0;
    if constexpr (IND == 1) {
        __syncthreads();  // the operators are no longer needed: the space holds the network's data
        short(*feat)[FB] = reinterpret_cast<short(*)[FB]>(lds);
        short(*hid)[HB] = reinterpret_cast<short(*)[HB]>(&feat[RECON_CELLS][0]);
        double *msc = reinterpret_cast<double *>(&hid[RECON_CELLS][0]);  // [4][32] momentum differences
        uint8_t *skip = reinterpret_cast<uint8_t *>(msc + 4 * RECON_CELLS);
        // thickness threads: their field's 17 features and size; momentum threads: their largest
        // stencil difference
        if (thick) {
            const int f = v == 3 ? 0 : 1;
            float x[18];
            if (valid) {
                const double h = f == 0 ? q.Q0h - m.Bbar[c] : q.Q0h;
                thick_features<R>(q.rhs, q.Q0h, h, x);
            } else {
#pragma unroll
                for (int k = 0; k < 18; k++) x[k] = 0.f;
            }
#pragma unroll
            for (int k = 0; k < 17; k++) feat[lane][17 * f + k] = to_bf16(x[k]);
            feat[lane][34 + f] = to_bf16(x[17]);
            if (f == 0) {
#pragma unroll
                for (int k = 0; k < 6; k++) feat[lane][38 + k] = to_bf16(valid ? m.igeo[k * T + c] : 0.f);
            } else {
#pragma unroll
                for (int k = MLP_IN; k < MLP_K; k++) feat[lane][k] = 0;
            }
        } else {
            msc[mom_slot(v) * RECON_CELLS + lane] = valid ? max_diff<R>(q.rhs) : 0.0;
        }
        __syncthreads();
        if (thick) {  // the layer's momentum feature: lower layer with eta1, upper with h2
            const int f = v == 3 ? 0 : 1, s0 = f == 0 ? 2 : 0;
            float y = 0.f;
            if (valid) {
                const double h = f == 0 ? q.Q0h - m.Bbar[c] : q.Q0h;
                const double sm = fmax(msc[s0 * RECON_CELLS + lane], msc[(s0 + 1) * RECON_CELLS + lane]);
                y = mom_feature(sm, h, p.G);
            }
            feat[lane][36 + f] = to_bf16(y);
        }
        __syncthreads();
        // waves 0 and 1 take one block of 32 hidden units each
        const int hw = threadIdx.x >> 6, hl = threadIdx.x & 63;
        if (hw < 2) mlp_layer1(feat, hid, hl, hw, ind.W1b, ind.P);
        __syncthreads();
        float *zp = reinterpret_cast<float *>(msc);  // [2][32] partial logits (msc is no longer read)
        if (hw < 2) {
            float z[16];
            mlp_layer2(hid, hl, hw, ind.W2b, ind.P, z);
            if ((hl & 31) == 0) {
                const int half = hl >> 5;
#pragma unroll
                for (int r = 0; r < 16; r++) zp[hw * RECON_CELLS + 8 * (r / 4) + 4 * half + (r % 4)] = z[r];
            }
        }
        __syncthreads();
        if (threadIdx.x < RECON_CELLS) {
            const float z = zp[threadIdx.x] + zp[RECON_CELLS + threadIdx.x] + ind.P[OFF_B3];
            skip[threadIdx.x] = z > ind.thr ? 1 : 0;
        }
        __syncthreads();
        lin = skip[lane] != 0;
        if (threadIdx.x < 32 && valid && ind.mask) ind.mask[c] = lin ? 1 : 0;
    }
    ReconOut<R> out;
    ReconComb<R> comb;
    if (valid) recon_cell<R>(m, p, lin, r0, v, thick, c, q, a, out, comb);
    // wet/dry layers exclude the indicator and the higher-order coupling (the library rejects the
    // combinations), so only the plain instance carries the band test and its registers
    if (IND == 0 && SRC == 0 && p.h_dry > 0 && valid && wd_band(m, p, Wh, v, c)) {
        // front band: the layer's cell average, thickness constant (the lower layer's level follows
        // the bottom), momentum the thickness times the desingularised velocity; r0 = 0 marks it
        const R *vt = tab<R>(m.vtx);
        const R gs[2] = {R(0.5 - 0.28867513459481288225), R(0.5 + 0.28867513459481288225)};
        const double gBx = v == 3 ? m.gB[c] : 0.0, gBy = v == 3 ? m.gB[T + c] : 0.0;
        const double mv = thick ? 0.0 : q.hl * wd_velocity(q.hl, (double)q.Q0, p.h_dry);
#pragma unroll
        for (int k = 0; k < 3; k++)
#pragma unroll
            for (int g = 0; g < 2; g++) {
                const int k1 = (k + 1) % 3, slot = 2 * k + g;
                const R x = vt[(2 * k) * T + c] + gs[g] * (vt[(2 * k1) * T + c] - vt[(2 * k) * T + c]);
                const R y = vt[(2 * k + 1) * T + c] + gs[g] * (vt[(2 * k1 + 1) * T + c] - vt[(2 * k + 1) * T + c]);
                out.v[slot] = thick ? q.Q0h + (double)q.hs * (gBx * (double)x + gBy * (double)y) : mv;
                out.gx[slot] = (R)gBx;
                out.gy[slot] = (R)gBy;
            }
        if (v == 3) r0[c] = R(0);
        if (v == 0) r0[T + c] = R(0);
    }
    __syncthreads();  // the space becomes the record tile
    if (valid) {
#pragma unroll
        for (int slot = 0; slot < 6; slot++) {
            const int i = 6 * lane + slot;
            if (thick)
                th[i].h[v == 3] = out.v[slot];
            else
                th[i].q[mom_slot(v)] = (R)out.v[slot];
            tt[i].g[2 * v] = out.gx[slot];
            tt[i].g[2 * v + 1] = out.gy[slot];
        }
    }
    __syncthreads();
    // copy out: 16-byte words of the valid cells' records
    const int nh = (int)(ncell * 6 * sizeof(GpHead<R>) / 16), nt = (int)(ncell * 6 * sizeof(GpTail<R>) / 16);
    const uint4 *sh = reinterpret_cast<const uint4 *>(th), *st = reinterpret_cast<const uint4 *>(tt);
    uint4 *dh = reinterpret_cast<uint4 *>(rec.head + 6 * c0), *dtl = reinterpret_cast<uint4 *>(rec.tail + 6 * c0);
    for (int i = threadIdx.x; i < nh; i += blockDim.x) dh[i] = sh[i];
    for (int i = threadIdx.x; i < nt; i += blockDim.x) dtl[i] = st[i];
    if constexpr (SRC == 1) {
        // Radon's 7-point rule (degree 5): the centroid, then two orbits (b, a, a) of barycentrics
        const R A1 = R(0.101286507323456338800987361915), B1 = R(0.797426985353087322398025276170);
        const R A2 = R(0.470142064105115089770441209513), B2 = R(0.059715871789769820459117580973);
        const R W0 = R(0.225), W1 = R(0.125939180544827152595683945500), W2 = R(0.132394152788506180737649387833);
        // [point of the batch][variable][3][cell]: four points, then three
        static_assert(4 * 6 * 3 * RECON_CELLS * (int)sizeof(R) <= LBYTES, "interior values exceed the LDS tile");
        R *sv = reinterpret_cast<R *>(lds);
        SrcGeo<R> geo;
        if (valid) src_geo<R>(m, c, a, q.hs, geo);
        // group 0: lower (h1 - mean) grad h2; 1: upper (h2 - mean) grad h1; 2 and 3: their rates
        const int gq = wv;
        const int ha = (gq == 0 || gq == 2) ? 3 : 0, hb = 3 - ha;  // deviation of h_a, gradient of h_b
        const int ta = ha == 3 ? 4 : 1, tb = ha == 3 ? 1 : 4;      // momenta of layer a, of layer b
        R acc[7] = {0, 0, 0, 0, 0, 0, 0};
        // loops kept rolled: the reconstruction's register budget (4 waves per SIMD) is the limit
#pragma unroll 1
        for (int b = 0; b < 2; b++) {
            const int q0 = 4 * b, nq = b == 0 ? 4 : 3;
            __syncthreads();  // the previous contents of the space have been read
            if (valid) {
#pragma unroll 1
                for (int j = 0; j < nq; j++) {
                    const int qi = q0 + j;
                    R l0, l1, l2;
                    if (qi == 0) {
                        l0 = l1 = l2 = R(1) / R(3);
                    } else if (qi <= 3) {
                        l0 = qi == 1 ? B1 : A1;
                        l1 = qi == 2 ? B1 : A1;
                        l2 = qi == 3 ? B1 : A1;
                    } else {
                        l0 = qi == 4 ? B2 : A2;
                        l1 = qi == 5 ? B2 : A2;
                        l2 = qi == 6 ? B2 : A2;
                    }
                    const R x = l0 * geo.vx[0] + l1 * geo.vx[1] + l2 * geo.vx[2];
                    const R y = l0 * geo.vy[0] + l1 * geo.vy[1] + l2 * geo.vy[2];
                    R o3[3];
                    src_point<R>(m, v, thick, c, a, comb, geo, q.hs, x, y, o3);
#pragma unroll
                    for (int k = 0; k < 3; k++) sv[((j * 6 + v) * 3 + k) * RECON_CELLS + lane] = o3[k];
                }
            }
            __syncthreads();
            if (valid && gq < 4) {
#pragma unroll 1
                for (int j = 0; j < nq; j++) {
                    const int qi = q0 + j;
                    const R wq = qi == 0 ? W0 : qi <= 3 ? W1 : W2;
                    auto at = [&](int vv, int k) { return sv[((j * 6 + vv) * 3 + k) * RECON_CELLS + lane]; };
                    const R f = at(ha, 0), gx = at(hb, 1), gy = at(hb, 2);
                    if (gq < 2) {
                        acc[0] += wq * f * gx;
                        acc[1] += wq * f * gy;
                    } else {
                        const R tau = -(at(ta, 0) + at(ta + 1, 0));
                        const R gtx = -(at(tb, 1) + at(tb + 1, 1)), gty = -(at(tb, 2) + at(tb + 1, 2));
                        acc[0] += wq * tau * gx;  // sum w tau_a grad h_b
                        acc[1] += wq * tau * gy;
                        acc[2] += wq * gx;        // sum w grad h_b
                        acc[3] += wq * gy;
                        acc[4] += wq * tau;       // mean of tau_a
                        acc[5] += wq * f * gtx;   // sum w (h_a - mean) grad tau_b
                        acc[6] += wq * f * gty;
                    }
                }
            }
        }
        if (valid && gq < 4) {
            // rates: sum w (tau_a - mean tau_a) grad h_b + sum w (h_a - mean) grad tau_b
            const R o0 = gq < 2 ? acc[0] : acc[0] - acc[4] * acc[2] + acc[5];
            const R o1 = gq < 2 ? acc[1] : acc[1] - acc[4] * acc[3] + acc[6];
            src[(2 * gq) * T + c] = o0;
            src[(2 * gq + 1) * T + c] = o1;
        }
    }
}

// --------------------------------------------------------------------------------------------
// interface force modelling (Sec. 2.3): edge-centre height of eta1 (lower-layer velocity) and of
// h2 (upper-layer velocity) from the two Gauss points' convex combinations (FP64: cheap, and the
// plane through them must be flat at rest)

// Cells whose plane gradient the flux can read: the force model blends it in with weight 1 - w,
// w = min(1, omega0/d0 of both sides) taken as 1 within 1e-12 of it, so only next to a cell whose
// weight ratio is below 1 - 1e-12.  A face neighbour beyond a wall is the cell's own mirror image.
template <typename R>
__global__ void k_need(MeshDev m, const R *__restrict__ r0, uint8_t *__restrict__ need)
{
    const int64_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= m.T) return;
    const int64_t T = m.T;
    bool bad = (double)r0[c] < W_ONE || (double)r0[T + c] < W_ONE;
#pragma unroll
    for (int l = 0; l < 3; l++) {
        const int32_t i = GKS_IX(m.sten[l * T + c], T + m.NG);
        if (i < T) bad = bad || (double)r0[i] < W_ONE || (double)r0[T + i] < W_ONE;
    }
    need[c] = bad ? 1 : 0;
}

template <typename R>
__global__ void k_hhat(MeshDev m, Phys p, const GpHead<R> *__restrict__ head, const uint8_t *__restrict__ need,
                       double *__restrict__ hmid)
{
    int64_t e = xcd_block() * blockDim.x + threadIdx.x;
    if (e >= m.E) return;
    const int64_t E = m.E;
    const int32_t L = GKS_IX(m.eL[e], m.T), Rc = m.eR[e] >= 0 ? GKS_IX(m.eR[e], m.T) : m.eR[e],
                  sl = m.eslot[e];
    if (!need[L] && (Rc < 0 || !need[Rc])) return;  // no plane gradient uses this edge
    const int kL = GKS_IX(sl & 3, 3), kR = GKS_IX(sl >> 2, 3);
    const R *en = tab<R>(m.en);
    const double nx = en[e], ny = en[E + e];
    double acc0 = 0, acc1 = 0;
#pragma unroll
    for (int g = 0; g < 2; g++) {
        const double Bg = m.eBgp[g * E + e];
        const int sL = 2 * kL + g, sR = 2 * kR + 1 - g;
        const GpHead<R> ql = head[6 * (int64_t)L + sL];
        GpHead<R> qr = ql;
        if (Rc >= 0) qr = head[6 * (int64_t)Rc + sR];
#pragma unroll
        for (int f = 0; f < 2; f++) {
            // f = 0: eta1 with the lower layer's momentum; f = 1: h2 with the upper layer's
            const int hq = f == 0 ? 1 : 0, mq = f == 0 ? 2 : 0;
            // a dry side (thickness at or below h_dry, or not positive) has no velocity
            const double zl = ql.h[hq];
            const double hl = f == 0 ? zl - Bg : zl;
            const double unl = (hl > p.h_dry && hl > 0) ? ((double)ql.q[mq] * nx + (double)ql.q[mq + 1] * ny) / hl : 0.0;
            double zr, hr, unr;
            if (Rc >= 0) {
                zr = qr.h[hq];
                hr = f == 0 ? zr - Bg : zr;
                unr = (hr > p.h_dry && hr > 0) ? ((double)qr.q[mq] * nx + (double)qr.q[mq + 1] * ny) / hr : 0.0;
            } else {  // mirror state across a wall; the same state across a free boundary
                zr = zl;
                hr = hl;
                unr = Rc == -1 ? -unl : unl;
            }
            // reading: xi is the kinetic fraction of particles moving from left to right (one half
            // when both sides are dry)
            const double lb = 2.0 / (p.G * (hl + hr));
            const double xi = (hl + hr > 0) ? 0.5 * erfc(-sqrt(lb) * 0.5 * (unl + unr)) : 0.5;
            const double hh = xi * zl + (1 - xi) * zr;
            if (f == 0) acc0 += 0.5 * hh; else acc1 += 0.5 * hh;
        }
    }
    hmid[e] = acc0;
    hmid[E + e] = acc1;
}

// gradient of the plane through the three edge-centre heights (Green-Gauss, exact for planes)
__global__ void k_plane(MeshDev m, const uint8_t *__restrict__ need, const double *__restrict__ hmid,
                        double *__restrict__ gP1)
{
    int64_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= m.T || !need[c]) return;
    const int64_t T = m.T, E = m.E;
    double s[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const int32_t code = m.cedge[k * T + c];
        const int64_t e = GKS_IX(code >= 0 ? code : ~code, m.E);
        const double gx = m.gg[(2 * k) * T + c], gy = m.gg[(2 * k + 1) * T + c];
        const double h0 = hmid[e], h1 = hmid[E + e];
        s[0] += gx * h0;
        s[1] += gy * h0;
        s[2] += gx * h1;
        s[3] += gy * h1;
    }
#pragma unroll
    for (int i = 0; i < 4; i++) gP1[i * T + c] = s[i];
}

// --------------------------------------------------------------------------------------------
// gas-kinetic evolution at one Gauss point for one layer (Sec. 2.2, Eq. SWE-2nd-order)
//
// Local frame: u along the edge normal.  Micro-slopes are Maxwellian-consistent (reading):
// a = alpha |c|^2 + beta c_u + gamma c_v with alpha = lam dh/h, beta = 2 lam dU, gamma = 2 lam dV,
// c = (u - U, v - V); the force term is -2 lam Phi . c.  Moments of the polynomial
//   P = a_n u + a_t v - 2 lam Phi . c
// over a (half-)Maxwellian are closed forms in the u-moments M_k and the centred v-moments.

// For the lower layer the bottom slope gB enters twice: in dh = d(eta1) - gB and in the force
// -G gB.  The |c|^2 part of the slope and the force part that carry gB are taken out of the
// polynomial P and added as the closed-form moments of
//   T_B = (gB_n/h)(2 c_u - lam |c|^2 u) + (gB_t/h)(2 c_v - lam |c|^2 v)
// (bottom_moments), whose momentum moments are exactly zero at rest in any precision, instead of
// two large terms that cancel.  The side record therefore carries the slopes of h (for beta,
// gamma) and of eta1 (for alpha), and the acceleration without its bottom part.
template <typename R>
struct SideL {
    R h, U, V;                    // state
    R ih;                         // 1/h
    R hn, ht, mnn, mnt, mtn, mtt;  // d/dn, d/dt of h, h U_n, h U_t
    R en, et;                     // d/dn, d/dt of the level whose |c|^2 slope enters P (h, or eta1)
    R pn, pt;                     // acceleration (without the bottom part for the lower layer)
};

template <typename R>
struct Slope {
    R an, bn, gn, at, bt, gt;
};

// ih = 1/h of the Maxwellian the slopes belong to
template <typename R>
__host__ __device__ inline Slope<R> slope_of(const SideL<R> &s, R ih, R U, R V, R lam)
{
    Slope<R> r;
    r.an = lam * s.en * ih;
    r.bn = 2 * lam * (s.mnn - U * s.hn) * ih;
    r.gn = 2 * lam * (s.mtn - V * s.hn) * ih;
    r.at = lam * s.et * ih;
    r.bt = 2 * lam * (s.mnt - U * s.ht) * ih;
    r.gt = 2 * lam * (s.mtt - V * s.ht) * ih;
    return r;
}

// out += <u^e psi T_B> for psi = (1, u, v) over a (half) Maxwellian with means (U, V), lam,
// th = 1/(2 lam) and u-moments M (the thickness cancels against the 1/h of T_B).  Closed forms
// from the moment recurrence M_{k+2} = U M_{k+1} + (k+1) th M_k and lam th = 1/2.
template <typename R>
__host__ __device__ inline void bottom_moments(R gn, R gt, R U, R V, R lam, R th, const R *M, int e, R *out)
{
    auto In = [&](int k) { return R(0.5 * (1 - k)) * M[k + 1] + R(0.5 * (k - 3)) * U * M[k]; };
    auto N1 = [&](int k) { return M[k + 1] - U * M[k]; };
    auto Jt = [&](int k) { return -V * (R(0.5 * (k + 2)) * M[k] - lam * U * N1(k)); };
    const R VV = V * V;
    auto Jv = [&](int k) {
        return M[k] * (R(0.5) * th - R(0.5) * VV - (VV + th) * R(0.5 * (k + 1))) + lam * U * (VV + th) * N1(k);
    };
    out[0] += gn * In(e) + gt * Jt(e);
    out[1] += gn * In(e + 1) + gt * Jt(e + 1);
    out[2] += gn * V * In(e) + gt * Jv(e);
}

// u-moments M_0..M_5 of the Gaussian (mean U, variance th = 1/(2 lam)) restricted to a half line
template <typename R>
__host__ __device__ inline void u_moments(R U, R th, R m0, R m1, R *M)
{
    M[0] = m0;
    M[1] = m1;
#pragma unroll
    for (int k = 2; k < 6; k++) M[k] = U * M[k - 1] + R(k - 1) * th * M[k - 2];
}

// moments of P (slope sl, force (pn, pt)) over a half Maxwellian with thickness h, means (U, V),
// lam, th = 1/(2 lam), u-moments M.  e = 0: <psi P>, e = 1: <u psi P>.
template <typename R>
__host__ __device__ inline void poly_moments(const Slope<R> &sl, R pn, R pt, R h, R U, R V, R lam, R th, const R *M, int e,
                                    R *out)
{
    R N1[5], N2[4];
#pragma unroll
    for (int k = 0; k < 5; k++) N1[k] = M[k + 1] - U * M[k];
#pragma unroll
    for (int k = 0; k < 4; k++) N2[k] = N1[k + 1] - U * N1[k];
    const R fn = sl.bt * V - 2 * lam * pn;
    const R q2 = sl.at * V + sl.gt;
    R Q[2];
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const int j = e + i;
        Q[i] = sl.an * N2[j + 1] + sl.at * V * N2[j] + sl.bn * N1[j + 1] + fn * N1[j] +
               th * (sl.an * M[j + 1] + q2 * M[j]);
    }
    const R Rv = th * (sl.gn * M[e + 1] + (sl.gt * V - 2 * lam * pt) * M[e] + sl.at * N2[e] + sl.bt * N1[e]) +
                 3 * th * th * sl.at * M[e];
    out[0] = h * Q[0];
    out[1] = h * Q[1];
    out[2] = h * (V * Q[0] + Rv);
}

// a*b + c*d with both products rounded before the sum (no fused multiply-add): for mirror-image
// left/right contributions the result is then exactly zero, as a contracted fma(a, b, c*d) is not
template <typename R>
__host__ __device__ inline R sum_products(R a, R b, R c, R d)
{
#pragma clang fp contract(off)
    const R p = a * b, q = c * d;
    return p + q;
}

__host__ __device__ inline float erfc_(float x) { return erfcf(x); }
__host__ __device__ inline double erfc_(double x) { return erfc(x); }
__host__ __device__ inline float erf_(float x) { return erff(x); }
__host__ __device__ inline double erf_(double x) { return erf(x); }
__host__ __device__ inline float exp_(float x) { return expf(x); }
__host__ __device__ inline double exp_(double x) { return exp(x); }
__host__ __device__ inline float sqrt_(float x) { return sqrtf(x); }
__host__ __device__ inline double sqrt_(double x) { return sqrt(x); }

// Outputs (local frame): F0 with the hydrostatic term 1/2 G hb^2 removed from its normal-momentum
// component, Ft, Wb (hb_dev = hb - (hL + hR)/2 in slot 0), Wbt.  hbase = (hL + hR)/2 in FP64; the
// interface thickness is hbase + hb_dev.
// AM selects the constants alpha_{k,m} of the acceleration term (Sec. 2.2, Eq. SWE-2nd-order):
// AM = 0 the weights read for these slopes (below), AM = 1 the paper's printed (1, 3/4, 1/4) on the
// flux moments of the acceleration term in both the equilibrium and the initial distributions'
// parts, 1 on the state moments.
// Wet/dry (h_dry > 0): a vacuum side comes with h = 1/h = U = V = 0 and no slopes, so that each of
// its terms is an exact zero; an interface whose equilibrium thickness hbase + hdev is at or below
// h_dry gives zero outputs and returns true (dry).  order1: first order in time, F0 the step's mean
// flux F(dt)/dt and Ft = 0 (the caller passes sides without slopes and accelerations).
template <typename R, int AM = 0, int WD = 0>
__host__ __device__ inline bool gks_point(const SideL<R> &sl, const SideL<R> &sr, double hbase, R gBn, R gBt, R G, R eps,
                                 R eps_num, R dt, R *F0, R *Ft, R *Wb, R *Wbt, bool order1 = false,
                                 double h_dry = 0.0)
{
    // the bottom's moments are added unconditionally: for the upper layer (and a flat bottom) the
    // slope is zero and they add exact zeros.  A branch on the slope diverges inside every wave
    // (lanes of both layers alternate) and kept 56 more registers live (222 against 166 in FP64:
    // 2 instead of 3 waves per SIMD).
    // reciprocals formed once (lam = 1/(G h)); 1/(2 sqrt(pi lam)) = sqrt(lam) th / sqrt(pi)
    const R iG = div_(R(1), G), ihL = sl.ih, ihR = sr.ih;
    const R lamL = iG * ihL, lamR = iG * ihR;
    const R thL = R(0.5) * G * sl.h, thR = R(0.5) * G * sr.h;
    const R ispi = R(0.56418958354775628695);  // 1/sqrt(pi)
    R ML[6], MR[6], eL, eR;
    // half-space masses from one error function per Gaussian: 1/2 erfc(-x) = 1/2 (1 + erf(x))
    // (exactly 1/2 at rest; where erf(x) is close to -1 the lost relative digits of the tiny mass
    // are below the absolute rounding of the moments it enters)
    {
        const R sq = sqrt_(lamL);
        eL = erf_(sq * sl.U);  // 2 (M0 - 1/2)
        const R m0 = R(0.5) + R(0.5) * eL;
        const R ex = exp_(-lamL * sl.U * sl.U) * sq * thL * ispi;
        u_moments(sl.U, thL, m0, sl.U * m0 + ex, ML);
    }
    {
        const R sq = sqrt_(lamR);
        eR = -erf_(sq * sr.U);
        const R m0 = R(0.5) + R(0.5) * eR;  // 1/2 erfc(x)
        const R ex = exp_(-lamR * sr.U * sr.U) * sq * thR * ispi;
        u_moments(sr.U, thR, m0, sr.U * m0 - ex, MR);
    }
    // interface equilibrium state: thickness as an FP64 base plus a deviation that is 0 at rest
    const R hdev = R(0.5) * (sl.h * eL + sr.h * eR);
    if constexpr (WD) {
        if (!(hbase + (double)hdev > h_dry)) {  // no particles at the interface
#pragma unroll
            for (int i = 0; i < 3; i++) F0[i] = Ft[i] = Wb[i] = Wbt[i] = R(0);
            return true;
        }
    }
    const R hb = (R)(hbase + (double)hdev);
    const R wb1 = sum_products(sl.h, ML[1], sr.h, MR[1]);
    const R wb2 = sum_products(sl.h * ML[0], sl.V, sr.h * MR[0], sr.V);
    // brackets of the initial (side) distributions first, so that the sides' moments are dead
    // before the interface equilibrium's are formed.  B4 = (.., D4 + P + B4p, ..)
    R B4[3], B5[3], t1[3], t2[3];
    B4[0] = wb1;
    // normal momentum: h U M1 parts plus the pressure-like part's excess over 1/2 G hb^2
    // (h^2 M0 summed over the sides minus hb^2: exactly zero at rest)
    {
        const R sq2 = sum_products(sl.h * sl.h, ML[0], sr.h * sr.h, MR[0]);
        const R hb2 = sum_products(hb, hb, R(0), R(0));
        B4[1] = sum_products(sl.h * sl.U, ML[1], sr.h * sr.U, MR[1]) + R(0.5) * G * (sq2 - hb2);
    }
    B4[2] = sum_products(sl.h * ML[1], sl.V, sr.h * MR[1], sr.V);
    {
        const Slope<R> aL = slope_of(sl, ihL, sl.U, sl.V, lamL), aR = slope_of(sr, ihR, sr.U, sr.V, lamR);
        poly_moments(aL, sl.pn, sl.pt, sl.h, sl.U, sl.V, lamL, thL, ML, 1, t1);
        poly_moments(aR, sr.pn, sr.pt, sr.h, sr.U, sr.V, lamR, thR, MR, 1, t2);
        bottom_moments(gBn, gBt, sl.U, sl.V, lamL, thL, ML, 1, t1);
        bottom_moments(gBn, gBt, sr.U, sr.V, lamR, thR, MR, 1, t2);
#pragma unroll
        for (int i = 0; i < 3; i++) B5[i] = t1[i] + t2[i];
        if constexpr (AM == 1) {
            // the paper's constants on the initial distributions' acceleration moments: (3/4 - 1) on
            // <u u>, (1/4 - 1) on <u v>; the moments are -2 Phi_n N1_2 / G and
            // -2 (V Phi_n N1_1 + th Phi_t M_1) / G over each side's own half Maxwellian
            const R pLn = sl.pn - G * gBn, pLt = sl.pt - G * gBt, pRn = sr.pn - G * gBn, pRt = sr.pt - G * gBt;
            const R L1 = ML[2] - sl.U * ML[1], L2 = ML[3] - sl.U * ML[2];
            const R R1 = MR[2] - sr.U * MR[1], R2 = MR[3] - sr.U * MR[2];
            B5[1] += R(0.5) * iG * sum_products(pLn, L2, pRn, R2);
            B5[2] += R(1.5) * iG * (sl.V * pLn * L1 + thL * pLt * ML[1] + sr.V * pRn * R1 + thR * pRt * MR[1]);
        }
    }
    const R ihb = div_(R(1), hb);
    const R Ub = wb1 * ihb, Vb = wb2 * ihb;
    const R lamb = iG * ihb, thb = R(0.5) * G * hb;
    R Mp[6], Mm[6];
    {
        const R sq = sqrt_(lamb);
        const R eb = erf_(sq * Ub);
        const R m0p = R(0.5) + R(0.5) * eb, m0m = R(0.5) - R(0.5) * eb;
        const R ex = exp_(-lamb * Ub * Ub) * sq * thb * ispi;
        u_moments(Ub, thb, m0p, Ub * m0p + ex, Mp);
        u_moments(Ub, thb, m0m, Ub * m0m - ex, Mm);
    }
    const Slope<R> bL = slope_of(sl, ihb, Ub, Vb, lamb), bR = slope_of(sr, ihb, Ub, Vb, lamb);
    // time slope of the interface equilibrium from compatibility
    R wt[3];
    poly_moments(bL, sl.pn, sl.pt, hb, Ub, Vb, lamb, thb, Mp, 0, t1);
    poly_moments(bR, sr.pn, sr.pt, hb, Ub, Vb, lamb, thb, Mm, 0, t2);
    bottom_moments(gBn, gBt, Ub, Vb, lamb, thb, Mp, 0, t1);
    bottom_moments(gBn, gBt, Ub, Vb, lamb, thb, Mm, 0, t2);
    // well-balance weights of the acceleration in the equilibrium part (Sec. 2.2, the constants
    // alpha_{k,m} of Eq. SWE-2nd-order), read as the weights that make the half-space moments of a
    // balanced level slope and acceleration vanish for these slopes: 3/4 on <1>, 5/4 on <u u> and
    // <u v>, 1 elsewhere; applied relative to the full-space moments, so only the jump between the
    // sides' accelerations is weighted.  With h lam = 1/G the acceleration's moments are
    // -2 Phi_n N1_e / G (mass), -2 Phi_n N1_{e+1} / G, -2 (V Phi_n N1_e + th Phi_t M_e) / G.
    const R aLn = sl.pn - G * gBn, aLt = sl.pt - G * gBt, aRn = sr.pn - G * gBn, aRt = sr.pt - G * gBt;
    const R N1p0 = Mp[1] - Ub * Mp[0], N1m0 = Mm[1] - Ub * Mm[0];
    // mass, state moment: weight 3/4 (the full-space moment is zero); the paper's constants leave
    // the state moments unweighted
#pragma unroll
    for (int i = 0; i < 3; i++) wt[i] = -(t1[i] + t2[i]);
    if constexpr (AM == 0) wt[0] -= sum_products(aLn, N1p0, aRn, N1m0) * (R(0.5) * iG);
    // brackets multiplying the five time coefficients; B1 and B4 split into a hydrostatic part
    // and the rest.  B1 = (hb Ub, hb Ub^2 + P, hb Ub Vb)
    R B1[3], B2[3], B3[3];
    B1[0] = hb * Ub;
    B1[1] = hb * Ub * Ub;  // pressure removed
    B1[2] = hb * Ub * Vb;
    poly_moments(bL, sl.pn, sl.pt, hb, Ub, Vb, lamb, thb, Mp, 1, t1);
    poly_moments(bR, sr.pn, sr.pt, hb, Ub, Vb, lamb, thb, Mm, 1, t2);
    bottom_moments(gBn, gBt, Ub, Vb, lamb, thb, Mp, 1, t1);
    bottom_moments(gBn, gBt, Ub, Vb, lamb, thb, Mm, 1, t2);
#pragma unroll
    for (int i = 0; i < 3; i++) B2[i] = t1[i] + t2[i];
    {
        const R N1p1 = Mp[2] - Ub * Mp[1], N1m1 = Mm[2] - Ub * Mm[1];
        const R N1p2 = Mp[3] - Ub * Mp[2], N1m2 = Mm[3] - Ub * Mm[2];
        if constexpr (AM == 0) {
            // flux moments: weight 5/4 on the two momentum components; full-space parts from
            // N1_1 = th, N1_2 = 2 U th, M_1 = U
            const R sn = aLn + aRn, st = aLt + aRt, q = R(-0.5) * iG;  // (5/4 - 1) (-2 / G)
            B2[1] += q * (sum_products(aLn, N1p2, aRn, N1m2) - sn * Ub * thb);
            B2[2] += q * (Vb * sum_products(aLn, N1p1, aRn, N1m1) + thb * sum_products(aLt, Mp[1], aRt, Mm[1]) -
                          R(0.5) * thb * (sn * Vb + st * Ub));
        } else {
            // the paper's constants: (3/4 - 1) on <u u>, (1/4 - 1) on <u v> of the whole term
            B2[1] += R(0.5) * iG * sum_products(aLn, N1p2, aRn, N1m2);
            B2[2] += R(1.5) * iG * (Vb * sum_products(aLn, N1p1, aRn, N1m1) + thb * sum_products(aLt, Mp[1], aRt, Mm[1]));
        }
    }
    {
        const R aA = lamb * wt[0] * ihb;
        const R bA = 2 * lamb * (wt[1] - Ub * wt[0]) * ihb;
        const R gA = 2 * lamb * (wt[2] - Vb * wt[0]) * ihb;
        const R mA = 2 * aA * thb;  // <A>
        B3[0] = hb * (Ub * mA + bA * thb);
        B3[1] = hb * (Ub * Ub * mA + 2 * Ub * bA * thb + 4 * aA * thb * thb);
        B3[2] = hb * (Ub * Vb * mA + Ub * gA * thb + Vb * bA * thb);
    }
    // collision time (Sec. 4) in units of dt, and the weights of F(dt), F(dt/2) giving the flux and
    // its time derivative; c01 + c04 = 1 and ct1 + ct4 = 0 exactly (the hydrostatic part of B1 and B4
    // carries weight 1 in F0 and 0 in Ft)
    const R pl = sl.h * sl.h, pr = sr.h * sr.h;
    const R r = eps + eps_num * fabs(div_(pl - pr, pl + pr));
    const R E2 = exp_(div_(R(-0.5), r)), E1 = E2 * E2, a1 = 1 - E1, a2 = 1 - E2;
    // first order: the step's mean flux, c01 + c04 = 1 still, no time derivative
    const bool o1 = WD && order1;
    const R c04 = o1 ? r * a1 : r * (4 * a2 - a1), c01 = 1 - c04;
    const R ct1 = o1 ? R(0) : 4 * r * (2 * a2 - a1), ct4 = -ct1;
    const R c02 = -r + r * r * (8 * a2 - 2 * a1) - 2 * r * E2 + r * E1;
    const R ct2 = 4 * (2 * r * r * (a1 - 2 * a2) + r * (E2 - E1));
    const R c03 = -r + r * r * (4 * a2 - a1), ct3 = 4 * (R(0.25) + r * r * (a1 - 2 * a2));
    const R c05 = r * (2 + 4 * r) * E2 - r * (1 + r) * E1 - 3 * r * r;
    const R ct5 = 4 * (r * (1 + r) * E1 - r * (1 + 2 * r) * E2 + r * r);
    const R idt = div_(R(1), dt);
#pragma unroll
    for (int i = 0; i < 3; i++) {
        F0[i] = c01 * B1[i] + c04 * B4[i] + dt * (c02 * B2[i] + c03 * B3[i] + c05 * B5[i]);
        Ft[i] = (ct1 * B1[i] + ct4 * B4[i]) * idt + ct2 * B2[i] + ct3 * B3[i] + ct5 * B5[i];
    }
    Wb[0] = hdev;
    Wb[1] = wb1;
    Wb[2] = wb2;
    Wbt[0] = wt[0];
    Wbt[1] = wt[1];
    Wbt[2] = wt[2];
    return false;
}

// Time derivative of one side's own state (h, m.n, m.t in the local frame) from the shallow-water
// equations on that side's data: minus the derivative of the normal and tangential fluxes plus
// h times the acceleration; the pressure term takes the slope of the level (eta1 for the lower
// layer, whose bottom slope it contains, h2 for the upper).
template <typename R>
__device__ inline void side_rate(const SideL<R> &q, R G, R *o)
{
    const R U = q.U, V = q.V, h = q.h;
    o[0] = -(q.mnn + q.mtt);
    o[1] = -(R(2) * U * q.mnn - U * U * q.hn + G * h * q.en) - (U * q.mtt + V * q.mnt - U * V * q.ht) + h * q.pn;
    o[2] = -(U * q.mtn + V * q.mnn - U * V * q.hn) - (R(2) * V * q.mtt - V * V * q.ht + G * h * q.et) + h * q.pt;
}

// one thread per (edge, Gauss point, layer); the two Gauss points of an edge are adjacent lanes
// STAGE 1 (the second stage) writes only what the second update reads: the mass fluxes, the time
// derivatives, the interface thicknesses and the coupling's Gauss-point thicknesses and rates; the
// momentum fluxes, the hydrostatic terms and the interface momenta keep the first stage's values.
// GM = 1: the discontinuous reading of the gradient update: besides the fluxes, each side's own
// state and time derivative, averaged over the edge's two Gauss points (left side in the rows of
// the interface state, right side in eoh rows 6-7 and eom rows 24-33)
// WD = 1: wet/dry layers (Phys::h_dry > 0): vacuum sides, first-order band edges, dry interfaces;
// a template argument so that the wet-only path carries none of it
template <typename R, int AM, int STAGE, int GM = 0, int WD = 0>
__global__ void __launch_bounds__(256) k_flux(MeshDev m, Phys p, GpRecs<R> rec,
                                              const R *__restrict__ r0, const double *__restrict__ gP1,
                                              double *__restrict__ eoh, R *__restrict__ eom)
{
    const int64_t idx = xcd_block() * blockDim.x + threadIdx.x;
    const int64_t e = idx >> 2;
    const int g = idx & 1, lay = (idx >> 1) & 1;  // lay 0: lower layer (h1), 1: upper (h2)
    if (e >= m.E) return;
    const int64_t T = m.T, E = m.E;
    const int sc = m.escen ? (int)GKS_IX(m.escen[e], m.S) : 0;
    const R dt = (R)p.scal[2 * sc];
    // a scenario that has reached its end time takes zero-length steps: nothing to evolve (both
    // lanes of a Gauss-point pair belong to the same edge and leave together)
    if (p.scal[2 * sc] == 0.0) return;
    const R chi = (R)p.chi[sc], G = (R)p.G;
    const int32_t L = GKS_IX(m.eL[e], m.T), Rc = m.eR[e] >= 0 ? GKS_IX(m.eR[e], m.T) : m.eR[e],
                  sl = m.eslot[e];
    const int kL = GKS_IX(sl & 3, 3), kR = GKS_IX(sl >> 2, 3);
    const int sL = 2 * kL + g, sR = 2 * kR + 1 - g;
    const R *en = tab<R>(m.en), *egB = tab<R>(m.egB);
    const R nx = en[e], ny = en[E + e], tx = -ny, ty = nx;
    const double Bg = m.eBgp[g * E + e];
    const R gBx = egB[e], gBy = egB[E + e];
    const int hq = lay == 0 ? 1 : 0;   // own thickness in the record (eta1 / h2)
    const int mq = lay == 0 ? 2 : 0;   // own momenta in the record
    const int gv = lay == 0 ? 3 : 0;   // own variables' gradients start at paper component gv
    const int fv = lay == 0 ? 0 : 3;   // the other layer's height drives this layer's force
    const int ff = lay == 0 ? 1 : 0;   // modelled field index (0: eta1, 1: h2)
    // nonlinear weight of the force model
    const R rL = r0[ff * T + L], rR = Rc >= 0 ? r0[ff * T + Rc] : rL;
    const R wf0 = fmin(R(1), fmin(rL, rR));
    const R wf = (double)wf0 < W_ONE ? wf0 : R(1);
    // wet/dry: at an edge of this layer's front band (r0 of its own field 0 on either side) the
    // evolution is of first order: the sides' states alone, no slopes, no acceleration
    const bool order1 = WD && (r0[(1 - ff) * T + L] == R(0) || (Rc >= 0 && r0[(1 - ff) * T + Rc] == R(0)));
    SideL<R> side[2];
    double h64[2];
#pragma unroll
    for (int s = 0; s < 2; s++) {
        if (s == 1 && Rc < 0) break;
        const int64_t cell = s == 0 ? L : Rc;
        const int slot = s == 0 ? sL : sR;
        const GpHead<R> *hp = rec.head + 6 * cell + slot;
        const R *rm = hp->q, *rg = rec.tail[6 * cell + slot].g;
        double hh = hp->h[hq];
        const R ex = rg[2 * gv], ey = rg[2 * gv + 1];  // slope of h2, or of eta1
        R hx = ex, hy = ey;
        if (lay == 0) {  // eta1 -> h1 with the single-valued bottom at the Gauss point
            hh -= Bg;
            hx -= gBx;
            hy -= gBy;
        }
        h64[s] = hh;
        const R mx = rm[mq], my = rm[mq + 1];
        const R mxx = rg[2 + 2 * gv], mxy = rg[3 + 2 * gv];
        const R myx = rg[4 + 2 * gv], myy = rg[5 + 2 * gv];
        const R fx = rg[2 * fv], fy = rg[2 * fv + 1];
        // the plane gradient enters only where the weight is below 1 (it is not computed elsewhere)
        R dfx = fx, dfy = fy;
        if (wf < R(1)) {
            const R px1 = (R)gP1[(2 * ff) * T + cell], py1 = (R)gP1[(2 * ff + 1) * T + cell];
            dfx = wf * fx + (1 - wf) * px1;
            dfy = wf * fy + (1 - wf) * py1;
        }
        R ax, ay;
        if (lay == 0) {  // lower layer: upper-layer thickness (chi weighted); the bottom part -G gB
            ax = -chi * G * dfx;  // of its acceleration enters through bottom_moments
            ay = -chi * G * dfy;
        } else {         // upper layer: slope of the interface level
            ax = -G * dfx;
            ay = -G * dfy;
        }
        SideL<R> &q = side[s];
        // wet/dry: a side at or below h_dry is a vacuum (every term of it an exact zero)
        const bool vac = WD && !(hh > p.h_dry);
        if (vac) h64[s] = 0.0;
        const R h = vac ? R(0) : (R)hh, ih = vac ? R(0) : div_(R(1), h);
        q.h = h;
        q.ih = ih;
        q.U = (mx * nx + my * ny) * ih;
        q.V = (mx * tx + my * ty) * ih;
        q.hn = hx * nx + hy * ny;
        q.ht = hx * tx + hy * ty;
        q.en = ex * nx + ey * ny;
        q.et = ex * tx + ey * ty;
        const R dmn_x = mxx * nx + myx * ny, dmn_y = mxy * nx + myy * ny;  // grad (m . n)
        const R dmt_x = mxx * tx + myx * ty, dmt_y = mxy * tx + myy * ty;  // grad (m . t)
        q.mnn = dmn_x * nx + dmn_y * ny;
        q.mnt = dmn_x * tx + dmn_y * ty;
        q.mtn = dmt_x * nx + dmt_y * ny;
        q.mtt = dmt_x * tx + dmt_y * ty;
        q.pn = ax * nx + ay * ny;
        q.pt = ax * tx + ay * ty;
        if (order1) {
            q.hn = q.ht = q.en = q.et = R(0);
            q.mnn = q.mnt = q.mtn = q.mtt = R(0);
            q.pn = q.pt = R(0);
        }
    }
    if (Rc == -1) {  // wall: mirror image of the left side
        side[1] = side[0];
        side[1].U = -side[0].U;
        side[1].hn = -side[0].hn;
        side[1].en = -side[0].en;
        side[1].mnt = -side[0].mnt;
        side[1].mtn = -side[0].mtn;
        side[1].pn = -side[0].pn;
        h64[1] = h64[0];
    } else if (Rc < 0) {  // free boundary: every component extended evenly across the edge
        side[1] = side[0];
        side[1].hn = -side[0].hn;
        side[1].en = -side[0].en;
        side[1].mnn = -side[0].mnn;
        side[1].mtn = -side[0].mtn;
        side[1].pn = -side[0].pn;
        h64[1] = h64[0];
    }
    const double hbase = 0.5 * (h64[0] + h64[1]);
    // single-valued bottom slope in the local frame (zero normal part at walls by construction)
    const R gBn = (lay == 0 && !order1) ? gBx * nx + gBy * ny : R(0);
    const R gBt = (lay == 0 && !order1) ? gBx * tx + gBy * ty : R(0);
    R F0[3], Ft[3], Wb[3], Wbt[3];
    const bool dry = gks_point<R, AM, WD>(side[0], side[1], hbase, gBn, gBt, G, (R)p.eps, (R)p.eps_num, dt, F0, Ft,
                                          Wb, Wbt, order1, p.h_dry);
    if (Rc == -1) {  // no mass crosses a wall
        F0[0] = 0;
        Ft[0] = 0;
    }
    // FP64 hydrostatic pieces: interface thickness and 1/2 G hb^2, averaged over the two points
    // (both zero at a dry interface)
    const double hb = dry ? 0.0 : hbase + (double)Wb[0];
    double P = 0.5 * p.G * hb * hb, H = hb, Hc = hbase;
    P = 0.5 * (P + __shfl_xor(P, 1));
    H = 0.5 * (H + __shfl_xor(H, 1));
    // the layer coupling's Gauss-point thickness (Sec. 3.2, Eq. SWE-source-discretization), read as
    // the mean of the two sides' reconstructed values, and its rate, the mean of the sides' -div(h U)
    Hc = 0.5 * (Hc + __shfl_xor(Hc, 1));
    R Hct = R(-0.5) * ((side[0].mnn + side[0].mtt) + (side[1].mnn + side[1].mtt));
    Hct = R(0.5) * (Hct + __shfl_xor(Hct, 1));
    // the rest back to the global frame, then averaged over the two Gauss points
    R out[11];
    out[0] = F0[0];
    out[1] = F0[1] * nx + F0[2] * tx;
    out[2] = F0[1] * ny + F0[2] * ty;
    out[3] = Ft[0];
    out[4] = Ft[1] * nx + Ft[2] * tx;
    out[5] = Ft[1] * ny + Ft[2] * ty;
    R side_out[5];  // GM = 1: the right side's momenta and rates (the left side's go in out[6..10])
    if constexpr (GM == 1) {
        H = h64[0];
        double Hr = h64[1];
#pragma unroll
        for (int s = 0; s < 2; s++) {
            R r[3];
            side_rate(side[s], G, r);
            R *o5 = s == 0 ? out + 6 : side_out;
            const R mn = side[s].h * side[s].U, mt = side[s].h * side[s].V;
            o5[0] = mn * nx + mt * tx;
            o5[1] = mn * ny + mt * ty;
            o5[2] = r[0];
            o5[3] = r[1] * nx + r[2] * tx;
            o5[4] = r[1] * ny + r[2] * ty;
        }
        H = 0.5 * (H + __shfl_xor(H, 1));
        Hr = 0.5 * (Hr + __shfl_xor(Hr, 1));
#pragma unroll
        for (int i = 0; i < 5; i++) side_out[i] = R(0.5) * (side_out[i] + __shfl_xor(side_out[i], 1));
        if (g == 0) eoh[(int64_t)(lay == 0 ? 7 : 6) * E + e] = Hr;
    } else {
        out[6] = Wb[1] * nx + Wb[2] * tx;
        out[7] = Wb[1] * ny + Wb[2] * ty;
        out[8] = Wbt[0];
        out[9] = Wbt[1] * nx + Wbt[2] * tx;
        out[10] = Wbt[1] * ny + Wbt[2] * ty;
    }
#pragma unroll
    for (int i = 0; i < 11; i++) out[i] = R(0.5) * (out[i] + __shfl_xor(out[i], 1));
    const int o = lay == 0 ? 3 : 0;  // paper component offset of this layer
    if (g == 0) {
        if constexpr (STAGE == 0) eoh[(int64_t)(lay == 0 ? 1 : 0) * E + e] = P;
        eoh[(int64_t)(lay == 0 ? 3 : 2) * E + e] = H;
        eoh[(int64_t)(lay == 0 ? 5 : 4) * E + e] = Hc;
#pragma unroll
        for (int i = 0; i < 3; i++)
            if (STAGE == 0 || i == 0) eom[(int64_t)(o + i) * E + e] = out[i];      // F0
#pragma unroll
        for (int i = 0; i < 3; i++) eom[(int64_t)(6 + o + i) * E + e] = out[3 + i];  // Ft
    } else {
        const int mo = lay == 0 ? 2 : 0;
        if constexpr (STAGE == 0) {
            eom[(int64_t)(12 + mo) * E + e] = out[6];  // Wb momenta
            eom[(int64_t)(13 + mo) * E + e] = out[7];
        }
#pragma unroll
        for (int i = 0; i < 3; i++) eom[(int64_t)(16 + o + i) * E + e] = out[8 + i];  // Wbt
        eom[(int64_t)(lay == 0 ? 23 : 22) * E + e] = Hct;
        if constexpr (GM == 1) {
            if constexpr (STAGE == 0) {
                eom[(int64_t)(24 + mo) * E + e] = side_out[0];
                eom[(int64_t)(25 + mo) * E + e] = side_out[1];
            }
#pragma unroll
            for (int i = 0; i < 3; i++) eom[(int64_t)(28 + o + i) * E + e] = side_out[2 + i];
        }
    }
}

// --------------------------------------------------------------------------------------------
// cell update: deterministic gather of the three edges in FP64, sources, S2O4 stage update

// stage 0: Ws = W + dt/2 L + dt^2/8 Lt, gWs = G + dt/2 Gt; carry Wc = W + dt L + dt^2/6 Lt, Gc = G
// stage 1: W = Wc + dt^2/3 Lt, gW = Gc + dt Gt
// STAGE is a template argument: the second stage needs only the time derivatives, the thickness
// fluxes and the interface thicknesses, so it neither loads nor sums the momentum fluxes, the
// hydrostatic terms and the interface momenta
// SRC = 1: the higher-order layer coupling: the cell-average thickness in place of the Gauss-point
// mean, its rate from the cell's mass flux, plus the interior correction src[8][T] of k_recon.
// GM = 1: the discontinuous reading of the gradient update: a cell takes the interface values of
// its own side of each edge (the right cell of an edge reads eoh rows 6-7 and eom rows 24-33).
template <typename R, int STAGE, int SRC = 0, int GM = 0>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_update(MeshDev m, Phys p, const double *__restrict__ eoh,
                                                const R *__restrict__ eom, const double *__restrict__ Whin,
                                                const R *__restrict__ Wmin, const R *__restrict__ gWin,
                                                double *__restrict__ Whout, R *__restrict__ Wmout,
                                                R *__restrict__ gWout, double *__restrict__ Wc, R *__restrict__ Gc,
                                                const R *__restrict__ src)
{
    constexpr int stage = STAGE;
    int64_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= m.T) return;
    const int64_t T = m.T, E = m.E, TG = m.T + m.NG;
    const int sc = m.cscen ? (int)GKS_IX(m.cscen[c], m.S) : 0;
    const double dt = p.scal[2 * sc], G = p.G, chi = p.chi[sc];
    if (dt == 0.0) {
        // the scenario has reached its end time: the state stays as it is (the stage's output is
        // its input; stage 0 also leaves the carry equal to it for stage 1)
#pragma unroll
        for (int v = 0; v < 6; v++) {
            const double w = stage == 0 ? ((v == 0) ? Whin[c] : (v == 3) ? Whin[TG + c] : (double)Wmin[mom_slot(v) * TG + c])
                                        : Wc[v * T + c];
            if (v == 0 || v == 3)
                Whout[(v == 3 ? TG : 0) + c] = w;
            else
                Wmout[mom_slot(v) * TG + c] = (R)w;
            if (stage == 0) Wc[v * T + c] = w;
#pragma unroll
            for (int d = 0; d < 2; d++) {
                const R g = stage == 0 ? gWin[(2 * v + d) * TG + c] : Gc[(2 * v + d) * T + c];
                gWout[(2 * v + d) * TG + c] = g;
                if (stage == 0) Gc[(2 * v + d) * T + c] = g;
            }
        }
        return;
    }
    double LF[6] = {0}, LFt[6] = {0}, GG[6][2] = {{0}}, GGt[6][2] = {{0}}, hs[2] = {0, 0}, hts[2] = {0, 0};
    // smallest acceptable new thickness, exclusive: 0, or -h_dry with wet/dry layers
    const double hneg = p.h_dry > 0 ? -p.h_dry : 0.0;
    double GC[2][2] = {{0, 0}}, GCt[2][2] = {{0, 0}};  // [0] lower, [1] upper: central thicknesses
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const int32_t code = m.cedge[k * T + c];
        const int64_t e = GKS_IX(code >= 0 ? code : ~code, m.E);
        const double f = m.fl[k * T + c], gx = m.gg[(2 * k) * T + c], gy = m.gg[(2 * k + 1) * T + c];
        // rows of this cell's interface values: shared, or those of its own side (GM = 1)
        const int64_t ho = (GM == 1 && code < 0) ? 4 * E : 0, mo = (GM == 1 && code < 0) ? 12 * E : 0;
        const double Hu = eoh[2 * E + ho + e], Hl = eoh[3 * E + ho + e];
        double Wb[6];
        Wb[0] = Hu;
        Wb[3] = Hl;
        if constexpr (stage == 0) {
            Wb[1] = eom[12 * E + mo + e];
            Wb[2] = eom[13 * E + mo + e];
            Wb[4] = eom[14 * E + mo + e];
            Wb[5] = eom[15 * E + mo + e];
        }
#pragma unroll
        for (int v = 0; v < 6; v++) {
            const bool mass = v == 0 || v == 3;
            if (stage == 0 || mass) {
                LF[v] -= f * (double)eom[(int64_t)v * E + e];
                GG[v][0] += gx * Wb[v];
                GG[v][1] += gy * Wb[v];
            }
            const double Ft = eom[(int64_t)(6 + v) * E + e];
            const double Wbt = eom[(int64_t)(16 + v) * E + mo + e];
            LFt[v] -= f * Ft;
            GGt[v][0] += gx * Wbt;
            GGt[v][1] += gy * Wbt;
        }
        if constexpr (stage == 0) {
            // hydrostatic part of the normal momentum flux, along the outward normal
            const double Pu = eoh[e], Pl = eoh[E + e];
            LF[1] -= gx * Pu;
            LF[2] -= gy * Pu;
            LF[4] -= gx * Pl;
            LF[5] -= gy * Pl;
        }
        const double Cu = eoh[4 * E + e], Cl = eoh[5 * E + e];
        const double Ctu = eom[22 * E + e], Ctl = eom[23 * E + e];
        GC[1][0] += gx * Cu;
        GC[1][1] += gy * Cu;
        GC[0][0] += gx * Cl;
        GC[0][1] += gy * Cl;
        GCt[1][0] += gx * Ctu;
        GCt[1][1] += gy * Ctu;
        GCt[0][0] += gx * Ctl;
        GCt[0][1] += gy * Ctl;
        hs[1] += Cu;
        hs[0] += Cl;
        hts[1] += Ctu;
        hts[0] += Ctl;
    }
    const double third = 1.0 / 3.0;
    hs[0] *= third; hs[1] *= third; hts[0] *= third; hts[1] *= third;  // [0] lower, [1] upper
    const double gBx = m.gB[c], gBy = m.gB[T + c];
    double Lt[6];
#pragma unroll
    for (int v = 0; v < 6; v++) Lt[v] = LFt[v];
    // bottom source rate via the thickness rates; layer coupling rate by the product rule
    Lt[1] += LF[0] * (-G * gBx);
    Lt[2] += LF[0] * (-G * gBy);
    Lt[4] += LF[3] * (-G * gBx);
    Lt[5] += LF[3] * (-G * gBy);
    if constexpr (SRC == 1) {
        // higher order: cell-average thicknesses, their rates from the mass fluxes
        const double h2a = Whin[c], h1a = Whin[TG + c] - m.Bbar[c];
        Lt[4] += -chi * G * (LF[3] * GC[1][0] + h1a * GCt[1][0] + (double)src[4 * T + c]);
        Lt[5] += -chi * G * (LF[3] * GC[1][1] + h1a * GCt[1][1] + (double)src[5 * T + c]);
        Lt[1] += -G * (LF[0] * GC[0][0] + h2a * GCt[0][0] + (double)src[6 * T + c]);
        Lt[2] += -G * (LF[0] * GC[0][1] + h2a * GCt[0][1] + (double)src[7 * T + c]);
    } else {
        Lt[4] += -chi * G * (hts[0] * GC[1][0] + hs[0] * GCt[1][0]);
        Lt[5] += -chi * G * (hts[0] * GC[1][1] + hs[0] * GCt[1][1]);
        Lt[1] += -G * (hts[1] * GC[0][0] + hs[1] * GCt[0][0]);
        Lt[2] += -G * (hts[1] * GC[0][1] + hs[1] * GCt[0][1]);
    }
    if constexpr (stage == 0) {
        double L[6];
#pragma unroll
        for (int v = 0; v < 6; v++) L[v] = LF[v];
        const double h2 = Whin[c], h1 = Whin[TG + c] - m.Bbar[c];
        // bottom source h_j (0, -G B_x, -G B_y) (Sec. 3.2) and layer coupling
        // (Eq. SWE-source-discretization) from the Gauss-point mean thickness and the Green-Gauss
        // derivative of the other layer's Gauss-point thickness (central values); the higher-order
        // form takes the cell average and adds the interior correction
        if constexpr (SRC == 1) {
            L[1] += h2 * (-G * gBx) - G * (h2 * GC[0][0] + (double)src[2 * T + c]);
            L[2] += h2 * (-G * gBy) - G * (h2 * GC[0][1] + (double)src[3 * T + c]);
            L[4] += h1 * (-G * gBx) - chi * G * (h1 * GC[1][0] + (double)src[c]);
            L[5] += h1 * (-G * gBy) - chi * G * (h1 * GC[1][1] + (double)src[T + c]);
        } else {
            L[1] += h2 * (-G * gBx) - G * hs[1] * GC[0][0];
            L[2] += h2 * (-G * gBy) - G * hs[1] * GC[0][1];
            L[4] += h1 * (-G * gBx) - chi * G * hs[0] * GC[1][0];
            L[5] += h1 * (-G * gBy) - chi * G * hs[0] * GC[1][1];
        }
        // the state carries grad(eta1) = grad(h1) + grad(B)
        GG[3][0] += gBx;
        GG[3][1] += gBy;
        bool bad = false;  // a new thickness <= 0 (or NaN), or a non-finite momentum (via their sum)
        double msum = 0;
#pragma unroll
        for (int v = 0; v < 6; v++) {
            const double w = (v == 0) ? Whin[c] : (v == 3) ? Whin[TG + c] : (double)Wmin[mom_slot(v) * TG + c];
            const double ws = w + 0.5 * dt * L[v] + 0.125 * dt * dt * Lt[v];
            if (v == 0 || v == 3)
                Whout[(v == 3 ? TG : 0) + c] = ws;
            else
                Wmout[mom_slot(v) * TG + c] = (R)ws;
            // a thickness <= 0 is bad, or with wet/dry layers one below -h_dry (a dry cell may hold
            // a rounding residue)
            if (v == 0) bad |= !(ws > hneg);
            else if (v == 3) bad |= !(ws - (w - h1) > hneg);  // w - h1: the cell's bottom mean
            else msum += ws;
            Wc[v * T + c] = w + dt * L[v] + (dt * dt / 6.0) * Lt[v];
#pragma unroll
            for (int d = 0; d < 2; d++) {
                gWout[(2 * v + d) * TG + c] = (R)(GG[v][d] + 0.5 * dt * GGt[v][d]);
                Gc[(2 * v + d) * T + c] = (R)GG[v][d];
            }
        }
        if (bad || !isfinite(msum)) atomicMin(p.bad, (unsigned long long)c);
    } else {
        bool bad = false;
        double msum = 0;
#pragma unroll
        for (int v = 0; v < 6; v++) {
            const double wn = Wc[v * T + c] + (dt * dt / 3.0) * Lt[v];
            if (v == 0 || v == 3)
                Whout[(v == 3 ? TG : 0) + c] = wn;
            else
                Wmout[mom_slot(v) * TG + c] = (R)wn;
            if (v == 0) bad |= !(wn > hneg);
            else if (v == 3) bad |= !(wn - m.Bbar[c] > hneg);
            else msum += wn;
#pragma unroll
            for (int d = 0; d < 2; d++)
                gWout[(2 * v + d) * TG + c] = (R)((double)Gc[(2 * v + d) * T + c] + dt * GGt[v][d]);
        }
        if (bad || !isfinite(msum)) atomicMin(p.bad, (unsigned long long)c);
    }
}

// --------------------------------------------------------------------------------------------
// time step: per-block maxima of the wave speed, then one block finishes (no atomics); batches of
// scenarios use one block per scenario

constexpr int DT_BLOCK = 256;

__device__ inline double block_max(double v, double *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (threadIdx.x < 64) {
        v = (lane < (int)(blockDim.x >> 6)) ? sh[lane] : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    }
    return v;
}

template <typename R>
__device__ inline double wave_speed(const MeshDev &m, const Phys &p, const double *Wh, const R *Wm, int64_t c)
{
    const int64_t TG = m.T + m.NG;
    const double h2 = Wh[c], h1 = Wh[TG + c] - m.Bbar[c];
    // velocities desingularised in thin layers (wet/dry; m / h otherwise), a dry cell may hold -0
    const double u2 = wd_velocity(h2, Wm[c], p.h_dry), v2 = wd_velocity(h2, Wm[TG + c], p.h_dry);
    const double u1 = wd_velocity(h1, Wm[2 * TG + c], p.h_dry), v1 = wd_velocity(h1, Wm[3 * TG + c], p.h_dry);
    const double s1 = sqrt(u1 * u1 + v1 * v1) + sqrt(p.G * fmax(h1, 0.0));
    const double s2 = sqrt(u2 * u2 + v2 * v2) + sqrt(p.G * fmax(h2, 0.0));
    return fmax(s1, s2);
}

template <typename R>
__global__ void __launch_bounds__(DT_BLOCK) k_dt_partial(MeshDev m, Phys p, const double *__restrict__ Wh,
                                                          const R *__restrict__ Wm, double *__restrict__ part)
{
    __shared__ double sh[DT_BLOCK / 64];
    double smax = 0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < m.T; c += (int64_t)gridDim.x * blockDim.x)
        smax = fmax(smax, wave_speed(m, p, Wh, Wm, c));
    smax = block_max(smax, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = smax;
}

__device__ inline void set_step(const MeshDev &m, const Phys &p, int s, double smax)
{
    double dt = p.cfl * m.sdxmin[s] / smax;
    const double t = p.scal[2 * s + 1];
    double tn = t + dt;
    if (tn > p.t_end[s]) {  // the last step ends exactly at t_end; none ever goes back
        dt = fmax(0.0, p.t_end[s] - t);
        tn = fmax(t, p.t_end[s]);
    }
    p.scal[2 * s] = dt;
    p.scal[2 * s + 1] = tn;
}

__global__ void __launch_bounds__(DT_BLOCK) k_dt_final(MeshDev m, Phys p, const double *__restrict__ part, int nparts)
{
    __shared__ double sh[DT_BLOCK / 64];
    double v = 0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) v = fmax(v, part[i]);
    v = block_max(v, sh);
    if (threadIdx.x == 0) set_step(m, p, 0, v);
}

// batches: one block per chunk of cells (the chunk's largest wave speed), then one block per
// scenario over its chunks
template <typename R>
__global__ void __launch_bounds__(DT_BLOCK) k_dt_chunk(MeshDev m, Phys p, const double *__restrict__ Wh,
                                                        const R *__restrict__ Wm, double *__restrict__ part)
{
    __shared__ double sh[DT_BLOCK / 64];
    const int ch = blockIdx.x;
    double smax = 0;
    const int64_t c0 = GKS_IX(m.cb[ch], m.T + 1), c1 = GKS_IX(m.cb[ch + 1], m.T + 1);
    for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x)
        smax = fmax(smax, wave_speed(m, p, Wh, Wm, c));
    smax = block_max(smax, sh);
    if (threadIdx.x == 0) part[ch] = smax;
}

__global__ void __launch_bounds__(64) k_dt_scenario(MeshDev m, Phys p, const double *__restrict__ part)
{
    const int s = blockIdx.x;
    double v = 0;
    const int i0 = (int)GKS_IX(m.sc0[s], m.NCH + 1), i1 = (int)GKS_IX(m.sc0[s + 1], m.NCH + 1);
    for (int i = i0 + threadIdx.x; i < i1; i += 64) v = fmax(v, part[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    if (threadIdx.x == 0) set_step(m, p, s, v);
}

// an explicit step of a single scenario, clipped like the CFL step so that t never passes t_end
__global__ void k_set_dt(Phys p, double dt)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double t = p.scal[1];
        double tn = t + dt;
        if (tn > p.t_end[0]) {
            dt = fmax(0.0, p.t_end[0] - t);
            tn = fmax(t, p.t_end[0]);
        }
        p.scal[0] = dt;
        p.scal[1] = tn;
    }
}

// per-layer mass of cells [c0, c1): fixed-order block sums (deterministic)
__global__ void __launch_bounds__(256) k_mass_partial(MeshDev m, const double *__restrict__ Wh, int64_t c0,
                                                      int64_t c1, double *__restrict__ part)
{
    __shared__ double sh[2][256];
    const int64_t TG = m.T + m.NG;
    double a = 0, b = 0;
    for (int64_t c = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < c1; c += (int64_t)gridDim.x * blockDim.x) {
        a += m.area[c] * Wh[c];
        b += m.area[c] * (Wh[TG + c] - m.Bbar[c]);
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sh[0][0];
        part[2 * blockIdx.x + 1] = sh[1][0];
    }
}

// Per-step diagnostics of a scenario's cells [c0, c1) (Sec. 3.2's well-balance property: a lake
// at rest keeps U = 0 and both levels flat): per block the largest speed |h U| / h of each layer
// (desingularised in thin layers when h_dry > 0, as in the time step) and the largest and smallest
// levels eta1 = h1 + B and eta2 = eta1 + h2, as six maxima (the minima negated); the host takes
// the maxima over the blocks.  Grid-stride over the cells.
template <typename R>
__global__ void __launch_bounds__(256) k_diag_partial(MeshDev m, const double *__restrict__ Wh,
                                                      const R *__restrict__ Wm, int64_t c0, int64_t c1,
                                                      double h_dry, double *__restrict__ part)
{
    __shared__ double sh[6][256];
    const int64_t TG = m.T + m.NG;
    double v[6] = {0.0, 0.0, -HUGE_VAL, -HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    for (int64_t c = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < c1; c += (int64_t)gridDim.x * blockDim.x) {
        const double h2 = Wh[c], e1 = Wh[TG + c], h1 = e1 - m.Bbar[c];
        const double m2x = Wm[c], m2y = Wm[TG + c], m1x = Wm[2 * TG + c], m1y = Wm[3 * TG + c];
        v[0] = fmax(v[0], wd_velocity(h2, sqrt(m2x * m2x + m2y * m2y), h_dry));
        v[1] = fmax(v[1], wd_velocity(h1, sqrt(m1x * m1x + m1y * m1y), h_dry));
        v[2] = fmax(v[2], e1);
        v[3] = fmax(v[3], -e1);
        v[4] = fmax(v[4], e1 + h2);
        v[5] = fmax(v[5], -(e1 + h2));
    }
#pragma unroll
    for (int k = 0; k < 6; k++) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < 6; k++) sh[k][threadIdx.x] = fmax(sh[k][threadIdx.x], sh[k][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

}  // namespace gks
