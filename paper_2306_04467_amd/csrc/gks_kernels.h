// Device kernels of one S2O4 stage of the compact gas-kinetic scheme (gfx950, wave64).
//
// Data layout (structure of arrays, index = component * stride + cell/edge):
//   state   W[6][TG], gW[12][TG]   TG = T + NG (ghost mirror cells appended), component 3 holds the
//                                  interface level eta1 = h1 + B (Sec. 3.2 water-level technique)
//   rec     [6 slots][6 comps][3][T] Gauss-point value and gradient of each reconstructed variable,
//                                  slot = 2 * local edge + Gauss point (cell's own orientation)
//   eo      [4][6][E]              per edge, both Gauss points averaged, global frame:
//                                  F0 (flux), Ft (its time derivative), Wb, Wbt (interface values)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gks {

struct MeshDev {
    int64_t T, E, NG;
    double dxmin;
    // cells
    const double *area, *hs, *vtx, *nbc, *fl, *gg, *Bbar, *gB, *M;
    const int32_t *cedge, *sten;
    // edges
    const int32_t *eL, *eR, *eslot;
    const double *en, *eBgp, *egB;
    // ghosts
    const int32_t *gsrc;
    const double *gR;
};

struct Phys {
    double G, chi, eps, eps_num, cfl, t_end;
    int linear;
};

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

// --------------------------------------------------------------------------------------------
// ghost mirror cells: state of the source cell seen through an orthogonal map R

__global__ void k_ghost_fill(MeshDev m, double *__restrict__ W, double *__restrict__ gW)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= m.NG) return;
    const int64_t TG = m.T + m.NG, s = m.gsrc[g], d = m.T + g;
    const double a = m.gR[g], b = m.gR[m.NG + g], c = m.gR[2 * m.NG + g], e = m.gR[3 * m.NG + g];
#pragma unroll
    for (int o = 0; o < 6; o += 3) {
        double h = W[o * TG + s], mx = W[(o + 1) * TG + s], my = W[(o + 2) * TG + s];
        W[o * TG + d] = h;
        W[(o + 1) * TG + d] = a * mx + b * my;
        W[(o + 2) * TG + d] = c * mx + e * my;
        double hx = gW[(2 * o) * TG + s], hy = gW[(2 * o + 1) * TG + s];
        gW[(2 * o) * TG + d] = a * hx + b * hy;
        gW[(2 * o + 1) * TG + d] = c * hx + e * hy;
        // momentum gradient G[i][j] = d m_i / d x_j  ->  R G R^T
        double g00 = gW[(2 * o + 2) * TG + s], g01 = gW[(2 * o + 3) * TG + s];
        double g10 = gW[(2 * o + 4) * TG + s], g11 = gW[(2 * o + 5) * TG + s];
        double r00 = a * g00 + b * g10, r01 = a * g01 + b * g11;
        double r10 = c * g00 + e * g10, r11 = c * g01 + e * g11;
        gW[(2 * o + 2) * TG + d] = r00 * a + r01 * b;
        gW[(2 * o + 3) * TG + d] = r00 * c + r01 * e;
        gW[(2 * o + 4) * TG + d] = r10 * a + r11 * b;
        gW[(2 * o + 5) * TG + d] = r10 * c + r11 * e;
    }
}

// --------------------------------------------------------------------------------------------
// compact reconstruction (Sec. 3.4): one thread per (cell, variable); 192 threads = 32 cells x 6

constexpr int RECON_CELLS = 32;

// STAGE_M: the block first copies its 32 cells' least-squares operators into LDS (coalesced), so
// the six variable-threads of a cell read them from LDS instead of six times through the caches.
template <bool STAGE_M>
__global__ void __launch_bounds__(192) k_recon(MeshDev m, Phys p, const double *__restrict__ W,
                                               const double *__restrict__ gW, double *__restrict__ rec,
                                               double *__restrict__ r0)
{
    const int lane = threadIdx.x & 31, v = threadIdx.x >> 5;
    const int64_t c = xcd_block() * RECON_CELLS + lane;
    const int64_t T = m.T, TG = m.T + m.NG;
    __shared__ double Ms[STAGE_M ? 153 * RECON_CELLS : 1];
    if (STAGE_M) {
        const int64_t c0 = xcd_block() * RECON_CELLS;
        for (int i = threadIdx.x; i < 153 * RECON_CELLS; i += blockDim.x) {
            const int k = i / RECON_CELLS, cl = i % RECON_CELLS;
            Ms[i] = (c0 + cl < T) ? m.M[(int64_t)k * T + c0 + cl] : 0.0;
        }
        __syncthreads();
    }
    if (c >= T) return;
    const double Q0 = W[v * TG + c];
    const double hs = m.hs[c];
    // right-hand side of the least-squares system: average differences, then scaled gradients
    double rhs[17];
    int32_t nb[9];
#pragma unroll
    for (int s = 0; s < 9; s++) {
        nb[s] = m.sten[s * T + c];
        rhs[s] = W[v * TG + nb[s]] - Q0;
    }
    rhs[9] = hs * gW[(2 * v) * TG + c];
    rhs[10] = hs * gW[(2 * v + 1) * TG + c];
#pragma unroll
    for (int l = 0; l < 3; l++) {
        rhs[11 + 2 * l] = hs * gW[(2 * v) * TG + nb[l]];
        rhs[12 + 2 * l] = hs * gW[(2 * v + 1) * TG + nb[l]];
    }
    double a[9];
#pragma unroll
    for (int k = 0; k < 9; k++) {
        double s = 0;
#pragma unroll
        for (int r = 0; r < 17; r++) {
            const double mk = STAGE_M ? Ms[(k * 17 + r) * RECON_CELLS + lane] : m.M[(k * 17 + r) * T + c];
            s = fma(mk, rhs[r], s);
        }
        a[k] = s;
    }
    // scaled vertices (centroid at the origin) and the cell means of the basis
    double vx[3], vy[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        vx[k] = m.vtx[(2 * k) * T + c];
        vy[k] = m.vtx[(2 * k + 1) * T + c];
    }
    double mxx = 0, mxy = 0, myy = 0, mx3 = 0, mx2y = 0, mxy2 = 0, my3 = 0;
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
    const double c12 = 1.0 / 12.0, c30 = 1.0 / 30.0;
    const double mean_const = a[2] * mxx * c12 + a[3] * mxy * c12 + a[4] * myy * c12 + a[5] * mx3 * c30 +
                              a[6] * mx2y * c30 + a[7] * mxy2 * c30 + a[8] * my3 * c30;
    // lower-order candidates (reading of the nonlinear compact reconstruction): planes through
    // the averages of {0, f0, f1}, {0, f1, f2}, {0, f2, f0} and the cell's own gradient
    double bx[4], by[4];
#pragma unroll
    for (int s = 0; s < 3; s++) {
        const int sa = s, sb = (s + 1) % 3;
        double ax_ = m.nbc[(2 * sa) * T + c], ay_ = m.nbc[(2 * sa + 1) * T + c];
        double bx_ = m.nbc[(2 * sb) * T + c], by_ = m.nbc[(2 * sb + 1) * T + c];
        double ra = rhs[sa], rb = rhs[sb];
        double inv = 1.0 / (ax_ * by_ - ay_ * bx_);
        bx[s] = (ra * by_ - ay_ * rb) * inv;
        by[s] = (ax_ * rb - ra * bx_) * inv;
    }
    bx[3] = rhs[9];
    by[3] = rhs[10];
    const double d0 = 0.8, dm = 0.05;
    double w0 = d0, wm[4] = {dm, dm, dm, dm};
    if (!p.linear) {
        // smoothness indicator of P^3 in scaled coordinates: the cell has area 1/2 there, so the
        // |Omega|^(|alpha|-1) weights become (1/2)^(|alpha|-1) and integrals are averages / 2.
        // First derivatives (quadratics): 6-point degree-4 rule; second (linear): edge midpoints.
        const double qa[2] = {0.445948490915964886, 0.091576213509770743};
        const double qw[2] = {0.223381589678011466, 1.0 / 3.0 - 0.223381589678011466};
        double s1 = 0;
#pragma unroll
        for (int r = 0; r < 2; r++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                double l0 = (j == 0) ? 1 - 2 * qa[r] : qa[r];
                double l1 = (j == 1) ? 1 - 2 * qa[r] : qa[r];
                double l2 = (j == 2) ? 1 - 2 * qa[r] : qa[r];
                double x = l0 * vx[0] + l1 * vx[1] + l2 * vx[2];
                double y = l0 * vy[0] + l1 * vy[1] + l2 * vy[2];
                double px = a[0] + 2 * a[2] * x + a[3] * y + 3 * a[5] * x * x + 2 * a[6] * x * y + a[7] * y * y;
                double py = a[1] + a[3] * x + 2 * a[4] * y + a[6] * x * x + 2 * a[7] * x * y + 3 * a[8] * y * y;
                s1 += qw[r] * (px * px + py * py);
            }
        double s2 = 0;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double x = 0.5 * (vx[j] + vx[(j + 1) % 3]), y = 0.5 * (vy[j] + vy[(j + 1) % 3]);
            double pxx = 2 * a[2] + 6 * a[5] * x + 2 * a[6] * y;
            double pxy = a[3] + 2 * a[6] * x + 2 * a[7] * y;
            double pyy = 2 * a[4] + 2 * a[7] * x + 6 * a[8] * y;
            s2 += (pxx * pxx + pxy * pxy + pyy * pyy) * (1.0 / 3.0);
        }
        double s3 = 36 * a[5] * a[5] + 4 * a[6] * a[6] + 4 * a[7] * a[7] + 36 * a[8] * a[8];
        double beta0 = 0.5 * s1 + 0.25 * s2 + 0.125 * s3;
        double tz = 0, bm[4];
#pragma unroll
        for (int s = 0; s < 4; s++) {
            bm[s] = 0.5 * (bx[s] * bx[s] + by[s] * by[s]);
            tz += fabs(beta0 - bm[s]);
        }
        tz *= 0.25;
        const double epsw = 1e-10 * fmax(Q0 * Q0, 1e-20);
        double t0 = d0 * (1 + tz / (beta0 + epsw)), sum = t0, tm[4];
#pragma unroll
        for (int s = 0; s < 4; s++) {
            tm[s] = dm * (1 + tz / (bm[s] + epsw));
            sum += tm[s];
        }
        const double isum = 1.0 / sum;
        w0 = t0 * isum;
#pragma unroll
        for (int s = 0; s < 4; s++) wm[s] = tm[s] * isum;
    }
    const double ratio = w0 / d0;
    if (v == 3) r0[c] = ratio;
    if (v == 0) r0[T + c] = ratio;
    // combined polynomial R = ratio (P0 - sum dm Pm) + sum wm Pm, Pm = Q0 + b . x
    double cm[4], sbx = 0, sby = 0;
#pragma unroll
    for (int s = 0; s < 4; s++) {
        cm[s] = wm[s] - ratio * dm;
        sbx += cm[s] * bx[s];
        sby += cm[s] * by[s];
    }
    const double ihs = 1.0 / hs;
    const double gs[2] = {0.5 - 0.28867513459481288225, 0.5 + 0.28867513459481288225};
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
        for (int g = 0; g < 2; g++) {
            const int k1 = (k + 1) % 3;
            double x = vx[k] + gs[g] * (vx[k1] - vx[k]);
            double y = vy[k] + gs[g] * (vy[k1] - vy[k]);
            double P = a[0] * x + a[1] * y + a[2] * x * x + a[3] * x * y + a[4] * y * y + a[5] * x * x * x +
                       a[6] * x * x * y + a[7] * x * y * y + a[8] * y * y * y - mean_const;
            double Px = a[0] + 2 * a[2] * x + a[3] * y + 3 * a[5] * x * x + 2 * a[6] * x * y + a[7] * y * y;
            double Py = a[1] + a[3] * x + 2 * a[4] * y + a[6] * x * x + 2 * a[7] * x * y + 3 * a[8] * y * y;
            // all candidates share the cell average Q0 (ratio + sum cm = 1)
            double val = Q0 + ratio * P + sbx * x + sby * y;
            double gx = (ratio * Px + sbx) * ihs, gy = (ratio * Py + sby) * ihs;
            const int slot = 2 * k + g;
            double *o = rec + ((int64_t)(slot * 6 + v) * 3) * T + c;
            o[0] = val;
            o[T] = gx;
            o[2 * T] = gy;
        }
}

// --------------------------------------------------------------------------------------------
// interface force modelling (Sec. 2.3): edge-centre height of eta1 (lower-layer velocity) and of
// h2 (upper-layer velocity) from the two Gauss points' convex combinations

__device__ inline double rec_at(const double *rec, int64_t T, int slot, int comp, int q, int64_t c)
{
    return rec[((int64_t)(slot * 6 + comp) * 3 + q) * T + c];
}

__global__ void k_hhat(MeshDev m, Phys p, const double *__restrict__ rec, double *__restrict__ hmid)
{
    int64_t e = xcd_block() * blockDim.x + threadIdx.x;
    if (e >= m.E) return;
    const int64_t T = m.T, E = m.E;
    const int32_t L = m.eL[e], R = m.eR[e], sl = m.eslot[e];
    const int kL = sl & 3, kR = sl >> 2;
    const double nx = m.en[e], ny = m.en[E + e];
    double acc0 = 0, acc1 = 0;
#pragma unroll
    for (int g = 0; g < 2; g++) {
        const double Bg = m.eBgp[g * E + e];
        const int sL = 2 * kL + g, sR = 2 * kR + 1 - g;
#pragma unroll
        for (int f = 0; f < 2; f++) {
            const int o = (f == 0) ? 3 : 0;
            double zl = rec_at(rec, T, sL, o, 0, L);
            double hl = (f == 0) ? zl - Bg : zl;
            double unl = (rec_at(rec, T, sL, o + 1, 0, L) * nx + rec_at(rec, T, sL, o + 2, 0, L) * ny) / hl;
            double zr, hr, unr;
            if (R >= 0) {
                zr = rec_at(rec, T, sR, o, 0, R);
                hr = (f == 0) ? zr - Bg : zr;
                unr = (rec_at(rec, T, sR, o + 1, 0, R) * nx + rec_at(rec, T, sR, o + 2, 0, R) * ny) / hr;
            } else {  // mirror state across the wall
                zr = zl;
                hr = hl;
                unr = -unl;
            }
            // reading: xi is the kinetic fraction of particles moving from left to right
            double lb = 2.0 / (p.G * (hl + hr));
            double xi = 0.5 * erfc(-sqrt(lb) * 0.5 * (unl + unr));
            double hh = xi * zl + (1 - xi) * zr;
            if (f == 0) acc0 += 0.5 * hh; else acc1 += 0.5 * hh;
        }
    }
    hmid[e] = acc0;
    hmid[E + e] = acc1;
}

// gradient of the plane through the three edge-centre heights (Green-Gauss, exact for planes)
__global__ void k_plane(MeshDev m, const double *__restrict__ hmid, double *__restrict__ gP1)
{
    int64_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= m.T) return;
    const int64_t T = m.T, E = m.E;
    double s[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        int32_t code = m.cedge[k * T + c];
        int64_t e = code >= 0 ? code : ~code;
        double gx = m.gg[(2 * k) * T + c], gy = m.gg[(2 * k + 1) * T + c];
        double h0 = hmid[e], h1 = hmid[E + e];
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

struct SideL {
    double h, U, V;               // state
    double hn, ht, mnn, mnt, mtn, mtt;  // d/dn, d/dt of h, h U_n, h U_t
    double pn, pt;                // acceleration
};

// u-moments M_0..M_5 of the Gaussian (mean U, variance th = 1/(2 lam)) restricted by sign s
__device__ inline void u_moments(double U, double th, double m0, double m1, double *M)
{
    M[0] = m0;
    M[1] = m1;
#pragma unroll
    for (int k = 2; k < 6; k++) M[k] = U * M[k - 1] + (k - 1) * th * M[k - 2];
}

// slope coefficients of one side's derivatives for a Maxwellian of state (h, U, V, lam)
struct Slope {
    double an, bn, gn, at, bt, gt;
};

__device__ inline Slope slope_of(const SideL &s, double h, double U, double V, double lam)
{
    Slope r;
    double ih = 1.0 / h;
    r.an = lam * s.hn * ih;
    r.bn = 2 * lam * (s.mnn - U * s.hn) * ih;
    r.gn = 2 * lam * (s.mtn - V * s.hn) * ih;
    r.at = lam * s.ht * ih;
    r.bt = 2 * lam * (s.mnt - U * s.ht) * ih;
    r.gt = 2 * lam * (s.mtt - V * s.ht) * ih;
    return r;
}

// moments of P (slope sl, force (pn, pt)) over a half Maxwellian with thickness h, means (U, V),
// lam, th = 1/(2 lam), u-moments M.  e = 0: <psi P>, e = 1: <u psi P>.
__device__ inline void poly_moments(const Slope &sl, double pn, double pt, double h, double U, double V,
                                    double lam, double th, const double *M, int e, double *out)
{
    double N1[5], N2[4];
#pragma unroll
    for (int k = 0; k < 5; k++) N1[k] = M[k + 1] - U * M[k];
#pragma unroll
    for (int k = 0; k < 4; k++) N2[k] = N1[k + 1] - U * N1[k];
    const double fn = sl.bt * V - 2 * lam * pn;
    const double q2 = sl.at * V + sl.gt;
    double Q[2], Rv;
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const int j = e + i;
        Q[i] = sl.an * N2[j + 1] + sl.at * V * N2[j] + sl.bn * N1[j + 1] + fn * N1[j] +
               th * (sl.an * M[j + 1] + q2 * M[j]);
    }
    Rv = th * (sl.gn * M[e + 1] + (sl.gt * V - 2 * lam * pt) * M[e] + sl.at * N2[e] + sl.bt * N1[e]) +
         3 * th * th * sl.at * M[e];
    out[0] = h * Q[0];
    out[1] = h * Q[1];
    out[2] = h * (V * Q[0] + Rv);
}

__device__ inline void gks_point(const SideL &sl, const SideL &sr, double G, double eps, double eps_num,
                                 double dt, double *F0, double *Ft, double *Wb, double *Wbt)
{
    const double lamL = 1.0 / (G * sl.h), lamR = 1.0 / (G * sr.h);
    const double thL = 0.5 * G * sl.h, thR = 0.5 * G * sr.h;
    const double spi = 1.7724538509055160273;  // sqrt(pi)
    double ML[6], MR[6];
    {
        double sq = sqrt(lamL);
        double m0 = 0.5 * erfc(-sq * sl.U);
        double ex = exp(-lamL * sl.U * sl.U) / (2 * spi * sq);
        u_moments(sl.U, thL, m0, sl.U * m0 + ex, ML);
    }
    {
        double sq = sqrt(lamR);
        double m0 = 0.5 * erfc(sq * sr.U);
        double ex = exp(-lamR * sr.U * sr.U) / (2 * spi * sq);
        u_moments(sr.U, thR, m0, sr.U * m0 - ex, MR);
    }
    // interface equilibrium state
    double wb0 = sl.h * ML[0] + sr.h * MR[0];
    double wb1 = sl.h * ML[1] + sr.h * MR[1];
    double wb2 = sl.h * ML[0] * sl.V + sr.h * MR[0] * sr.V;
    const double hb = wb0, Ub = wb1 / hb, Vb = wb2 / hb;
    const double lamb = 1.0 / (G * hb), thb = 0.5 * G * hb;
    double Mp[6], Mm[6];
    {
        double sq = sqrt(lamb);
        double m0p = 0.5 * erfc(-sq * Ub), m0m = 0.5 * erfc(sq * Ub);
        double ex = exp(-lamb * Ub * Ub) / (2 * spi * sq);
        u_moments(Ub, thb, m0p, Ub * m0p + ex, Mp);
        u_moments(Ub, thb, m0m, Ub * m0m - ex, Mm);
    }
    const Slope bL = slope_of(sl, hb, Ub, Vb, lamb), bR = slope_of(sr, hb, Ub, Vb, lamb);
    // time slope of the interface equilibrium from compatibility
    double t1[3], t2[3], wt[3];
    poly_moments(bL, sl.pn, sl.pt, hb, Ub, Vb, lamb, thb, Mp, 0, t1);
    poly_moments(bR, sr.pn, sr.pt, hb, Ub, Vb, lamb, thb, Mm, 0, t2);
#pragma unroll
    for (int i = 0; i < 3; i++) wt[i] = -(t1[i] + t2[i]);
    // brackets multiplying the five time coefficients
    double B1[3], B2[3], B3[3], B4[3], B5[3];
    B1[0] = hb * Ub;
    B1[1] = hb * (Ub * Ub + thb);
    B1[2] = hb * Ub * Vb;
    poly_moments(bL, sl.pn, sl.pt, hb, Ub, Vb, lamb, thb, Mp, 1, t1);
    poly_moments(bR, sr.pn, sr.pt, hb, Ub, Vb, lamb, thb, Mm, 1, t2);
#pragma unroll
    for (int i = 0; i < 3; i++) B2[i] = t1[i] + t2[i];
    {
        const double ih = 1.0 / hb;
        const double aA = lamb * wt[0] * ih;
        const double bA = 2 * lamb * (wt[1] - Ub * wt[0]) * ih;
        const double gA = 2 * lamb * (wt[2] - Vb * wt[0]) * ih;
        const double mA = 2 * aA * thb;  // <A>
        B3[0] = hb * (Ub * mA + bA * thb);
        B3[1] = hb * (Ub * Ub * mA + 2 * Ub * bA * thb + 4 * aA * thb * thb);
        B3[2] = hb * (Ub * Vb * mA + Ub * gA * thb + Vb * bA * thb);
    }
    B4[0] = sl.h * ML[1] + sr.h * MR[1];
    B4[1] = sl.h * ML[2] + sr.h * MR[2];
    B4[2] = sl.h * ML[1] * sl.V + sr.h * MR[1] * sr.V;
    {
        const Slope aL = slope_of(sl, sl.h, sl.U, sl.V, lamL), aR = slope_of(sr, sr.h, sr.U, sr.V, lamR);
        poly_moments(aL, sl.pn, sl.pt, sl.h, sl.U, sl.V, lamL, thL, ML, 1, t1);
        poly_moments(aR, sr.pn, sr.pt, sr.h, sr.U, sr.V, lamR, thR, MR, 1, t2);
#pragma unroll
        for (int i = 0; i < 3; i++) B5[i] = t1[i] + t2[i];
    }
    // collision time (Sec. 4) in units of dt, and the flux / flux-rate weights of F(dt), F(dt/2)
    const double pl = sl.h * sl.h, pr = sr.h * sr.h;
    const double r = eps + eps_num * fabs((pl - pr) / (pl + pr));
    const double E2 = exp(-0.5 / r), E1 = E2 * E2, a1 = 1 - E1, a2 = 1 - E2;
    const double c01 = 1 - 4 * r * a2 + r * a1, ct1 = 4 * r * (2 * a2 - a1);
    const double c04 = r * (4 * a2 - a1), ct4 = 4 * r * (a1 - 2 * a2);
    const double c02 = -r + r * r * (8 * a2 - 2 * a1) - 2 * r * E2 + r * E1;
    const double ct2 = 4 * (2 * r * r * (a1 - 2 * a2) + r * (E2 - E1));
    const double c03 = -r + r * r * (4 * a2 - a1), ct3 = 4 * (0.25 + r * r * (a1 - 2 * a2));
    const double c05 = r * (2 + 4 * r) * E2 - r * (1 + r) * E1 - 3 * r * r;
    const double ct5 = 4 * (r * (1 + r) * E1 - r * (1 + 2 * r) * E2 + r * r);
    const double idt = 1.0 / dt;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        F0[i] = c01 * B1[i] + c04 * B4[i] + dt * (c02 * B2[i] + c03 * B3[i] + c05 * B5[i]);
        Ft[i] = (ct1 * B1[i] + ct4 * B4[i]) * idt + ct2 * B2[i] + ct3 * B3[i] + ct5 * B5[i];
    }
    Wb[0] = wb0;
    Wb[1] = wb1;
    Wb[2] = wb2;
    Wbt[0] = wt[0];
    Wbt[1] = wt[1];
    Wbt[2] = wt[2];
}

// one thread per (edge, Gauss point, layer); the two Gauss points of an edge are adjacent lanes
__global__ void __launch_bounds__(256) k_flux(MeshDev m, Phys p, const double *__restrict__ dtp,
                                              const double *__restrict__ rec, const double *__restrict__ r0,
                                              const double *__restrict__ gP1, double *__restrict__ eo)
{
    const int64_t idx = xcd_block() * blockDim.x + threadIdx.x;
    const int64_t e = idx >> 2;
    const int g = idx & 1, lay = (idx >> 1) & 1;  // lay 0: lower layer (h1), 1: upper (h2)
    if (e >= m.E) return;
    const int64_t T = m.T, E = m.E;
    const double dt = dtp[0];
    const int32_t L = m.eL[e], R = m.eR[e], sl = m.eslot[e];
    const int kL = sl & 3, kR = sl >> 2;
    const int sL = 2 * kL + g, sR = 2 * kR + 1 - g;
    const double nx = m.en[e], ny = m.en[E + e], tx = -ny, ty = nx;
    const double Bg = m.eBgp[g * E + e];
    const double gBx = m.egB[e], gBy = m.egB[E + e];
    const int o = lay == 0 ? 3 : 0;   // own variables in the state / records
    const int fo = lay == 0 ? 0 : 3;  // the other layer's height drives this layer's force
    const int ff = lay == 0 ? 1 : 0;  // modelled field index (0: eta1, 1: h2)
    // nonlinear weight of the force model
    double rL = r0[ff * T + L], rR = R >= 0 ? r0[ff * T + R] : rL;
    const double wf = fmin(1.0, fmin(rL, rR));
    SideL side[2];
#pragma unroll
    for (int s = 0; s < 2; s++) {
        if (s == 1 && R < 0) break;
        const int cell = s == 0 ? L : R, slot = s == 0 ? sL : sR;
        double h = rec_at(rec, T, slot, o, 0, cell);
        double hx = rec_at(rec, T, slot, o, 1, cell), hy = rec_at(rec, T, slot, o, 2, cell);
        if (lay == 0) {  // eta1 -> h1 with the single-valued bottom at the Gauss point
            h -= Bg;
            hx -= gBx;
            hy -= gBy;
        }
        const double mx = rec_at(rec, T, slot, o + 1, 0, cell), my = rec_at(rec, T, slot, o + 2, 0, cell);
        const double mxx = rec_at(rec, T, slot, o + 1, 1, cell), mxy = rec_at(rec, T, slot, o + 1, 2, cell);
        const double myx = rec_at(rec, T, slot, o + 2, 1, cell), myy = rec_at(rec, T, slot, o + 2, 2, cell);
        const double fx = rec_at(rec, T, slot, fo, 1, cell), fy = rec_at(rec, T, slot, fo, 2, cell);
        const double px1 = gP1[(2 * ff) * T + cell], py1 = gP1[(2 * ff + 1) * T + cell];
        const double dfx = wf * fx + (1 - wf) * px1, dfy = wf * fy + (1 - wf) * py1;
        double ax, ay;
        if (lay == 0) {  // lower layer: bottom slope and upper-layer thickness (chi weighted)
            ax = -p.G * gBx - p.chi * p.G * dfx;
            ay = -p.G * gBy - p.chi * p.G * dfy;
        } else {         // upper layer: slope of the interface level
            ax = -p.G * dfx;
            ay = -p.G * dfy;
        }
        SideL &q = side[s];
        q.h = h;
        q.U = (mx * nx + my * ny) / h;
        q.V = (mx * tx + my * ty) / h;
        q.hn = hx * nx + hy * ny;
        q.ht = hx * tx + hy * ty;
        const double dmn_x = mxx * nx + myx * ny, dmn_y = mxy * nx + myy * ny;  // grad (m . n)
        const double dmt_x = mxx * tx + myx * ty, dmt_y = mxy * tx + myy * ty;  // grad (m . t)
        q.mnn = dmn_x * nx + dmn_y * ny;
        q.mnt = dmn_x * tx + dmn_y * ty;
        q.mtn = dmt_x * nx + dmt_y * ny;
        q.mtt = dmt_x * tx + dmt_y * ty;
        q.pn = ax * nx + ay * ny;
        q.pt = ax * tx + ay * ty;
    }
    if (R < 0) {  // wall: mirror image of the left side
        side[1] = side[0];
        side[1].U = -side[0].U;
        side[1].hn = -side[0].hn;
        side[1].mnt = -side[0].mnt;
        side[1].mtn = -side[0].mtn;
        side[1].pn = -side[0].pn;
    }
    double F0[3], Ft[3], Wb[3], Wbt[3];
    gks_point(side[0], side[1], p.G, p.eps, p.eps_num, dt, F0, Ft, Wb, Wbt);
    if (R < 0) {
        F0[0] = 0;
        Ft[0] = 0;
    }
    // back to the global frame, then average the edge's two Gauss points (weights 1/2)
    double out[12];
    const double *src[4] = {F0, Ft, Wb, Wbt};
#pragma unroll
    for (int q = 0; q < 4; q++) {
        out[3 * q] = src[q][0];
        out[3 * q + 1] = src[q][1] * nx + src[q][2] * tx;
        out[3 * q + 2] = src[q][1] * ny + src[q][2] * ty;
    }
#pragma unroll
    for (int i = 0; i < 12; i++) out[i] = 0.5 * (out[i] + __shfl_xor(out[i], 1));
    // lane g = 0 stores F0, Ft; lane g = 1 stores Wb, Wbt
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const int qq = 2 * g + q;
#pragma unroll
        for (int i = 0; i < 3; i++) eo[((int64_t)(qq * 6 + o + i)) * E + e] = out[3 * qq + i];
    }
}

// --------------------------------------------------------------------------------------------
// cell update: deterministic gather of the three edges, sources, S2O4 stage update

// stage 0: Ws = W + dt/2 L + dt^2/8 Lt, gWs = G + dt/2 Gt; carry Wc = W + dt L + dt^2/6 Lt, Gc = G
// stage 1: W = Wc + dt^2/3 Lt, gW = Gc + dt Gt
__global__ void __launch_bounds__(256) k_update(MeshDev m, Phys p, int stage, const double *__restrict__ dtp,
                                                const double *__restrict__ eo, const double *__restrict__ Win,
                                                double *__restrict__ Wout, double *__restrict__ gWout,
                                                double *__restrict__ Wc, double *__restrict__ Gc)
{
    int64_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= m.T) return;
    const int64_t T = m.T, E = m.E, TG = m.T + m.NG;
    const double dt = dtp[0], G = p.G;
    double LF[6] = {0}, LFt[6] = {0}, GG[6][2] = {{0}}, GGt[6][2] = {{0}}, hs[2] = {0, 0}, hts[2] = {0, 0};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        int32_t code = m.cedge[k * T + c];
        int64_t e = code >= 0 ? code : ~code;
        const double f = m.fl[k * T + c], gx = m.gg[(2 * k) * T + c], gy = m.gg[(2 * k + 1) * T + c];
#pragma unroll
        for (int v = 0; v < 6; v++) {
            const double F0 = eo[(0 * 6 + v) * E + e], Ft = eo[(1 * 6 + v) * E + e];
            const double Wb = eo[(2 * 6 + v) * E + e], Wbt = eo[(3 * 6 + v) * E + e];
            LF[v] -= f * F0;
            LFt[v] -= f * Ft;
            GG[v][0] += gx * Wb;
            GG[v][1] += gy * Wb;
            GGt[v][0] += gx * Wbt;
            GGt[v][1] += gy * Wbt;
            if (v == 0) { hs[1] += Wb; hts[1] += Wbt; }
            if (v == 3) { hs[0] += Wb; hts[0] += Wbt; }
        }
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
    Lt[4] += -p.chi * G * (hts[0] * GG[0][0] + hs[0] * GGt[0][0]);
    Lt[5] += -p.chi * G * (hts[0] * GG[0][1] + hs[0] * GGt[0][1]);
    Lt[1] += -G * (hts[1] * GG[3][0] + hs[1] * GGt[3][0]);
    Lt[2] += -G * (hts[1] * GG[3][1] + hs[1] * GGt[3][1]);
    if (stage == 0) {
        double L[6];
#pragma unroll
        for (int v = 0; v < 6; v++) L[v] = LF[v];
        const double h2 = Win[0 * TG + c], h1 = Win[3 * TG + c] - m.Bbar[c];
        // bottom source h_j (0, -G B_x, -G B_y) (Sec. 3.2) and layer coupling
        // (Eq. SWE-source-discretization) from the Gauss-point mean thickness and the Green-Gauss
        // derivative of the other layer's interface thickness
        L[1] += h2 * (-G * gBx) - G * hs[1] * GG[3][0];
        L[2] += h2 * (-G * gBy) - G * hs[1] * GG[3][1];
        L[4] += h1 * (-G * gBx) - p.chi * G * hs[0] * GG[0][0];
        L[5] += h1 * (-G * gBy) - p.chi * G * hs[0] * GG[0][1];
        // the state carries grad(eta1) = grad(h1) + grad(B)
        GG[3][0] += gBx;
        GG[3][1] += gBy;
#pragma unroll
        for (int v = 0; v < 6; v++) {
            const double w = Win[v * TG + c];
            Wout[v * TG + c] = w + 0.5 * dt * L[v] + 0.125 * dt * dt * Lt[v];
            Wc[v * T + c] = w + dt * L[v] + (dt * dt / 6.0) * Lt[v];
#pragma unroll
            for (int d = 0; d < 2; d++) {
                gWout[(2 * v + d) * TG + c] = GG[v][d] + 0.5 * dt * GGt[v][d];
                Gc[(2 * v + d) * T + c] = GG[v][d];
            }
        }
    } else {
#pragma unroll
        for (int v = 0; v < 6; v++) {
            Wout[v * TG + c] = Wc[v * T + c] + (dt * dt / 3.0) * Lt[v];
#pragma unroll
            for (int d = 0; d < 2; d++) gWout[(2 * v + d) * TG + c] = Gc[(2 * v + d) * T + c] + dt * GGt[v][d];
        }
    }
}

// --------------------------------------------------------------------------------------------
// time step: per-block maxima of the wave speed, then one block finishes (no atomics)

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

__global__ void __launch_bounds__(DT_BLOCK) k_dt_partial(MeshDev m, Phys p, const double *__restrict__ W,
                                                          double *__restrict__ part)
{
    __shared__ double sh[DT_BLOCK / 64];
    const int64_t T = m.T, TG = m.T + m.NG;
    double smax = 0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < T; c += (int64_t)gridDim.x * blockDim.x) {
        const double h2 = W[c], h1 = W[3 * TG + c] - m.Bbar[c];
        const double u2 = W[TG + c] / h2, v2 = W[2 * TG + c] / h2;
        const double u1 = W[4 * TG + c] / h1, v1 = W[5 * TG + c] / h1;
        const double s1 = sqrt(u1 * u1 + v1 * v1) + sqrt(p.G * h1);
        const double s2 = sqrt(u2 * u2 + v2 * v2) + sqrt(p.G * h2);
        smax = fmax(smax, fmax(s1, s2));
    }
    smax = block_max(smax, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = smax;
}

// scal[0] = dt of this step, scal[1] = time at the end of this step
__global__ void __launch_bounds__(DT_BLOCK) k_dt_final(MeshDev m, Phys p, const double *__restrict__ part,
                                                        int nparts, double *__restrict__ scal)
{
    __shared__ double sh[DT_BLOCK / 64];
    double v = 0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) v = fmax(v, part[i]);
    v = block_max(v, sh);
    if (threadIdx.x == 0) {
        double dt = p.cfl * m.dxmin / v;
        const double t = scal[1];
        if (t + dt > p.t_end) dt = p.t_end - t;
        scal[0] = dt;
        scal[1] = t + dt;
    }
}

__global__ void k_set_dt(double *scal, double dt)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        scal[0] = dt;
        scal[1] += dt;
    }
}

// per-layer mass: fixed-order block sums (deterministic)
__global__ void __launch_bounds__(256) k_mass_partial(MeshDev m, const double *__restrict__ W,
                                                      double *__restrict__ part)
{
    __shared__ double sh[2][256];
    const int64_t T = m.T, TG = m.T + m.NG;
    double a = 0, b = 0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < T; c += (int64_t)gridDim.x * blockDim.x) {
        a += m.area[c] * W[c];
        b += m.area[c] * (W[3 * TG + c] - m.Bbar[c]);
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

}  // namespace gks
