// Host-side mesh preprocessing: connectivity, compact stencils with mirror ghost cells, scaled
// geometry and the least-squares reconstruction operators (Sec. 3.4), all in FP64.
#include "mesh_setup.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <thread>
#include <tuple>
#include <unordered_map>

namespace gks {
namespace {

// x' = [a b; c d] x + (tx, ty)
struct Aff {
    double a, b, c, d, tx, ty;
};

Aff aff_id() { return {1, 0, 0, 1, 0, 0}; }
Aff aff_shift(double x, double y) { return {1, 0, 0, 1, x, y}; }

// outer(inner(x))
Aff aff_then(const Aff &o, const Aff &i)
{
    return {o.a * i.a + o.b * i.c, o.a * i.b + o.b * i.d, o.c * i.a + o.d * i.c, o.c * i.b + o.d * i.d,
            o.a * i.tx + o.b * i.ty + o.tx, o.c * i.tx + o.d * i.ty + o.ty};
}

// reflection across the line through p and q
Aff aff_reflect(double px, double py, double qx, double qy)
{
    double ux = qx - px, uy = qy - py, l = std::hypot(ux, uy);
    ux /= l;
    uy /= l;
    Aff r{ux * ux - uy * uy, 2 * ux * uy, 2 * ux * uy, uy * uy - ux * ux, 0, 0};
    r.tx = px - (r.a * px + r.b * py);
    r.ty = py - (r.c * px + r.d * py);
    return r;
}

void aff_apply(const Aff &f, double x, double y, double &X, double &Y)
{
    X = f.a * x + f.b * y + f.tx;
    Y = f.c * x + f.d * y + f.ty;
}

bool aff_is_translation(const Aff &f)
{
    return std::fabs(f.a - 1) < 1e-12 && std::fabs(f.b) < 1e-12 && std::fabs(f.c) < 1e-12 &&
           std::fabs(f.d - 1) < 1e-12;
}

// scaled cubic basis about the owner's centroid: xi, eta, xi^2, xi eta, eta^2, xi^3, xi^2 eta,
// xi eta^2, eta^3 (the polynomial space of Eq. Recons-poly; the scaling only rescales columns)
void basis(double x, double y, double *f, double *fx, double *fy)
{
    f[0] = x; f[1] = y; f[2] = x * x; f[3] = x * y; f[4] = y * y;
    f[5] = x * x * x; f[6] = x * x * y; f[7] = x * y * y; f[8] = y * y * y;
    fx[0] = 1; fx[1] = 0; fx[2] = 2 * x; fx[3] = y; fx[4] = 0;
    fx[5] = 3 * x * x; fx[6] = 2 * x * y; fx[7] = y * y; fx[8] = 0;
    fy[0] = 0; fy[1] = 1; fy[2] = 0; fy[3] = x; fy[4] = 2 * y;
    fy[5] = 0; fy[6] = x * x; fy[7] = 2 * x * y; fy[8] = 3 * y * y;
}

// averages over a triangle of the basis and its derivatives: 7-point rule (vertices 1/20, edge
// midpoints 2/15, centroid 9/20), exact for cubics
void tri_basis_avg(const double v[3][2], double *f, double *fx, double *fy)
{
    for (int k = 0; k < 9; k++) f[k] = fx[k] = fy[k] = 0;
    double pts[7][2], w[7];
    for (int i = 0; i < 3; i++) {
        pts[i][0] = v[i][0];
        pts[i][1] = v[i][1];
        w[i] = 1.0 / 20.0;
        pts[3 + i][0] = 0.5 * (v[i][0] + v[(i + 1) % 3][0]);
        pts[3 + i][1] = 0.5 * (v[i][1] + v[(i + 1) % 3][1]);
        w[3 + i] = 2.0 / 15.0;
    }
    pts[6][0] = (v[0][0] + v[1][0] + v[2][0]) / 3.0;
    pts[6][1] = (v[0][1] + v[1][1] + v[2][1]) / 3.0;
    w[6] = 9.0 / 20.0;
    for (int p = 0; p < 7; p++) {
        double b[9], bx[9], by[9];
        basis(pts[p][0], pts[p][1], b, bx, by);
        for (int k = 0; k < 9; k++) {
            f[k] += w[p] * b[k];
            fx[k] += w[p] * bx[k];
            fy[k] += w[p] * by[k];
        }
    }
}

// cell means of the basis for a triangle whose centroid is the origin: quadratic monomials
// average to (1/12) sum over vertices, cubic ones to (1/30) sum over vertices
void centroid_means(const double v[3][2], double *mean)
{
    double s[9] = {0};
    for (int i = 0; i < 3; i++) {
        double x = v[i][0], y = v[i][1];
        s[2] += x * x; s[3] += x * y; s[4] += y * y;
        s[5] += x * x * x; s[6] += x * x * y; s[7] += x * y * y; s[8] += y * y * y;
    }
    mean[0] = mean[1] = 0;
    for (int k = 2; k < 5; k++) mean[k] = s[k] / 12.0;
    for (int k = 5; k < 9; k++) mean[k] = s[k] / 30.0;
}

// least-squares operator M (9 x 17) = R^-1 Q^T of A (17 x 9) by Givens rotations
void lsq_operator(double A[17][9], double *M)
{
    double Qt[17][17];
    for (int i = 0; i < 17; i++)
        for (int j = 0; j < 17; j++) Qt[i][j] = (i == j) ? 1.0 : 0.0;
    for (int j = 0; j < 9; j++) {
        for (int i = 16; i > j; i--) {
            double x = A[j][j], y = A[i][j];
            if (y == 0) continue;
            double r = std::hypot(x, y), c = x / r, s = y / r;
            for (int k = 0; k < 9; k++) {
                double p = A[j][k], q = A[i][k];
                A[j][k] = c * p + s * q;
                A[i][k] = -s * p + c * q;
            }
            for (int k = 0; k < 17; k++) {
                double p = Qt[j][k], q = Qt[i][k];
                Qt[j][k] = c * p + s * q;
                Qt[i][k] = -s * p + c * q;
            }
        }
    }
    for (int r = 0; r < 17; r++) {
        double col[9];
        for (int i = 8; i >= 0; i--) {
            double s = Qt[i][r];
            for (int k = i + 1; k < 9; k++) s -= A[i][k] * col[k];
            col[i] = s / A[i][i];
        }
        for (int i = 0; i < 9; i++) M[i * 17 + r] = col[i];
    }
}

}  // namespace

int build_host_mesh(const double *xy, int64_t nn, const int32_t *tri, int64_t nt, const double *B,
                    int bc, const double *L, HostMesh &m, std::string &err)
{
    if (nn <= 0 || nt <= 0 || !xy || !tri) {
        err = "empty mesh";
        return 1;
    }
    for (int64_t i = 0; i < 3 * nt; i++)
        if (tri[i] < 0 || tri[i] >= nn) {
            err = "triangle references a node out of range";
            return 1;
        }
    const bool periodic = (bc == 1), freebc = (bc == 2);
    if (bc < 0 || bc > 2) {
        err = "unknown boundary kind";
        return 1;
    }
    if (periodic && (!L || !(L[0] > 0) || !(L[1] > 0))) {
        err = "periodic mesh needs positive periods";
        return 1;
    }
    auto X = [&](int64_t c, int k, double &x, double &y) {
        int32_t v = tri[3 * c + (k % 3)];
        x = xy[2 * v];
        y = xy[2 * v + 1];
    };
    auto Bn = [&](int64_t c, int k) { return B ? B[tri[3 * c + (k % 3)]] : 0.0; };

    // node identification under the periodic wrap
    std::vector<int64_t> canon(nn);
    if (periodic) {
        std::unordered_map<uint64_t, int64_t> seen;
        seen.reserve(2 * nn);
        for (int64_t i = 0; i < nn; i++) {
            uint64_t key[2];
            for (int d = 0; d < 2; d++) {
                double f = xy[2 * i + d] / L[d];
                f -= std::floor(f);
                long long q = std::llround(f * 1073741824.0);
                if (q >= 1073741824LL) q -= 1073741824LL;
                key[d] = (uint64_t)q;
            }
            uint64_t k = (key[0] << 32) | key[1];
            auto it = seen.find(k);
            if (it == seen.end()) {
                seen.emplace(k, i);
                canon[i] = i;
            } else {
                canon[i] = it->second;
            }
        }
    } else {
        for (int64_t i = 0; i < nn; i++) canon[i] = i;
    }

    // cells
    m.nt = nt;
    m.area.assign(nt, 0);
    m.hs.assign(nt, 0);
    m.vtx.assign(6 * nt, 0);
    m.Bbar.assign(nt, 0);
    m.gB.assign(2 * nt, 0);
    std::vector<double> cx(nt), cy(nt);
    m.dxmin = 1e300;
    for (int64_t c = 0; c < nt; c++) {
        double x[3], y[3];
        for (int k = 0; k < 3; k++) X(c, k, x[k], y[k]);
        double ar = 0.5 * ((x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]));
        if (!(ar > 0) || !std::isfinite(ar)) {
            err = "inverted or degenerate triangle " + std::to_string(c);
            return 1;
        }
        m.area[c] = ar;
        cx[c] = (x[0] + x[1] + x[2]) / 3.0;
        cy[c] = (y[0] + y[1] + y[2]) / 3.0;
        double hs = std::sqrt(2.0 * ar);
        m.hs[c] = hs;
        double lmax = 0;
        for (int k = 0; k < 3; k++) {
            m.vtx[(2 * k) * nt + c] = (x[k] - cx[c]) / hs;
            m.vtx[(2 * k + 1) * nt + c] = (y[k] - cy[c]) / hs;
            lmax = std::max(lmax, std::hypot(x[(k + 1) % 3] - x[k], y[(k + 1) % 3] - y[k]));
        }
        m.dxmin = std::min(m.dxmin, 2.0 * ar / lmax);
        double b0 = Bn(c, 0), b1 = Bn(c, 1), b2 = Bn(c, 2);
        m.Bbar[c] = (b0 + b1 + b2) / 3.0;
        // plane through the three vertex values
        double a11 = x[1] - x[0], a12 = y[1] - y[0], a21 = x[2] - x[0], a22 = y[2] - y[0];
        double r1 = b1 - b0, r2 = b2 - b0, det = a11 * a22 - a12 * a21;
        m.gB[c] = (r1 * a22 - a12 * r2) / det;
        m.gB[nt + c] = (a11 * r2 - r1 * a21) / det;
    }

    // edges: first incidence is the left cell
    std::unordered_map<uint64_t, int64_t> emap;
    emap.reserve(3 * nt);
    std::vector<int32_t> eL, eR, ekL, ekR;
    std::vector<uint8_t> eup;  // direction of the edge in its left cell: from the smaller node id
    std::vector<int32_t> cedge(3 * nt);
    for (int64_t c = 0; c < nt; c++)
        for (int k = 0; k < 3; k++) {
            uint64_t a = canon[tri[3 * c + k]], b = canon[tri[3 * c + (k + 1) % 3]];
            if (a == b) {
                err = "degenerate edge";
                return 1;
            }
            uint64_t key = (std::min(a, b) << 32) | std::max(a, b);
            auto it = emap.find(key);
            if (it == emap.end()) {
                int64_t e = (int64_t)eL.size();
                emap.emplace(key, e);
                eup.push_back(a < b ? 1 : 0);
                eL.push_back((int32_t)c);
                ekL.push_back(k);
                eR.push_back(-1);
                ekR.push_back(-1);
                cedge[3 * c + k] = (int32_t)e;
            } else {
                int64_t e = it->second;
                if (eR[e] >= 0) {
                    err = "edge shared by more than two triangles";
                    return 1;
                }
                if ((a < b ? 1 : 0) == eup[e]) {
                    err = "edge traversed in the same direction by two triangles (overlapping or "
                          "inconsistently oriented triangles)";
                    return 1;
                }
                eR[e] = (int32_t)c;
                ekR[e] = k;
                cedge[3 * c + k] = ~(int32_t)e;
            }
        }
    const int64_t ne = (int64_t)eL.size();
    m.ne = ne;
    m.eL = eL;
    m.eR = eR;
    m.eslot.assign(ne, 0);
    m.en.assign(2 * ne, 0);
    m.eBgp.assign(2 * ne, 0);
    m.egB.assign(2 * ne, 0);
    std::vector<Aff> eshift(ne, aff_id());  // right cell's coordinates -> left cell's frame
    std::vector<double> elen(ne);
    const double s0 = 0.5 - std::sqrt(3.0) / 6.0, s1 = 0.5 + std::sqrt(3.0) / 6.0;
    for (int64_t e = 0; e < ne; e++) {
        if (eR[e] < 0 && periodic) {
            err = "unpaired boundary edge on a periodic mesh";
            return 1;
        }
        m.eslot[e] = ekL[e] | ((eR[e] >= 0 ? ekR[e] : 0) << 2);
        double px, py, qx, qy;
        X(eL[e], ekL[e], px, py);
        X(eL[e], ekL[e] + 1, qx, qy);
        double len = std::hypot(qx - px, qy - py);
        elen[e] = len;
        double nx = (qy - py) / len, ny = (px - qx) / len;
        m.en[e] = nx;
        m.en[ne + e] = ny;
        double bp = Bn(eL[e], ekL[e]), bq = Bn(eL[e], ekL[e] + 1);
        m.eBgp[e] = (1 - s0) * bp + s0 * bq;
        m.eBgp[ne + e] = (1 - s1) * bp + s1 * bq;
        double gLx = m.gB[eL[e]], gLy = m.gB[nt + eL[e]], gRx, gRy;
        if (eR[e] >= 0) {
            double rx, ry, rqx, rqy;
            X(eR[e], ekR[e] + 1, rx, ry);  // the right cell's copy of node p
            X(eR[e], ekR[e], rqx, rqy);    // ... and of node q
            eshift[e] = aff_shift(px - rx, py - ry);
            if (std::fabs(rqx + (px - rx) - qx) > 1e-9 * (1 + std::fabs(qx)) ||
                std::fabs(rqy + (py - ry) - qy) > 1e-9 * (1 + std::fabs(qy))) {
                err = "the two cells of an edge do not share its end points (up to the periodic shift)";
                return 1;
            }
            gRx = m.gB[eR[e]];
            gRy = m.gB[nt + eR[e]];
        } else {
            // mirror of the left cell across the wall: (I - 2 n n^T) grad B
            double dn = gLx * nx + gLy * ny;
            gRx = gLx - 2 * dn * nx;
            gRy = gLy - 2 * dn * ny;
        }
        m.egB[e] = 0.5 * (gLx + gRx);
        m.egB[ne + e] = 0.5 * (gLy + gRy);
    }

    // per-cell edge factors
    m.cedge = std::vector<int32_t>(3 * nt);
    m.fl.assign(3 * nt, 0);
    m.gg.assign(6 * nt, 0);
    for (int64_t c = 0; c < nt; c++)
        for (int k = 0; k < 3; k++) {
            int32_t code = cedge[3 * c + k];
            int64_t e = code >= 0 ? code : ~code;
            double sg = code >= 0 ? 1.0 : -1.0;
            m.cedge[k * nt + c] = code;
            double f = sg * elen[e] / m.area[c];
            m.fl[k * nt + c] = f;
            m.gg[(2 * k) * nt + c] = f * m.en[e];
            m.gg[(2 * k + 1) * nt + c] = f * m.en[ne + e];
        }

    // neighbour image across local edge k of cell c
    auto neighbour = [&](int64_t c, int k, int64_t &n, Aff &T, int &back) {
        int32_t code = cedge[3 * c + k];
        if (code >= 0) {
            int64_t e = code;
            if (eR[e] < 0) {  // wall: the cell mirrored across the edge
                double px, py, qx, qy;
                X(c, k, px, py);
                X(c, k + 1, qx, qy);
                n = c;
                T = aff_reflect(px, py, qx, qy);
                back = k;
            } else {
                n = eR[e];
                T = eshift[e];
                back = ekR[e];
            }
        } else {
            int64_t e = ~code;
            n = eL[e];
            T = aff_shift(-eshift[e].tx, -eshift[e].ty);
            back = ekL[e];
        }
    };

    // stencils and ghost cells
    std::map<std::tuple<int64_t, long long, long long, long long, long long>, int64_t> ghost_of;
    std::vector<int32_t> gsrc;
    std::vector<double> gR;
    auto index_of = [&](int64_t n, const Aff &T) -> int32_t {
        if (aff_is_translation(T)) return (int32_t)n;
        auto key = std::make_tuple(n, std::llround(T.a * 1e9), std::llround(T.b * 1e9),
                                   std::llround(T.c * 1e9), std::llround(T.d * 1e9));
        auto it = ghost_of.find(key);
        if (it != ghost_of.end()) return (int32_t)(nt + it->second);
        int64_t g = (int64_t)gsrc.size();
        ghost_of.emplace(key, g);
        gsrc.push_back((int32_t)n);
        gR.push_back(T.a);
        gR.push_back(T.b);
        gR.push_back(T.c);
        gR.push_back(T.d);
        // the map of the momentum vector: the same reflection across walls; none across free
        // boundaries, where every component extends evenly like a scalar
        gR.push_back(freebc ? 1.0 : T.a);
        gR.push_back(freebc ? 0.0 : T.b);
        gR.push_back(freebc ? 0.0 : T.c);
        gR.push_back(freebc ? 1.0 : T.d);
        return (int32_t)(nt + g);
    };
    m.sten.assign(9 * nt, 0);
    m.nbc.assign(6 * nt, 0);
    m.cand.assign(nt, 0);
    m.M.assign(153 * nt, 0);
    // stencil images and least-squares operators: independent per cell, computed by a pool of host
    // threads; the images' linear parts are kept to number the ghost cells serially afterwards
    struct SlotImage {
        int64_t cell;
        double a, b, c, d;
    };
    std::vector<SlotImage> slots(9 * (size_t)nt);
    auto cell_work = [&](int64_t c) {
        int64_t img_cell[10];
        Aff img_T[10];
        img_cell[0] = c;
        img_T[0] = aff_id();
        int64_t face[3];
        Aff faceT[3];
        int backk[3];
        for (int k = 0; k < 3; k++) neighbour(c, k, face[k], faceT[k], backk[k]);
        // product ordering: face neighbours 0..2, then the second ring of each
        for (int k = 0; k < 3; k++) {
            img_cell[1 + k] = face[k];
            img_T[1 + k] = faceT[k];
            for (int q = 1; q <= 2; q++) {
                int64_t n2;
                Aff T2;
                int b2;
                neighbour(face[k], (backk[k] + q) % 3, n2, T2, b2);
                img_cell[4 + 2 * k + (q - 1)] = n2;
                img_T[4 + 2 * k + (q - 1)] = aff_then(faceT[k], T2);
            }
        }
        for (int s = 0; s < 9; s++) {
            const Aff &T = img_T[1 + s];
            slots[9 * (size_t)c + s] = {img_cell[1 + s], T.a, T.b, T.c, T.d};
        }
        // least-squares rows in scaled coordinates about the centroid
        const double hs = m.hs[c];
        double v0[3][2];
        for (int k = 0; k < 3; k++) {
            v0[k][0] = m.vtx[(2 * k) * nt + c];
            v0[k][1] = m.vtx[(2 * k + 1) * nt + c];
        }
        double mean0[9];
        centroid_means(v0, mean0);
        double A[17][9];
        for (int l = 0; l < 10; l++) {
            double v[3][2];
            for (int k = 0; k < 3; k++) {
                double x, y, Xm, Ym;
                X(img_cell[l], k, x, y);
                aff_apply(img_T[l], x, y, Xm, Ym);
                v[k][0] = (Xm - cx[c]) / hs;
                v[k][1] = (Ym - cy[c]) / hs;
            }
            double f[9], fx[9], fy[9];
            tri_basis_avg(v, f, fx, fy);
            if (l >= 1)
                for (int k = 0; k < 9; k++) A[l - 1][k] = f[k] - mean0[k];
            if (l <= 3)
                for (int k = 0; k < 9; k++) {
                    A[9 + 2 * l][k] = fx[k];
                    A[10 + 2 * l][k] = fy[k];
                }
            if (l >= 1 && l <= 3) {
                m.nbc[(2 * (l - 1)) * nt + c] = (v[0][0] + v[1][0] + v[2][0]) / 3.0;
                m.nbc[(2 * (l - 1) + 1) * nt + c] = (v[0][1] + v[1][1] + v[2][1]) / 3.0;
            }
        }
        // plane candidates of the nonlinear reconstruction: sub-stencils {0, s, s+1} whose centroid
        // offsets are not nearly parallel
        uint8_t cm = 0;
        for (int s = 0; s < 3; s++) {
            const int sb = (s + 1) % 3;
            const double ax = m.nbc[(2 * s) * nt + c], ay = m.nbc[(2 * s + 1) * nt + c];
            const double bx = m.nbc[(2 * sb) * nt + c], by = m.nbc[(2 * sb + 1) * nt + c];
            const double cross = ax * by - ay * bx;
            if (std::fabs(cross) >= PLANE_SINE_MIN * std::sqrt((ax * ax + ay * ay) * (bx * bx + by * by)))
                cm |= (uint8_t)(1u << s);
        }
        m.cand[c] = cm;
        double Mc[153];
        lsq_operator(A, Mc);
        for (int i = 0; i < 153; i++) m.M[(int64_t)i * nt + c] = Mc[i];
    };
    {
        const int64_t nthr = std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(),
                                                                       (nt + 4095) / 4096}));
        std::vector<std::thread> pool;
        for (int64_t t = 0; t < nthr; t++)
            pool.emplace_back([&, t] {
                for (int64_t c = t * nt / nthr; c < (t + 1) * nt / nthr; c++) cell_work(c);
            });
        for (auto &th : pool) th.join();
    }
    for (int64_t c = 0; c < nt; c++)
        for (int s = 0; s < 9; s++) {
            const SlotImage &im = slots[9 * (size_t)c + s];
            m.sten[s * nt + c] = index_of(im.cell, Aff{im.a, im.b, im.c, im.d, 0, 0});
        }
    m.ng = (int64_t)gsrc.size();
    m.gsrc = gsrc;
    m.igeo.assign(6 * nt, 0);
    for (int64_t c = 0; c < nt; c++) {
        for (int l = 0; l < 3; l++) {
            const int32_t i = m.sten[l * nt + c];
            const int64_t src = i < nt ? i : m.gsrc[i - nt];
            m.igeo[l * nt + c] = m.area[src] / m.area[c];
        }
        for (int k = 0; k < 3; k++) m.igeo[(3 + k) * nt + c] = std::fabs(m.fl[k * nt + c]) * m.area[c] / m.hs[c];
    }
    m.gR.assign(8 * std::max<int64_t>(m.ng, 1), 0);
    for (int64_t g = 0; g < m.ng; g++)
        for (int i = 0; i < 8; i++) m.gR[i * m.ng + g] = gR[8 * g + i];
    if (freebc)
        for (int64_t e = 0; e < ne; e++)
            if (m.eR[e] < 0) m.eR[e] = -2;
    m.S = 1;
    m.scell = {0, nt};
    m.sdxmin = {m.dxmin};
    return 0;
}

}  // namespace gks

namespace gks {

HostMesh concat_host_meshes(const std::vector<const HostMesh *> &parts)
{
    HostMesh o;
    o.S = (int32_t)parts.size();
    for (const HostMesh *p : parts) {
        o.nt += p->nt;
        o.ne += p->ne;
        o.ng += p->ng;
    }
    const int64_t T = o.nt, E = o.ne, NG = o.ng;
    auto cells = [&](std::vector<double> &dst, int width, std::vector<double> HostMesh::*src) {
        dst.assign((size_t)width * T, 0);
        int64_t off = 0;
        for (const HostMesh *p : parts) {
            for (int w = 0; w < width; w++)
                for (int64_t c = 0; c < p->nt; c++) dst[w * T + off + c] = (p->*src)[w * p->nt + c];
            off += p->nt;
        }
    };
    auto edges = [&](std::vector<double> &dst, int width, std::vector<double> HostMesh::*src) {
        dst.assign((size_t)width * E, 0);
        int64_t off = 0;
        for (const HostMesh *p : parts) {
            for (int w = 0; w < width; w++)
                for (int64_t e = 0; e < p->ne; e++) dst[w * E + off + e] = (p->*src)[w * p->ne + e];
            off += p->ne;
        }
    };
    cells(o.area, 1, &HostMesh::area);
    cells(o.hs, 1, &HostMesh::hs);
    cells(o.vtx, 6, &HostMesh::vtx);
    cells(o.nbc, 6, &HostMesh::nbc);
    cells(o.fl, 3, &HostMesh::fl);
    cells(o.gg, 6, &HostMesh::gg);
    cells(o.Bbar, 1, &HostMesh::Bbar);
    cells(o.gB, 2, &HostMesh::gB);
    cells(o.M, 153, &HostMesh::M);
    cells(o.igeo, 6, &HostMesh::igeo);
    o.cand.assign(T, 0);
    {
        int64_t off = 0;
        for (const HostMesh *p : parts) {
            for (int64_t c = 0; c < p->nt; c++) o.cand[off + c] = p->cand[c];
            off += p->nt;
        }
    }
    edges(o.en, 2, &HostMesh::en);
    edges(o.eBgp, 2, &HostMesh::eBgp);
    edges(o.egB, 2, &HostMesh::egB);
    o.cedge.assign(3 * T, 0);
    o.sten.assign(9 * T, 0);
    o.eL.assign(E, 0);
    o.eR.assign(E, 0);
    o.eslot.assign(E, 0);
    o.gsrc.assign(NG, 0);
    o.gR.assign(8 * std::max<int64_t>(NG, 1), 0);
    o.cscen.assign(T, 0);
    o.escen.assign(E, 0);
    o.scell.assign(o.S + 1, 0);
    o.sdxmin.assign(o.S, 0);
    int64_t coff = 0, eoff = 0, goff = 0;
    for (int32_t s = 0; s < o.S; s++) {
        const HostMesh *p = parts[s];
        o.scell[s] = coff;
        o.sdxmin[s] = p->dxmin;
        // a cell index of the part: real cells shift by coff, ghost cells move behind all real cells
        auto cell_index = [&](int32_t i) -> int32_t {
            return i < p->nt ? (int32_t)(coff + i) : (int32_t)(T + goff + (i - p->nt));
        };
        for (int64_t c = 0; c < p->nt; c++) {
            o.cscen[coff + c] = s;
            for (int k = 0; k < 3; k++) {
                int32_t code = p->cedge[k * p->nt + c];
                o.cedge[k * T + coff + c] = code >= 0 ? (int32_t)(code + eoff) : ~(int32_t)(~code + eoff);
            }
            for (int k = 0; k < 9; k++) o.sten[k * T + coff + c] = cell_index(p->sten[k * p->nt + c]);
        }
        for (int64_t e = 0; e < p->ne; e++) {
            o.escen[eoff + e] = s;
            o.eL[eoff + e] = (int32_t)(p->eL[e] + coff);
            o.eR[eoff + e] = p->eR[e] >= 0 ? (int32_t)(p->eR[e] + coff) : p->eR[e];
            o.eslot[eoff + e] = p->eslot[e];
        }
        for (int64_t g = 0; g < p->ng; g++) {
            o.gsrc[goff + g] = (int32_t)(p->gsrc[g] + coff);
            for (int i = 0; i < 8; i++) o.gR[i * NG + goff + g] = p->gR[i * p->ng + g];
        }
        coff += p->nt;
        eoff += p->ne;
        goff += p->ng;
    }
    o.scell[o.S] = T;
    o.dxmin = *std::min_element(o.sdxmin.begin(), o.sdxmin.end());
    return o;
}

}  // namespace gks
