/*
 * Oracle: plain FP64 CPU implementation of the compact gas-kinetic scheme for the two-layer
 * shallow water equations on triangles (Zhao, Gan & Xu).  TEST INFRASTRUCTURE ONLY: loaded by the
 * tests, the smoke check and the CPU-baseline leg of the benchmark, never by the product.  It
 * shares no source with the HIP library and is written for clarity, not speed: dense loops,
 * explicit quadrature, one cell / edge / Gauss point at a time.  The independent per-cell and
 * per-edge loops carry OpenMP pragmas; every iteration writes only its own outputs and every sum
 * is taken in a fixed order inside one iteration, so results do not depend on the thread count.
 *
 * Points where the paper defers to companion papers or is silent are filled in by the readings
 * listed in the design notes of the repository; each is marked "reading:" where it is used.
 */
#include "gks_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define NV 6
#define NS 10       /* stencil cells (Sec. 3.4, Eq. Recons-stencil) */
#define NROW 17     /* 9 averages + 2 x 4 gradients */
#define NDOF 9      /* a_1 .. a_9 */
/* Loops over fewer cells or edges than this run on one thread: on small meshes the threads
 * cost more than the work.  Every iteration is independent, so the count changes no result. */
#define OMP_MIN_ITEMS 4096

/* ----------------------------------------------------------------------------------------- */
/* affine maps x -> R x + t: periodic translations and wall mirror images of cells             */

typedef struct {
    double R[2][2];
    double t[2];
} amap;

static amap map_id(void)
{
    amap a;
    a.R[0][0] = 1; a.R[0][1] = 0; a.R[1][0] = 0; a.R[1][1] = 1;
    a.t[0] = 0; a.t[1] = 0;
    return a;
}

static amap map_shift(double dx, double dy)
{
    amap a = map_id();
    a.t[0] = dx;
    a.t[1] = dy;
    return a;
}

/* x -> a(b(x)) */
static amap map_compose(amap a, amap b)
{
    amap c;
    for (int i = 0; i < 2; i++) {
        for (int j = 0; j < 2; j++) c.R[i][j] = a.R[i][0] * b.R[0][j] + a.R[i][1] * b.R[1][j];
        c.t[i] = a.R[i][0] * b.t[0] + a.R[i][1] * b.t[1] + a.t[i];
    }
    return c;
}

/* reflection across the line through p and q */
static amap map_mirror(const double *p, const double *q)
{
    double dx = q[0] - p[0], dy = q[1] - p[1];
    double L = sqrt(dx * dx + dy * dy);
    dx /= L;
    dy /= L;
    amap a;
    a.R[0][0] = 2 * dx * dx - 1; a.R[0][1] = 2 * dx * dy;
    a.R[1][0] = 2 * dx * dy;     a.R[1][1] = 2 * dy * dy - 1;
    a.t[0] = p[0] - (a.R[0][0] * p[0] + a.R[0][1] * p[1]);
    a.t[1] = p[1] - (a.R[1][0] * p[0] + a.R[1][1] * p[1]);
    return a;
}

static void map_point(const amap *a, const double *x, double *y)
{
    double y0 = a->R[0][0] * x[0] + a->R[0][1] * x[1] + a->t[0];
    double y1 = a->R[1][0] * x[0] + a->R[1][1] * x[1] + a->t[1];
    y[0] = y0;
    y[1] = y1;
}

static void map_vec(const double R[2][2], const double *x, double *y)
{
    double y0 = R[0][0] * x[0] + R[0][1] * x[1];
    double y1 = R[1][0] * x[0] + R[1][1] * x[1];
    y[0] = y0;
    y[1] = y1;
}

/* ----------------------------------------------------------------------------------------- */

struct om_mesh {
    int nn, nt, ne;
    double *xy, *B;
    int *tri;
    int periodic;
    int free_bc; /* boundary edges are free (zero-gradient) instead of walls */
    double Lx, Ly;
    /* cells */
    double *area, *cx, *cy, *Bbar, *Bx, *By, *dX;
    int *c_edge; /* [nt][3] edge of local edge k (vertex k -> vertex k+1) */
    int *c_side; /* [nt][3] 0: the cell is the edge's left cell, 1: right cell */
    /* edges */
    int *e_cell; /* [ne][2] left, right (-1: wall) */
    int *e_lk;   /* [ne][2] local edge index in the left / right cell */
    double *e_n, *e_len;
    double *e_Bgp;  /* [ne][2] bottom at the two Gauss points, in the left cell's orientation */
    amap *e_shift;  /* [ne] maps the right cell's coordinates into the left cell's frame */
    /* reconstruction */
    int *st_cell;   /* [nt][10] */
    amap *st_map;   /* [nt][10] */
    double *M;      /* [nt][9][17] */
};

/* Gauss points on an edge p->q: p + s (q - p), s = 1/2 -+ sqrt(3)/6, weights 1/2 (Sec. 3.1,
 * Eq. SWE-semi-flux with q = 2). */
static const double GP_S[2] = {0.5 - 0.28867513459481288225, 0.5 + 0.28867513459481288225};

static void vtx(const om_mesh *m, int c, int k, double *p)
{
    int v = m->tri[3 * c + (k % 3)];
    p[0] = m->xy[2 * v];
    p[1] = m->xy[2 * v + 1];
}

/* ----------------------------------------------------------------------------------------- */
/* quadrature over a triangle: collapsed (Duffy) Gauss-Legendre product rule, 5 x 5 points,   */
/* exact for polynomials of degree <= 9; returns averages                                     */

static double QX[25], QY[25], QW[25];
static int quad_ready = 0;

static void quad_init(void)
{
    if (quad_ready) return;
    const double g[5] = {-0.90617984593866399280, -0.53846931010568309104, 0.0,
                         0.53846931010568309104, 0.90617984593866399280};
    const double w[5] = {0.23692688505618908751, 0.47862867049936646804, 0.56888888888888888889,
                         0.47862867049936646804, 0.23692688505618908751};
    double tot = 0;
    for (int i = 0; i < 5; i++) {
        for (int j = 0; j < 5; j++) {
            double s = 0.5 * (g[i] + 1), r = 0.5 * (g[j] + 1);
            QX[5 * i + j] = s;
            QY[5 * i + j] = r * (1 - s);
            QW[5 * i + j] = 0.25 * w[i] * w[j] * (1 - s);
            tot += QW[5 * i + j];
        }
    }
    for (int k = 0; k < 25; k++) QW[k] /= tot;
    quad_ready = 1;
}

/* physical quadrature points of triangle (a, b, c) */
static void quad_points(const double *a, const double *b, const double *c, double *px, double *py)
{
    for (int k = 0; k < 25; k++) {
        px[k] = a[0] + QX[k] * (b[0] - a[0]) + QY[k] * (c[0] - a[0]);
        py[k] = a[1] + QX[k] * (b[1] - a[1]) + QY[k] * (c[1] - a[1]);
    }
}

/* ----------------------------------------------------------------------------------------- */
/* polynomial basis of the P^3 reconstruction (Sec. 3.4, Eq. Recons-poly / Recons-eqs):       */
/* monomials in (dx, dy) = x - x0 with Taylor factors, made zero-mean over cell 0             */

static void mono(double dx, double dy, double *m)
{
    m[0] = dx;
    m[1] = dy;
    m[2] = 0.5 * dx * dx;
    m[3] = dx * dy;
    m[4] = 0.5 * dy * dy;
    m[5] = dx * dx * dx / 6.0;
    m[6] = 0.5 * dx * dx * dy;
    m[7] = 0.5 * dx * dy * dy;
    m[8] = dy * dy * dy / 6.0;
}

static void mono_dx(double dx, double dy, double *m)
{
    m[0] = 1;
    m[1] = 0;
    m[2] = dx;
    m[3] = dy;
    m[4] = 0;
    m[5] = 0.5 * dx * dx;
    m[6] = dx * dy;
    m[7] = 0.5 * dy * dy;
    m[8] = 0;
}

static void mono_dy(double dx, double dy, double *m)
{
    m[0] = 0;
    m[1] = 1;
    m[2] = 0;
    m[3] = dx;
    m[4] = dy;
    m[5] = 0;
    m[6] = 0.5 * dx * dx;
    m[7] = dx * dy;
    m[8] = 0.5 * dy * dy;
}

/* averages over triangle (a,b,c) of the monomials and of their x / y derivatives, about x0 */
static void tri_mono_avgs(const double *a, const double *b, const double *c, const double *x0,
                          double *avg, double *avgx, double *avgy)
{
    double px[25], py[25], mm[9], mx[9], my[9];
    quad_points(a, b, c, px, py);
    for (int k = 0; k < 9; k++) avg[k] = avgx[k] = avgy[k] = 0;
    for (int q = 0; q < 25; q++) {
        double dx = px[q] - x0[0], dy = py[q] - x0[1];
        mono(dx, dy, mm);
        mono_dx(dx, dy, mx);
        mono_dy(dx, dy, my);
        for (int k = 0; k < 9; k++) {
            avg[k] += QW[q] * mm[k];
            avgx[k] += QW[q] * mx[k];
            avgy[k] += QW[q] * my[k];
        }
    }
}

/* ----------------------------------------------------------------------------------------- */
/* mesh construction                                                                          */

typedef struct {
    long long a, b;
    int cell, k;
} halfedge;

static int he_cmp(const void *x, const void *y)
{
    const halfedge *p = (const halfedge *)x, *q = (const halfedge *)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    if (p->cell != q->cell) return p->cell < q->cell ? -1 : 1;
    return p->k - q->k;
}

typedef struct {
    long long kx, ky;
    int id;
} nodekey;

static int nk_cmp(const void *x, const void *y)
{
    const nodekey *p = (const nodekey *)x, *q = (const nodekey *)y;
    if (p->kx != q->kx) return p->kx < q->kx ? -1 : 1;
    if (p->ky != q->ky) return p->ky < q->ky ? -1 : 1;
    return p->id - q->id;
}

static double wrap(double x, double L)
{
    double w = x - L * floor(x / L);
    if (L - w < 1e-9 * L) w = 0;
    return w;
}

/* image of the neighbour of cell c across its local edge k: cell id, map from that cell's
 * coordinates into c's frame, and the neighbour's local index of the shared edge */
static void nb_image(const om_mesh *m, int c, int k, int *nc, amap *T, int *back)
{
    int e = m->c_edge[3 * c + k];
    if (m->c_side[3 * c + k] == 0) {
        int r = m->e_cell[2 * e + 1];
        if (r < 0) { /* reading: beyond a wall or a free boundary edge lies the mirror image of the
                      * cell itself (its state seen through image_state) */
            double p[2], q[2];
            vtx(m, c, k, p);
            vtx(m, c, k + 1, q);
            *nc = c;
            *T = map_mirror(p, q);
            *back = k;
            return;
        }
        *nc = r;
        *T = m->e_shift[e];
        *back = m->e_lk[2 * e + 1];
    } else {
        *nc = m->e_cell[2 * e];
        *T = map_shift(-m->e_shift[e].t[0], -m->e_shift[e].t[1]);
        *back = m->e_lk[2 * e];
    }
}

static void image_vertices(const om_mesh *m, int c, const amap *T, double v[3][2])
{
    for (int k = 0; k < 3; k++) {
        double p[2];
        vtx(m, c, k, p);
        map_point(T, p, v[k]);
    }
}

/* Householder QR of A (17 x 9, row-major) and M = R^-1 Q1^T (9 x 17): the least-squares solution
 * operator (A^T A)^-1 A^T of Sec. 3.4. */
static void lsq_solve_matrix(const double *Ain, double *M)
{
    double A[NROW][NDOF], Qt[NROW][NROW];
    memcpy(A, Ain, sizeof(A));
    for (int i = 0; i < NROW; i++)
        for (int j = 0; j < NROW; j++) Qt[i][j] = (i == j);
    for (int k = 0; k < NDOF; k++) {
        double nrm = 0;
        for (int i = k; i < NROW; i++) nrm += A[i][k] * A[i][k];
        nrm = sqrt(nrm);
        double alpha = A[k][k] > 0 ? -nrm : nrm;
        double v[NROW];
        for (int i = 0; i < NROW; i++) v[i] = 0;
        for (int i = k; i < NROW; i++) v[i] = A[i][k];
        v[k] -= alpha;
        double vv = 0;
        for (int i = k; i < NROW; i++) vv += v[i] * v[i];
        if (vv == 0) continue;
        for (int j = 0; j < NDOF; j++) {
            double s = 0;
            for (int i = k; i < NROW; i++) s += v[i] * A[i][j];
            s = 2 * s / vv;
            for (int i = k; i < NROW; i++) A[i][j] -= s * v[i];
        }
        for (int j = 0; j < NROW; j++) {
            double s = 0;
            for (int i = k; i < NROW; i++) s += v[i] * Qt[i][j];
            s = 2 * s / vv;
            for (int i = k; i < NROW; i++) Qt[i][j] -= s * v[i];
        }
    }
    /* back substitution R M = Q1^T */
    for (int j = 0; j < NROW; j++) {
        for (int i = NDOF - 1; i >= 0; i--) {
            double s = Qt[i][j];
            for (int l = i + 1; l < NDOF; l++) s -= A[i][l] * M[l * NROW + j];
            M[i * NROW + j] = s / A[i][i];
        }
    }
}

static void build_lsq(om_mesh *m, int c)
{
    double x0[2] = {m->cx[c], m->cy[c]};
    double h = sqrt(2.0 * m->area[c]); /* reading: the scale h of the gradient rows */
    double v0[3][2], off[9], ox[9], oy[9];
    amap I = map_id();
    image_vertices(m, c, &I, v0);
    tri_mono_avgs(v0[0], v0[1], v0[2], x0, off, ox, oy);
    double A[NROW * NDOF];
    for (int l = 0; l < NS; l++) {
        double v[3][2], av[9], ax[9], ay[9];
        image_vertices(m, m->st_cell[NS * c + l], &m->st_map[NS * c + l], v);
        tri_mono_avgs(v[0], v[1], v[2], x0, av, ax, ay);
        if (l >= 1)
            for (int k = 0; k < 9; k++) A[(l - 1) * NDOF + k] = av[k] - off[k];
        if (l <= 3)
            for (int k = 0; k < 9; k++) {
                A[(9 + 2 * l) * NDOF + k] = h * ax[k];
                A[(10 + 2 * l) * NDOF + k] = h * ay[k];
            }
    }
    lsq_solve_matrix(A, m->M + (size_t)c * NDOF * NROW);
}

om_mesh *om_mesh_new(const double *node_xy, int nn, const int *tri, int nt, const double *node_B,
                     int bc, double Lx, double Ly)
{
    if (bc < 0 || bc > 2) return NULL;
    const int periodic = bc == 1;
    quad_init();
    om_mesh *m = (om_mesh *)calloc(1, sizeof(om_mesh));
    m->nn = nn;
    m->nt = nt;
    m->periodic = periodic;
    m->free_bc = bc == 2;
    m->Lx = Lx;
    m->Ly = Ly;
    m->xy = (double *)malloc(sizeof(double) * 2 * nn);
    m->B = (double *)malloc(sizeof(double) * nn);
    m->tri = (int *)malloc(sizeof(int) * 3 * nt);
    memcpy(m->xy, node_xy, sizeof(double) * 2 * nn);
    memcpy(m->tri, tri, sizeof(int) * 3 * nt);
    for (int i = 0; i < nn; i++) m->B[i] = node_B ? node_B[i] : 0.0;

    /* node identification (periodic: nodes that coincide after wrapping) */
    int *canon = (int *)malloc(sizeof(int) * nn);
    if (periodic) {
        nodekey *keys = (nodekey *)malloc(sizeof(nodekey) * nn);
        for (int i = 0; i < nn; i++) {
            keys[i].kx = llround(wrap(node_xy[2 * i], Lx) / Lx * 1e7);
            keys[i].ky = llround(wrap(node_xy[2 * i + 1], Ly) / Ly * 1e7);
            if (keys[i].kx == 10000000LL) keys[i].kx = 0;
            if (keys[i].ky == 10000000LL) keys[i].ky = 0;
            keys[i].id = i;
        }
        qsort(keys, nn, sizeof(nodekey), nk_cmp);
        int rep = -1;
        for (int i = 0; i < nn; i++) {
            if (i == 0 || keys[i].kx != keys[i - 1].kx || keys[i].ky != keys[i - 1].ky) rep = keys[i].id;
            canon[keys[i].id] = rep;
        }
        free(keys);
    } else {
        for (int i = 0; i < nn; i++) canon[i] = i;
    }

    /* cell geometry */
    m->area = (double *)malloc(sizeof(double) * nt);
    m->cx = (double *)malloc(sizeof(double) * nt);
    m->cy = (double *)malloc(sizeof(double) * nt);
    m->Bbar = (double *)malloc(sizeof(double) * nt);
    m->Bx = (double *)malloc(sizeof(double) * nt);
    m->By = (double *)malloc(sizeof(double) * nt);
    m->dX = (double *)malloc(sizeof(double) * nt);
    for (int c = 0; c < nt; c++) {
        double a[2], b[2], d[2];
        vtx(m, c, 0, a);
        vtx(m, c, 1, b);
        vtx(m, c, 2, d);
        double ar = 0.5 * ((b[0] - a[0]) * (d[1] - a[1]) - (b[1] - a[1]) * (d[0] - a[0]));
        if (!(ar > 0)) {
            om_mesh_free(m);
            free(canon);
            return NULL;
        }
        m->area[c] = ar;
        m->cx[c] = (a[0] + b[0] + d[0]) / 3.0;
        m->cy[c] = (a[1] + b[1] + d[1]) / 3.0;
        double Ba = m->B[tri[3 * c]], Bb = m->B[tri[3 * c + 1]], Bd = m->B[tri[3 * c + 2]];
        /* reading: the discretised bottom is the continuous piecewise-linear interpolant of the
         * node values; its cell average is the vertex mean and its gradient is constant. */
        m->Bbar[c] = (Ba + Bb + Bd) / 3.0;
        m->Bx[c] = (Ba * (b[1] - d[1]) + Bb * (d[1] - a[1]) + Bd * (a[1] - b[1])) / (2 * ar);
        m->By[c] = (Ba * (d[0] - b[0]) + Bb * (a[0] - d[0]) + Bd * (b[0] - a[0])) / (2 * ar);
        double lmax = 0;
        for (int k = 0; k < 3; k++) {
            double p[2], q[2];
            vtx(m, c, k, p);
            vtx(m, c, k + 1, q);
            double l = sqrt((q[0] - p[0]) * (q[0] - p[0]) + (q[1] - p[1]) * (q[1] - p[1]));
            if (l > lmax) lmax = l;
        }
        m->dX[c] = 2 * ar / lmax; /* reading: cell size = smallest altitude */
    }

    /* edges from paired half-edges */
    halfedge *he = (halfedge *)malloc(sizeof(halfedge) * 3 * nt);
    for (int c = 0; c < nt; c++)
        for (int k = 0; k < 3; k++) {
            long long a = canon[tri[3 * c + k]], b = canon[tri[3 * c + (k + 1) % 3]];
            halfedge *h = &he[3 * c + k];
            h->a = a < b ? a : b;
            h->b = a < b ? b : a;
            h->cell = c;
            h->k = k;
        }
    qsort(he, 3 * nt, sizeof(halfedge), he_cmp);
    m->c_edge = (int *)malloc(sizeof(int) * 3 * nt);
    m->c_side = (int *)malloc(sizeof(int) * 3 * nt);
    m->e_cell = (int *)malloc(sizeof(int) * 6 * nt);
    m->e_lk = (int *)malloc(sizeof(int) * 6 * nt);
    m->e_n = (double *)malloc(sizeof(double) * 6 * nt);
    m->e_len = (double *)malloc(sizeof(double) * 3 * nt);
    m->e_Bgp = (double *)malloc(sizeof(double) * 6 * nt);
    m->e_shift = (amap *)malloc(sizeof(amap) * 3 * nt);
    int ne = 0, bad = 0;
    for (int i = 0; i < 3 * nt;) {
        int j = i + 1;
        while (j < 3 * nt && he[j].a == he[i].a && he[j].b == he[i].b) j++;
        int cnt = j - i;
        if (cnt > 2 || (cnt == 1 && periodic)) {
            bad = 1;
            break;
        }
        int e = ne++;
        int L = he[i].cell, kL = he[i].k;
        double p[2], q[2];
        vtx(m, L, kL, p);
        vtx(m, L, kL + 1, q);
        double len = sqrt((q[0] - p[0]) * (q[0] - p[0]) + (q[1] - p[1]) * (q[1] - p[1]));
        m->e_cell[2 * e] = L;
        m->e_lk[2 * e] = kL;
        m->e_len[e] = len;
        m->e_n[2 * e] = (q[1] - p[1]) / len; /* outward for the counter-clockwise left cell */
        m->e_n[2 * e + 1] = -(q[0] - p[0]) / len;
        double Bp = m->B[tri[3 * L + kL]], Bq = m->B[tri[3 * L + (kL + 1) % 3]];
        for (int g = 0; g < 2; g++) m->e_Bgp[2 * e + g] = (1 - GP_S[g]) * Bp + GP_S[g] * Bq;
        m->c_edge[3 * L + kL] = e;
        m->c_side[3 * L + kL] = 0;
        if (cnt == 2) {
            int R = he[i + 1].cell, kR = he[i + 1].k;
            m->e_cell[2 * e + 1] = R;
            m->e_lk[2 * e + 1] = kR;
            m->c_edge[3 * R + kR] = e;
            m->c_side[3 * R + kR] = 1;
            double r1[2];
            vtx(m, R, kR + 1, r1); /* the right cell's copy of the left cell's vertex kL */
            m->e_shift[e] = map_shift(p[0] - r1[0], p[1] - r1[1]);
        } else {
            m->e_cell[2 * e + 1] = -1;
            m->e_lk[2 * e + 1] = -1;
            m->e_shift[e] = map_id();
        }
        i = j;
    }
    free(he);
    free(canon);
    m->ne = ne;
    if (bad) {
        om_mesh_free(m);
        return NULL;
    }

    /* compact stencils: the cell, its three face neighbours, and their other neighbours
     * (Sec. 3.4, Eq. Recons-stencil; images carry the periodic / mirror map into the cell frame) */
    m->st_cell = (int *)malloc(sizeof(int) * NS * nt);
    m->st_map = (amap *)malloc(sizeof(amap) * NS * nt);
    for (int c = 0; c < nt; c++) {
        int *sc = m->st_cell + NS * c;
        amap *sm = m->st_map + NS * c;
        sc[0] = c;
        sm[0] = map_id();
        for (int k = 0; k < 3; k++) {
            int n1, back;
            amap T1;
            nb_image(m, c, k, &n1, &T1, &back);
            sc[1 + k] = n1;
            sm[1 + k] = T1;
            for (int q = 1; q <= 2; q++) {
                int n2, b2;
                amap T2;
                nb_image(m, n1, (back + q) % 3, &n2, &T2, &b2);
                sc[4 + 2 * k + (q - 1)] = n2;
                sm[4 + 2 * k + (q - 1)] = map_compose(T1, T2);
            }
        }
    }
    m->M = (double *)malloc(sizeof(double) * (size_t)nt * NDOF * NROW);
#pragma omp parallel for schedule(dynamic, 256) if(nt >= OMP_MIN_ITEMS)
    for (int c = 0; c < nt; c++) build_lsq(m, c);
    return m;
}

void om_mesh_free(om_mesh *m)
{
    if (!m) return;
    free(m->xy); free(m->B); free(m->tri);
    free(m->area); free(m->cx); free(m->cy); free(m->Bbar); free(m->Bx); free(m->By); free(m->dX);
    free(m->c_edge); free(m->c_side); free(m->e_cell); free(m->e_lk); free(m->e_n);
    free(m->e_len); free(m->e_Bgp); free(m->e_shift); free(m->st_cell); free(m->st_map);
    free(m->M);
    free(m);
}

int om_mesh_n_edges(const om_mesh *m) { return m->ne; }

void om_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

int om_max_threads(void) { return omp_get_max_threads(); }

/* Interface height of the force model (Sec. 2.3): the convex combination of the two sides' heights
 * whose weight xi is, in this reading, the fraction of the particles of the interface Maxwellian
 * (mean normal velocity (unl + unr) / 2, lambda = 2 / (G (hl + hr))) that move from the left
 * side to the right one, 1/2 erfc(-sqrt(lambda) (unl + unr) / 2). */
double om_edge_height(double zl, double zr, double hl, double hr, double unl, double unr, double G)
{
    if (!(hl + hr > 0)) return 0.5 * (zl + zr); /* both sides dry: no particles to weigh */
    double lamb = 2 / (G * (hl + hr));
    double xi = 0.5 * erfc(-sqrt(lamb) * 0.5 * (unl + unr));
    return xi * zl + (1 - xi) * zr;
}

/* Gradient of the plane through the values hk[k] at the centres of cell c's local edges k (edge k
 * joins vertices k and k + 1): the cell average of the gradient by Gauss's theorem, exact for a
 * plane (Sec. 2.3 extended to two dimensions). */
void om_plane_gradient(const om_mesh *m, int c, const double *hk, double *out)
{
    double s[2] = {0, 0};
    for (int k = 0; k < 3; k++) {
        int e = m->c_edge[3 * c + k];
        double sg = m->c_side[3 * c + k] == 0 ? 1.0 : -1.0;
        s[0] += sg * m->e_len[e] * m->e_n[2 * e] * hk[k];
        s[1] += sg * m->e_len[e] * m->e_n[2 * e + 1] * hk[k];
    }
    out[0] = s[0] / m->area[c];
    out[1] = s[1] / m->area[c];
}

void om_cell_geometry(const om_mesh *m, double *area, double *cx, double *cy)
{
    for (int c = 0; c < m->nt; c++) {
        area[c] = m->area[c];
        cx[c] = m->cx[c];
        cy[c] = m->cy[c];
    }
}

void om_stencil(const om_mesh *m, int c, int *cells, double *maps)
{
    for (int l = 0; l < NS; l++) {
        const amap *a = &m->st_map[NS * c + l];
        cells[l] = m->st_cell[NS * c + l];
        maps[6 * l + 0] = a->R[0][0];
        maps[6 * l + 1] = a->R[0][1];
        maps[6 * l + 2] = a->R[1][0];
        maps[6 * l + 3] = a->R[1][1];
        maps[6 * l + 4] = a->t[0];
        maps[6 * l + 5] = a->t[1];
    }
}

void om_lsq_matrix(const om_mesh *m, int c, double *M)
{
    memcpy(M, m->M + (size_t)c * NDOF * NROW, sizeof(double) * NDOF * NROW);
}

/* ----------------------------------------------------------------------------------------- */
/* reconstruction (Sec. 3.4)                                                                  */

/* variables of cell n seen through the map R (linear part of its image map): six averages in the
 * reconstruction's variable set (eta1 = h1 + B replaces h1, Sec. 3.2 water-level technique) and
 * their gradients [6][2].  Scalars keep their value; gradients of scalars rotate with R.  With
 * vec != 0 momenta rotate with R and their gradients as R (grad m) R^T (walls: the momentum is a
 * vector that reflects); with vec = 0 (free boundaries) every momentum component extends evenly
 * like a scalar: value kept, gradient (grad m) R^T. */
static void image_state(const om_mesh *m, int n, const double R[2][2], int vec, const double *W,
                        const double *gW, double *q, double *gq)
{
    int T = m->nt;
    double w[NV], g[NV][2];
    for (int v = 0; v < NV; v++) {
        w[v] = W[v * T + n];
        g[v][0] = gW[(2 * v) * T + n];
        g[v][1] = gW[(2 * v + 1) * T + n];
    }
    w[3] += m->Bbar[n];
    g[3][0] += m->Bx[n];
    g[3][1] += m->By[n];
    for (int layer = 0; layer < 2; layer++) {
        int o = 3 * layer;
        const double I[2][2] = {{1, 0}, {0, 1}};
        const double(*V)[2] = vec ? R : I; /* the map of momentum vectors */
        double mv[2] = {w[o + 1], w[o + 2]}, rm[2];
        map_vec(V, mv, rm);
        q[o] = w[o];
        q[o + 1] = rm[0];
        q[o + 2] = rm[1];
        map_vec(R, g[o], gq + 2 * o);
        /* grad of momentum: Gm[a][d] = d m_a / d x_d  ->  V Gm R^T */
        double Gm[2][2] = {{g[o + 1][0], g[o + 1][1]}, {g[o + 2][0], g[o + 2][1]}};
        double RG[2][2], RGRt[2][2];
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++) RG[i][j] = V[i][0] * Gm[0][j] + V[i][1] * Gm[1][j];
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++) RGRt[i][j] = RG[i][0] * R[j][0] + RG[i][1] * R[j][1];
        gq[2 * (o + 1)] = RGRt[0][0];
        gq[2 * (o + 1) + 1] = RGRt[0][1];
        gq[2 * (o + 2)] = RGRt[1][0];
        gq[2 * (o + 2) + 1] = RGRt[1][1];
    }
}

/* smoothness indicator of the cubic: sum over 1 <= |alpha| <= 3 of |Omega|^(|alpha|-1) times the
 * integral over the cell of (D^alpha P)^2 (reading of the nonlinear compact reconstruction) */
static double beta_cubic(const double *a, const double v0[3][2], const double *x0, double area)
{
    double px[25], py[25];
    quad_points(v0[0], v0[1], v0[2], px, py);
    double s1 = 0, s2 = 0;
    for (int q = 0; q < 25; q++) {
        double dx = px[q] - x0[0], dy = py[q] - x0[1];
        double Px = a[0] + a[2] * dx + a[3] * dy + 0.5 * a[5] * dx * dx + a[6] * dx * dy + 0.5 * a[7] * dy * dy;
        double Py = a[1] + a[3] * dx + a[4] * dy + 0.5 * a[6] * dx * dx + a[7] * dx * dy + 0.5 * a[8] * dy * dy;
        double Pxx = a[2] + a[5] * dx + a[6] * dy;
        double Pxy = a[3] + a[6] * dx + a[7] * dy;
        double Pyy = a[4] + a[7] * dx + a[8] * dy;
        s1 += QW[q] * (Px * Px + Py * Py);
        s2 += QW[q] * (Pxx * Pxx + Pxy * Pxy + Pyy * Pyy);
    }
    double s3 = a[5] * a[5] + a[6] * a[6] + a[7] * a[7] + a[8] * a[8];
    /* QW are averages: integral = area * average */
    return area * s1 + area * area * s2 + area * area * area * s3;
}

/* One variable's reconstruction in a cell as a function of position (offset d from the centroid):
 * R(d) = Q0 + theta (ratio (P(d) - Q0) + sum_s c_s (P_s(d) - Q0)), P the P^3 fit, P_s the plane
 * candidates, c_s = omega_s - ratio d_s (the nonlinear combination, Sec. 3.4), theta the positivity
 * safeguard's factor.  Kept for the interior quadrature of the higher-order layer coupling. */
typedef struct {
    double Q0, ratio, theta, a[NDOF], off[NDOF], cs[4], b[4][2];
} rfun;

/* value, first and second derivatives (R, R_x, R_y, R_xx, R_xy, R_yy) of a reconstruction at d */
static void rfun_eval(const rfun *r, double dx, double dy, double *o)
{
    double mm[9], mx[9], my[9];
    mono(dx, dy, mm);
    mono_dx(dx, dy, mx);
    mono_dy(dx, dy, my);
    double P = 0, Px = 0, Py = 0;
    for (int k = 0; k < 9; k++) {
        P += r->a[k] * (mm[k] - r->off[k]);
        Px += r->a[k] * mx[k];
        Py += r->a[k] * my[k];
    }
    /* second derivatives of the Taylor monomials dx^2/2, dx dy, dy^2/2, dx^3/6, dx^2 dy/2,
     * dx dy^2/2, dy^3/6 */
    double Pxx = r->a[2] + r->a[5] * dx + r->a[6] * dy;
    double Pxy = r->a[3] + r->a[6] * dx + r->a[7] * dy;
    double Pyy = r->a[4] + r->a[7] * dx + r->a[8] * dy;
    double dev = r->ratio * P, gx = r->ratio * Px, gy = r->ratio * Py;
    for (int s = 0; s < 4; s++) {
        dev += r->cs[s] * (r->b[s][0] * dx + r->b[s][1] * dy);
        gx += r->cs[s] * r->b[s][0];
        gy += r->cs[s] * r->b[s][1];
    }
    const double th = r->theta;
    o[0] = r->Q0 + th * dev;
    o[1] = th * gx;
    o[2] = th * gy;
    o[3] = th * r->ratio * Pxx;
    o[4] = th * r->ratio * Pxy;
    o[5] = th * r->ratio * Pyy;
}

/* Higher-order layer coupling (Sec. 3.2, Eq. SWE-source-discretization and the remark after it
 * that more integration points raise its order).  The cell average of h_a grad h_b splits
 * exactly into  mean(h_a) mean(grad h_b) + mean((h_a - mean h_a) grad h_b);  the first product is
 * the paper's form with the exact cell average in place of the Gauss-point mean, the second is the
 * correction integrated here over the cell's own reconstructions, with the oracle's 25-point rule
 * (exact for these degree-5 products).  The time derivative follows by the product rule with the
 * thickness rate h_t = -div(h U) of the reconstructed momenta.  corr[8]:
 *   0,1  mean((h1 - mean h1) grad h2)      2,3  mean((h2 - mean h2) grad h1)
 *   4,5  its time derivative (lower)       6,7  its time derivative (upper)
 * (h1 = eta1 - B with the cell's linear bottom). */
static void coupling_correction(const om_mesh *m, int c, const rfun *rf, double *corr)
{
    quad_init();
    double v0[3][2], px[25], py[25];
    amap I = map_id();
    image_vertices(m, c, &I, v0);
    quad_points(v0[0], v0[1], v0[2], px, py);
    const double x0 = m->cx[c], y0 = m->cy[c], Bx = m->Bx[c], By = m->By[c];
    double f1[25], f2[25], g1[25][2], g2[25][2], t1[25], t2[25], gt1[25][2], gt2[25][2];
    double t1m = 0, t2m = 0;
    for (int q = 0; q < 25; q++) {
        double dx = px[q] - x0, dy = py[q] - y0, e[NV][6];
        for (int v = 0; v < NV; v++) rfun_eval(&rf[v], dx, dy, e[v]);
        f2[q] = e[0][0] - rf[0].Q0;
        g2[q][0] = e[0][1];
        g2[q][1] = e[0][2];
        f1[q] = (e[3][0] - rf[3].Q0) - (Bx * dx + By * dy);
        g1[q][0] = e[3][1] - Bx;
        g1[q][1] = e[3][2] - By;
        /* thickness rates -div(h U) and their gradients, from the momentum reconstructions */
        t2[q] = -(e[1][1] + e[2][2]);
        gt2[q][0] = -(e[1][3] + e[2][4]);
        gt2[q][1] = -(e[1][4] + e[2][5]);
        t1[q] = -(e[4][1] + e[5][2]);
        gt1[q][0] = -(e[4][3] + e[5][4]);
        gt1[q][1] = -(e[4][4] + e[5][5]);
        t1m += QW[q] * t1[q];
        t2m += QW[q] * t2[q];
    }
    for (int k = 0; k < 8; k++) corr[k] = 0;
    for (int q = 0; q < 25; q++)
        for (int d = 0; d < 2; d++) {
            corr[d] += QW[q] * f1[q] * g2[q][d];
            corr[2 + d] += QW[q] * f2[q] * g1[q][d];
            corr[4 + d] += QW[q] * ((t1[q] - t1m) * g2[q][d] + f1[q] * gt2[q][d]);
            corr[6 + d] += QW[q] * ((t2[q] - t2m) * g1[q][d] + f2[q] * gt1[q][d]);
        }
}

double om_cell_velocity(double h, double m, double h_dry)
{
    const double hs = OM_THIN * h_dry; /* desingularised below the thin-layer thickness */
    if (!(h_dry > 0) || h >= hs) return m / h;
    double h2 = h * h, d2 = hs * hs;
    return sqrt(2.0) * h * m / sqrt(h2 * h2 + d2 * d2);
}

static void reconstruct_cell(const om_mesh *m, int c, const double *W, const double *gW, int linear, double G,
                             double h_dry, double *val, double *grad, double *r0, double *corr)
{
    const double dlin = 0.05; /* reading: linear weight of each lower-order candidate */
    rfun rf[NV];
    double x0[2] = {m->cx[c], m->cy[c]};
    double area = m->area[c];
    double h = sqrt(2.0 * area);
    double q[NS][NV], gq[NS][NV][2], cen[NS][2];
    for (int l = 0; l < NS; l++) {
        int n = m->st_cell[NS * c + l];
        const amap *T = &m->st_map[NS * c + l];
        image_state(m, n, T->R, !m->free_bc, W, gW, q[l], &gq[l][0][0]);
        double cn[2] = {m->cx[n], m->cy[n]};
        map_point(T, cn, cen[l]);
    }
    double v0[3][2], off[9], ox[9], oy[9];
    amap I = map_id();
    image_vertices(m, c, &I, v0);
    tri_mono_avgs(v0[0], v0[1], v0[2], x0, off, ox, oy);
    const double *M = m->M + (size_t)c * NDOF * NROW;
    /* Gauss points of the cell */
    double gp[6][2];
    for (int k = 0; k < 3; k++)
        for (int g = 0; g < 2; g++) {
            gp[2 * k + g][0] = v0[k][0] + GP_S[g] * (v0[(k + 1) % 3][0] - v0[k][0]);
            gp[2 * k + g][1] = v0[k][1] + GP_S[g] * (v0[(k + 1) % 3][1] - v0[k][1]);
        }
    for (int v = 0; v < NV; v++) {
        double Q0 = q[0][v];
        double rhs[NROW], a[NDOF];
        for (int l = 1; l < NS; l++) rhs[l - 1] = q[l][v] - Q0;
        for (int l = 0; l < 4; l++) {
            rhs[9 + 2 * l] = h * gq[l][v][0];
            rhs[10 + 2 * l] = h * gq[l][v][1];
        }
        for (int i = 0; i < NDOF; i++) {
            double s = 0;
            for (int j = 0; j < NROW; j++) s += M[i * NROW + j] * rhs[j];
            a[i] = s;
        }
        /* lower-order candidates: planes through the averages of {0,i,j}, {0,j,k}, {0,k,i}
         * (face neighbours are stencil slots 1..3) and the cell's own gradient.  Reading: a
         * sub-stencil whose two centroid offsets are nearly parallel (the sine of the angle between
         * them below 0.2) does not determine a plane and is not a candidate; its linear weight
         * goes to P^3.  Such a plane's slope is huge, and the combination below subtracts
         * (omega_0 / d_0) d_m P_m even when the plane's own weight has dropped to zero. */
        double b[4][2], dm[4];
        for (int s = 0; s < 3; s++) {
            int la = 1 + s, lb = 1 + (s + 1) % 3;
            double ax = cen[la][0] - x0[0], ay = cen[la][1] - x0[1];
            double bx = cen[lb][0] - x0[0], by = cen[lb][1] - x0[1];
            double ra = q[la][v] - Q0, rb = q[lb][v] - Q0;
            double det = ax * by - ay * bx;
            if (fabs(det) >= OM_PLANE_SINE_MIN * sqrt((ax * ax + ay * ay) * (bx * bx + by * by))) {
                dm[s] = dlin;
                b[s][0] = (ra * by - ay * rb) / det;
                b[s][1] = (ax * rb - ra * bx) / det;
            } else {
                dm[s] = 0;
                b[s][0] = b[s][1] = 0;
            }
        }
        dm[3] = dlin;
        b[3][0] = gq[0][v][0];
        b[3][1] = gq[0][v][1];
        int ncand = 0;
        for (int s = 0; s < 4; s++) ncand += dm[s] > 0;
        const double d0 = ncand == 4 ? 0.8 : ncand == 3 ? 0.85 : ncand == 2 ? 0.9 : 0.95; /* 1 - ncand dlin */
        double w0 = d0, wm[4] = {dm[0], dm[1], dm[2], dm[3]};
        if (!linear) {
            double beta0 = beta_cubic(a, v0, x0, area);
            double betam[4], tauz = 0;
            for (int s = 0; s < 4; s++) {
                betam[s] = area * (b[s][0] * b[s][0] + b[s][1] * b[s][1]);
                if (dm[s] > 0) tauz += fabs(beta0 - betam[s]);
            }
            tauz /= ncand;
            /* reading: the floor of the smoothness indicators carries the variable's scale, the
             * level itself for a thickness and 1e-8 h sqrt(G h) of the layer for a momentum, with
             * the relative factor 1e-18: the weights leave their linear values once a variable
             * varies by about 1e-9 of its scale */
            double S2 = 1e-20;
            if (v != 0 && v != 3) {
                double hl = W[(v < 3 ? 0 : 3) * m->nt + c];
                S2 = 1e-16 * G * hl * hl * hl;
            }
            double eps = 1e-18 * fmax(Q0 * Q0, S2);
            double wt0 = d0 * (1 + tauz / (beta0 + eps)), wts[4], sum = wt0;
            for (int s = 0; s < 4; s++) {
                wts[s] = dm[s] * (1 + tauz / (betam[s] + eps));
                sum += wts[s];
            }
            w0 = wt0 / sum;
            for (int s = 0; s < 4; s++) wm[s] = wts[s] / sum;
        }
        r0[v] = w0 / d0;
        for (int p = 0; p < 6; p++) {
            double dx = gp[p][0] - x0[0], dy = gp[p][1] - x0[1];
            double mm[9], mx[9], my[9];
            mono(dx, dy, mm);
            mono_dx(dx, dy, mx);
            mono_dy(dx, dy, my);
            double P = Q0, Px = 0, Py = 0;
            for (int k = 0; k < 9; k++) {
                P += a[k] * (mm[k] - off[k]);
                Px += a[k] * mx[k];
                Py += a[k] * my[k];
            }
            double R = (w0 / d0) * P, Rx = (w0 / d0) * Px, Ry = (w0 / d0) * Py;
            for (int s = 0; s < 4; s++) {
                double Pm = Q0 + b[s][0] * dx + b[s][1] * dy;
                double coef = wm[s] - (w0 / d0) * dm[s];
                R += coef * Pm;
                Rx += coef * b[s][0];
                Ry += coef * b[s][1];
            }
            val[p * NV + v] = R;
            grad[(p * NV + v) * 2] = Rx;
            grad[(p * NV + v) * 2 + 1] = Ry;
        }
        /* positivity safeguard (not in the paper): where a layer thickness at a Gauss point would
         * fall below a tenth of the cell's average, the reconstruction's deviation from the
         * average is scaled down (Zhang-Shu scaling) until it does not; the lower layer's
         * thickness is eta1 minus the piecewise-linear bottom.  At rest and in ordinary flows the
         * factor is 1 and nothing changes. */
        if (v == 0 || v == 3) {
            double hbar = v == 0 ? Q0 : Q0 - m->Bbar[c], floor_h = 0.1 * hbar, theta = 1.0;
            for (int p = 0; p < 6; p++) {
                double dev = val[p * NV + v] - Q0;
                double bdev = v == 3 ? m->Bx[c] * (gp[p][0] - x0[0]) + m->By[c] * (gp[p][1] - x0[1]) : 0.0;
                if (dev < 0) theta = fmin(theta, fmax(0.0, (hbar - bdev - floor_h) / -dev));
            }
            if (theta < 1.0)
                for (int p = 0; p < 6; p++) {
                    val[p * NV + v] = Q0 + theta * (val[p * NV + v] - Q0);
                    grad[(p * NV + v) * 2] *= theta;
                    grad[(p * NV + v) * 2 + 1] *= theta;
                }
            rf[v].theta = theta;
        } else {
            rf[v].theta = 1.0;
        }
        rf[v].Q0 = Q0;
        rf[v].ratio = w0 / d0;
        for (int k = 0; k < NDOF; k++) {
            rf[v].a[k] = a[k];
            rf[v].off[k] = off[k];
        }
        for (int s = 0; s < 4; s++) {
            rf[v].cs[s] = wm[s] - (w0 / d0) * dm[s];
            rf[v].b[s][0] = b[s][0];
            rf[v].b[s][1] = b[s][1];
        }
    }
    /* wet/dry reading: in the front band of a layer -- the cell or one of its face neighbours has
     * that layer thinner than OM_THIN h_dry -- the layer is reconstructed as its cell average,
     * thickness constant (the lower layer's level then follows the bottom) and momentum the
     * thickness times the cell's desingularised velocity, all gradients at the Gauss points those
     * of these constant fields.  Its high-order weight ratio r0 is set to 0 (never 0 otherwise):
     * the force model then takes the plane gradient at its edges, and the evolution there is of
     * first order in space and time */
    if (h_dry > 0)
        for (int o = 0; o < NV; o += 3) {
            double hbar = o == 0 ? q[0][0] : q[0][3] - m->Bbar[c];
            double hk[4], hmax = 0;
            for (int l = 0; l < 4; l++) {
                int n = m->st_cell[NS * c + l];
                hk[l] = o == 0 ? q[l][0] : q[l][3] - m->Bbar[n];
                hmax = fmax(hmax, hk[l]);
            }
            int band = 0;
            for (int l = 0; l < 4; l++) band |= hk[l] < OM_THIN * h_dry || hk[l] < OM_FRONT * hmax;
            /* the lower layer thinner than the bottom's rise across the cell: its shoreline lies
             * inside the cell (a partially flooded cell) */
            if (o == 3) band |= hbar < h * sqrt(m->Bx[c] * m->Bx[c] + m->By[c] * m->By[c]);
            if (!band) continue;
            double Uc = om_cell_velocity(hbar, q[0][o + 1], h_dry), Vc = om_cell_velocity(hbar, q[0][o + 2], h_dry);
            for (int p = 0; p < 6; p++) {
                double bdev = o == 3 ? m->Bx[c] * (gp[p][0] - x0[0]) + m->By[c] * (gp[p][1] - x0[1]) : 0.0;
                val[p * NV + o] = q[0][o] + bdev;
                val[p * NV + o + 1] = hbar * Uc;
                val[p * NV + o + 2] = hbar * Vc;
                grad[(p * NV + o) * 2] = o == 3 ? m->Bx[c] : 0.0;
                grad[(p * NV + o) * 2 + 1] = o == 3 ? m->By[c] : 0.0;
                for (int k = 2; k < 6; k++) grad[(p * NV + o) * 2 + k] = 0.0;
            }
            for (int v = o; v < o + 3; v++) rf[v].theta = 0.0;
            r0[o] = 0.0;
        }
    if (corr) coupling_correction(m, c, rf, corr);
}

void om_reconstruct_cell(const om_mesh *m, int c, const double *W, const double *gW, int linear, double G,
                         double *val, double *grad, double *r0)
{
    reconstruct_cell(m, c, W, gW, linear, G, 0.0, val, grad, r0, NULL);
}

void om_coupling_correction(const om_mesh *m, int c, const double *W, const double *gW, int linear, double G,
                            double *corr)
{
    double val[36], grad[72], r0[6];
    reconstruct_cell(m, c, W, gW, linear, G, 0.0, val, grad, r0, corr);
}

/* ----------------------------------------------------------------------------------------- */
/* gas-kinetic evolution at one Gauss point (Sec. 2.2, Eq. SWE-2nd-order), local frame         */

void om_moments(double U, double lam, int half, int K, double *out)
{
    double m0, m1;
    if (half == 0) {
        m0 = 1;
        m1 = U;
    } else if (half > 0) {
        m0 = 0.5 * erfc(-sqrt(lam) * U);
        m1 = U * m0 + exp(-lam * U * U) / (2 * sqrt(M_PI * lam));
    } else {
        m0 = 0.5 * erfc(sqrt(lam) * U);
        m1 = U * m0 - exp(-lam * U * U) / (2 * sqrt(M_PI * lam));
    }
    out[0] = m0;
    if (K > 1) out[1] = m1;
    for (int k = 2; k < K; k++) out[k] = U * out[k - 1] + (k - 1) / (2 * lam) * out[k - 2];
}

void om_time_integrals(double d, double tau, double *g)
{
    double E = exp(-d / tau);
    g[0] = d - tau * (1 - E);
    g[1] = -tau * d + 2 * tau * tau * (1 - E) - tau * d * E;
    g[2] = d * d / 2 - tau * d + tau * tau * (1 - E);
    g[3] = tau * (1 - E);
    g[4] = tau * (d + tau) * E - tau * tau;
}

#define PD 6
typedef struct {
    double c[PD][PD]; /* coefficient of u^i v^j */
} poly;

static void p_zero(poly *p) { memset(p, 0, sizeof(poly)); }

/* p += s * slope(u, v) with slope = lam (dh/h) ((u-U)^2 + (v-V)^2) + 2 lam ((u-U) dU + (v-V) dV):
 * the spatial or time derivative of ln g for the Maxwellian g(h, U, V), lam = 1/(G h)
 * (reading: Maxwellian-consistent slopes) */
static void p_add_slope(poly *p, double s, double lam, double h, double U, double V, double dh,
                        double dhU, double dhV)
{
    double dU = (dhU - U * dh) / h, dV = (dhV - V * dh) / h;
    double A = lam * dh / h, Bc = 2 * lam;
    /* A (u^2 - 2Uu + U^2 + v^2 - 2Vv + V^2) + Bc (u dU - U dU + v dV - V dV) */
    p->c[2][0] += s * A;
    p->c[0][2] += s * A;
    p->c[1][0] += s * (-2 * U * A + Bc * dU);
    p->c[0][1] += s * (-2 * V * A + Bc * dV);
    p->c[0][0] += s * (A * (U * U + V * V) - Bc * (U * dU + V * dV));
}

/* out += u * p  or  v * p */
static void p_add_mul_u(poly *out, const poly *p)
{
    for (int i = 0; i + 1 < PD; i++)
        for (int j = 0; j < PD; j++) out->c[i + 1][j] += p->c[i][j];
}
static void p_add_mul_v(poly *out, const poly *p)
{
    for (int i = 0; i < PD; i++)
        for (int j = 0; j + 1 < PD; j++) out->c[i][j + 1] += p->c[i][j];
}

/* combined polynomial a_n u + a_t v - 2 lam_g (Phi_n (u - Ug) + Phi_t (v - Vg)) for the Maxwellian
 * (lam_g, h_g, Ug, Vg) and the derivatives of one side */
static void p_micro(poly *out, double lam, double h, double U, double V, const double *side)
{
    poly an, at;
    p_zero(&an);
    p_zero(&at);
    p_add_slope(&an, 1, lam, h, U, V, side[3], side[5], side[7]);
    p_add_slope(&at, 1, lam, h, U, V, side[4], side[6], side[8]);
    p_zero(out);
    p_add_mul_u(out, &an);
    p_add_mul_v(out, &at);
    /* reading: the well-balance constants alpha are all 1 with these slopes */
    out->c[1][0] += -2 * lam * side[9];
    out->c[0][1] += -2 * lam * side[10];
    out->c[0][0] += 2 * lam * (side[9] * U + side[10] * V);
}

/* <u^e psi_m p> over the Maxwellian with thickness h, u-moments mu and v-moments nv */
static void p_moment3(const poly *p, int e, double h, const double *mu, const double *nv, double *o)
{
    o[0] = o[1] = o[2] = 0;
    for (int i = 0; i < PD; i++)
        for (int j = 0; j < PD; j++) {
            double c = p->c[i][j];
            if (c == 0) continue;
            o[0] += c * mu[i + e] * nv[j];
            o[1] += c * mu[i + e + 1] * nv[j];
            o[2] += c * mu[i + e] * nv[j + 1];
        }
    o[0] *= h;
    o[1] *= h;
    o[2] *= h;
}

#define NM (PD + 3)

typedef struct {
    double B[5][3];   /* the five moment brackets multiplying Gamma_1..Gamma_5 */
    double Wb[3], Wbt[3];
} gks_brackets;

/* Well-balance weights of the acceleration term in the interface equilibrium's part of the
 * evolution solution (Sec. 2.2, Eq. SWE-2nd-order, the constants alpha_{k,m}).  Reading: they
 * are the weights that make the half-space moments of a balanced pair -- the |c|^2 slope of a
 * level and the equal and opposite acceleration -2 lambda Phi . (u - U) -- vanish for this
 * reading's Maxwellian-consistent slopes: (3/4, 1, 1) for the moments <psi_m> and (1, 5/4, 5/4)
 * for <u psi_m> (m: mass, normal, tangential momentum).  The correction is taken relative to the
 * full-space moments, so it vanishes where the two sides agree and the scheme stays consistent;
 * it only acts on the jump between the sides' accelerations. */
static const double ALPHA_W[2][3] = {{0.75, 1.0, 1.0}, {1.0, 1.25, 1.25}};

static void alpha_correction(const double *sL, const double *sR, double lamb, double hb, double Ub, double Vb,
                             const double *mub, const double *mubp, const double *mubm, const double *nvb, int e,
                             double *d)
{
    double fL[11] = {0}, fR[11] = {0};
    for (int i = 9; i < 11; i++) {
        fL[i] = sL[i];
        fR[i] = sR[i];
    }
    poly FL, FR;
    p_micro(&FL, lamb, hb, Ub, Vb, fL); /* the acceleration term alone */
    p_micro(&FR, lamb, hb, Ub, Vb, fR);
    double lp[3], rm[3], lf[3], rf[3];
    p_moment3(&FL, e, hb, mubp, nvb, lp);
    p_moment3(&FR, e, hb, mubm, nvb, rm);
    p_moment3(&FL, e, hb, mub, nvb, lf);
    p_moment3(&FR, e, hb, mub, nvb, rf);
    for (int k = 0; k < 3; k++) d[k] = (ALPHA_W[e][k] - 1) * (lp[k] + rm[k] - 0.5 * (lf[k] + rf[k]));
}

/* The paper's printed constants (Sec. 2.2, Eq. SWE-2nd-order), as an alternative reading
 * (alpha_mode 1): alpha_{1,m} = (1, 3/4, 1/4) weight the acceleration term -2 lam Phi . (u - U)
 * in the flux moments <u psi_m> (m: mass, normal, tangential momentum) of both the interface
 * equilibrium's part (C2 term) and the initial distributions' part (C5 term); alpha_{2,m} = 1 for
 * the state moments, so the time slope of the interface equilibrium is unweighted.  Returns the
 * changes of the C2 and C5 brackets. */
static const double ALPHA_PAPER[3] = {1.0, 0.75, 0.25};

static void alpha_paper(const double *sL, const double *sR, double G, double lamb, double hb, double Ub,
                        double Vb, const double *mubp, const double *mubm, const double *nvb, double *d2,
                        double *d5)
{
    double fL[11] = {0}, fR[11] = {0};
    for (int i = 9; i < 11; i++) {
        fL[i] = sL[i];
        fR[i] = sR[i];
    }
    poly FL, FR;
    double lp[3], rm[3];
    p_micro(&FL, lamb, hb, Ub, Vb, fL); /* acceleration over the interface equilibrium */
    p_micro(&FR, lamb, hb, Ub, Vb, fR);
    p_moment3(&FL, 1, hb, mubp, nvb, lp);
    p_moment3(&FR, 1, hb, mubm, nvb, rm);
    for (int k = 0; k < 3; k++) d2[k] = (ALPHA_PAPER[k] - 1) * (lp[k] + rm[k]);
    double hL = sL[0], UL = sL[1], VL = sL[2], hR = sR[0], UR = sR[1], VR = sR[2];
    for (int k = 0; k < 3; k++) lp[k] = rm[k] = 0; /* a vacuum side has no particles */
    if (hL > 0) {
        double lamL = 1 / (G * hL), muLp[NM], nvL[NM];
        om_moments(UL, lamL, +1, NM, muLp);
        om_moments(VL, lamL, 0, NM, nvL);
        p_micro(&FL, lamL, hL, UL, VL, fL); /* acceleration over each side's own Maxwellian */
        p_moment3(&FL, 1, hL, muLp, nvL, lp);
    }
    if (hR > 0) {
        double lamR = 1 / (G * hR), muRm[NM], nvR[NM];
        om_moments(UR, lamR, -1, NM, muRm);
        om_moments(VR, lamR, 0, NM, nvR);
        p_micro(&FR, lamR, hR, UR, VR, fR);
        p_moment3(&FR, 1, hR, muRm, nvR, rm);
    }
    for (int k = 0; k < 3; k++) d5[k] = (ALPHA_PAPER[k] - 1) * (lp[k] + rm[k]);
}

static void gks_brackets_eval(const double *sL, const double *sR, double G, int alpha_mode, gks_brackets *o)
{
    double hL = sL[0], UL = sL[1], VL = sL[2];
    double hR = sR[0], UR = sR[1], VR = sR[2];
    /* a side at zero thickness is a vacuum: its moments are zero (its record is all zeros) */
    const int wetL = hL > 0, wetR = hR > 0;
    double lamL = wetL ? 1 / (G * hL) : 0, lamR = wetR ? 1 / (G * hR) : 0;
    double muLp[NM] = {0}, muRm[NM] = {0}, nvL[NM] = {0}, nvR[NM] = {0};
    if (wetL) {
        om_moments(UL, lamL, +1, NM, muLp);
        om_moments(VL, lamL, 0, NM, nvL);
    }
    if (wetR) {
        om_moments(UR, lamR, -1, NM, muRm);
        om_moments(VR, lamR, 0, NM, nvR);
    }
    /* interface state: particles from the left moving right plus from the right moving left */
    double Wb[3];
    Wb[0] = hL * muLp[0] + hR * muRm[0];
    Wb[1] = hL * muLp[1] + hR * muRm[1];
    Wb[2] = hL * muLp[0] * VL + hR * muRm[0] * VR;
    if (!(Wb[0] > 0)) { /* no particles at the interface */
        memset(o, 0, sizeof(*o));
        return;
    }
    double hb = Wb[0], Ub = Wb[1] / hb, Vb = Wb[2] / hb, lamb = 1 / (G * hb);
    double mub[NM], mubp[NM], mubm[NM], nvb[NM];
    om_moments(Ub, lamb, 0, NM, mub);
    om_moments(Ub, lamb, +1, NM, mubp);
    om_moments(Ub, lamb, -1, NM, mubm);
    om_moments(Vb, lamb, 0, NM, nvb);
    /* slopes of the equilibrium at the interface built with each side's derivatives */
    poly PbL, PbR, PL, PR, one;
    p_micro(&PbL, lamb, hb, Ub, Vb, sL);
    p_micro(&PbR, lamb, hb, Ub, Vb, sR);
    if (wetL)
        p_micro(&PL, lamL, hL, UL, VL, sL);
    else
        p_zero(&PL);
    if (wetR)
        p_micro(&PR, lamR, hR, UR, VR, sR);
    else
        p_zero(&PR);
    p_zero(&one);
    one.c[0][0] = 1;
    /* time slope of the interface equilibrium from compatibility */
    double t1[3], t2[3], Wbt[3], da[3];
    p_moment3(&PbL, 0, hb, mubp, nvb, t1);
    p_moment3(&PbR, 0, hb, mubm, nvb, t2);
    if (alpha_mode == 0)
        alpha_correction(sL, sR, lamb, hb, Ub, Vb, mub, mubp, mubm, nvb, 0, da);
    else
        da[0] = da[1] = da[2] = 0; /* the paper's alpha_{2,m} = 1 */
    for (int k = 0; k < 3; k++) Wbt[k] = -(t1[k] + t2[k] + da[k]);
    poly Abar;
    p_zero(&Abar);
    p_add_slope(&Abar, 1, lamb, hb, Ub, Vb, Wbt[0], Wbt[1], Wbt[2]);
    p_moment3(&one, 1, hb, mub, nvb, o->B[0]);
    p_moment3(&PbL, 1, hb, mubp, nvb, t1);
    p_moment3(&PbR, 1, hb, mubm, nvb, t2);
    double d5[3] = {0, 0, 0};
    if (alpha_mode == 0)
        alpha_correction(sL, sR, lamb, hb, Ub, Vb, mub, mubp, mubm, nvb, 1, da);
    else
        alpha_paper(sL, sR, G, lamb, hb, Ub, Vb, mubp, mubm, nvb, da, d5);
    for (int k = 0; k < 3; k++) o->B[1][k] = t1[k] + t2[k] + da[k];
    p_moment3(&Abar, 1, hb, mub, nvb, o->B[2]);
    p_moment3(&one, 1, hL, muLp, nvL, t1);
    p_moment3(&one, 1, hR, muRm, nvR, t2);
    for (int k = 0; k < 3; k++) o->B[3][k] = t1[k] + t2[k];
    p_moment3(&PL, 1, hL, muLp, nvL, t1);
    p_moment3(&PR, 1, hR, muRm, nvR, t2);
    for (int k = 0; k < 3; k++) o->B[4][k] = t1[k] + t2[k] + d5[k];
    for (int k = 0; k < 3; k++) {
        o->Wb[k] = Wb[k];
        o->Wbt[k] = Wbt[k];
    }
}

void om_side_rate(const double *sd, double G, double *Wt)
{
    if (!(sd[0] > 0)) { /* a vacuum side */
        Wt[0] = Wt[1] = Wt[2] = 0;
        return;
    }
    double h = sd[0], U = sd[1], V = sd[2], lam = 1 / (G * h);
    double mu[NM], nv[NM];
    om_moments(U, lam, 0, NM, mu);
    om_moments(V, lam, 0, NM, nv);
    poly P;
    p_micro(&P, lam, h, U, V, sd);
    p_moment3(&P, 0, h, mu, nv, Wt);
    for (int k = 0; k < 3; k++) Wt[k] = -Wt[k];
}

void om_gks_point_integrated(const double *sL, const double *sR, double G, double delta,
                             double tau, double *F)
{
    gks_brackets br;
    gks_brackets_eval(sL, sR, G, 0, &br);
    double g[5];
    om_time_integrals(delta, tau, g);
    for (int k = 0; k < 3; k++) {
        F[k] = 0;
        for (int i = 0; i < 5; i++) F[k] += g[i] * br.B[i][k];
    }
}

void om_gks_point_mode(const double *sL, const double *sR, double G, double dt, double eps,
                       double eps_num, int alpha_mode, double *F0, double *Ft, double *Wb, double *Wbt)
{
    om_gks_point_wd(sL, sR, G, dt, eps, eps_num, alpha_mode, 0.0, 0, F0, Ft, Wb, Wbt);
}

void om_gks_point_wd(const double *sL, const double *sR, double G, double dt, double eps,
                     double eps_num, int alpha_mode, double h_dry, int order1, double *F0, double *Ft,
                     double *Wb, double *Wbt)
{
    gks_brackets br;
    gks_brackets_eval(sL, sR, G, alpha_mode, &br);
    if (!(br.Wb[0] > h_dry)) { /* a dry interface passes nothing */
        for (int k = 0; k < 3; k++) F0[k] = Ft[k] = Wb[k] = Wbt[k] = 0;
        return;
    }
    /* collision time with the pressure-jump term (Sec. 4) */
    double pl = sL[0] * sL[0], pr = sR[0] * sR[0];
    double tau = eps * dt + eps_num * fabs((pl - pr) / (pl + pr)) * dt;
    double g1[5], g2[5], F1[3], F2[3];
    om_time_integrals(dt, tau, g1);
    om_time_integrals(0.5 * dt, tau, g2);
    for (int k = 0; k < 3; k++) {
        F1[k] = F2[k] = 0;
        for (int i = 0; i < 5; i++) {
            F1[k] += g1[i] * br.B[i][k];
            F2[k] += g2[i] * br.B[i][k];
        }
        /* flux and its time derivative from F(dt) and F(dt/2) for a linear-in-time flux; at first
         * order the step's mean flux with no time derivative */
        F0[k] = order1 ? F1[k] / dt : (4 * F2[k] - F1[k]) / dt;
        Ft[k] = order1 ? 0.0 : 4 * (F1[k] - 2 * F2[k]) / (dt * dt);
        Wb[k] = br.Wb[k];
        Wbt[k] = br.Wbt[k];
    }
}

void om_gks_point(const double *sL, const double *sR, double G, double dt, double eps,
                  double eps_num, double *F0, double *Ft, double *Wb, double *Wbt)
{
    om_gks_point_mode(sL, sR, G, dt, eps, eps_num, 0, F0, Ft, Wb, Wbt);
}

/* ----------------------------------------------------------------------------------------- */
/* time step (Sec. 4)                                                                         */

double om_dt(const om_mesh *m, const om_params *p, const double *W)
{
    int T = m->nt;
    double dxmin = 1e300, smax = 0;
    for (int c = 0; c < T; c++) {
        if (m->dX[c] < dxmin) dxmin = m->dX[c];
        for (int layer = 0; layer < 2; layer++) {
            int o = 3 * layer;
            double h = W[o * T + c];
            double U = om_cell_velocity(h, W[(o + 1) * T + c], p->h_dry);
            double V = om_cell_velocity(h, W[(o + 2) * T + c], p->h_dry);
            double s = sqrt(U * U + V * V) + sqrt(p->G * fmax(h, 0.0)); /* a dry cell may hold -0 */
            if (s > smax) smax = s;
        }
    }
    return p->cfl * dxmin / smax;
}

/* ----------------------------------------------------------------------------------------- */
/* one stage of the spatial operator                                                          */

/* mirror of a Gauss-point record across the boundary edge with unit normal n (R = I - 2 n n^T):
 * vec != 0 a wall (momentum reflected), vec = 0 a free boundary (every component even) */
static void mirror_record(const double *n, int vec, const double *val, const double *grad, double *mval,
                          double *mgrad)
{
    double R[2][2] = {{1 - 2 * n[0] * n[0], -2 * n[0] * n[1]}, {-2 * n[0] * n[1], 1 - 2 * n[1] * n[1]}};
    const double I[2][2] = {{1, 0}, {0, 1}};
    const double(*V)[2] = vec ? R : I;
    for (int layer = 0; layer < 2; layer++) {
        int o = 3 * layer;
        mval[o] = val[o];
        double mv[2] = {val[o + 1], val[o + 2]}, rm[2];
        map_vec(V, mv, rm);
        mval[o + 1] = rm[0];
        mval[o + 2] = rm[1];
        map_vec(R, grad + 2 * o, mgrad + 2 * o);
        double Gm[2][2] = {{grad[2 * (o + 1)], grad[2 * (o + 1) + 1]}, {grad[2 * (o + 2)], grad[2 * (o + 2) + 1]}};
        double RG[2][2];
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++) RG[i][j] = V[i][0] * Gm[0][j] + V[i][1] * Gm[1][j];
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++) mgrad[2 * (o + 1 + i) + j] = RG[i][0] * R[j][0] + RG[i][1] * R[j][1];
    }
}

int om_operator_src(const om_mesh *m, const om_params *p, double dt, const double *W, const double *gW,
                    double *Lo, double *Lto, double *GWo, double *GWto, double *So, double *Sto)
{
    int T = m->nt, E = m->ne;
    const double G = p->G, chi = p->chi;
    const int src4 = p->src_order == 4;
    /* 1. reconstruction at the Gauss points of every cell (and, for the higher-order coupling,
     *    the interior correction of each cell) */
    double *val = (double *)malloc(sizeof(double) * (size_t)T * 36);
    double *grd = (double *)malloc(sizeof(double) * (size_t)T * 72);
    double *r0 = (double *)malloc(sizeof(double) * (size_t)T * 6);
    double *corr = src4 ? (double *)malloc(sizeof(double) * (size_t)T * 8) : NULL;
#pragma omp parallel for schedule(dynamic, 256) if(T >= OMP_MIN_ITEMS)
    for (int c = 0; c < T; c++)
        reconstruct_cell(m, c, W, gW, p->linear, p->G, p->h_dry, val + (size_t)c * 36, grd + (size_t)c * 72, r0 + (size_t)c * 6,
                         src4 ? corr + (size_t)c * 8 : NULL);

    /* side records of edge e, Gauss point g (edge orientation), side s: pointers or mirrors */
#define REC_VAL(c, k, g) (val + (size_t)(c) * 36 + (2 * (k) + (g)) * 6)
#define REC_GRD(c, k, g) (grd + (size_t)(c) * 72 + (2 * (k) + (g)) * 12)

    /* 2. interface modelling of the heights that drive the layer forces (Sec. 2.3):
     *    field 0 = eta1 = h1 + B with layer-1 velocities, field 1 = h2 with layer-2 velocities */
    double *hmid = (double *)malloc(sizeof(double) * (size_t)E * 2);
#pragma omp parallel for schedule(static) if(E >= OMP_MIN_ITEMS)
    for (int e = 0; e < E; e++) {
        int L = m->e_cell[2 * e], R = m->e_cell[2 * e + 1];
        int kL = m->e_lk[2 * e], kR = m->e_lk[2 * e + 1];
        const double *n = m->e_n + 2 * e;
        double acc[2] = {0, 0};
        for (int g = 0; g < 2; g++) {
            const double *vl = REC_VAL(L, kL, g);
            double vr[6], gr[12];
            if (R >= 0) {
                memcpy(vr, REC_VAL(R, kR, 1 - g), sizeof(vr));
            } else {
                mirror_record(n, !m->free_bc, vl, REC_GRD(L, kL, g), vr, gr);
            }
            double Bg = m->e_Bgp[2 * e + g];
            for (int f = 0; f < 2; f++) {
                int o = f == 0 ? 3 : 0; /* eta1 lives in slot 3, h2 in slot 0 */
                double hl = f == 0 ? vl[3] - Bg : vl[0], hr = f == 0 ? vr[3] - Bg : vr[0];
                /* a dry side (wet/dry reading) has no velocity */
                double unl = hl > p->h_dry && hl > 0 ? (vl[o + 1] * n[0] + vl[o + 2] * n[1]) / hl : 0.0;
                double unr = hr > p->h_dry && hr > 0 ? (vr[o + 1] * n[0] + vr[o + 2] * n[1]) / hr : 0.0;
                acc[f] += 0.5 * om_edge_height(vl[o], vr[o], hl, hr, unl, unr, G);
            }
        }
        hmid[2 * e] = acc[0];
        hmid[2 * e + 1] = acc[1];
    }
    /* gradient of the plane through the three edge-centre values of each cell */
    double *gP1 = (double *)malloc(sizeof(double) * (size_t)T * 4);
#pragma omp parallel for schedule(static) if(T >= OMP_MIN_ITEMS)
    for (int c = 0; c < T; c++) {
        for (int f = 0; f < 2; f++) {
            double hk[3];
            for (int k = 0; k < 3; k++) hk[k] = hmid[2 * m->c_edge[3 * c + k] + f];
            om_plane_gradient(m, c, hk, gP1 + 4 * c + 2 * f);
        }
    }

    /* 3. gas-kinetic evolution at every Gauss point of every edge, both layers */
    double *eo = (double *)malloc(sizeof(double) * (size_t)E * 2 * 2 * 26);
#define EO(e, g, layer) (eo + (((size_t)(e) * 2 + (g)) * 2 + (layer)) * 26)
#pragma omp parallel for schedule(dynamic, 256) if(E >= OMP_MIN_ITEMS)
    for (int e = 0; e < E; e++) {
        int L = m->e_cell[2 * e], R = m->e_cell[2 * e + 1];
        int kL = m->e_lk[2 * e], kR = m->e_lk[2 * e + 1];
        const double *n = m->e_n + 2 * e;
        double t[2] = {-n[1], n[0]};
        double Rm[2][2] = {{1 - 2 * n[0] * n[0], -2 * n[0] * n[1]}, {-2 * n[0] * n[1], 1 - 2 * n[1] * n[1]}};
        double gBL[2] = {m->Bx[L], m->By[L]}, gBR[2], gPL[4], gPR[4];
        for (int i = 0; i < 4; i++) gPL[i] = gP1[4 * L + i];
        double rL[2] = {r0[6 * L + 3], r0[6 * L + 0]}, rR[2];
        if (R >= 0) {
            gBR[0] = m->Bx[R];
            gBR[1] = m->By[R];
            for (int i = 0; i < 4; i++) gPR[i] = gP1[4 * R + i];
            rR[0] = r0[6 * R + 3];
            rR[1] = r0[6 * R + 0];
        } else {
            map_vec(Rm, gBL, gBR);
            map_vec(Rm, gPL, gPR);
            map_vec(Rm, gPL + 2, gPR + 2);
            rR[0] = rL[0];
            rR[1] = rL[1];
        }
        /* reading: single-valued bottom slope at the interface (the test-only switch gives each
         * side its own cell's slope instead) */
        double gB[2] = {0.5 * (gBL[0] + gBR[0]), 0.5 * (gBL[1] + gBR[1])};
        double gBs[2][2];
        for (int d = 0; d < 2; d++) {
            gBs[0][d] = p->per_side_gb ? gBL[d] : gB[d];
            gBs[1][d] = p->per_side_gb ? gBR[d] : gB[d];
        }
        /* reading: nonlinear weight of the force model from the cells' high-order weights */
        double wf[2];
        for (int f = 0; f < 2; f++) {
            wf[f] = fmin(1.0, fmin(rL[f], rR[f]));
            /* within 1e-12 of 1 the blend changes the acceleration by less than its rounding */
            if (wf[f] >= 1.0 - 1e-12) wf[f] = 1.0;
        }
        for (int g = 0; g < 2; g++) {
            double vs[2][6], gs[2][12];
            memcpy(vs[0], REC_VAL(L, kL, g), sizeof(vs[0]));
            memcpy(gs[0], REC_GRD(L, kL, g), sizeof(gs[0]));
            if (R >= 0) {
                memcpy(vs[1], REC_VAL(R, kR, 1 - g), sizeof(vs[1]));
                memcpy(gs[1], REC_GRD(R, kR, 1 - g), sizeof(gs[1]));
            } else {
                mirror_record(n, !m->free_bc, vs[0], gs[0], vs[1], gs[1]);
            }
            double Bg = m->e_Bgp[2 * e + g];
            double side[2][2][11]; /* [layer: 0 lower, 1 upper][side][...] */
            for (int s = 0; s < 2; s++) {
                const double *gP = s == 0 ? gPL : gPR;
                /* modelled derivatives (Sec. 2.3 nonlinear combination) */
                double deta[2], dh2[2];
                for (int d = 0; d < 2; d++) {
                    deta[d] = wf[0] * gs[s][2 * 3 + d] + (1 - wf[0]) * gP[d];
                    dh2[d] = wf[1] * gs[s][2 * 0 + d] + (1 - wf[1]) * gP[2 + d];
                }
                /* accelerations (Sec. 2.1 source terms over h): lower layer feels the bottom and
                 * the upper layer's thickness, upper layer the interface level */
                double phi1[2], phi2[2];
                for (int d = 0; d < 2; d++) {
                    phi1[d] = -G * gBs[s][d] - chi * G * dh2[d];
                    phi2[d] = -G * deta[d];
                }
                for (int layer = 0; layer < 2; layer++) {
                    int o = layer == 0 ? 3 : 0;
                    double h = layer == 0 ? vs[s][3] - Bg : vs[s][0];
                    double dh[2];
                    for (int d = 0; d < 2; d++) dh[d] = layer == 0 ? gs[s][2 * 3 + d] - gBs[s][d] : gs[s][d];
                    const double *dm1 = gs[s] + 2 * (o + 1), *dm2 = gs[s] + 2 * (o + 2);
                    const double *phi = layer == 0 ? phi1 : phi2;
                    double mx = vs[s][o + 1], my = vs[s][o + 2];
                    double *sd = side[layer][s];
                    if (p->h_dry > 0 && !(h > p->h_dry)) { /* wet/dry reading: a dry side is a vacuum */
                        for (int i = 0; i < 11; i++) sd[i] = 0.0;
                        continue;
                    }
                    sd[0] = h;
                    sd[1] = (mx * n[0] + my * n[1]) / h;
                    sd[2] = (mx * t[0] + my * t[1]) / h;
                    sd[3] = dh[0] * n[0] + dh[1] * n[1];
                    sd[4] = dh[0] * t[0] + dh[1] * t[1];
                    /* derivatives of the rotated momenta (hU_n, hU_t) */
                    double dmn_x = dm1[0] * n[0] + dm2[0] * n[1], dmn_y = dm1[1] * n[0] + dm2[1] * n[1];
                    double dmt_x = dm1[0] * t[0] + dm2[0] * t[1], dmt_y = dm1[1] * t[0] + dm2[1] * t[1];
                    sd[5] = dmn_x * n[0] + dmn_y * n[1];
                    sd[6] = dmn_x * t[0] + dmn_y * t[1];
                    sd[7] = dmt_x * n[0] + dmt_y * n[1];
                    sd[8] = dmt_x * t[0] + dmt_y * t[1];
                    sd[9] = phi[0] * n[0] + phi[1] * n[1];
                    sd[10] = phi[0] * t[0] + phi[1] * t[1];
                }
            }
            for (int layer = 0; layer < 2; layer++) {
                /* wet/dry reading: at an edge of the layer's front band (r0 = 0 on either side) the
                 * evolution is of first order: the sides' states alone, no slopes, no acceleration,
                 * and the step's mean flux */
                const int order1 = p->h_dry > 0 && (rL[layer] == 0.0 || rR[layer] == 0.0);
                if (order1)
                    for (int s = 0; s < 2; s++)
                        for (int i = 3; i < 11; i++) side[layer][s][i] = 0.0;
                double F0[3], Ft[3], Wb[3], Wbt[3];
                om_gks_point_wd(side[layer][0], side[layer][1], G, dt, p->eps, p->eps_num, p->alpha_mode,
                                p->h_dry, order1, F0, Ft, Wb, Wbt);
                if (R < 0 && !m->free_bc) { /* reflecting wall: no mass crosses */
                    F0[0] = 0;
                    Ft[0] = 0;
                }
                double *out = EO(e, g, layer);
                const double *src[4] = {F0, Ft, Wb, Wbt};
                for (int q = 0; q < 4; q++) {
                    out[3 * q] = src[q][0];
                    out[3 * q + 1] = src[q][1] * n[0] + src[q][2] * t[0];
                    out[3 * q + 2] = src[q][1] * n[1] + src[q][2] * t[1];
                }
                /* reading of the Gauss-point thicknesses in the layer coupling (Sec. 3.2, Eq.
                 * SWE-source-discretization): the mean of the two sides' reconstructed values, and
                 * for its time derivative the mean of the sides' own rates -div(h U) */
                const double *a = side[layer][0], *b = side[layer][1];
                out[12] = 0.5 * (a[0] + b[0]);
                out[13] = -0.5 * ((a[5] + a[8]) + (b[5] + b[8]));
                /* the discontinuous reading of the gradient update (Sec. 3.3, the values W^l, W^r
                 * at the inner sides): each side's own state and its own time derivative, in the
                 * global frame (14..19 left side, 20..25 right side) */
                for (int s = 0; s < 2; s++) {
                    const double *sd = side[layer][s];
                    double Ws[3] = {sd[0], sd[0] * sd[1], sd[0] * sd[2]}, Wst[3];
                    om_side_rate(sd, G, Wst);
                    double *o6 = out + 14 + 6 * s;
                    o6[0] = Ws[0];
                    o6[1] = Ws[1] * n[0] + Ws[2] * t[0];
                    o6[2] = Ws[1] * n[1] + Ws[2] * t[1];
                    o6[3] = Wst[0];
                    o6[4] = Wst[1] * n[0] + Wst[2] * t[0];
                    o6[5] = Wst[1] * n[1] + Wst[2] * t[1];
                }
            }
        }
    }

    /* 4. cell gather: flux divergence, Green-Gauss gradients of the interface values, sources */
#pragma omp parallel for schedule(static) if(T >= OMP_MIN_ITEMS)
    for (int c = 0; c < T; c++) {
        double LF[6] = {0}, LFt[6] = {0}, GG[6][2] = {{0}}, GGt[6][2] = {{0}};
        double hsum[6] = {0}, htsum[6] = {0};
        double GGc[6][2] = {{0}}, GGct[6][2] = {{0}}; /* central Gauss-point thicknesses (slots 0, 3) */
        double inv = 1.0 / m->area[c];
        for (int k = 0; k < 3; k++) {
            int e = m->c_edge[3 * c + k];
            double sg = m->c_side[3 * c + k] == 0 ? 1.0 : -1.0;
            double ln = m->e_len[e];
            const double *n = m->e_n + 2 * e;
            for (int layer = 0; layer < 2; layer++) {
                int o = layer == 0 ? 3 : 0;
                for (int v = 0; v < 3; v++) {
                    double F0 = 0, Ft = 0, Wb = 0, Wbt = 0;
                    /* interface value of the gradient update: the evolution's W-bar, or the value
                     * on this cell's own side of the edge */
                    const int wo = p->grad_mode == 1 ? (sg > 0 ? 14 : 20) : 6;
                    for (int g = 0; g < 2; g++) {
                        const double *q = EO(e, g, layer);
                        F0 += 0.5 * q[v];
                        Ft += 0.5 * q[3 + v];
                        Wb += 0.5 * q[wo + v];
                        Wbt += 0.5 * q[wo + 3 + v];
                    }
                    LF[o + v] -= sg * ln * F0 * inv;
                    LFt[o + v] -= sg * ln * Ft * inv;
                    for (int d = 0; d < 2; d++) {
                        GG[o + v][d] += sg * ln * n[d] * Wb * inv;
                        GGt[o + v][d] += sg * ln * n[d] * Wbt * inv;
                    }
                    if (v == 0) {
                        double hc = 0, hct = 0;
                        for (int g = 0; g < 2; g++) {
                            hc += 0.5 * EO(e, g, layer)[12];
                            hct += 0.5 * EO(e, g, layer)[13];
                        }
                        for (int d = 0; d < 2; d++) {
                            GGc[o][d] += sg * ln * n[d] * hc * inv;
                            GGct[o][d] += sg * ln * n[d] * hct * inv;
                        }
                        hsum[o] += hc / 3.0;
                        htsum[o] += hct / 3.0;
                    }
                }
            }
        }
        double L[6], Lt[6];
        for (int v = 0; v < 6; v++) {
            L[v] = LF[v];
            Lt[v] = LFt[v];
        }
        double gB[2] = {m->Bx[c], m->By[c]};
        /* bottom source h_j (0, -G B_x, -G B_y) (Sec. 3.2) and its time derivative through the
         * cell's thickness rate */
        for (int d = 0; d < 2; d++) {
            L[1 + d] += W[0 * T + c] * (-G * gB[d]);
            L[4 + d] += W[3 * T + c] * (-G * gB[d]);
            Lt[1 + d] += LF[0] * (-G * gB[d]);
            Lt[4 + d] += LF[3] * (-G * gB[d]);
        }
        /* layer coupling (Sec. 3.2, Eq. SWE-source-discretization): Gauss-point mean thickness of
         * one layer times the Green-Gauss derivative of the other, from the central Gauss-point
         * thicknesses; its time derivative by the product rule.  Higher order (the paper's remark
         * on more integration points): the cell average of the thickness in place of the
         * Gauss-point mean, its rate from the cell's mass flux, plus the interior correction. */
        double S[4], St[4];
        for (int d = 0; d < 2; d++) {
            if (src4) {
                const double *cc = corr + (size_t)c * 8;
                double h1 = W[3 * T + c], h2 = W[0 * T + c]; /* cell-average thicknesses */
                S[d] = -chi * G * (h1 * GGc[0][d] + cc[d]);
                St[d] = -chi * G * (LF[3] * GGc[0][d] + h1 * GGct[0][d] + cc[4 + d]);
                S[2 + d] = -G * (h2 * GGc[3][d] + cc[2 + d]);
                St[2 + d] = -G * (LF[0] * GGc[3][d] + h2 * GGct[3][d] + cc[6 + d]);
            } else {
                S[d] = -chi * G * hsum[3] * GGc[0][d];
                St[d] = -chi * G * (htsum[3] * GGc[0][d] + hsum[3] * GGct[0][d]);
                S[2 + d] = -G * hsum[0] * GGc[3][d];
                St[2 + d] = -G * (htsum[0] * GGc[3][d] + hsum[0] * GGct[3][d]);
            }
            L[4 + d] += S[d];
            Lt[4 + d] += St[d];
            L[1 + d] += S[2 + d];
            Lt[1 + d] += St[2 + d];
        }
        if (So)
            for (int k = 0; k < 4; k++) {
                So[(size_t)k * T + c] = S[k];
                Sto[(size_t)k * T + c] = St[k];
            }
        for (int v = 0; v < 6; v++) {
            Lo[v * T + c] = L[v];
            Lto[v * T + c] = Lt[v];
            for (int d = 0; d < 2; d++) {
                GWo[(2 * v + d) * T + c] = GG[v][d];
                GWto[(2 * v + d) * T + c] = GGt[v][d];
            }
        }
    }
    free(val);
    free(grd);
    free(r0);
    free(corr);
    free(hmid);
    free(gP1);
    free(eo);
    return 0;
}

int om_operator(const om_mesh *m, const om_params *p, double dt, const double *W, const double *gW,
                double *Lo, double *Lto, double *GWo, double *GWto)
{
    return om_operator_src(m, p, dt, W, gW, Lo, Lto, GWo, GWto, NULL, NULL);
}

/* ----------------------------------------------------------------------------------------- */
/* S2O4 step (Sec. 3.3)                                                                       */

void om_s2o4_stage(int n, double dt, const double *W, const double *L, const double *Lt, double *out)
{
    for (int i = 0; i < n; i++) out[i] = W[i] + 0.5 * dt * L[i] + 0.125 * dt * dt * Lt[i];
}

void om_s2o4_final(int n, double dt, const double *W, const double *L, const double *Lt, const double *Lt2,
                   double *out)
{
    for (int i = 0; i < n; i++) out[i] = W[i] + dt * L[i] + dt * dt / 6.0 * Lt[i] + dt * dt / 3.0 * Lt2[i];
}

int om_step(const om_mesh *m, const om_params *p, double dt, int nstages, const double *W,
            const double *gW, double *Wout, double *gWout)
{
    size_t T = m->nt;
    double *L = (double *)malloc(sizeof(double) * 6 * T), *Lt = (double *)malloc(sizeof(double) * 6 * T);
    double *G = (double *)malloc(sizeof(double) * 12 * T), *Gt = (double *)malloc(sizeof(double) * 12 * T);
    om_operator(m, p, dt, W, gW, L, Lt, G, Gt);
    if (nstages == 1) {
        om_s2o4_stage((int)(6 * T), dt, W, L, Lt, Wout);
        for (size_t i = 0; i < 12 * T; i++) gWout[i] = G[i] + 0.5 * dt * Gt[i];
    } else {
        double *Ws = (double *)malloc(sizeof(double) * 6 * T), *gWs = (double *)malloc(sizeof(double) * 12 * T);
        om_s2o4_stage((int)(6 * T), dt, W, L, Lt, Ws);
        for (size_t i = 0; i < 12 * T; i++) gWs[i] = G[i] + 0.5 * dt * Gt[i];
        double *L2 = (double *)malloc(sizeof(double) * 6 * T), *Lt2 = (double *)malloc(sizeof(double) * 6 * T);
        double *G2 = (double *)malloc(sizeof(double) * 12 * T), *Gt2 = (double *)malloc(sizeof(double) * 12 * T);
        om_operator(m, p, dt, Ws, gWs, L2, Lt2, G2, Gt2);
        om_s2o4_final((int)(6 * T), dt, W, L, Lt, Lt2, Wout);
        for (size_t i = 0; i < 12 * T; i++) gWout[i] = G[i] + dt * Gt2[i];
        free(Ws); free(gWs); free(L2); free(Lt2); free(G2); free(Gt2);
    }
    free(L); free(Lt); free(G); free(Gt);
    return 0;
}

void om_mass(const om_mesh *m, const double *W, double *mass)
{
    int T = m->nt;
    mass[0] = mass[1] = 0;
    for (int c = 0; c < T; c++) {
        mass[0] += m->area[c] * W[0 * T + c];
        mass[1] += m->area[c] * W[3 * T + c];
    }
}

/* ----------------------------------------------------------------------------------------- */
/* learned smoothness indicator: features and the multilayer perceptron                       */

#define MLP_IN 44
#define MLP_H 64

void om_features(const om_mesh *m, double G, const double *W, const double *gW, double *X)
{
#pragma omp parallel for schedule(static) if(m->nt >= OMP_MIN_ITEMS)
    for (int c = 0; c < m->nt; c++) {
        double q[NS][NV], gq[NS][NV][2];
        for (int l = 0; l < NS; l++) {
            int n = m->st_cell[NS * c + l];
            image_state(m, n, m->st_map[NS * c + l].R, !m->free_bc, W, gW, q[l], &gq[l][0][0]);
        }
        double h = sqrt(2.0 * m->area[c]);
        double *x = X + (size_t)c * MLP_IN;
        const int fields[2] = {3, 0}; /* eta1, h2 */
        const double thick[2] = {W[3 * m->nt + c], W[c]}; /* h1, h2 of the cell */
        for (int f = 0; f < 2; f++) {
            int v = fields[f];
            double Q0 = q[0][v], s = 0;
            for (int l = 1; l < NS; l++) s = fmax(s, fabs(q[l][v] - Q0));
            s += 1e-12 * fabs(Q0);
            for (int l = 1; l < NS; l++) x[17 * f + l - 1] = (q[l][v] - Q0) / s;
            for (int l = 0; l < 4; l++)
                for (int d = 0; d < 2; d++) x[17 * f + 9 + 2 * l + d] = h * gq[l][v][d] / s;
            /* size of the variation against the layer thickness */
            x[34 + f] = log10(s / thick[f]) / 4.0;
            /* momentum variation of the same layer against h sqrt(G h) */
            double cm = thick[f] * sqrt(G * thick[f]), sm = 0;
            for (int l = 1; l < NS; l++)
                for (int k = 1; k <= 2; k++) sm = fmax(sm, fabs(q[l][v + k] - q[0][v + k]));
            x[36 + f] = log10((sm + 1e-12 * cm) / cm) / 4.0;
        }
        for (int l = 1; l <= 3; l++) x[38 + l - 1] = m->area[m->st_cell[NS * c + l]] / m->area[c];
        for (int k = 0; k < 3; k++) x[41 + k] = m->e_len[m->c_edge[3 * c + k]] / h;
    }
}

/* hidden activations of one sample (ReLU layers) */
static void mlp_hidden(const double *P, const double *x, double *a1, double *h1, double *a2, double *h2)
{
    const double *W1 = P, *b1 = W1 + MLP_IN * MLP_H, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H;
    for (int j = 0; j < MLP_H; j++) {
        double s = b1[j];
        for (int i = 0; i < MLP_IN; i++) s += x[i] * W1[i * MLP_H + j];
        a1[j] = s;
        h1[j] = s > 0 ? s : 0;
    }
    for (int j = 0; j < MLP_H; j++) {
        double s = b2[j];
        for (int i = 0; i < MLP_H; i++) s += h1[i] * W2[i * MLP_H + j];
        a2[j] = s;
        h2[j] = s > 0 ? s : 0;
    }
}

void om_mlp_forward(const double *P, const double *X, int B, double *z)
{
    const double *w3 = P + MLP_IN * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H, *b3 = w3 + MLP_H;
    for (int s = 0; s < B; s++) {
        double a1[MLP_H], h1[MLP_H], a2[MLP_H], h2[MLP_H];
        mlp_hidden(P, X + (size_t)s * MLP_IN, a1, h1, a2, h2);
        double zz = b3[0];
        for (int j = 0; j < MLP_H; j++) zz += h2[j] * w3[j];
        z[s] = zz;
    }
}

/* v rounded to single precision, then to 8 significant bits (bfloat16), ties to even */
static double round_bf16(double v)
{
    float f = (float)v;
    if (f == 0.0f || !isfinite(f)) return (double)f;
    int e;
    double m = frexp((double)f, &e); /* f = m 2^e, 0.5 <= |m| < 1 */
    return ldexp(nearbyint(ldexp(m, 8)), e - 8);
}

void om_mlp_forward_bf16(const double *P, const double *X, int B, double *z)
{
    const double *W1 = P, *b1 = W1 + MLP_IN * MLP_H, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H;
    const double *w3 = b2 + MLP_H, *b3 = w3 + MLP_H;
    for (int s = 0; s < B; s++) {
        const double *x = X + (size_t)s * MLP_IN;
        double h1[MLP_H], zz = b3[0];
        for (int j = 0; j < MLP_H; j++) {
            double a = 0;
            for (int i = 0; i < MLP_IN; i++) a += round_bf16(x[i]) * round_bf16(W1[i * MLP_H + j]);
            a = (double)(float)a + b1[j];
            h1[j] = round_bf16(a > 0 ? a : 0);
        }
        for (int j = 0; j < MLP_H; j++) {
            double a = 0;
            for (int i = 0; i < MLP_H; i++) a += h1[i] * round_bf16(W2[i * MLP_H + j]);
            a += b2[j];
            zz += (a > 0 ? a : 0) * w3[j];
        }
        z[s] = zz;
    }
}

/* gradient of the mean logistic loss by backpropagation (chain rule, one sample at a time) */
double om_mlp_grad(const double *P, const double *X, const double *y, int B, double *grad)
{
    const int n1 = MLP_IN * MLP_H, n2 = MLP_H * MLP_H;
    const double *W2 = P + n1 + MLP_H, *w3 = W2 + n2 + MLP_H, *b3 = w3 + MLP_H;
    double *gW1 = grad, *gb1 = gW1 + n1, *gW2 = gb1 + MLP_H, *gb2 = gW2 + n2, *gw3 = gb2 + MLP_H, *gb3 = gw3 + MLP_H;
    for (int i = 0; i < n1 + MLP_H + n2 + MLP_H + MLP_H + 1; i++) grad[i] = 0;
    double loss = 0;
    for (int s = 0; s < B; s++) {
        const double *x = X + (size_t)s * MLP_IN;
        double a1[MLP_H], h1[MLP_H], a2[MLP_H], h2[MLP_H];
        mlp_hidden(P, x, a1, h1, a2, h2);
        double z = b3[0];
        for (int j = 0; j < MLP_H; j++) z += h2[j] * w3[j];
        /* softplus(z) - y z, written to avoid overflow */
        loss += (z > 0 ? z + log1p(exp(-z)) : log1p(exp(z))) - y[s] * z;
        double dz = (1.0 / (1.0 + exp(-z)) - y[s]) / B;
        double d2[MLP_H], d1[MLP_H];
        gb3[0] += dz;
        for (int j = 0; j < MLP_H; j++) {
            gw3[j] += dz * h2[j];
            d2[j] = a2[j] > 0 ? dz * w3[j] : 0;
            gb2[j] += d2[j];
        }
        for (int i = 0; i < MLP_H; i++) {
            double acc = 0;
            for (int j = 0; j < MLP_H; j++) {
                gW2[i * MLP_H + j] += h1[i] * d2[j];
                acc += W2[i * MLP_H + j] * d2[j];
            }
            d1[i] = a1[i] > 0 ? acc : 0;
            gb1[i] += d1[i];
        }
        for (int i = 0; i < MLP_IN; i++)
            for (int j = 0; j < MLP_H; j++) gW1[i * MLP_H + j] += x[i] * d1[j];
    }
    return loss / B;
}
