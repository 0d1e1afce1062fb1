/* Sanitizer driver for the oracle: builds a periodic lattice and a wall mesh with a bottom,
 * runs nonlinear steps (on the wall mesh also with a dry upper layer, wet/dry reading), the
 * force-model pieces, features and the network's gradient.  Built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py; exits 0 when every
 * call ran and every result is finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "gks_oracle.h"

static int lattice(int n, double L, double jit, double *xy, int *tri)
{
    unsigned s = 12345u;
    for (int i = 0; i <= n; i++)
        for (int j = 0; j <= n; j++) {
            double dx = 0, dy = 0;
            if (jit > 0 && i > 0 && i < n && j > 0 && j < n) {
                s = s * 1103515245u + 12345u;
                dx = jit * L / n * (((s >> 8) & 0xffff) / 32768.0 - 1.0);
                s = s * 1103515245u + 12345u;
                dy = jit * L / n * (((s >> 8) & 0xffff) / 32768.0 - 1.0);
            }
            xy[2 * (i * (n + 1) + j)] = i * L / n + dx;
            xy[2 * (i * (n + 1) + j) + 1] = j * L / n + dy;
        }
    int t = 0;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            int a = i * (n + 1) + j, b = (i + 1) * (n + 1) + j, c = (i + 1) * (n + 1) + j + 1, d = i * (n + 1) + j + 1;
            tri[3 * t] = a; tri[3 * t + 1] = b; tri[3 * t + 2] = c; t++;
            tri[3 * t] = a; tri[3 * t + 1] = c; tri[3 * t + 2] = d; t++;
        }
    return t;
}

static int finite_all(const double *v, long n)
{
    for (long i = 0; i < n; i++)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static int run(int periodic, int wetdry)
{
    const int n = 8;
    const double L = periodic ? 2.0 : 1.0;
    int nn = (n + 1) * (n + 1);
    double *xy = malloc(sizeof(double) * 2 * nn), *B = malloc(sizeof(double) * nn);
    int *tri = malloc(sizeof(int) * 6 * n * n);
    int nt = lattice(n, L, periodic ? 0.0 : 0.25, xy, tri);
    for (int i = 0; i < nn; i++) {
        double x = xy[2 * i] - 0.5 * L, y = xy[2 * i + 1] - 0.5 * L;
        B[i] = periodic ? 0.0 : 0.3 * exp(-20 * (x * x + y * y));
    }
    om_mesh *m = om_mesh_new(xy, nn, tri, nt, B, periodic, L, L);
    if (!m) return 1;
    double *W = calloc(6 * nt, sizeof(double)), *gW = calloc(12 * nt, sizeof(double));
    double *W2 = calloc(6 * nt, sizeof(double)), *gW2 = calloc(12 * nt, sizeof(double));
    double *area = malloc(sizeof(double) * nt), *cx = malloc(sizeof(double) * nt), *cy = malloc(sizeof(double) * nt);
    om_cell_geometry(m, area, cx, cy);
    for (int c = 0; c < nt; c++) {
        W[c] = wetdry ? (cx[c] < 0.5 * L ? 0.2 : 0.0) : 0.2 + (cx[c] < 0.5 * L ? 0.05 : 0.0);
        W[3 * nt + c] = 0.8 + 0.02 * sin(3 * cx[c]);
        W[4 * nt + c] = 0.01 * cos(2 * cy[c]);
    }
    /* both alpha modes, both layer-coupling orders and both gradient-update readings: the
     * periodic run takes the paper's constants and the higher-order coupling, the wall run the
     * discontinuous interface values */
    om_params p = {9.81, 0.95, 0.3, 0.05, 5.0, 0, 0, periodic ? 1 : 0, periodic ? 4 : 2, periodic ? 0 : 1,
                   wetdry ? 1e-6 : 0.0};
    for (int k = 0; k < 3; k++) {
        double dt = om_dt(m, &p, W);
        om_step(m, &p, dt, 2, W, gW, W2, gW2);
        double *t = W; W = W2; W2 = t;
        t = gW; gW = gW2; gW2 = t;
    }
    int ok = finite_all(W, 6 * nt) && finite_all(gW, 12 * nt);
    double mass[2];
    om_mass(m, W, mass);
    double hk[3] = {0.1, 0.2, 0.4}, g2[2];
    om_plane_gradient(m, 0, hk, g2);
    double val[36], grad[72], r0[6];
    om_reconstruct_cell(m, nt / 2, W, gW, 0, 9.81, val, grad, r0);
    double side[11] = {0.7, 0.2, -0.1, 0.05, -0.02, 0.01, 0.03, -0.04, 0.02, -0.3, 0.1}, st[3];
    om_side_rate(side, 9.81, st);
    double corr[8];
    om_coupling_correction(m, nt / 2, W, gW, 0, 9.81, corr);
    double *X = calloc((size_t)44 * nt, sizeof(double));
    om_features(m, 9.81, W, gW, X);
    double *P = calloc(7105, sizeof(double)), *gr = calloc(7105, sizeof(double)), *y = calloc(nt, sizeof(double)),
           *z = calloc(nt, sizeof(double));
    for (int i = 0; i < 7105; i++) P[i] = 0.01 * sin(i);
    double loss = om_mlp_grad(P, X, y, nt, gr);
    om_mlp_forward(P, X, nt, z);
    om_mlp_forward_bf16(P, X, nt, z);
    /* with a dry layer the indicator's features (scaled by the thickness) and the higher-order
     * coupling are not defined (the library rejects them with wet/dry layers): run, not checked */
    ok = ok && isfinite(mass[0]) && isfinite(mass[1]) &&
         (wetdry || (isfinite(loss) && finite_all(X, 44L * nt) && finite_all(gr, 7105) && finite_all(val, 36) &&
                     finite_all(g2, 2) && finite_all(corr, 8) && finite_all(st, 3)));
    om_mesh_free(m);
    free(xy); free(B); free(tri); free(W); free(gW); free(W2); free(gW2); free(area); free(cx); free(cy);
    free(X); free(P); free(gr); free(y); free(z);
    return ok ? 0 : 2;
}

int main(void)
{
    int r = run(1, 0);
    if (r == 0) r = run(0, 0);
    if (r == 0) r = run(0, 1);
    printf("oracle driver: %s\n", r == 0 ? "ok" : "failed");
    return r;
}
