// Sanitizer driver for the library's host mesh setup (least-squares operators, stencils, ghosts,
// batch concatenation): wall and periodic lattices, then a batch of both.  Built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py (host code only).
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "mesh_setup.h"

static void lattice(int n, double L, double jit, std::vector<double> &xy, std::vector<int32_t> &tri)
{
    unsigned s = 777u;
    xy.clear();
    tri.clear();
    for (int i = 0; i <= n; i++)
        for (int j = 0; j <= n; j++) {
            double dx = 0, dy = 0;
            if (jit > 0 && i > 0 && i < n && j > 0 && j < n) {
                s = s * 1103515245u + 12345u;
                dx = jit * L / n * (((s >> 8) & 0xffff) / 32768.0 - 1.0);
                s = s * 1103515245u + 12345u;
                dy = jit * L / n * (((s >> 8) & 0xffff) / 32768.0 - 1.0);
            }
            xy.push_back(i * L / n + dx);
            xy.push_back(j * L / n + dy);
        }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            int a = i * (n + 1) + j, b = (i + 1) * (n + 1) + j, c = (i + 1) * (n + 1) + j + 1, d = i * (n + 1) + j + 1;
            tri.insert(tri.end(), {a, b, c, a, c, d});
        }
}

int main()
{
    std::vector<double> xy, B;
    std::vector<int32_t> tri;
    gks::HostMesh wall, per;
    std::string err;
    lattice(12, 1.0, 0.25, xy, tri);
    B.assign(xy.size() / 2, 0.0);
    for (size_t i = 0; i < B.size(); i++) B[i] = 0.2 * std::exp(-30 * ((xy[2 * i] - 0.5) * (xy[2 * i] - 0.5)));
    if (gks::build_host_mesh(xy.data(), (int64_t)B.size(), tri.data(), (int64_t)tri.size() / 3, B.data(), 0, nullptr,
                             wall, err) != 0) {
        std::printf("wall mesh: %s\n", err.c_str());
        return 1;
    }
    lattice(6, 2.0, 0.0, xy, tri);
    const double L[2] = {2.0, 2.0};
    if (gks::build_host_mesh(xy.data(), (int64_t)xy.size() / 2, tri.data(), (int64_t)tri.size() / 3, nullptr, 1, L,
                             per, err) != 0) {
        std::printf("periodic mesh: %s\n", err.c_str());
        return 1;
    }
    gks::HostMesh both = gks::concat_host_meshes({&wall, &per});
    double s = 0;
    for (double v : both.M) s += std::fabs(v);
    const bool ok = std::isfinite(s) && both.nt == wall.nt + per.nt && both.ng == wall.ng + per.ng;
    std::printf("mesh driver: %s (%lld cells, %lld ghosts)\n", ok ? "ok" : "failed", (long long)both.nt,
                (long long)both.ng);
    return ok ? 0 : 2;
}
