// C ABI of the GKS library: mesh / state lifetime, stage orchestration, host <-> device copies.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gks.h"
#include "gks_kernels.h"
#include "mesh_setup.h"

#ifndef GKS_RECON_STAGE_M
#define GKS_RECON_STAGE_M false
#endif

namespace {

thread_local std::string g_err;

gks_status fail(gks_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

#define HIP_OK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(GKS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
hipError_t upload(const std::vector<T> &h, T **d, std::vector<void *> &owned)
{
    size_t n = std::max<size_t>(h.size(), 1);
    hipError_t e = hipMalloc((void **)d, n * sizeof(T));
    if (e != hipSuccess) return e;
    owned.push_back(*d);
    if (!h.empty()) e = hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

struct gks_mesh {
    gks::MeshDev d{};
    std::vector<void *> owned;
    std::vector<double> Bbar, gB, area;  // host copies for state conversion
    int device = 0;
};

struct gks_state {
    const gks_mesh *mesh = nullptr;
    gks::Phys p{};
    hipStream_t stream = nullptr;
    double *Wa = nullptr, *gWa = nullptr, *Wb = nullptr, *gWb = nullptr;
    double *Wc = nullptr, *Gc = nullptr, *rec = nullptr, *r0 = nullptr, *hmid = nullptr, *gP1 = nullptr;
    double *eo = nullptr, *scal = nullptr, *part = nullptr;
    int nparts = 0;
    int half = 0;  // 1 between stage 0 and stage 1: the latest state is W^{n+1/2} (Wb)
    std::vector<void *> owned;
    // optional kernel timing: an event pair around every launch, per kernel class
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct Rec {
        int kernel;
        hipEvent_t a, b;
    };
    std::vector<Rec> prof;
};

namespace {

hipEvent_t next_event(gks_state *s)
{
    if (s->ev_used == s->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        s->ev_pool.push_back(e);
    }
    return s->ev_pool[s->ev_used++];
}

// runs launch() on the state's stream, bracketed by events when profiling is on
template <typename F>
void timed(gks_state *s, int kernel, F &&launch)
{
    if (!s->prof_on) {
        launch();
        return;
    }
    hipEvent_t a = next_event(s), b = next_event(s);
    if (a && b) (void)hipEventRecord(a, s->stream);
    launch();
    if (a && b) {
        (void)hipEventRecord(b, s->stream);
        s->prof.push_back({kernel, a, b});
    }
}

}  // namespace

extern "C" {

const char *gks_last_error(void) { return g_err.c_str(); }

gks_status gks_mesh_create(const double *node_xy, int64_t n_nodes, const int32_t *tri, int64_t n_tri,
                           const double *node_B, int32_t bc, const double *periodic_L, gks_mesh **out)
{
    if (!out || !node_xy || !tri || n_nodes <= 0 || n_tri <= 0) return fail(GKS_EINVAL, "bad mesh arguments");
    if (bc != GKS_BC_WALL && bc != GKS_BC_PERIODIC) return fail(GKS_EINVAL, "unknown boundary kind");
    if (n_tri > (int64_t)1 << 29) return fail(GKS_EINVAL, "mesh too large for 32-bit cell indices");
    *out = nullptr;
    gks::HostMesh hm;
    std::string err;
    if (gks::build_host_mesh(node_xy, n_nodes, tri, n_tri, node_B, bc, periodic_L, hm, err) != 0)
        return fail(GKS_EMESH, err);
    gks_mesh *m = new gks_mesh();
    HIP_OK(hipGetDevice(&m->device));
    gks::MeshDev &d = m->d;
    d.T = hm.nt;
    d.E = hm.ne;
    d.NG = hm.ng;
    d.dxmin = hm.dxmin;
    std::vector<void *> &o = m->owned;
    hipError_t e = hipSuccess;
#define UP(field, vec)                                                \
    if (e == hipSuccess) {                                            \
        e = upload(hm.vec, const_cast<std::remove_const_t<std::remove_pointer_t<decltype(d.field)>> **>(&d.field), o); \
    }
    UP(area, area) UP(hs, hs) UP(vtx, vtx) UP(nbc, nbc) UP(fl, fl) UP(gg, gg) UP(Bbar, Bbar) UP(gB, gB)
    UP(M, M) UP(cedge, cedge) UP(sten, sten) UP(eL, eL) UP(eR, eR) UP(eslot, eslot) UP(en, en)
    UP(eBgp, eBgp) UP(egB, egB) UP(gsrc, gsrc) UP(gR, gR)
#undef UP
    if (e != hipSuccess) {
        gks_mesh_destroy(m);
        return fail(GKS_ENOMEM, std::string("mesh upload: ") + hipGetErrorString(e));
    }
    m->Bbar = hm.Bbar;
    m->gB = hm.gB;
    m->area = hm.area;
    *out = m;
    return GKS_OK;
}

void gks_mesh_destroy(gks_mesh *m)
{
    if (!m) return;
    for (void *p : m->owned) (void)hipFree(p);
    delete m;
}

gks_status gks_mesh_info(const gks_mesh *m, int64_t *n_tri, int64_t *n_edges, int64_t *n_ghost)
{
    if (!m) return fail(GKS_EINVAL, "null mesh");
    if (n_tri) *n_tri = m->d.T;
    if (n_edges) *n_edges = m->d.E;
    if (n_ghost) *n_ghost = m->d.NG;
    return GKS_OK;
}

gks_status gks_state_init(const gks_mesh *mesh, const gks_params *prm, const double *W0, const double *gradW0,
                          void *stream, gks_state **out)
{
    if (!mesh || !prm || !W0 || !gradW0 || !out) return fail(GKS_EINVAL, "null argument");
    if (prm->precision != GKS_FP64) return fail(GKS_EUNSUPPORTED, "only GKS_FP64 in this build");
    if (!(prm->G > 0) || !(prm->cfl > 0) || !(prm->chi > 0) || !(prm->eps > 0) || !(prm->eps_num >= 0))
        return fail(GKS_EINVAL, "bad physical parameters");
    *out = nullptr;
    const int64_t T = mesh->d.T, TG = T + mesh->d.NG, E = mesh->d.E;
    // host conversion: the device state carries eta1 = h1 + B and grad(eta1)
    std::vector<double> w(6 * TG, 0.0), g(12 * TG, 0.0);
    for (int v = 0; v < 6; v++)
        for (int64_t c = 0; c < T; c++) {
            double x = W0[v * T + c];
            if (!std::isfinite(x) || ((v == 0 || v == 3) && !(x > 0)))
                return fail(GKS_ENONFINITE, "bad initial value at component " + std::to_string(v) + ", cell " +
                                                std::to_string(c));
            w[v * TG + c] = v == 3 ? x + mesh->Bbar[c] : x;
            for (int d = 0; d < 2; d++) {
                double y = gradW0[(2 * v + d) * T + c];
                if (!std::isfinite(y)) return fail(GKS_ENONFINITE, "non-finite initial gradient");
                g[(2 * v + d) * TG + c] = v == 3 ? y + mesh->gB[d * T + c] : y;
            }
        }
    gks_state *s = new gks_state();
    s->mesh = mesh;
    s->p.G = prm->G;
    s->p.chi = prm->chi;
    s->p.eps = prm->eps;
    s->p.eps_num = prm->eps_num;
    s->p.cfl = prm->cfl;
    s->p.t_end = prm->t_end > 0 ? prm->t_end : 1e300;
    s->p.linear = prm->linear;
    s->stream = (hipStream_t)stream;
    s->nparts = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (T + gks::DT_BLOCK - 1) / gks::DT_BLOCK));
    struct Buf {
        double **p;
        size_t n;
    } bufs[] = {{&s->Wa, 6 * (size_t)TG}, {&s->gWa, 12 * (size_t)TG}, {&s->Wb, 6 * (size_t)TG},
                {&s->gWb, 12 * (size_t)TG}, {&s->Wc, 6 * (size_t)T}, {&s->Gc, 12 * (size_t)T},
                {&s->rec, 108 * (size_t)T}, {&s->r0, 2 * (size_t)T}, {&s->hmid, 2 * (size_t)E},
                {&s->gP1, 4 * (size_t)T}, {&s->eo, 24 * (size_t)E}, {&s->scal, 2},
                {&s->part, 2 * (size_t)std::max(s->nparts, 1024)}};
    for (auto &b : bufs) {
        hipError_t e = hipMalloc((void **)b.p, b.n * sizeof(double));
        if (e != hipSuccess) {
            gks_state_destroy(s);
            return fail(GKS_ENOMEM, std::string("state allocation: ") + hipGetErrorString(e));
        }
        s->owned.push_back(*b.p);
    }
    double scal0[2] = {0.0, 0.0};
    HIP_OK(hipMemcpy(s->Wa, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(s->gWa, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(s->scal, scal0, sizeof(scal0), hipMemcpyHostToDevice));
    HIP_OK(hipMemset(s->Wb, 0, 6 * (size_t)TG * sizeof(double)));
    HIP_OK(hipMemset(s->gWb, 0, 12 * (size_t)TG * sizeof(double)));
    *out = s;
    return GKS_OK;
}

void gks_state_destroy(gks_state *s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    for (void *p : s->owned) (void)hipFree(p);
    delete s;
}

gks_status gks_profile(gks_state *s, int32_t enable)
{
    if (!s) return fail(GKS_EINVAL, "null state");
    HIP_OK(hipStreamSynchronize(s->stream));
    s->prof.clear();
    s->ev_used = 0;
    s->prof_on = enable != 0;
    return GKS_OK;
}

gks_status gks_profile_read(gks_state *s, int32_t kernel, double *total_ms, int64_t *launches)
{
    if (!s || kernel < 0 || kernel >= GKS_KERNEL_COUNT) return fail(GKS_EINVAL, "bad profile query");
    HIP_OK(hipStreamSynchronize(s->stream));
    double tot = 0;
    int64_t n = 0;
    for (const auto &r : s->prof)
        if (r.kernel == kernel) {
            float ms = 0;
            HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
            tot += ms;
            n++;
        }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = n;
    return GKS_OK;
}

static gks_status run_stage(gks_state *s, int stage)
{
    const gks::MeshDev &m = s->mesh->d;
    hipStream_t st = s->stream;
    double *Win = stage == 0 ? s->Wa : s->Wb, *gWin = stage == 0 ? s->gWa : s->gWb;
    double *Wout = stage == 0 ? s->Wb : s->Wa, *gWout = stage == 0 ? s->gWb : s->gWa;
    if (m.NG > 0)
        timed(s, GKS_KERNEL_GHOST, [&] {
            hipLaunchKernelGGL(gks::k_ghost_fill, dim3(blocks(m.NG, 256)), dim3(256), 0, st, m, Win, gWin);
        });
    timed(s, GKS_KERNEL_RECON, [&] {
        hipLaunchKernelGGL(gks::k_recon<GKS_RECON_STAGE_M>, dim3(blocks(m.T, gks::RECON_CELLS)), dim3(192), 0, st,
                           m, s->p, Win, gWin, s->rec, s->r0);
    });
    timed(s, GKS_KERNEL_HHAT, [&] {
        hipLaunchKernelGGL(gks::k_hhat, dim3(blocks(m.E, 256)), dim3(256), 0, st, m, s->p, s->rec, s->hmid);
    });
    timed(s, GKS_KERNEL_PLANE, [&] {
        hipLaunchKernelGGL(gks::k_plane, dim3(blocks(m.T, 256)), dim3(256), 0, st, m, s->hmid, s->gP1);
    });
    timed(s, GKS_KERNEL_FLUX, [&] {
        hipLaunchKernelGGL(gks::k_flux, dim3(blocks(4 * m.E, 256)), dim3(256), 0, st, m, s->p, s->scal, s->rec,
                           s->r0, s->gP1, s->eo);
    });
    timed(s, GKS_KERNEL_UPDATE, [&] {
        hipLaunchKernelGGL(gks::k_update, dim3(blocks(m.T, 256)), dim3(256), 0, st, m, s->p, stage, s->scal,
                           s->eo, Win, Wout, gWout, s->Wc, s->Gc);
    });
    HIP_OK(hipGetLastError());
    s->half = stage == 0;
    return GKS_OK;
}

static gks_status compute_dt(gks_state *s)
{
    const gks::MeshDev &m = s->mesh->d;
    timed(s, GKS_KERNEL_DT, [&] {
        hipLaunchKernelGGL(gks::k_dt_partial, dim3(s->nparts), dim3(gks::DT_BLOCK), 0, s->stream, m, s->p, s->Wa,
                           s->part);
        hipLaunchKernelGGL(gks::k_dt_final, dim3(1), dim3(gks::DT_BLOCK), 0, s->stream, m, s->p, s->part,
                           s->nparts, s->scal);
    });
    HIP_OK(hipGetLastError());
    return GKS_OK;
}

gks_status gks_stage(gks_state *s, int32_t stage, const double *dt)
{
    if (!s || (stage != 0 && stage != 1)) return fail(GKS_EINVAL, "bad stage arguments");
    if (stage == 1 && !s->half) return fail(GKS_EINVAL, "stage 1 must follow stage 0");
    if (stage == 0 && s->half) return fail(GKS_EINVAL, "stage 0 must follow stage 1");
    if (stage == 0) {
        if (dt) {
            if (!(*dt > 0) || !std::isfinite(*dt)) return fail(GKS_EINVAL, "dt must be positive");
            hipLaunchKernelGGL(gks::k_set_dt, dim3(1), dim3(1), 0, s->stream, s->scal, *dt);
            HIP_OK(hipGetLastError());
        } else {
            gks_status r = compute_dt(s);
            if (r != GKS_OK) return r;
        }
    } else if (dt) {
        return fail(GKS_EINVAL, "stage 1 reuses the step size of stage 0");
    }
    return run_stage(s, stage);
}

gks_status gks_step(gks_state *s, int32_t n_steps, double *dt_last)
{
    if (!s || n_steps < 0) return fail(GKS_EINVAL, "bad step arguments");
    if (s->half) return fail(GKS_EINVAL, "a step cannot start between stage 0 and stage 1");
    for (int i = 0; i < n_steps; i++) {
        gks_status r = compute_dt(s);
        if (r == GKS_OK) r = run_stage(s, 0);
        if (r == GKS_OK) r = run_stage(s, 1);
        if (r != GKS_OK) return r;
    }
    if (dt_last) {
        double sc[2];
        HIP_OK(hipMemcpyAsync(sc, s->scal, sizeof(sc), hipMemcpyDeviceToHost, s->stream));
        HIP_OK(hipStreamSynchronize(s->stream));
        *dt_last = sc[0];
    }
    return GKS_OK;
}

gks_status gks_state_read(const gks_state *s, double *W, double *gradW, double *t)
{
    if (!s) return fail(GKS_EINVAL, "null state");
    const gks_mesh *mesh = s->mesh;
    const int64_t T = mesh->d.T, TG = T + mesh->d.NG;
    const double *Wsrc = s->half ? s->Wb : s->Wa, *gWsrc = s->half ? s->gWb : s->gWa;
    HIP_OK(hipStreamSynchronize(s->stream));
    if (W) {
        std::vector<double> w(6 * TG);
        HIP_OK(hipMemcpy(w.data(), Wsrc, w.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int v = 0; v < 6; v++)
            for (int64_t c = 0; c < T; c++) W[v * T + c] = v == 3 ? w[v * TG + c] - mesh->Bbar[c] : w[v * TG + c];
    }
    if (gradW) {
        std::vector<double> g(12 * TG);
        HIP_OK(hipMemcpy(g.data(), gWsrc, g.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int v = 0; v < 6; v++)
            for (int d = 0; d < 2; d++)
                for (int64_t c = 0; c < T; c++)
                    gradW[(2 * v + d) * T + c] =
                        v == 3 ? g[(2 * v + d) * TG + c] - mesh->gB[d * T + c] : g[(2 * v + d) * TG + c];
    }
    if (t) {
        double sc[2];
        HIP_OK(hipMemcpy(sc, s->scal, sizeof(sc), hipMemcpyDeviceToHost));
        *t = s->half ? sc[1] - 0.5 * sc[0] : sc[1];
    }
    return GKS_OK;
}

gks_status gks_state_mass(const gks_state *s, double mass[2])
{
    if (!s || !mass) return fail(GKS_EINVAL, "null argument");
    const gks::MeshDev &m = s->mesh->d;
    const int nb = 256;
    hipLaunchKernelGGL(gks::k_mass_partial, dim3(nb), dim3(256), 0, s->stream, m, s->half ? s->Wb : s->Wa,
                       s->part);
    HIP_OK(hipGetLastError());
    std::vector<double> part(2 * nb);
    HIP_OK(hipMemcpyAsync(part.data(), s->part, part.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_OK(hipStreamSynchronize(s->stream));
    mass[0] = mass[1] = 0;
    for (int b = 0; b < nb; b++) {
        mass[0] += part[2 * b];
        mass[1] += part[2 * b + 1];
    }
    return GKS_OK;
}

}  // extern "C"
