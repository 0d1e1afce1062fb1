// C ABI of the GKS library: mesh / state lifetime, stage orchestration, batched stepping with HIP
// graphs, host <-> device copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/gks.h"
#include "gks_indicator.h"
#include "gks_kernels.h"
#include "mesh_setup.h"

namespace {

thread_local std::string g_err;

gks_status fail(gks_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

// the body of an entry point: C++ exceptions (a failed host allocation) become status codes and
// never cross the C boundary
template <typename F>
gks_status guarded(F &&body)
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(GKS_ENOMEM, "host allocation failed");
    } catch (const std::exception &x) {
        return fail(GKS_EDEVICE, std::string("internal error: ") + x.what());
    }
}

#define HIP_OK(expr)                                                                                      \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) return fail(GKS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
hipError_t upload(const std::vector<T> &h, const T **d, std::vector<void *> &owned)
{
    size_t n = std::max<size_t>(h.size(), 1);
    T *p = nullptr;
    hipError_t e = hipMalloc((void **)&p, n * sizeof(T));
    if (e != hipSuccess) return e;
    owned.push_back(p);
    *d = p;
    if (!h.empty()) e = hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

hipError_t upload_f32(const std::vector<double> &h, const void **d, std::vector<void *> &owned)
{
    std::vector<float> f(h.begin(), h.end());
    const float *p = nullptr;
    hipError_t e = upload(f, &p, owned);
    *d = p;
    return e;
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

constexpr int64_t DT_CHUNK = 4096;  // cells per block of the batched time step

// bytes of the head and of the tail of one Gauss-point record
size_t head_bytes(int prec) { return prec == GKS_FP64 ? sizeof(gks::GpHead<double>) : sizeof(gks::GpHead<float>); }
size_t rec_bytes(int prec)
{
    return head_bytes(prec) + (prec == GKS_FP64 ? sizeof(gks::GpTail<double>) : sizeof(gks::GpTail<float>));
}

// the two record arrays inside one allocation of 6 T records: heads, then tails
template <typename R>
gks::GpRecs<R> recs_of(void *base, int64_t T)
{
    gks::GpHead<R> *h = static_cast<gks::GpHead<R> *>(base);
    return {h, reinterpret_cast<gks::GpTail<R> *>(h + 6 * T)};
}

}  // namespace

struct gks_mesh {
    gks::HostMesh host;             // kept for concatenation into batches and for state conversion
    gks::MeshDev d64{}, d32{};      // device tables; bulk tables as double / as float
    bool has32 = false;
    std::vector<void *> owned;
    int device = 0;
};

struct gks_state {
    const gks_mesh *mesh = nullptr;
    int prec = GKS_FP64;
    gks::MeshDev md{};
    gks::Phys p{};
    hipStream_t stream = nullptr;
    double *Wh[2] = {nullptr, nullptr};
    void *Wm[2] = {nullptr, nullptr}, *gW[2] = {nullptr, nullptr};
    double *Wc = nullptr, *hmid = nullptr, *gP1 = nullptr;
    double *eoh = nullptr;
    void *Gc = nullptr, *rec = nullptr, *r0 = nullptr, *eom = nullptr;  // rec: GpRec[6T]
    double *scal = nullptr, *part = nullptr, *chi = nullptr, *tend = nullptr;
    uint8_t *smooth = nullptr;  // skip mask of the reconstruction (learned indicator)
    uint8_t *need = nullptr;    // cells whose plane gradient of the force model is used
    unsigned long long *bad = nullptr;  // first cell updated to a non-finite / non-positive state
    bool src4 = false;          // higher-order layer coupling
    bool gm1 = false;           // discontinuous interface values in the gradient update
    void *src = nullptr;        // its interior correction [8][T] (real), written by the reconstruction
    // threads per block of the edge and cell kernels (per kernel class), chosen by gks_autotune
    int bs[GKS_KERNEL_COUNT] = {256, 192, 256, 256, 256, 256, 256, 256};
    int nparts = 0;
    // learned indicator: parameters, bf16 copies of the weight matrices, threshold
    bool ind_on = false;
    float ind_thr = 0;
    float *ind_P = nullptr, *ind_logit = nullptr;
    short *ind_W1b = nullptr, *ind_W2b = nullptr;
    // second reconstruction (linear) for labels
    void *lab_rec = nullptr, *lab_r0 = nullptr;
    uint8_t *lab_y = nullptr;
    int half = 0;  // 1 between stage 0 and stage 1: the latest state is W^{n+1/2}
    std::vector<void *> owned;
    // graph of one full step, replayed by gks_batch_step
    hipStream_t gstream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};
    bool capturing = false;
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

// runs launch() on stream st, bracketed by events when profiling is on (never inside a capture)
template <typename F>
void timed(gks_state *s, hipStream_t st, int kernel, F &&launch)
{
    if (!s->prof_on || s->capturing) {
        launch();
        return;
    }
    hipEvent_t a = next_event(s), b = next_event(s);
    if (a && b) (void)hipEventRecord(a, st);
    launch();
    if (a && b) {
        (void)hipEventRecord(b, st);
        s->prof.push_back({kernel, a, b});
    }
}

template <typename R, int SRC>
void launch_recon(gks_state *s, int stage, hipStream_t st, const double *Whin, const R *Wmin, const R *gWin)
{
    const gks::MeshDev &m = s->md;
    const dim3 g(blocks(m.T, gks::RECON_CELLS)), t(192);
    R *src = SRC ? (R *)s->src : nullptr;
    if (s->ind_on) {
        const gks::IndArgs ia{s->ind_W1b, s->ind_W2b, s->ind_P, s->ind_thr, s->smooth};
        if (stage == 1)  // the second stage reuses the decisions of the step's first stage
            hipLaunchKernelGGL((gks::k_recon<R, 2, SRC>), g, t, 0, st, m, s->p, Whin, Wmin, gWin, ia,
                               recs_of<R>(s->rec, m.T), (R *)s->r0, src);
        else
            hipLaunchKernelGGL((gks::k_recon<R, 1, SRC>), g, t, 0, st, m, s->p, Whin, Wmin, gWin, ia,
                               recs_of<R>(s->rec, m.T), (R *)s->r0, src);
    } else
        hipLaunchKernelGGL((gks::k_recon<R, 0, SRC>), g, t, 0, st, m, s->p, Whin, Wmin, gWin, gks::IndArgs{},
                           recs_of<R>(s->rec, m.T), (R *)s->r0, src);
}

template <typename R, int AM, int STAGE, int GM>
void launch_flux_gm(gks_state *s, hipStream_t st)
{
    const gks::MeshDev &m = s->md;
    const int b = s->bs[GKS_KERNEL_FLUX];
    if (s->p.h_dry > 0)
        hipLaunchKernelGGL((gks::k_flux<R, AM, STAGE, GM, 1>), dim3(blocks(4 * m.E, b)), dim3(b), 0, st, m, s->p,
                           recs_of<R>(s->rec, m.T), (const R *)s->r0, s->gP1, s->eoh, (R *)s->eom);
    else
        hipLaunchKernelGGL((gks::k_flux<R, AM, STAGE, GM, 0>), dim3(blocks(4 * m.E, b)), dim3(b), 0, st, m, s->p,
                           recs_of<R>(s->rec, m.T), (const R *)s->r0, s->gP1, s->eoh, (R *)s->eom);
}

template <typename R, int AM, int STAGE>
void launch_flux(gks_state *s, hipStream_t st)
{
    if (s->gm1)
        launch_flux_gm<R, AM, STAGE, 1>(s, st);
    else
        launch_flux_gm<R, AM, STAGE, 0>(s, st);
}

template <typename R, int SRC, int GM>
void launch_update_gm(gks_state *s, int stage, hipStream_t st, const double *Whin, const R *Wmin, const R *gWin,
                      double *Whout, R *Wmout, R *gWout)
{
    const gks::MeshDev &m = s->md;
    const int b = s->bs[GKS_KERNEL_UPDATE];
    const R *src = SRC ? (const R *)s->src : nullptr;
    if (stage == 0)
        hipLaunchKernelGGL((gks::k_update<R, 0, SRC, GM>), dim3(blocks(m.T, b)), dim3(b), 0, st, m, s->p, s->eoh,
                           (const R *)s->eom, Whin, Wmin, gWin, Whout, Wmout, gWout, s->Wc, (R *)s->Gc, src);
    else
        hipLaunchKernelGGL((gks::k_update<R, 1, SRC, GM>), dim3(blocks(m.T, b)), dim3(b), 0, st, m, s->p, s->eoh,
                           (const R *)s->eom, Whin, Wmin, gWin, Whout, Wmout, gWout, s->Wc, (R *)s->Gc, src);
}

template <typename R, int SRC>
void launch_update(gks_state *s, int stage, hipStream_t st, const double *Whin, const R *Wmin, const R *gWin,
                   double *Whout, R *Wmout, R *gWout)
{
    if (s->gm1)
        launch_update_gm<R, SRC, 1>(s, stage, st, Whin, Wmin, gWin, Whout, Wmout, gWout);
    else
        launch_update_gm<R, SRC, 0>(s, stage, st, Whin, Wmin, gWin, Whout, Wmout, gWout);
}

template <typename R>
void launch_stage(gks_state *s, int stage, hipStream_t st)
{
    const gks::MeshDev &m = s->md;
    const int in = stage == 0 ? 0 : 1, out = 1 - in;
    double *Whin = s->Wh[in];
    R *Wmin = (R *)s->Wm[in], *gWin = (R *)s->gW[in];
    double *Whout = s->Wh[out];
    R *Wmout = (R *)s->Wm[out], *gWout = (R *)s->gW[out];
    if (m.NG > 0)
        timed(s, st, GKS_KERNEL_GHOST, [&] {
            const int b = s->bs[GKS_KERNEL_GHOST];
            hipLaunchKernelGGL(gks::k_ghost_fill<R>, dim3(blocks(m.NG, b)), dim3(b), 0, st, m, Whin, Wmin, gWin);
        });
    timed(s, st, GKS_KERNEL_RECON, [&] {
        if (s->src4)
            launch_recon<R, 1>(s, stage, st, Whin, Wmin, gWin);
        else
            launch_recon<R, 0>(s, stage, st, Whin, Wmin, gWin);
    });
    timed(s, st, GKS_KERNEL_HHAT, [&] {
        const int b = s->bs[GKS_KERNEL_HHAT];
        hipLaunchKernelGGL(gks::k_need<R>, dim3(blocks(m.T, b)), dim3(b), 0, st, m, (const R *)s->r0, s->need);
        hipLaunchKernelGGL(gks::k_hhat<R>, dim3(blocks(m.E, b)), dim3(b), 0, st, m, s->p,
                           (const gks::GpHead<R> *)s->rec, s->need, s->hmid);
    });
    timed(s, st, GKS_KERNEL_PLANE, [&] {
        const int b = s->bs[GKS_KERNEL_PLANE];
        hipLaunchKernelGGL(gks::k_plane, dim3(blocks(m.T, b)), dim3(b), 0, st, m, s->need, s->hmid, s->gP1);
    });
    timed(s, st, GKS_KERNEL_FLUX, [&] {
        if (s->p.alpha_mode == 0) {
            if (stage == 0)
                launch_flux<R, 0, 0>(s, st);
            else
                launch_flux<R, 0, 1>(s, st);
        } else {
            if (stage == 0)
                launch_flux<R, 1, 0>(s, st);
            else
                launch_flux<R, 1, 1>(s, st);
        }
    });
    timed(s, st, GKS_KERNEL_UPDATE, [&] {
        if (s->src4)
            launch_update<R, 1>(s, stage, st, Whin, Wmin, gWin, Whout, Wmout, gWout);
        else
            launch_update<R, 0>(s, stage, st, Whin, Wmin, gWin, Whout, Wmout, gWout);
    });
}

template <typename R>
void launch_dt(gks_state *s, hipStream_t st)
{
    const gks::MeshDev &m = s->md;
    timed(s, st, GKS_KERNEL_DT, [&] {
        if (m.S == 1) {
            hipLaunchKernelGGL(gks::k_dt_partial<R>, dim3(s->nparts), dim3(gks::DT_BLOCK), 0, st, m, s->p, s->Wh[0],
                               (const R *)s->Wm[0], s->part);
            hipLaunchKernelGGL(gks::k_dt_final, dim3(1), dim3(gks::DT_BLOCK), 0, st, m, s->p, s->part, s->nparts);
        } else {
            hipLaunchKernelGGL(gks::k_dt_chunk<R>, dim3(m.NCH), dim3(gks::DT_BLOCK), 0, st, m, s->p, s->Wh[0],
                               (const R *)s->Wm[0], s->part);
            hipLaunchKernelGGL(gks::k_dt_scenario, dim3(m.S), dim3(64), 0, st, m, s->p, s->part);
        }
    });
}

void stage_any(gks_state *s, int stage, hipStream_t st)
{
    if (s->prec == GKS_FP64)
        launch_stage<double>(s, stage, st);
    else
        launch_stage<float>(s, stage, st);
}

void dt_any(gks_state *s, hipStream_t st)
{
    if (s->prec == GKS_FP64)
        launch_dt<double>(s, st);
    else
        launch_dt<float>(s, st);
}

// The least-squares operators as the reconstruction reads them: block-major, each block of
// RECON_CELLS cells holding its 153 rows of RECON_CELLS entries as one contiguous span
// ([ceil(T / RECON_CELLS)][153][RECON_CELLS], the last block padded with zeros), so that a block's
// operators stream in as one piece.  The host mesh keeps them row-major [153][T].
std::vector<double> operators_block_major(const gks::HostMesh &h)
{
    const int64_t T = h.nt, C = gks::RECON_CELLS, nb = (T + C - 1) / C;
    std::vector<double> out((size_t)(nb * 153 * C), 0.0);
    for (int64_t b = 0; b < nb; b++)
        for (int64_t j = 0; j < 153; j++)
            for (int64_t l = 0; l < C && b * C + l < T; l++) out[(size_t)((b * 153 + j) * C + l)] = h.M[(size_t)(j * T + b * C + l)];
    return out;
}

gks_status upload_mesh(gks_mesh *m)
{
    const gks::HostMesh &h = m->host;
    gks::MeshDev &d = m->d64;
    d.T = h.nt;
    d.E = h.ne;
    d.NG = h.ng;
    d.S = h.S;
    std::vector<void *> &o = m->owned;
    hipError_t e = hipSuccess;
    auto up = [&](auto &vec, auto **field) {
        if (e == hipSuccess) e = upload(vec, field, o);
    };
    up(h.area, &d.area);
    up(h.Bbar, &d.Bbar);
    up(h.gB, &d.gB);
    up(h.fl, &d.fl);
    up(h.gg, &d.gg);
    up(h.eBgp, &d.eBgp);
    up(h.gR, &d.gR);
    up(h.sdxmin, &d.sdxmin);
    up(h.cedge, &d.cedge);
    up(h.sten, &d.sten);
    up(h.eL, &d.eL);
    up(h.eR, &d.eR);
    up(h.eslot, &d.eslot);
    up(h.gsrc, &d.gsrc);
    up(h.scell, &d.scell);
    up(h.cand, &d.cand);
    const double *M = nullptr, *hs = nullptr, *vtx = nullptr, *nbc = nullptr, *en = nullptr, *egB = nullptr;
    {
        const std::vector<double> Mb = operators_block_major(h);
        up(Mb, &M);
    }
    up(h.hs, &hs);
    up(h.vtx, &vtx);
    up(h.nbc, &nbc);
    up(h.en, &en);
    up(h.egB, &egB);
    d.M = M;
    d.hs = hs;
    d.vtx = vtx;
    d.nbc = nbc;
    d.en = en;
    d.egB = egB;
    {
        const void *ig = nullptr;
        if (e == hipSuccess) e = upload_f32(h.igeo, &ig, o);
        d.igeo = static_cast<const float *>(ig);
    }
    if (h.S > 1) {
        up(h.cscen, &d.cscen);
        up(h.escen, &d.escen);
        // time-step chunks: at most DT_CHUNK cells, never across a scenario boundary
        std::vector<int64_t> cb{0};
        std::vector<int32_t> sc0{0};
        for (int32_t sn = 0; sn < h.S; sn++) {
            for (int64_t c = h.scell[sn] + DT_CHUNK; c < h.scell[sn + 1]; c += DT_CHUNK) cb.push_back(c);
            cb.push_back(h.scell[sn + 1]);
            sc0.push_back((int32_t)cb.size() - 1);
        }
        d.NCH = (int32_t)cb.size() - 1;
        up(cb, &d.cb);
        up(sc0, &d.sc0);
    } else {
        d.cscen = d.escen = nullptr;
        d.cb = nullptr;
        d.sc0 = nullptr;
        d.NCH = 0;
    }
    if (e != hipSuccess) return fail(GKS_ENOMEM, std::string("mesh upload: ") + hipGetErrorString(e));
    m->d32 = d;
    return GKS_OK;
}

gks_status ensure_f32(gks_mesh *m)
{
    if (m->has32) return GKS_OK;
    const gks::HostMesh &h = m->host;
    gks::MeshDev &d = m->d32;
    hipError_t e = hipSuccess;
    std::vector<void *> &o = m->owned;
    if (e == hipSuccess) e = upload_f32(operators_block_major(h), &d.M, o);
    if (e == hipSuccess) e = upload_f32(h.hs, &d.hs, o);
    if (e == hipSuccess) e = upload_f32(h.vtx, &d.vtx, o);
    if (e == hipSuccess) e = upload_f32(h.nbc, &d.nbc, o);
    if (e == hipSuccess) e = upload_f32(h.en, &d.en, o);
    if (e == hipSuccess) e = upload_f32(h.egB, &d.egB, o);
    if (e != hipSuccess) return fail(GKS_ENOMEM, std::string("mesh upload: ") + hipGetErrorString(e));
    m->has32 = true;
    return GKS_OK;
}

// checkpoint: a fixed header, then the raw device state (levels and thicknesses in FP64, momenta
// and gradients in the state's precision, ghosts included), the per-scenario (dt, t) pairs and
// the non-finite flag
struct CkptHeader {
    uint32_t magic, version;
    int32_t prec, S;
    int64_t T, NG;
};
constexpr uint32_t CKPT_MAGIC = 0x474b5331u;  // "GKS1"

int64_t ckpt_bytes(const gks_state *s)
{
    const gks::HostMesh &h = s->mesh->host;
    const int64_t TG = h.nt + h.ng, rs = s->prec == GKS_FP64 ? 8 : 4;
    return (int64_t)sizeof(CkptHeader) + 2 * TG * 8 + 16 * TG * rs + 2 * (int64_t)h.S * 8 + 8;
}

// the non-finite flag of a state whose stream has been synchronised: GKS_ENONFINITE naming the
// first bad cell, or GKS_OK
gks_status check_bad(const gks_state *s, int64_t *first)
{
    unsigned long long v = ~0ull;
    HIP_OK(hipMemcpy(&v, s->bad, 8, hipMemcpyDeviceToHost));
    if (first) *first = v == ~0ull ? -1 : (int64_t)v;
    if (v == ~0ull) return GKS_OK;
    return fail(GKS_ENONFINITE, "non-finite value or non-positive layer thickness after an update, first at cell " +
                                    std::to_string(v));
}

template <typename R>
void to_real(const std::vector<double> &src, std::vector<unsigned char> &dst)
{
    dst.resize(src.size() * sizeof(R));
    R *p = reinterpret_cast<R *>(dst.data());
    for (size_t i = 0; i < src.size(); i++) p[i] = (R)src[i];
}

template <typename R>
void from_real(const std::vector<unsigned char> &src, std::vector<double> &dst)
{
    const R *p = reinterpret_cast<const R *>(src.data());
    dst.resize(src.size() / sizeof(R));
    for (size_t i = 0; i < dst.size(); i++) dst[i] = (double)p[i];
}

}  // namespace

extern "C" {

const char *gks_last_error(void) { return g_err.c_str(); }

gks_status gks_mesh_create(const double *node_xy, int64_t n_nodes, const int32_t *tri, int64_t n_tri,
                           const double *node_B, int32_t bc, const double *periodic_L, gks_mesh **out)
{
    return guarded([&]() -> gks_status {
        if (!out || !node_xy || !tri || n_nodes <= 0 || n_tri <= 0) return fail(GKS_EINVAL, "bad mesh arguments");
        if (bc != GKS_BC_WALL && bc != GKS_BC_PERIODIC && bc != GKS_BC_FREE)
            return fail(GKS_EINVAL, "unknown boundary kind");
        if (n_tri > (int64_t)1 << 29) return fail(GKS_EINVAL, "mesh too large for 32-bit cell indices");
        *out = nullptr;
        gks_mesh *m = new gks_mesh();
        std::string err;
        if (gks::build_host_mesh(node_xy, n_nodes, tri, n_tri, node_B, bc, periodic_L, m->host, err) != 0) {
            delete m;
            return fail(GKS_EMESH, err);
        }
        if (hipGetDevice(&m->device) != hipSuccess) {
            delete m;
            return fail(GKS_EDEVICE, "no HIP device");
        }
        gks_status r = upload_mesh(m);
        if (r != GKS_OK) {
            gks_mesh_destroy(m);
            return r;
        }
        *out = m;
        return GKS_OK;
    });
}

gks_status gks_mesh_batch(const gks_mesh *const *meshes, int32_t n, gks_mesh **out)
{
    return guarded([&]() -> gks_status {
        if (!meshes || n <= 0 || !out) return fail(GKS_EINVAL, "bad batch arguments");
        *out = nullptr;
        std::vector<const gks::HostMesh *> parts;
        int64_t T = 0;
        for (int32_t i = 0; i < n; i++) {
            if (!meshes[i]) return fail(GKS_EINVAL, "null mesh in batch");
            if (meshes[i]->host.S != 1) return fail(GKS_EINVAL, "batches cannot be nested");
            parts.push_back(&meshes[i]->host);
            T += meshes[i]->host.nt + meshes[i]->host.ng;
        }
        if (T > (int64_t)1 << 30) return fail(GKS_EINVAL, "batch too large for 32-bit cell indices");
        gks_mesh *m = new gks_mesh();
        m->host = gks::concat_host_meshes(parts);
        if (hipGetDevice(&m->device) != hipSuccess) {
            delete m;
            return fail(GKS_EDEVICE, "no HIP device");
        }
        gks_status r = upload_mesh(m);
        if (r != GKS_OK) {
            gks_mesh_destroy(m);
            return r;
        }
        *out = m;
        return GKS_OK;
    });
}

void gks_mesh_destroy(gks_mesh *m)
{
    if (!m) return;
    for (void *p : m->owned) (void)hipFree(p);
    delete m;
}

gks_status gks_mesh_info(const gks_mesh *m, int64_t *n_tri, int64_t *n_edges, int64_t *n_ghost, int32_t *n_scen)
{
    return guarded([&]() -> gks_status {
        if (!m) return fail(GKS_EINVAL, "null mesh");
        if (n_tri) *n_tri = m->host.nt;
        if (n_edges) *n_edges = m->host.ne;
        if (n_ghost) *n_ghost = m->host.ng;
        if (n_scen) *n_scen = m->host.S;
        return GKS_OK;
    });
}

gks_status gks_mesh_scenario(const gks_mesh *m, int32_t s, int64_t *first_cell, int64_t *n_cells)
{
    return guarded([&]() -> gks_status {
        if (!m || s < 0 || s >= m->host.S) return fail(GKS_EINVAL, "bad scenario index");
        if (first_cell) *first_cell = m->host.scell[s];
        if (n_cells) *n_cells = m->host.scell[s + 1] - m->host.scell[s];
        return GKS_OK;
    });
}

gks_status gks_state_init(const gks_mesh *mesh_c, const gks_params *prm, const double *W0, const double *gradW0,
                          void *stream, gks_state **out)
{
    return guarded([&]() -> gks_status {
        if (!mesh_c || !prm || !W0 || !gradW0 || !out) return fail(GKS_EINVAL, "null argument");
        gks_mesh *mesh = const_cast<gks_mesh *>(mesh_c);
        const gks::HostMesh &h = mesh->host;
        const int32_t S = h.S;
        for (int32_t s = 0; s < S; s++) {
            const gks_params &q = prm[s];
            if (q.precision != GKS_FP64 && q.precision != GKS_FP32_MIXED)
                return fail(GKS_EUNSUPPORTED, "unknown precision");
            if (!(q.G > 0) || !(q.cfl > 0) || !(q.chi > 0) || !(q.eps > 0) || !(q.eps_num >= 0))
                return fail(GKS_EINVAL, "bad physical parameters");
            if (q.alpha_mode != 0 && q.alpha_mode != 1) return fail(GKS_EINVAL, "unknown alpha_mode");
            if (q.src_order != 0 && q.src_order != 2 && q.src_order != 4)
                return fail(GKS_EINVAL, "src_order must be 2 (or 0) or 4");
            if (q.grad_mode != 0 && q.grad_mode != 1) return fail(GKS_EINVAL, "grad_mode must be 0 or 1");
            if (!(q.h_dry >= 0) || !std::isfinite(q.h_dry)) return fail(GKS_EINVAL, "h_dry must be finite and >= 0");
            if (q.h_dry > 0 && q.src_order == 4)
                return fail(GKS_EINVAL, "wet/dry layers (h_dry > 0) need the second-order layer coupling");
            if (q.G != prm[0].G || q.cfl != prm[0].cfl || q.eps != prm[0].eps || q.eps_num != prm[0].eps_num ||
                q.precision != prm[0].precision || q.linear != prm[0].linear || q.alpha_mode != prm[0].alpha_mode ||
                (q.src_order == 4) != (prm[0].src_order == 4) || q.grad_mode != prm[0].grad_mode ||
                q.h_dry != prm[0].h_dry)
                return fail(GKS_EINVAL, "scenarios of a batch share G, cfl, eps, eps_num, precision, linear, "
                                        "alpha_mode, src_order, grad_mode and h_dry");
        }
        *out = nullptr;
        const int prec = prm[0].precision;
        if (prec == GKS_FP32_MIXED) {
            gks_status r = ensure_f32(mesh);
            if (r != GKS_OK) return r;
        }
        const int64_t T = h.nt, TG = T + h.ng, E = h.ne;
        // host conversion: the device state carries eta1 = h1 + B and grad(eta1)
        std::vector<double> wh(2 * TG, 0.0), wm(4 * TG, 0.0), g(12 * TG, 0.0);
        for (int v = 0; v < 6; v++)
            for (int64_t c = 0; c < T; c++) {
                double x = W0[v * T + c];
                // a layer thickness must be positive, or >= 0 with wet/dry layers
                if (!std::isfinite(x) || ((v == 0 || v == 3) && !(x > 0 || (prm[0].h_dry > 0 && x >= 0))))
                    return fail(GKS_ENONFINITE, "bad initial value at component " + std::to_string(v) + ", cell " +
                                                    std::to_string(c));
                if (v == 0) wh[c] = x;
                else if (v == 3) wh[TG + c] = x + h.Bbar[c];
                else wm[(v < 3 ? v - 1 : v - 2) * TG + c] = x;
                for (int d = 0; d < 2; d++) {
                    double y = gradW0[(2 * v + d) * T + c];
                    if (!std::isfinite(y)) return fail(GKS_ENONFINITE, "non-finite initial gradient");
                    g[(2 * v + d) * TG + c] = v == 3 ? y + h.gB[d * T + c] : y;
                }
            }
        gks_state *s = new gks_state();
        s->mesh = mesh;
        s->prec = prec;
        s->src4 = prm[0].src_order == 4;
        s->gm1 = prm[0].grad_mode == 1;
        s->md = prec == GKS_FP64 ? mesh->d64 : mesh->d32;
        s->stream = (hipStream_t)stream;
        s->nparts = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (T + gks::DT_BLOCK - 1) / gks::DT_BLOCK));
        const size_t rs = prec == GKS_FP64 ? sizeof(double) : sizeof(float);
        const size_t uT = (size_t)T, uTG = (size_t)TG, uE = (size_t)E, uS = (size_t)S;
        struct Buf {
            void **p;
            size_t bytes;
        } bufs[] = {{(void **)&s->Wh[0], 2 * uTG * 8}, {(void **)&s->Wh[1], 2 * uTG * 8}, {&s->Wm[0], 4 * uTG * rs},
                    {&s->Wm[1], 4 * uTG * rs}, {&s->gW[0], 12 * uTG * rs}, {&s->gW[1], 12 * uTG * rs},
                    {(void **)&s->Wc, 6 * uT * 8}, {&s->Gc, 12 * uT * rs}, {&s->rec, 6 * uT * rec_bytes(prec)},
                    {&s->r0, 2 * uT * rs}, {(void **)&s->hmid, 2 * uE * 8},
                    {(void **)&s->gP1, 4 * uT * 8}, {(void **)&s->need, uT}, {(void **)&s->eoh, (s->gm1 ? 8 : 6) * uE * 8},
                    {&s->eom, (s->gm1 ? 34 : 24) * uE * rs},
                    {(void **)&s->scal, 2 * uS * 8}, {(void **)&s->part, 2 * (size_t)std::max<int64_t>(std::max(s->nparts, 1024), mesh->d64.NCH) * 8},
                    {(void **)&s->chi, uS * 8}, {(void **)&s->tend, uS * 8}, {(void **)&s->bad, 8},
                    {&s->src, s->src4 ? 8 * uT * rs : 8}};
        for (auto &b : bufs) {
            hipError_t e = hipMalloc(b.p, std::max<size_t>(b.bytes, 8));
            if (e != hipSuccess) {
                gks_state_destroy(s);
                return fail(GKS_ENOMEM, std::string("state allocation: ") + hipGetErrorString(e));
            }
            s->owned.push_back(*b.p);
        }
        std::vector<double> chi(S), tend(S), scal(2 * S, 0.0);
        for (int32_t i = 0; i < S; i++) {
            chi[i] = prm[i].chi;
            tend[i] = prm[i].t_end > 0 ? prm[i].t_end : 1e300;
        }
        s->p.G = prm[0].G;
        s->p.eps = prm[0].eps;
        s->p.eps_num = prm[0].eps_num;
        s->p.cfl = prm[0].cfl;
        s->p.linear = prm[0].linear;
        s->p.alpha_mode = prm[0].alpha_mode;
        s->p.h_dry = prm[0].h_dry;
        s->p.chi = s->chi;
        s->p.t_end = s->tend;
        s->p.scal = s->scal;
        s->p.bad = s->bad;
        std::vector<unsigned char> bm, bg;
        if (prec == GKS_FP64) {
            to_real<double>(wm, bm);
            to_real<double>(g, bg);
        } else {
            to_real<float>(wm, bm);
            to_real<float>(g, bg);
        }
        // a failed copy releases the partly built state
        const gks_status r = [&]() -> gks_status {
            HIP_OK(hipMemcpy(s->Wh[0], wh.data(), wh.size() * 8, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(s->Wm[0], bm.data(), bm.size(), hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(s->gW[0], bg.data(), bg.size(), hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(s->chi, chi.data(), S * 8, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(s->tend, tend.data(), S * 8, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(s->scal, scal.data(), 2 * S * 8, hipMemcpyHostToDevice));
            const unsigned long long none = ~0ull;
            HIP_OK(hipMemcpy(s->bad, &none, 8, hipMemcpyHostToDevice));
            HIP_OK(hipMemset(s->Wh[1], 0, 2 * TG * 8));
            HIP_OK(hipMemset(s->Wm[1], 0, 4 * TG * rs));
            HIP_OK(hipMemset(s->gW[1], 0, 12 * TG * rs));
            return GKS_OK;
        }();
        if (r != GKS_OK) {
            gks_state_destroy(s);
            return r;
        }
        *out = s;
        return GKS_OK;
    });
}

void gks_state_destroy(gks_state *s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    if (s->gstream) (void)hipStreamSynchronize(s->gstream);
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    for (hipEvent_t e : s->gev)
        if (e) (void)hipEventDestroy(e);
    if (s->gstream) (void)hipStreamDestroy(s->gstream);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    for (void *p : s->owned) (void)hipFree(p);
    delete s;
}

gks_status gks_profile(gks_state *s, int32_t enable)
{
    return guarded([&]() -> gks_status {
        if (!s) return fail(GKS_EINVAL, "null state");
        HIP_OK(hipStreamSynchronize(s->stream));
        s->prof.clear();
        s->ev_used = 0;
        s->prof_on = enable != 0;
        return GKS_OK;
    });
}

gks_status gks_profile_read(gks_state *s, int32_t kernel, double *total_ms, int64_t *launches)
{
    return guarded([&]() -> gks_status {
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
    });
}

gks_status gks_stage(gks_state *s, int32_t stage, const double *dt)
{
    return guarded([&]() -> gks_status {
        if (!s || (stage != 0 && stage != 1)) return fail(GKS_EINVAL, "bad stage arguments");
        if (stage == 1 && !s->half) return fail(GKS_EINVAL, "stage 1 must follow stage 0");
        if (stage == 0 && s->half) return fail(GKS_EINVAL, "stage 0 must follow stage 1");
        if (stage == 0) {
            if (dt) {
                if (s->md.S != 1) return fail(GKS_EINVAL, "an explicit dt needs a single-scenario state");
                if (!(*dt > 0) || !std::isfinite(*dt)) return fail(GKS_EINVAL, "dt must be positive");
                hipLaunchKernelGGL(gks::k_set_dt, dim3(1), dim3(1), 0, s->stream, s->p, *dt);
            } else {
                dt_any(s, s->stream);
            }
        } else if (dt) {
            return fail(GKS_EINVAL, "stage 1 reuses the step size of stage 0");
        }
        stage_any(s, stage, s->stream);
        HIP_OK(hipGetLastError());
        s->half = stage == 0;
        return GKS_OK;
    });
}

gks_status gks_step(gks_state *s, int32_t n_steps, double *dt_last)
{
    return guarded([&]() -> gks_status {
        if (!s || n_steps < 0) return fail(GKS_EINVAL, "bad step arguments");
        if (s->half) return fail(GKS_EINVAL, "a step cannot start between stage 0 and stage 1");
        for (int i = 0; i < n_steps; i++) {
            dt_any(s, s->stream);
            stage_any(s, 0, s->stream);
            stage_any(s, 1, s->stream);
            HIP_OK(hipGetLastError());
        }
        if (dt_last) {
            double sc[2];
            HIP_OK(hipMemcpyAsync(sc, s->scal, sizeof(sc), hipMemcpyDeviceToHost, s->stream));
            HIP_OK(hipStreamSynchronize(s->stream));
            *dt_last = sc[0];
            return check_bad(s, nullptr);
        }
        return GKS_OK;
    });
}

gks_status gks_batch_step(gks_state *s, int32_t n_steps)
{
    return guarded([&]() -> gks_status {
        if (!s || n_steps < 0) return fail(GKS_EINVAL, "bad step arguments");
        if (s->half) return fail(GKS_EINVAL, "a step cannot start between stage 0 and stage 1");
        if (!s->gexec) {
            // capture one full step (every scenario's dt, both stages) on a private stream
            HIP_OK(hipStreamCreateWithFlags(&s->gstream, hipStreamNonBlocking));
            HIP_OK(hipEventCreateWithFlags(&s->gev[0], hipEventDisableTiming));
            HIP_OK(hipEventCreateWithFlags(&s->gev[1], hipEventDisableTiming));
            s->capturing = true;
            HIP_OK(hipStreamBeginCapture(s->gstream, hipStreamCaptureModeThreadLocal));
            dt_any(s, s->gstream);
            stage_any(s, 0, s->gstream);
            stage_any(s, 1, s->gstream);
            hipError_t e = hipStreamEndCapture(s->gstream, &s->graph);
            s->capturing = false;
            HIP_OK(e);
            HIP_OK(hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0));
        }
        // order the graph replays after the work already queued on the state's stream, and later
        // work on that stream after them
        HIP_OK(hipEventRecord(s->gev[0], s->stream));
        HIP_OK(hipStreamWaitEvent(s->gstream, s->gev[0], 0));
        for (int i = 0; i < n_steps; i++) HIP_OK(hipGraphLaunch(s->gexec, s->gstream));
        HIP_OK(hipEventRecord(s->gev[1], s->gstream));
        HIP_OK(hipStreamWaitEvent(s->stream, s->gev[1], 0));
        return GKS_OK;
    });
}

gks_status gks_state_read(const gks_state *s, double *W, double *gradW, double *t)
{
    return guarded([&]() -> gks_status {
        if (!s) return fail(GKS_EINVAL, "null state");
        const gks::HostMesh &h = s->mesh->host;
        const int64_t T = h.nt, TG = T + h.ng;
        const int b = s->half ? 1 : 0;
        const size_t rs = s->prec == GKS_FP64 ? 8 : 4;
        HIP_OK(hipStreamSynchronize(s->stream));
        if (W) {
            std::vector<double> wh(2 * TG), wm;
            std::vector<unsigned char> raw(4 * TG * rs);
            HIP_OK(hipMemcpy(wh.data(), s->Wh[b], wh.size() * 8, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(raw.data(), s->Wm[b], raw.size(), hipMemcpyDeviceToHost));
            if (s->prec == GKS_FP64) from_real<double>(raw, wm); else from_real<float>(raw, wm);
            for (int64_t c = 0; c < T; c++) {
                W[c] = wh[c];
                W[3 * T + c] = wh[TG + c] - h.Bbar[c];
                W[T + c] = wm[c];
                W[2 * T + c] = wm[TG + c];
                W[4 * T + c] = wm[2 * TG + c];
                W[5 * T + c] = wm[3 * TG + c];
            }
        }
        if (gradW) {
            std::vector<double> g;
            std::vector<unsigned char> raw(12 * TG * rs);
            HIP_OK(hipMemcpy(raw.data(), s->gW[b], raw.size(), hipMemcpyDeviceToHost));
            if (s->prec == GKS_FP64) from_real<double>(raw, g); else from_real<float>(raw, g);
            for (int v = 0; v < 6; v++)
                for (int d = 0; d < 2; d++)
                    for (int64_t c = 0; c < T; c++)
                        gradW[(2 * v + d) * T + c] = v == 3 ? g[(2 * v + d) * TG + c] - h.gB[d * T + c] : g[(2 * v + d) * TG + c];
        }
        if (t) return gks_state_time(s, 0, t, nullptr);
        return check_bad(s, nullptr);
    });
}

gks_status gks_state_time(const gks_state *s, int32_t scen, double *t, double *dt)
{
    return guarded([&]() -> gks_status {
        if (!s || scen < 0 || scen >= s->md.S) return fail(GKS_EINVAL, "bad scenario index");
        double sc[2];
        HIP_OK(hipStreamSynchronize(s->stream));
        HIP_OK(hipMemcpy(sc, s->scal + 2 * scen, sizeof(sc), hipMemcpyDeviceToHost));
        if (t) *t = s->half ? sc[1] - 0.5 * sc[0] : sc[1];
        if (dt) *dt = sc[0];
        return check_bad(s, nullptr);
    });
}

gks_status gks_state_mass(const gks_state *s, int32_t scen, double mass[2])
{
    return guarded([&]() -> gks_status {
        if (!s || !mass || scen < -1 || scen >= s->md.S) return fail(GKS_EINVAL, "bad mass query");
        const gks::HostMesh &h = s->mesh->host;
        const int64_t c0 = scen < 0 ? 0 : h.scell[scen], c1 = scen < 0 ? h.nt : h.scell[scen + 1];
        const int nb = 256;
        hipLaunchKernelGGL(gks::k_mass_partial, dim3(nb), dim3(256), 0, s->stream, s->md, s->Wh[s->half ? 1 : 0], c0, c1,
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
        return check_bad(s, nullptr);
    });
}

gks_status gks_state_diagnostics(const gks_state *s, int32_t scen, double out[8])
{
    return guarded([&]() -> gks_status {
        if (!s || !out || scen < 0 || scen >= s->md.S) return fail(GKS_EINVAL, "bad diagnostics query");
        const gks::HostMesh &h = s->mesh->host;
        const int64_t c0 = h.scell[scen], c1 = h.scell[scen + 1];
        const int nb = 256;  // 6 values per block: the state's part buffer holds at least 2048
        const int b = s->half ? 1 : 0;
        hipLaunchKernelGGL(gks::k_mass_partial, dim3(nb), dim3(256), 0, s->stream, s->md, s->Wh[b], c0, c1, s->part);
        HIP_OK(hipGetLastError());
        std::vector<double> mpart(2 * nb), dpart(6 * nb);
        HIP_OK(hipMemcpyAsync(mpart.data(), s->part, mpart.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        if (s->prec == GKS_FP64)
            hipLaunchKernelGGL(gks::k_diag_partial<double>, dim3(nb), dim3(256), 0, s->stream, s->md, s->Wh[b],
                               (const double *)s->Wm[b], c0, c1, s->p.h_dry, s->part);
        else
            hipLaunchKernelGGL(gks::k_diag_partial<float>, dim3(nb), dim3(256), 0, s->stream, s->md, s->Wh[b],
                               (const float *)s->Wm[b], c0, c1, s->p.h_dry, s->part);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(dpart.data(), s->part, dpart.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        double sc[2];
        HIP_OK(hipMemcpyAsync(sc, s->scal + 2 * scen, sizeof(sc), hipMemcpyDeviceToHost, s->stream));
        HIP_OK(hipStreamSynchronize(s->stream));
        out[0] = s->half ? sc[1] - 0.5 * sc[0] : sc[1];
        out[1] = sc[0];
        out[2] = out[3] = 0;
        for (int k = 0; k < nb; k++) {
            out[2] += mpart[2 * k];
            out[3] += mpart[2 * k + 1];
        }
        double mx[6] = {0.0, 0.0, -HUGE_VAL, -HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
        for (int k = 0; k < nb; k++)
            for (int q = 0; q < 6; q++) mx[q] = std::max(mx[q], dpart[6 * k + q]);
        out[4] = mx[0];
        out[5] = mx[1];
        out[6] = mx[2] + mx[3];  // max - min of eta1
        out[7] = mx[4] + mx[5];  // max - min of eta2
        return check_bad(s, nullptr);
    });
}

gks_status gks_debug_bounds(int32_t reset, int32_t *violations)
{
    return guarded([&]() -> gks_status {
#ifdef GKS_CHECKED
        unsigned int v = 0;
        HIP_OK(hipDeviceSynchronize());
        HIP_OK(hipMemcpyFromSymbol(&v, HIP_SYMBOL(gks::oob_flag), sizeof(v)));
        if (violations) *violations = (int32_t)v;
        if (reset) {
            const unsigned int zero = 0;
            HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(gks::oob_flag), &zero, sizeof(zero)));
        }
        return GKS_OK;
#else
        (void)reset;
        if (violations) *violations = -1;
        return fail(GKS_EUNSUPPORTED, "index checks are compiled into the checked build only");
#endif
    });
}

gks_status gks_state_check(const gks_state *s, int64_t *first_bad)
{
    return guarded([&]() -> gks_status {
        if (!s) return fail(GKS_EINVAL, "null state");
        HIP_OK(hipStreamSynchronize(s->stream));
        return check_bad(s, first_bad);
    });
}

gks_status gks_state_checkpoint_size(const gks_state *s, int64_t *bytes)
{
    return guarded([&]() -> gks_status {
        if (!s || !bytes) return fail(GKS_EINVAL, "null argument");
        *bytes = ckpt_bytes(s);
        return GKS_OK;
    });
}

gks_status gks_state_save(const gks_state *s, void *blob, int64_t bytes)
{
    return guarded([&]() -> gks_status {
        if (!s || !blob) return fail(GKS_EINVAL, "null argument");
        if (s->half) return fail(GKS_EINVAL, "a checkpoint cannot be taken between stage 0 and stage 1");
        if (bytes < ckpt_bytes(s)) return fail(GKS_EINVAL, "checkpoint buffer too small");
        const gks::HostMesh &h = s->mesh->host;
        const int64_t TG = h.nt + h.ng, rs = s->prec == GKS_FP64 ? 8 : 4;
        CkptHeader hd{CKPT_MAGIC, 1u, s->prec, h.S, h.nt, h.ng};
        unsigned char *p = static_cast<unsigned char *>(blob);
        std::memcpy(p, &hd, sizeof(hd));
        p += sizeof(hd);
        HIP_OK(hipStreamSynchronize(s->stream));
        HIP_OK(hipMemcpy(p, s->Wh[0], 2 * TG * 8, hipMemcpyDeviceToHost));
        p += 2 * TG * 8;
        HIP_OK(hipMemcpy(p, s->Wm[0], 4 * TG * rs, hipMemcpyDeviceToHost));
        p += 4 * TG * rs;
        HIP_OK(hipMemcpy(p, s->gW[0], 12 * TG * rs, hipMemcpyDeviceToHost));
        p += 12 * TG * rs;
        HIP_OK(hipMemcpy(p, s->scal, 2 * (size_t)h.S * 8, hipMemcpyDeviceToHost));
        p += 2 * (size_t)h.S * 8;
        HIP_OK(hipMemcpy(p, s->bad, 8, hipMemcpyDeviceToHost));
        return GKS_OK;
    });
}

gks_status gks_state_load(gks_state *s, const void *blob, int64_t bytes)
{
    return guarded([&]() -> gks_status {
        if (!s || !blob) return fail(GKS_EINVAL, "null argument");
        if (bytes < ckpt_bytes(s)) return fail(GKS_EINVAL, "checkpoint too short for this state");
        const gks::HostMesh &h = s->mesh->host;
        CkptHeader hd;
        std::memcpy(&hd, blob, sizeof(hd));
        if (hd.magic != CKPT_MAGIC || hd.version != 1u) return fail(GKS_EINVAL, "not a checkpoint of this library");
        if (hd.prec != s->prec || hd.S != h.S || hd.T != h.nt || hd.NG != h.ng)
            return fail(GKS_EINVAL, "checkpoint of another mesh or precision");
        const int64_t TG = h.nt + h.ng, rs = s->prec == GKS_FP64 ? 8 : 4;
        const unsigned char *p = static_cast<const unsigned char *>(blob) + sizeof(hd);
        HIP_OK(hipStreamSynchronize(s->stream));
        HIP_OK(hipMemcpy(s->Wh[0], p, 2 * TG * 8, hipMemcpyHostToDevice));
        p += 2 * TG * 8;
        HIP_OK(hipMemcpy(s->Wm[0], p, 4 * TG * rs, hipMemcpyHostToDevice));
        p += 4 * TG * rs;
        HIP_OK(hipMemcpy(s->gW[0], p, 12 * TG * rs, hipMemcpyHostToDevice));
        p += 12 * TG * rs;
        HIP_OK(hipMemcpy(s->scal, p, 2 * (size_t)h.S * 8, hipMemcpyHostToDevice));
        p += 2 * (size_t)h.S * 8;
        HIP_OK(hipMemcpy(s->bad, p, 8, hipMemcpyHostToDevice));
        s->half = 0;
        return GKS_OK;
    });
}

}  // extern "C"

namespace {

// the record arrays repacked into the component-major layouts documented for gks_state_buffer
template <typename R>
gks_status read_buffer(const gks_state *s, int32_t which, void *dst)
{
    const int64_t T = s->md.T, E = s->md.E;
    if (which == GKS_BUF_R0) {
        HIP_OK(hipMemcpy(dst, s->r0, (size_t)(2 * T) * sizeof(R), hipMemcpyDeviceToHost));
        return GKS_OK;
    }
    if (which == GKS_BUF_RECH || which == GKS_BUF_RECM) {
        std::vector<gks::GpHead<R>> hd((size_t)(6 * T));
        std::vector<gks::GpTail<R>> tl((size_t)(6 * T));
        const gks::GpRecs<R> rr = recs_of<R>(s->rec, T);
        HIP_OK(hipMemcpy(hd.data(), rr.head, hd.size() * sizeof(gks::GpHead<R>), hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(tl.data(), rr.tail, tl.size() * sizeof(gks::GpTail<R>), hipMemcpyDeviceToHost));
        for (int64_t c = 0; c < T; c++)
            for (int slot = 0; slot < 6; slot++) {
                const gks::GpHead<R> &h = hd[6 * c + slot];
                const gks::GpTail<R> &t = tl[6 * c + slot];
                if (which == GKS_BUF_RECH) {
                    for (int q = 0; q < 2; q++) static_cast<double *>(dst)[(slot * 2 + q) * T + c] = h.h[q];
                } else {
                    R *d = static_cast<R *>(dst);
                    for (int q = 0; q < 4; q++) d[(slot * 16 + q) * T + c] = h.q[q];
                    for (int q = 0; q < 12; q++) d[(slot * 16 + 4 + q) * T + c] = t.g[q];
                }
            }
        return GKS_OK;
    }
    if (which == GKS_BUF_EOH) {
        HIP_OK(hipMemcpy(dst, s->eoh, (size_t)(6 * E) * 8, hipMemcpyDeviceToHost));
    } else {
        HIP_OK(hipMemcpy(dst, s->eom, (size_t)(24 * E) * sizeof(R), hipMemcpyDeviceToHost));
    }
    return GKS_OK;
}

}  // namespace

extern "C" gks_status gks_state_buffer(const gks_state *s, int32_t which, void *dst, int64_t bytes)
{
    return guarded([&]() -> gks_status {
        if (!s || !dst || which < 0 || which >= GKS_BUF_COUNT) return fail(GKS_EINVAL, "bad buffer query");
        const int64_t T = s->md.T, E = s->md.E;
        const int64_t rs = s->prec == GKS_FP64 ? 8 : 4;
        int64_t need = 0;
        switch (which) {
        case GKS_BUF_RECH: need = 12 * T * 8; break;
        case GKS_BUF_RECM: need = 96 * T * rs; break;
        case GKS_BUF_R0: need = 2 * T * rs; break;
        case GKS_BUF_EOH: need = 6 * E * 8; break;
        case GKS_BUF_SKIP: need = T; break;
        case GKS_BUF_SRC: need = 8 * T * rs; break;
        default: need = 24 * E * rs; break;
        }
        if (bytes < need) return fail(GKS_EINVAL, "buffer too small: " + std::to_string(need) + " bytes needed");
        HIP_OK(hipStreamSynchronize(s->stream));
        if (which == GKS_BUF_SRC) {
            if (!s->src4) return fail(GKS_EINVAL, "the state uses the second-order layer coupling (src_order 2)");
            HIP_OK(hipMemcpy(dst, s->src, (size_t)need, hipMemcpyDeviceToHost));
            return GKS_OK;
        }
        if (which == GKS_BUF_SKIP) {
            if (!s->smooth) return fail(GKS_EINVAL, "the indicator has never been switched on");
            HIP_OK(hipMemcpy(dst, s->smooth, (size_t)T, hipMemcpyDeviceToHost));
            return GKS_OK;
        }
        return s->prec == GKS_FP64 ? read_buffer<double>(s, which, dst) : read_buffer<float>(s, which, dst);
    });
}

// ---------------------------------------------------------------------------------------------
// learned smoothness indicator and its trainer

namespace {

gks_status state_alloc(gks_state *s, void **p, size_t bytes)
{
    if (*p) return GKS_OK;
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 8));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(GKS_ENOMEM, std::string("indicator allocation: ") + hipGetErrorString(e));
    }
    s->owned.push_back(*p);
    return GKS_OK;
}

// refresh the ghost cells of the latest state (they are otherwise refreshed at the start of a stage)
template <typename R>
void ghost_latest(gks_state *s, int b)
{
    const gks::MeshDev &m = s->md;
    if (m.NG > 0)
        hipLaunchKernelGGL(gks::k_ghost_fill<R>, dim3(blocks(m.NG, 256)), dim3(256), 0, s->stream, m, s->Wh[b],
                           (R *)s->Wm[b], (R *)s->gW[b]);
}

template <typename R>
void launch_features(gks_state *s, float *X)
{
    const int b = s->half ? 1 : 0;
    ghost_latest<R>(s, b);
    hipLaunchKernelGGL(gks::k_features<R>, dim3(blocks(s->md.T, 256)), dim3(256), 0, s->stream, s->md, s->p.G,
                       s->Wh[b], (const R *)s->Wm[b], (const R *)s->gW[b], X);
}

template <typename R>
void launch_labels(gks_state *s, double tol)
{
    const gks::MeshDev &m = s->md;
    const int b = s->half ? 1 : 0;
    ghost_latest<R>(s, b);
    gks::Phys pn = s->p, pl = s->p;
    pn.linear = 0;
    pl.linear = 1;
    const dim3 g(blocks(m.T, gks::RECON_CELLS)), t(192);
    hipLaunchKernelGGL((gks::k_recon<R, 0>), g, t, 0, s->stream, m, pn, s->Wh[b], (const R *)s->Wm[b],
                       (const R *)s->gW[b], gks::IndArgs{}, recs_of<R>(s->rec, m.T), (R *)s->r0, nullptr);
    hipLaunchKernelGGL((gks::k_recon<R, 0>), g, t, 0, s->stream, m, pl, s->Wh[b], (const R *)s->Wm[b],
                       (const R *)s->gW[b], gks::IndArgs{}, recs_of<R>(s->lab_rec, m.T), (R *)s->lab_r0, nullptr);
    hipLaunchKernelGGL(gks::k_label<R>, dim3(blocks(m.T, 256)), dim3(256), 0, s->stream, m, s->p.G, tol, s->Wh[b],
                       (const gks::GpHead<R> *)s->rec, (const gks::GpHead<R> *)s->lab_rec, s->lab_y);
}

gks_status labels_any(gks_state *s, double tol)
{
    if (!(tol >= 0) || !std::isfinite(tol)) return fail(GKS_EINVAL, "label tolerance must be finite and >= 0");
    const size_t T = (size_t)s->md.T, rs = s->prec == GKS_FP64 ? 8 : 4;
    gks_status r = state_alloc(s, &s->lab_rec, 6 * T * rec_bytes(s->prec));
    if (r == GKS_OK) r = state_alloc(s, &s->lab_r0, 2 * T * rs);
    if (r == GKS_OK) r = state_alloc(s, (void **)&s->lab_y, T);
    if (r != GKS_OK) return r;
    if (s->prec == GKS_FP64)
        launch_labels<double>(s, tol);
    else
        launch_labels<float>(s, tol);
    HIP_OK(hipGetLastError());
    return GKS_OK;
}

void drop_graph(gks_state *s)
{
    if (s->gstream) (void)hipStreamSynchronize(s->gstream);
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->gexec = nullptr;
    s->graph = nullptr;
}

// splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number generators", 2014)
uint64_t splitmix64(uint64_t &x)
{
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

}  // namespace

struct gks_trainer {
    hipStream_t stream = nullptr;
    int device = 0;
    int64_t cap = 0, n = 0, npos = 0;
    int32_t maxB = 0;
    int64_t adam_t = 0;
    float *X = nullptr, *Y = nullptr, *logit = nullptr;
    int32_t *perm = nullptr;
    float *P = nullptr, *g = nullptr, *mo = nullptr, *ve = nullptr;
    float *H1 = nullptr, *H2 = nullptr, *D1 = nullptr, *D2 = nullptr, *DZ = nullptr, *L = nullptr, *loss = nullptr;
    short *W1b = nullptr, *W2b = nullptr;
    std::vector<void *> owned;
};

namespace {

// forward, back-propagation and weight gradients of the minibatch tr->perm[off .. off + B)
void train_grad(gks_trainer *tr, int64_t off, int B, float *loss_out)
{
    const int32_t *idx = tr->perm + off;
    hipLaunchKernelGGL(gks::k_mlp_forward_delta, dim3(blocks(B, gks::TRAIN_BLOCK)), dim3(gks::TRAIN_BLOCK), 0,
                       tr->stream, tr->P, tr->X, tr->Y, idx, B, tr->H1, tr->H2, tr->D1, tr->D2, tr->DZ, tr->L);
    hipLaunchKernelGGL(gks::k_mlp_weight_grad, dim3(blocks(gks::MLP_NP, 64)), dim3(64), 0, tr->stream, tr->X, idx, B,
                       tr->H1, tr->H2, tr->D1, tr->D2, tr->DZ, tr->g);
    hipLaunchKernelGGL(gks::k_mean, dim3(1), dim3(256), 0, tr->stream, tr->L, B, loss_out);
}

gks_status trainer_logits(gks_trainer *tr)
{
    hipLaunchKernelGGL(gks::k_weights_bf16, dim3(blocks(gks::MLP_H * gks::MLP_H, 256)), dim3(256), 0, tr->stream, tr->P,
                       tr->W1b, tr->W2b);
    if (tr->n > 0)
        hipLaunchKernelGGL(gks::k_mlp_infer, dim3(blocks(tr->n, 32 * gks::IND_WAVES)), dim3(64 * gks::IND_WAVES), 0,
                           tr->stream, tr->X, tr->n, tr->W1b, tr->W2b, tr->P, tr->logit);
    HIP_OK(hipGetLastError());
    return GKS_OK;
}

}  // namespace

extern "C" {

gks_status gks_indicator_set(gks_state *s, const float *params, float threshold)
{
    return guarded([&]() -> gks_status {
        if (!s) return fail(GKS_EINVAL, "null state");
        if (!params) {
            if (s->ind_on) drop_graph(s);
            s->ind_on = false;
            return GKS_OK;
        }
        if (!std::isfinite(threshold)) return fail(GKS_EINVAL, "threshold must be finite");
        if (s->p.h_dry > 0)
            return fail(GKS_EINVAL, "the learned indicator is not trained for wet/dry layers (h_dry > 0)");
        for (int i = 0; i < gks::MLP_NP; i++)
            if (!std::isfinite(params[i])) return fail(GKS_ENONFINITE, "non-finite indicator parameter");
        const size_t T = (size_t)s->md.T;
        gks_status r = state_alloc(s, (void **)&s->ind_P, gks::MLP_NP * sizeof(float));
        if (r == GKS_OK) r = state_alloc(s, (void **)&s->ind_W1b, gks::MLP_K * gks::MLP_H * sizeof(short));
        if (r == GKS_OK) r = state_alloc(s, (void **)&s->ind_W2b, gks::MLP_H * gks::MLP_H * sizeof(short));
        if (r == GKS_OK) r = state_alloc(s, (void **)&s->ind_logit, T * sizeof(float));
        if (r == GKS_OK) r = state_alloc(s, (void **)&s->smooth, T);
        if (r != GKS_OK) return r;
        // the captured graph (if any) holds the launches without the indicator
        drop_graph(s);
        HIP_OK(hipStreamSynchronize(s->stream));
        HIP_OK(hipMemcpy(s->ind_P, params, gks::MLP_NP * sizeof(float), hipMemcpyHostToDevice));
        hipLaunchKernelGGL(gks::k_weights_bf16, dim3(blocks(gks::MLP_H * gks::MLP_H, 256)), dim3(256), 0, s->stream,
                           s->ind_P, s->ind_W1b, s->ind_W2b);
        HIP_OK(hipGetLastError());
        s->ind_thr = threshold;
        s->ind_on = true;
        return GKS_OK;
    });
}

gks_status gks_indicator_eval(gks_state *s, float *logits, uint8_t *mask, int64_t *n_skip)
{
    return guarded([&]() -> gks_status {
        if (!s) return fail(GKS_EINVAL, "null state");
        if (!s->ind_on) return fail(GKS_EINVAL, "the indicator is off");
        const gks::MeshDev &m = s->md;
        const int b = s->half ? 1 : 0;
        if (s->prec == GKS_FP64) {
            ghost_latest<double>(s, b);
            hipLaunchKernelGGL(gks::k_indicator<double>, dim3(blocks(m.T, 32 * gks::IND_WAVES)),
                               dim3(64 * gks::IND_WAVES), 0, s->stream, m, s->p.G, s->Wh[b], (const double *)s->Wm[b],
                               (const double *)s->gW[b], s->ind_W1b, s->ind_W2b, s->ind_P, s->ind_thr, s->smooth,
                               s->ind_logit);
        } else {
            ghost_latest<float>(s, b);
            hipLaunchKernelGGL(gks::k_indicator<float>, dim3(blocks(m.T, 32 * gks::IND_WAVES)),
                               dim3(64 * gks::IND_WAVES), 0, s->stream, m, s->p.G, s->Wh[b], (const float *)s->Wm[b],
                               (const float *)s->gW[b], s->ind_W1b, s->ind_W2b, s->ind_P, s->ind_thr, s->smooth,
                               s->ind_logit);
        }
        HIP_OK(hipGetLastError());
        HIP_OK(hipStreamSynchronize(s->stream));
        const size_t T = (size_t)m.T;
        if (logits) HIP_OK(hipMemcpy(logits, s->ind_logit, T * sizeof(float), hipMemcpyDeviceToHost));
        if (mask || n_skip) {
            std::vector<uint8_t> mk(T);
            HIP_OK(hipMemcpy(mk.data(), s->smooth, T, hipMemcpyDeviceToHost));
            if (mask) std::memcpy(mask, mk.data(), T);
            if (n_skip) {
                int64_t k = 0;
                for (uint8_t v : mk) k += v;
                *n_skip = k;
            }
        }
        return GKS_OK;
    });
}

gks_status gks_state_features(gks_state *s, float *X)
{
    return guarded([&]() -> gks_status {
        if (!s || !X) return fail(GKS_EINVAL, "null argument");
        const size_t T = (size_t)s->md.T;
        float *d = nullptr;
        HIP_OK(hipMalloc((void **)&d, T * gks::MLP_IN * sizeof(float)));
        if (s->prec == GKS_FP64)
            launch_features<double>(s, d);
        else
            launch_features<float>(s, d);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e == hipSuccess) e = hipMemcpy(X, d, T * gks::MLP_IN * sizeof(float), hipMemcpyDeviceToHost);
        (void)hipFree(d);
        if (e != hipSuccess) return fail(GKS_EDEVICE, std::string("features: ") + hipGetErrorString(e));
        return GKS_OK;
    });
}

gks_status gks_state_labels(gks_state *s, double tol, uint8_t *y)
{
    return guarded([&]() -> gks_status {
        if (!s || !y) return fail(GKS_EINVAL, "null argument");
        gks_status r = labels_any(s, tol);
        if (r != GKS_OK) return r;
        HIP_OK(hipStreamSynchronize(s->stream));
        HIP_OK(hipMemcpy(y, s->lab_y, (size_t)s->md.T, hipMemcpyDeviceToHost));
        return GKS_OK;
    });
}

gks_status gks_trainer_create(int64_t capacity, int32_t max_batch, const float *params0, void *stream,
                              gks_trainer **out)
{
    return guarded([&]() -> gks_status {
        if (!out || !params0 || capacity <= 0 || max_batch <= 0 || capacity > ((int64_t)1 << 31) - 1)
            return fail(GKS_EINVAL, "bad trainer arguments");
        *out = nullptr;
        for (int i = 0; i < gks::MLP_NP; i++)
            if (!std::isfinite(params0[i])) return fail(GKS_ENONFINITE, "non-finite initial parameter");
        gks_trainer *t = new gks_trainer();
        t->stream = (hipStream_t)stream;
        t->cap = capacity;
        t->maxB = max_batch;
        if (hipGetDevice(&t->device) != hipSuccess) {
            delete t;
            return fail(GKS_EDEVICE, "no HIP device");
        }
        const size_t C = (size_t)capacity, B = (size_t)max_batch, NP = gks::MLP_NP;
        struct Buf {
            void **p;
            size_t bytes;
        } bufs[] = {{(void **)&t->X, C * gks::MLP_IN * 4}, {(void **)&t->Y, C * 4}, {(void **)&t->logit, C * 4},
                    {(void **)&t->perm, C * 4}, {(void **)&t->P, NP * 4}, {(void **)&t->g, NP * 4},
                    {(void **)&t->mo, NP * 4}, {(void **)&t->ve, NP * 4}, {(void **)&t->H1, B * gks::MLP_H * 4},
                    {(void **)&t->H2, B * 64 * 4}, {(void **)&t->D1, B * 64 * 4}, {(void **)&t->D2, B * 64 * 4},
                    {(void **)&t->DZ, B * 4}, {(void **)&t->L, B * 4}, {(void **)&t->loss, (C / 1 + 1) * 4},
                    {(void **)&t->W1b, (size_t)gks::MLP_K * gks::MLP_H * 2},
                    {(void **)&t->W2b, (size_t)gks::MLP_H * gks::MLP_H * 2}};
        for (auto &b : bufs) {
            hipError_t e = hipMalloc(b.p, std::max<size_t>(b.bytes, 8));
            if (e != hipSuccess) {
                gks_trainer_destroy(t);
                return fail(GKS_ENOMEM, std::string("trainer allocation: ") + hipGetErrorString(e));
            }
            t->owned.push_back(*b.p);
        }
        std::vector<float> zero(NP, 0.f);
        hipError_t e = hipMemcpy(t->P, params0, NP * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(t->mo, zero.data(), NP * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(t->ve, zero.data(), NP * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            gks_trainer_destroy(t);
            return fail(GKS_EDEVICE, std::string("trainer upload: ") + hipGetErrorString(e));
        }
        *out = t;
        return GKS_OK;
    });
}

void gks_trainer_destroy(gks_trainer *t)
{
    if (!t) return;
    (void)hipStreamSynchronize(t->stream);
    for (void *p : t->owned) (void)hipFree(p);
    delete t;
}

gks_status gks_trainer_add(gks_trainer *t, const float *X, const uint8_t *y, int64_t n)
{
    return guarded([&]() -> gks_status {
        if (!t || n < 0 || (n > 0 && (!X || !y))) return fail(GKS_EINVAL, "bad sample arguments");
        if (t->n + n > t->cap) return fail(GKS_EINVAL, "trainer capacity exceeded");
        std::vector<float> yf((size_t)n);
        int64_t pos = 0;
        for (int64_t i = 0; i < n; i++) {
            if (y[i] > 1) return fail(GKS_EINVAL, "labels must be 0 or 1");
            yf[i] = (float)y[i];
            pos += y[i];
        }
        for (int64_t i = 0; i < n * gks::MLP_IN; i++)
            if (!std::isfinite(X[i])) return fail(GKS_ENONFINITE, "non-finite feature");
        HIP_OK(hipStreamSynchronize(t->stream));
        HIP_OK(hipMemcpy(t->X + t->n * gks::MLP_IN, X, (size_t)n * gks::MLP_IN * 4, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(t->Y + t->n, yf.data(), (size_t)n * 4, hipMemcpyHostToDevice));
        t->n += n;
        t->npos += pos;
        return GKS_OK;
    });
}

gks_status gks_trainer_add_state(gks_trainer *t, gks_state *s, double tol, int64_t *n_added)
{
    return guarded([&]() -> gks_status {
        if (!t || !s) return fail(GKS_EINVAL, "null argument");
        if (s->mesh->device != t->device) return fail(GKS_EINVAL, "state and trainer live on different devices");
        const int64_t T = s->md.T;
        if (t->n + T > t->cap) return fail(GKS_EINVAL, "trainer capacity exceeded");
        HIP_OK(hipStreamSynchronize(t->stream));
        if (s->prec == GKS_FP64)
            launch_features<double>(s, t->X + t->n * gks::MLP_IN);
        else
            launch_features<float>(s, t->X + t->n * gks::MLP_IN);
        gks_status r = labels_any(s, tol);
        if (r != GKS_OK) return r;
        hipLaunchKernelGGL(gks::k_u8_to_f32, dim3(blocks(T, 256)), dim3(256), 0, s->stream, s->lab_y, T, t->Y + t->n);
        HIP_OK(hipGetLastError());
        std::vector<uint8_t> y((size_t)T);
        HIP_OK(hipStreamSynchronize(s->stream));
        HIP_OK(hipMemcpy(y.data(), s->lab_y, (size_t)T, hipMemcpyDeviceToHost));
        int64_t pos = 0;
        for (uint8_t v : y) pos += v;
        t->n += T;
        t->npos += pos;
        if (n_added) *n_added = T;
        return GKS_OK;
    });
}

gks_status gks_trainer_info(const gks_trainer *t, int64_t *n_samples, int64_t *n_positive)
{
    return guarded([&]() -> gks_status {
        if (!t) return fail(GKS_EINVAL, "null trainer");
        if (n_samples) *n_samples = t->n;
        if (n_positive) *n_positive = t->npos;
        return GKS_OK;
    });
}

gks_status gks_trainer_grad(gks_trainer *t, const int32_t *idx, int32_t B, float *loss, float *grad)
{
    return guarded([&]() -> gks_status {
        if (!t || !idx || B < 1 || B > t->maxB) return fail(GKS_EINVAL, "bad gradient arguments");
        for (int32_t i = 0; i < B; i++)
            if (idx[i] < 0 || idx[i] >= t->n) return fail(GKS_EINVAL, "sample index out of range");
        HIP_OK(hipStreamSynchronize(t->stream));
        HIP_OK(hipMemcpy(t->perm, idx, (size_t)B * 4, hipMemcpyHostToDevice));
        train_grad(t, 0, B, t->loss);
        HIP_OK(hipGetLastError());
        HIP_OK(hipStreamSynchronize(t->stream));
        if (loss) HIP_OK(hipMemcpy(loss, t->loss, 4, hipMemcpyDeviceToHost));
        if (grad) HIP_OK(hipMemcpy(grad, t->g, gks::MLP_NP * 4, hipMemcpyDeviceToHost));
        return GKS_OK;
    });
}

gks_status gks_trainer_fit(gks_trainer *t, int32_t epochs, int32_t batch, float lr, uint64_t seed,
                           float *epoch_loss)
{
    return guarded([&]() -> gks_status {
        if (!t || epochs < 0 || batch < 1 || batch > t->maxB || !(lr > 0) || !std::isfinite(lr))
            return fail(GKS_EINVAL, "bad training arguments");
        if (t->n == 0) return fail(GKS_EINVAL, "no samples");
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const int64_t n = t->n, nb = (n + batch - 1) / batch;
        std::vector<int32_t> perm((size_t)n);
        std::vector<float> bl((size_t)nb);
        uint64_t state = seed;
        for (int32_t ep = 0; ep < epochs; ep++) {
            for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
            for (int64_t i = n - 1; i > 0; i--) {
                const int64_t j = (int64_t)(splitmix64(state) % (uint64_t)(i + 1));
                std::swap(perm[i], perm[j]);
            }
            HIP_OK(hipStreamSynchronize(t->stream));
            HIP_OK(hipMemcpy(t->perm, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice));
            for (int64_t k = 0; k < nb; k++) {
                const int64_t off = k * batch;
                const int B = (int)std::min<int64_t>(batch, n - off);
                train_grad(t, off, B, t->loss + k);
                t->adam_t++;
                const float c1 = 1.f - std::pow(b1, (float)t->adam_t), c2 = 1.f - std::pow(b2, (float)t->adam_t);
                hipLaunchKernelGGL(gks::k_adam, dim3(blocks(gks::MLP_NP, 256)), dim3(256), 0, t->stream, t->P, t->g, t->mo,
                                   t->ve, lr, b1, b2, eps, c1, c2);
            }
            HIP_OK(hipGetLastError());
            if (epoch_loss) {
                HIP_OK(hipStreamSynchronize(t->stream));
                HIP_OK(hipMemcpy(bl.data(), t->loss, (size_t)nb * 4, hipMemcpyDeviceToHost));
                double acc = 0;
                for (float v : bl) acc += v;
                epoch_loss[ep] = (float)(acc / (double)nb);
            }
        }
        HIP_OK(hipStreamSynchronize(t->stream));
        return GKS_OK;
    });
}

gks_status gks_trainer_params(const gks_trainer *t, float *params)
{
    return guarded([&]() -> gks_status {
        if (!t || !params) return fail(GKS_EINVAL, "null argument");
        HIP_OK(hipStreamSynchronize(t->stream));
        HIP_OK(hipMemcpy(params, t->P, gks::MLP_NP * 4, hipMemcpyDeviceToHost));
        return GKS_OK;
    });
}

gks_status gks_trainer_logits(gks_trainer *t, float *logits)
{
    return guarded([&]() -> gks_status {
        if (!t || !logits) return fail(GKS_EINVAL, "null argument");
        gks_status r = trainer_logits(t);
        if (r != GKS_OK) return r;
        HIP_OK(hipStreamSynchronize(t->stream));
        HIP_OK(hipMemcpy(logits, t->logit, (size_t)t->n * 4, hipMemcpyDeviceToHost));
        return GKS_OK;
    });
}

gks_status gks_trainer_threshold(gks_trainer *t, double max_false_skip, float *threshold)
{
    return guarded([&]() -> gks_status {
        if (!t || !threshold || !(max_false_skip >= 0) || !(max_false_skip <= 1))
            return fail(GKS_EINVAL, "bad threshold arguments");
        if (t->n == 0) return fail(GKS_EINVAL, "no samples");
        gks_status r = trainer_logits(t);
        if (r != GKS_OK) return r;
        const size_t n = (size_t)t->n;
        std::vector<float> z(n), y(n);
        HIP_OK(hipStreamSynchronize(t->stream));
        HIP_OK(hipMemcpy(z.data(), t->logit, n * 4, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(y.data(), t->Y, n * 4, hipMemcpyDeviceToHost));
        std::vector<float> neg;
        for (size_t i = 0; i < n; i++)
            if (y[i] < 0.5f) neg.push_back(z[i]);
        const size_t allowed = (size_t)std::floor(max_false_skip * (double)n);
        if (allowed >= neg.size()) {
            *threshold = -FLT_MAX;
            return GKS_OK;
        }
        // skip iff z > threshold: at most `allowed` label-0 logits may lie above it
        std::sort(neg.begin(), neg.end(), [](float a, float b) { return a > b; });
        *threshold = neg[allowed];
        return GKS_OK;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// launch-shape autotuner

extern "C" gks_status gks_autotune(gks_state *s, int32_t reps, int32_t *chosen)
{
    return guarded([&]() -> gks_status {
        if (!s || reps < 1) return fail(GKS_EINVAL, "bad autotune arguments");
        if (s->half) return fail(GKS_EINVAL, "autotune cannot start between stage 0 and stage 1");
        const gks::HostMesh &h = s->mesh->host;
        const int64_t TG = h.nt + h.ng;
        const size_t rs = s->prec == GKS_FP64 ? 8 : 4;
        const size_t nb[4] = {2 * (size_t)TG * 8, 4 * (size_t)TG * rs, 12 * (size_t)TG * rs, 2 * (size_t)h.S * 8};
        void *src[4] = {s->Wh[0], s->Wm[0], s->gW[0], s->scal};
        void *save[4] = {nullptr, nullptr, nullptr, nullptr};
        gks_status r = GKS_OK;
        HIP_OK(hipStreamSynchronize(s->stream));
        for (int i = 0; i < 4 && r == GKS_OK; i++)
            if (hipMalloc(&save[i], nb[i]) != hipSuccess) r = fail(GKS_ENOMEM, "autotune state copy");
        auto copy = [&](bool restore) {
            for (int i = 0; i < 4; i++)
                (void)hipMemcpyAsync(restore ? src[i] : save[i], restore ? save[i] : src[i], nb[i], hipMemcpyDeviceToDevice,
                                     s->stream);
        };
        const bool prof_was = s->prof_on;
        if (r == GKS_OK) {
            copy(false);
            drop_graph(s);
            const int tuned[5] = {GKS_KERNEL_GHOST, GKS_KERNEL_HHAT, GKS_KERNEL_PLANE, GKS_KERNEL_FLUX, GKS_KERNEL_UPDATE};
            const int cand[3] = {64, 128, 256};
            for (int k : tuned) {
                if (k == GKS_KERNEL_GHOST && h.ng == 0) continue;
                double best = 1e300;
                int pick = s->bs[k];
                for (int b : cand) {
                    s->bs[k] = b;
                    copy(true);
                    s->prof.clear();
                    s->ev_used = 0;
                    s->prof_on = true;
                    for (int i = 0; i < reps; i++) {
                        dt_any(s, s->stream);
                        stage_any(s, 0, s->stream);
                        stage_any(s, 1, s->stream);
                    }
                    if (hipStreamSynchronize(s->stream) != hipSuccess) {
                        r = fail(GKS_EDEVICE, "autotune run failed");
                        break;
                    }
                    double tot = 0;
                    for (const auto &rec : s->prof)
                        if (rec.kernel == k) {
                            float ms = 0;
                            (void)hipEventElapsedTime(&ms, rec.a, rec.b);
                            tot += ms;
                        }
                    if (tot < best) {
                        best = tot;
                        pick = b;
                    }
                }
                s->bs[k] = pick;
                if (r != GKS_OK) break;
            }
            copy(true);
            (void)hipStreamSynchronize(s->stream);
        }
        s->prof.clear();
        s->ev_used = 0;
        s->prof_on = prof_was;
        for (void *p : save)
            if (p) (void)hipFree(p);
        if (r == GKS_OK && chosen)
            for (int k = 0; k < GKS_KERNEL_COUNT; k++) chosen[k] = s->bs[k];
        return r;
    });
}

// ---------------------------------------------------------------------------------------------
// allocation-free mass query: the block partial sums of k_mass_partial go to a file-scope device
// array instead of the state's buffer

namespace {

constexpr int MASS_PARTS = 256;  // blocks of the mass reduction, one (upper, lower) pair each
constexpr int MAX_DEVICES = 64;

// 4 KiB on every device the library runs on, held until the process ends.  In host code the name
// is only a stand-in for the symbol: kernels and copies use the address from scratch_of().
static __device__ __align__(256) double scratch[2 * MASS_PARTS];

std::mutex g_scratch_mu;
double *g_scratch[MAX_DEVICES] = {};

// this device's copy of scratch, looked up once per device with that device current
gks_status scratch_of(int dev, double **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(GKS_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        int prev = 0;
        HIP_OK(hipGetDevice(&prev));
        if (prev != dev) HIP_OK(hipSetDevice(dev));
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != dev) (void)hipSetDevice(prev);
        if (e != hipSuccess || !p) return fail(GKS_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return GKS_OK;
}

}  // namespace

extern "C" gks_status gks_state_mass_noalloc(const gks_state *s, int32_t scen, double mass[2])
{
    return guarded([&]() -> gks_status {
        if (!s || !mass || scen < -1 || scen >= s->md.S) return fail(GKS_EINVAL, "bad mass query");
        double *part_d = nullptr;
        gks_status st = scratch_of(s->mesh->device, &part_d);
        if (st != GKS_OK) return st;
        const gks::HostMesh &h = s->mesh->host;
        const int64_t c0 = scen < 0 ? 0 : h.scell[scen], c1 = scen < 0 ? h.nt : h.scell[scen + 1];
        // every block writes its pair, so nothing needs clearing; the grid strides over any number
        // of cells, so every mesh fits the fixed-size scratch
        hipLaunchKernelGGL(gks::k_mass_partial, dim3(MASS_PARTS), dim3(256), 0, s->stream, s->md,
                           s->Wh[s->half ? 1 : 0], c0, c1, part_d);
        HIP_OK(hipGetLastError());
        double part[2 * MASS_PARTS];
        HIP_OK(hipMemcpyAsync(part, part_d, sizeof(part), hipMemcpyDeviceToHost, s->stream));
        HIP_OK(hipStreamSynchronize(s->stream));
        mass[0] = mass[1] = 0;
        for (int b = 0; b < MASS_PARTS; b++) {
            mass[0] += part[2 * b];
            mass[1] += part[2 * b + 1];
        }
        return GKS_OK;
    });
}
