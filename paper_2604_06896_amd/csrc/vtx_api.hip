// Host side of the libvtx C ABI: validation and staging of the half-edge
// table, workspace ownership, the relaxation and CG drivers (device loops
// captured as HIP graphs, host polls an 8-byte status per chunk), and the
// hypergradient entry point.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "vtx_launch.h"

namespace vtx {
int tissue_topology_changed(vtx_tissue t, hipStream_t s);
}

using namespace vtx;

// ------------------------------------------------- allocation-free scratch
// Fixed device scratch of vtx_energy_forces_noalloc: the per-tile partial
// sums and two loop control blocks of one fused evaluation, for tissues of
// up to kNoAllocVerts vertices (a 3-valent periodic tissue has half as many
// cells).  Every GPU the library runs on holds one copy until the process
// ends.  In host code `scratch` names a host-side stand-in; its device
// address comes from hipGetSymbolAddress (noalloc_scratch).
namespace {
constexpr int64_t kNoAllocVerts = 1 << 18;
constexpr size_t kNoAllocMpartBytes = 16 * (size_t)((kNoAllocVerts + kTileV - 1) / kTileV);
constexpr size_t kNoAllocCtlOffset = (kNoAllocMpartBytes + 255) & ~(size_t)255;
constexpr size_t kNoAllocBytes = kNoAllocCtlOffset + ((2 * sizeof(LoopCtl) + 255) & ~(size_t)255);
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Clears the two control blocks in the scratch (a kernel, not a memset, so a
// caller may capture the call in a graph).
__global__ void k_clear_ctl(LoopCtl *ctl) {
    const int n = (int)(2 * sizeof(LoopCtl) / sizeof(uint32_t));
    uint32_t *w = reinterpret_cast<uint32_t *>(ctl);
    for (int i = threadIdx.x; i < n; i += blockDim.x) w[i] = 0u;
}

struct vtx_tissue_s {
    DevTissue d;
    Workspace w;
    TileTables tiles;    // fused evaluation; rebuilt in stream order after topology changes
    int64_t n_vert, n_cell, n_edge, n_he;
    double *ep_buf;      // two position buffers for EP (double-sized)
    int64_t t1_cap;
};

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            return fail(VTX_E_HIP, "%s failed: %s", #x, hipGetErrorString(e_));            \
    } while (0)

int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VTX_E_HIP, "%s: %s", what, hipGetErrorString(e));
    return VTX_OK;
}

bool mode_ok(int m) { return m == VTX_F32 || m == VTX_F64 || m == VTX_MIXED; }

ParamsRaw raw(const vtx_params *p) {
    ParamsRaw r{p->KA, p->A0, p->KP, p->P0, p->lam, p->KA_s, p->A0_s, p->KP_s, p->P0_s, p->lam_s};
    return r;
}

// Host copy of the staged layouts.
struct Staged {
    std::vector<int32_t> he_edge, edge_he, row_ptr, row_cap, corner, corner_he, nsides, cell_he;
    std::vector<int32_t> star, star_he;
};

int validate_and_stage(const int32_t *he, int64_t n_he, int64_t n_vert, int64_t n_cell,
                       Staged &S) {
    if (n_he <= 0 || n_he % 2 || n_vert <= 0 || n_cell <= 0)
        return fail(VTX_E_ARG, "bad sizes n_he=%lld n_vert=%lld n_cell=%lld", (long long)n_he,
                    (long long)n_vert, (long long)n_cell);
    if (n_vert >= (int64_t)kIdMask || n_he >= (int64_t)INT32_MAX / 2 || n_cell >= INT32_MAX)
        return fail(VTX_E_CAPACITY, "tissue too large (n_vert must be < 2^28)");
    auto R = [&](int64_t h, int c) { return he[8 * h + c]; };
    for (int64_t h = 0; h < n_he; ++h) {
        for (int c : {HP, HN, HT})
            if (R(h, c) < 0 || R(h, c) >= n_he)
                return fail(VTX_E_TOPOLOGY, "half-edge %lld: index out of range", (long long)h);
        if (R(h, HS) < 0 || R(h, HS) >= n_vert || R(h, HG) < 0 || R(h, HG) >= n_vert)
            return fail(VTX_E_TOPOLOGY, "half-edge %lld: vertex out of range", (long long)h);
        if (R(h, HF) < 0 || R(h, HF) >= n_cell)
            return fail(VTX_E_TOPOLOGY, "half-edge %lld: face out of range", (long long)h);
        if (R(h, HOX) < -1 || R(h, HOX) > 1 || R(h, HOY) < -1 || R(h, HOY) > 1)
            return fail(VTX_E_TOPOLOGY, "half-edge %lld: offset not in {-1,0,1}", (long long)h);
        const int64_t t = R(h, HT);
        if (t == h || R(t, HT) != h)
            return fail(VTX_E_TOPOLOGY, "half-edge %lld: twin is not an involution", (long long)h);
        if (R(t, HS) != R(h, HG) || R(t, HG) != R(h, HS) || R(t, HOX) != -R(h, HOX) ||
            R(t, HOY) != -R(h, HOY))
            return fail(VTX_E_TOPOLOGY, "half-edge %lld: twin does not reverse it", (long long)h);
        if (R(R(h, HN), HP) != h || R(R(h, HP), HN) != h)
            return fail(VTX_E_TOPOLOGY, "half-edge %lld: prev/next not inverse", (long long)h);
        if (R(R(h, HN), HS) != R(h, HG))
            return fail(VTX_E_TOPOLOGY, "half-edge %lld: source(next) != target", (long long)h);
        if (R(R(h, HN), HF) != R(h, HF))
            return fail(VTX_E_TOPOLOGY, "half-edge %lld: next leaves the face", (long long)h);
        if (R(h, HS) == R(h, HG))
            return fail(VTX_E_TOPOLOGY, "half-edge %lld joins a vertex to itself", (long long)h);
    }
    // edges: ascending lower half-edge id
    S.he_edge.assign(n_he, -1);
    S.edge_he.clear();
    for (int64_t h = 0; h < n_he; ++h) {
        const int64_t t = R(h, HT);
        if (h < t) {
            S.he_edge[h] = S.he_edge[t] = (int32_t)S.edge_he.size();
            S.edge_he.push_back((int32_t)h);
        }
    }
    // faces
    std::vector<int64_t> count(n_cell, 0);
    S.cell_he.assign(n_cell, -1);
    for (int64_t h = 0; h < n_he; ++h) {
        const int c = R(h, HF);
        if (S.cell_he[c] < 0) S.cell_he[c] = (int32_t)h;
        ++count[c];
    }
    S.nsides.assign(n_cell, 0);
    S.row_ptr.assign(n_cell + 1, 0);
    for (int64_t c = 0; c < n_cell; ++c) {
        if (S.cell_he[c] < 0) return fail(VTX_E_TOPOLOGY, "cell %lld has no half-edge", (long long)c);
        int64_t n = 0, h = S.cell_he[c];
        int sx = 0, sy = 0;
        do {
            sx += R(h, HOX);
            sy += R(h, HOY);
            h = R(h, HN);
            ++n;
        } while (h != S.cell_he[c] && n <= n_he);
        if (n != count[c])
            return fail(VTX_E_TOPOLOGY, "cell %lld is not a single cycle", (long long)c);
        if (n < 3) return fail(VTX_E_TOPOLOGY, "cell %lld has fewer than 3 sides", (long long)c);
        if (sx || sy)
            return fail(VTX_E_TOPOLOGY, "cell %lld: image offsets do not close", (long long)c);
        S.nsides[c] = (int32_t)n;
        S.row_ptr[c + 1] = S.row_ptr[c] + (int32_t)n;
    }
    S.row_cap.assign(S.nsides.begin(), S.nsides.end());
    // corner rows: compact rows, room to re-compact them with kRowSlack spare
    // slots each, then a relocation pool of n_he + 1024 slots
    const int64_t cap_total = 2 * n_he + kRowSlack * n_cell + 1024;
    if (cap_total >= INT32_MAX) return fail(VTX_E_CAPACITY, "tissue too large");
    S.corner.assign(cap_total, 0);
    S.corner_he.assign(cap_total, 0);
    for (int64_t c = 0; c < n_cell; ++c) {
        int64_t h = S.cell_he[c], k = S.row_ptr[c];
        int wx = 0, wy = 0;
        do {
            if (wx < -1 || wx > 1 || wy < -1 || wy > 1)
                return fail(VTX_E_CAPACITY, "cell %lld spans more than one periodic image",
                            (long long)c);
            S.corner[k] = pack_id(R(h, HS), wx, wy);
            S.corner_he[k] = (int32_t)h;
            wx += R(h, HOX);
            wy += R(h, HOY);
            h = R(h, HN);
            ++k;
        } while (h != S.cell_he[c]);
    }
    // vertex stars
    std::vector<int32_t> out_he(n_vert, -1), out_n(n_vert, 0);
    for (int64_t h = 0; h < n_he; ++h) {
        const int v = R(h, HS);
        if (out_he[v] < 0) out_he[v] = (int32_t)h;
        ++out_n[v];
    }
    S.star.assign(9 * n_vert, 0);
    S.star_he.assign(3 * n_vert, 0);
    for (int64_t v = 0; v < n_vert; ++v) {
        if (out_n[v] != 3)
            return fail(VTX_E_TOPOLOGY, "vertex %lld has %d edges (3 required)", (long long)v,
                        out_n[v]);
        int64_t h = out_he[v];
        for (int k = 0; k < 3; ++k) {
            if (R(h, HS) != v)
                return fail(VTX_E_TOPOLOGY, "vertex %lld: star does not close", (long long)v);
            S.star_he[k * n_vert + v] = (int32_t)h;
            S.star[star_nb_at(n_vert, k, v)] = pack_id(R(h, HG), R(h, HOX), R(h, HOY));
            S.star[star_cell_at(n_vert, k, v)] = R(h, HF);
            S.star[star_edge_at(n_vert, k, v)] = S.he_edge[h];
            h = R(R(h, HP), HT);
        }
        if (h != out_he[v])
            return fail(VTX_E_TOPOLOGY, "vertex %lld: star does not close", (long long)v);
    }
    return VTX_OK;
}

template <typename T>
int upload(T **dst, const std::vector<T> &src) {
    HIPCHK(hipMalloc((void **)dst, std::max<size_t>(1, src.size()) * sizeof(T)));
    if (!src.empty()) HIPCHK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return VTX_OK;
}

int upload_into(int32_t *dst, const std::vector<int32_t> &src) {
    HIPCHK(hipMemcpy(dst, src.data(), src.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    return VTX_OK;
}

void free_tissue(vtx_tissue t) {
    if (!t) return;
    DevTissue &d = t->d;
    void *ptrs[] = {d.he, d.he_edge, d.edge_he, d.row_ptr, d.row_cap, d.pool_top, d.corner,
                    d.corner_he, d.nsides,
                    d.cell_he, d.star, d.star_he, t->w.xbuf,
                    t->w.cap, t->w.cell_aux, t->w.partials, t->w.partials2, t->w.mpart,
                    t->w.t1_list,
                    t->w.ctl, t->w.cg, t->w.scal, t->ep_buf,
                    t->tiles.cells, t->tiles.info, t->tiles.halo, t->tiles.cstart,
                    t->tiles.corners, t->tiles.fstar, t->tiles.fe};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (t->w.ctl_host) (void)hipHostFree(t->w.ctl_host);
    if (t->w.cap_stream) (void)hipStreamDestroy(t->w.cap_stream);
    delete t;
}

int reset_ctl(vtx_tissue t, int which, const LoopCtl &init, hipStream_t s) {
    t->w.ctl_host[which] = init;
    HIPCHK(hipMemcpyAsync(t->w.ctl + which, t->w.ctl_host + which, sizeof(LoopCtl),
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return VTX_OK;
}

int read_ctl(vtx_tissue t, int which, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(t->w.ctl_host + which, t->w.ctl + which, sizeof(LoopCtl),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return VTX_OK;
}

size_t pos_bytes(vtx_tissue t, int mode) {
    return (size_t)t->n_vert * 2 * (mode == VTX_F32 ? sizeof(float) : sizeof(double));
}

// Device loop driver: capture `chunk` steps of `body` once, replay until the
// control block reports done.
template <typename Body>
int run_loop(vtx_tissue t, int chunk, int64_t max_steps, hipStream_t s, Body body) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    HIPCHK(hipStreamBeginCapture(t->w.cap_stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < chunk; ++k) body(k, t->w.cap_stream);
    hipError_t ce = hipStreamEndCapture(t->w.cap_stream, &g);
    if (ce != hipSuccess) return fail(VTX_E_HIP, "graph capture: %s", hipGetErrorString(ce));
    ce = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (ce != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(VTX_E_HIP, "graph instantiate: %s", hipGetErrorString(ce));
    }
    int rc = VTX_OK;
    for (int64_t done_steps = 0;; done_steps += chunk) {
        hipError_t e = hipGraphLaunch(ge, s);
        if (e == hipSuccess) e = hipMemcpyAsync(t->w.ctl_host, t->w.ctl, sizeof(LoopCtl),
                                                hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            rc = fail(VTX_E_HIP, "device loop: %s", hipGetErrorString(e));
            break;
        }
        if (t->w.ctl_host[0].done) break;
        if (done_steps + chunk >= max_steps + 2 * (int64_t)chunk) {
            rc = fail(VTX_E_HIP, "device loop did not report completion");
            break;
        }
    }
    (void)hipGraphExecDestroy(ge);
    (void)hipGraphDestroy(g);
    return rc;
}

int relax_impl(vtx_tissue t, int mode, void *X, const vtx_params *p, const vtx_relax_opts *o,
               vtx_relax_result *res, hipStream_t s) {
    if (!(o->eta > 0) || !(o->tol >= 0) || o->patience < 1 || o->max_iter < 1)
        return fail(VTX_E_ARG, "relax options: eta > 0, tol >= 0, patience >= 1, max_iter >= 1");
    RelaxArgs ra{};
    ra.eta = o->eta;
    ra.t1_enable = o->t1_enable != 0;
    ra.l_min = o->l_min;
    ra.l_new = o->l_new;
    ra.beta = o->beta;
    ra.X_target = o->X_target;
    ra.g_lin = o->g_lin;
    ra.nudge = o->beta != 0.0 ? (o->X_target ? 1 : (o->g_lin ? 2 : 0)) : 0;
    if (o->beta != 0.0 && ra.nudge == 0)
        return fail(VTX_E_ARG, "a nudge needs X_target or g_lin");
    if (ra.nudge && ra.t1_enable) return fail(VTX_E_ARG, "a nudge cannot be combined with T1");
    if (ra.t1_enable && !(o->l_min > 0 && o->l_new > 0))
        return fail(VTX_E_ARG, "T1 needs l_min > 0 and l_new > 0");
    LoopCtl c{};
    c.status = VTX_NOT_CONVERGED;
    c.max_iter = o->max_iter;
    c.patience = o->patience;
    c.tol = o->tol;
    int rc = reset_ctl(t, 0, c, s);
    if (rc) return rc;
    if (ra.nudge == 2) {
        double *mean = (double *)((char *)t->w.ctl + offsetof(LoopCtl, nudge_mean));
        launch_mean_pos(t->w, VTX_F64, (int)t->n_vert, o->g_lin, mean, s);
        if ((rc = check_launch("nudge mean"))) return rc;
    }
    int chunk = o->chunk > 0 ? o->chunk : 256;
    chunk += chunk & 1;  // even: every replay starts on the caller's buffer
    void *bufs[2] = {X, t->w.xbuf};
    rc = run_loop(t, chunk, o->max_iter, s, [&](int k, hipStream_t cs) {
        const int cur = k & 1;
        launch_relax_iter(t->d, t->w, mode, bufs[cur], bufs[cur ^ 1], cur, raw(p), ra, cs);
    });
    if (ra.t1_enable) {
        const int rt = vtx::tissue_topology_changed(t, s);
        if (!rc) rc = rt;
    }
    if (rc) return rc;
    const LoopCtl &h = t->w.ctl_host[0];
    if (h.result_buf == 1) HIPCHK(hipMemcpyAsync(X, t->w.xbuf, pos_bytes(t, mode),
                                                 hipMemcpyDeviceToDevice, s));
    // energy (and nudge energy) at the returned positions
    launch_eval(t->d, t->w, mode, X, raw(p), t->w.scal + 4, nullptr, nullptr, s);
    if (ra.nudge == 1) launch_v2v(t->d, t->w, mode, X, o->X_target, t->w.scal + 5, nullptr, s);
    if (ra.nudge == 2)
        launch_dot_pos(t->w, mode, (int)t->n_vert, (const double *)o->g_lin, X, t->w.scal + 5, s);
    if ((rc = check_launch("final energy"))) return rc;
    double e[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(e, t->w.scal + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (res) {
        res->iters = h.iter;
        res->n_t1 = h.n_t1;
        res->n_stretch = h.n_stretch;
        res->max_f = h.last_maxf;
        res->energy = e[0] + (ra.nudge ? o->beta * e[1] : 0.0);
        res->status = h.status == VTX_E_NONFINITE ? VTX_NOT_CONVERGED : h.status;
    }
    if (h.t1_overflow == 1) return fail(VTX_E_CAPACITY, "T1 pass: too many pending re-checks");
    if (h.t1_overflow == 2)
        return fail(VTX_E_CAPACITY, "T1 pass: corner-row pool exhausted or a cell spans two images");
    if (h.status == VTX_E_NONFINITE) return fail(VTX_E_NONFINITE, "non-finite forces in relaxation");
    return VTX_OK;
}

}  // namespace

namespace vtx {
const DevTissue &tissue_dev(vtx_tissue t) { return t->d; }
const Workspace &tissue_ws(vtx_tissue t) { return t->w; }
int64_t tissue_size(vtx_tissue t) { return t->n_vert; }
int64_t tissue_cells(vtx_tissue t) { return t->n_cell; }
double *tissue_ep_buf(vtx_tissue t) { return t->ep_buf; }
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }
int tissue_topology_changed(vtx_tissue t, hipStream_t s) {
    launch_tile_build(t->d, t->tiles, s);
    return check_launch("tile tables");
}
}  // namespace vtx

extern "C" {

const char *vtx_last_error(void) { return g_err.c_str(); }

int vtx_tissue_create(const int32_t *he, int64_t n_he, int64_t n_vert, int64_t n_cell, double Lx,
                      double Ly, vtx_tissue *out) {
    if (!he || !out) return fail(VTX_E_ARG, "null argument");
    if (!(Lx > 0) || !(Ly > 0) || !std::isfinite(Lx) || !std::isfinite(Ly))
        return fail(VTX_E_ARG, "box sides must be positive and finite");
    *out = nullptr;
    Staged S;
    int rc = validate_and_stage(he, n_he, n_vert, n_cell, S);
    if (rc) return rc;
    vtx_tissue t = new vtx_tissue_s();
    std::memset(&t->d, 0, sizeof t->d);
    std::memset(&t->w, 0, sizeof t->w);
    t->ep_buf = nullptr;
    t->n_vert = n_vert;
    t->n_cell = n_cell;
    t->n_he = n_he;
    t->n_edge = (int64_t)S.edge_he.size();
    DevTissue &d = t->d;
    d.n_vert = (int32_t)n_vert;
    d.n_cell = (int32_t)n_cell;
    d.n_edge = (int32_t)t->n_edge;
    d.n_he = (int32_t)n_he;
    d.Lx = Lx;
    d.Ly = Ly;
    std::vector<int32_t> hev(he, he + 8 * n_he);
#define UP(dst, v)                       \
    if ((rc = upload(&dst, v))) {        \
        free_tissue(t);                  \
        return rc;                       \
    }
    UP(d.he, hev);
    UP(d.he_edge, S.he_edge);
    UP(d.edge_he, S.edge_he);
    UP(d.row_ptr, S.row_ptr);
    UP(d.row_cap, S.row_cap);
    {
        const std::vector<int32_t> pt{(int32_t)(n_he + kRowSlack * n_cell)};
        UP(d.pool_top, pt);
    }
    d.pool_start = (int32_t)(n_he + kRowSlack * n_cell);
    d.corner_cap = (int32_t)S.corner.size();
    UP(d.corner, S.corner);
    UP(d.corner_he, S.corner_he);
    UP(d.nsides, S.nsides);
    UP(d.cell_he, S.cell_he);
    UP(d.star, S.star);
    UP(d.star_he, S.star_he);
#undef UP
    int64_t t1cap = 1;
    while (t1cap < t->n_edge) t1cap <<= 1;
    t->t1_cap = t1cap;
    const int64_t nb = std::max<int64_t>(
        1024, (std::max(n_vert, std::max(n_cell, t->n_edge)) + kBlock - 1) / kBlock);
    Workspace &w = t->w;
    hipError_t e = hipSuccess;
    auto A = [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(bytes, 16));
    };
    A(&w.xbuf, 16 * (size_t)n_vert);
    A((void **)&w.cap, 16 * (size_t)n_cell);
    A((void **)&w.cell_aux, 16 * (size_t)n_cell);
    A((void **)&w.partials, 16 * (size_t)nb);
    A((void **)&w.partials2, 16 * (size_t)nb);
    A((void **)&w.mpart, 16 * (size_t)nb);
    A((void **)&w.t1_list, 4 * (size_t)t1cap);
    A((void **)&w.ctl, 2 * sizeof(LoopCtl));
    A((void **)&w.cg, 6 * 16 * (size_t)n_vert);  // CG: 4 vectors, MINRES: 6
    A((void **)&w.scal, 16 * sizeof(double));
    A((void **)&t->ep_buf, 2 * 16 * (size_t)n_vert);
    const size_t n_tiles = (size_t)n_tiles_for(n_vert);
    A((void **)&t->tiles.cells, 4 * (size_t)kTileCap * n_tiles);
    A((void **)&t->tiles.info, 16 * n_tiles);
    A((void **)&t->tiles.halo, 4 * (size_t)kHaloCap * n_tiles);
    A((void **)&t->tiles.cstart, 2 * (size_t)kCstartPad * n_tiles);
    A((void **)&t->tiles.corners, 2 * (size_t)kCornerCap * n_tiles);
    A((void **)&t->tiles.fstar, 16 * (size_t)n_vert);
    A((void **)&t->tiles.fe, 8 * (size_t)n_vert);
    if (e == hipSuccess) e = hipHostMalloc((void **)&w.ctl_host, 2 * sizeof(LoopCtl), 0);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&w.cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) {
        LoopCtl z{};
        w.ctl_host[0] = z;
        w.ctl_host[1] = z;
        e = hipMemcpy(w.ctl, w.ctl_host, 2 * sizeof(LoopCtl), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) {
        launch_tile_build(d, t->tiles, nullptr);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    if (e != hipSuccess) {
        free_tissue(t);
        return fail(VTX_E_HIP, "workspace allocation: %s", hipGetErrorString(e));
    }
    *out = t;
    return VTX_OK;
}

int vtx_tissue_destroy(vtx_tissue t) {
    if (!t) return fail(VTX_E_ARG, "null tissue");
    (void)hipDeviceSynchronize();
    free_tissue(t);
    return VTX_OK;
}

int vtx_tissue_sizes(vtx_tissue t, int64_t *n_vert, int64_t *n_cell, int64_t *n_edge,
                     int64_t *n_he) {
    if (!t) return fail(VTX_E_ARG, "null tissue");
    if (n_vert) *n_vert = t->n_vert;
    if (n_cell) *n_cell = t->n_cell;
    if (n_edge) *n_edge = t->n_edge;
    if (n_he) *n_he = t->n_he;
    return VTX_OK;
}

int vtx_tissue_tile_stats(vtx_tissue t, int64_t *stats) {
    if (!t || !stats) return fail(VTX_E_ARG, "null argument");
    const int64_t nt = n_tiles_for(t->n_vert);
    std::vector<int4> info((size_t)nt);
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(info.data(), t->tiles.info, sizeof(int4) * (size_t)nt,
                     hipMemcpyDeviceToHost));
    for (int k = 0; k < 5; ++k) stats[k] = 0;
    stats[0] = nt;
    for (const int4 &i : info) {
        stats[1] += i.x;
        stats[2] += i.y;
        stats[3] += i.w;
        stats[4] += i.z;
    }
    return VTX_OK;
}

int vtx_tissue_get_topology(vtx_tissue t, int32_t *he_out) {
    if (!t || !he_out) return fail(VTX_E_ARG, "null argument");
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(he_out, t->d.he, 8 * sizeof(int32_t) * t->n_he, hipMemcpyDeviceToHost));
    return VTX_OK;
}

int vtx_tissue_set_topology(vtx_tissue t, const int32_t *he) {
    if (!t || !he) return fail(VTX_E_ARG, "null argument");
    Staged S;
    int rc = validate_and_stage(he, t->n_he, t->n_vert, t->n_cell, S);
    if (rc) return rc;
    if ((int64_t)S.edge_he.size() != t->n_edge) return fail(VTX_E_TOPOLOGY, "edge count changed");
    HIPCHK(hipDeviceSynchronize());
    std::vector<int32_t> hev(he, he + 8 * t->n_he);
    DevTissue &d = t->d;
    if ((rc = upload_into(d.he, hev)) || (rc = upload_into(d.he_edge, S.he_edge)) ||
        (rc = upload_into(d.edge_he, S.edge_he)) || (rc = upload_into(d.row_ptr, S.row_ptr)) ||
        (rc = upload_into(d.row_cap, S.row_cap)) ||
        (rc = upload_into(d.pool_top, std::vector<int32_t>{d.pool_start})) ||
        (rc = upload_into(d.corner, S.corner)) || (rc = upload_into(d.corner_he, S.corner_he)) ||
        (rc = upload_into(d.nsides, S.nsides)) || (rc = upload_into(d.cell_he, S.cell_he)) ||
        (rc = upload_into(d.star, S.star)) || (rc = upload_into(d.star_he, S.star_he)))
        return rc;
    // synchronous like the uploads: the tables are complete on return, for
    // callers on any stream
    if ((rc = vtx::tissue_topology_changed(t, nullptr))) return rc;
    HIPCHK(hipDeviceSynchronize());
    return VTX_OK;
}

int vtx_energy_forces(vtx_tissue t, int32_t mode, const void *X, const vtx_params *p,
                      double *E_dev, void *F, double *maxf_dev, void *stream) {
    if (!t || !X || !p || !mode_ok(mode)) return fail(VTX_E_ARG, "bad argument");
    launch_eval_fused(t->d, t->w, t->tiles, mode, X, raw(p), E_dev, F, maxf_dev,
                      (hipStream_t)stream);
    return check_launch("vtx_energy_forces");
}

}  // extern "C"

namespace {
// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept; NULL on failure.
unsigned char *noalloc_scratch(int *err) {
    static std::mutex mu;
    static unsigned char *addr[64] = {nullptr};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= 64) {
        *err = fail(VTX_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            *err = fail(VTX_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return nullptr;
        }
        addr[dev] = (unsigned char *)ptr;
    }
    return addr[dev];
}
}  // namespace

extern "C" {

int vtx_energy_forces_noalloc(vtx_tissue t, int32_t mode, const void *X, const vtx_params *p,
                              double *E_dev, void *F, double *maxf_dev, void *stream) {
    if (!t || !X || !p || !mode_ok(mode)) return fail(VTX_E_ARG, "bad argument");
    if (t->n_vert > kNoAllocVerts)
        return fail(VTX_E_CAPACITY,
                    "vtx_energy_forces_noalloc: %lld vertices exceed its fixed scratch (at most "
                    "%lld vertices)",
                    (long long)t->n_vert, (long long)kNoAllocVerts);
    int rc = VTX_OK;
    unsigned char *base = noalloc_scratch(&rc);
    if (!base) return rc;
    hipStream_t s = (hipStream_t)stream;
    Workspace w{};
    w.mpart = (double *)base;
    w.ctl = (LoopCtl *)(base + kNoAllocCtlOffset);
    hipLaunchKernelGGL(k_clear_ctl, dim3(1), dim3(64), 0, s, w.ctl);
    launch_eval_fused(t->d, w, t->tiles, mode, X, raw(p), E_dev, F, maxf_dev, s);
    return check_launch("vtx_energy_forces_noalloc");
}

int vtx_cell_coeffs(vtx_tissue t, int32_t mode, const void *X, const vtx_params *p,
                    void *coeffs, void *stream) {
    if (!t || !X || !p || !coeffs || !mode_ok(mode)) return fail(VTX_E_ARG, "bad argument");
    launch_cell_pass(t->d, t->w, mode, X, raw(p), coeffs, (hipStream_t)stream);
    return check_launch("vtx_cell_coeffs");
}

int vtx_vertex_forces(vtx_tissue t, int32_t mode, const void *X, const vtx_params *p,
                      const void *coeffs, void *F, double *maxf_dev, void *stream) {
    if (!t || !X || !p || !coeffs || !mode_ok(mode)) return fail(VTX_E_ARG, "bad argument");
    launch_vertex_pass(t->d, t->w, mode, X, raw(p), coeffs, F, maxf_dev, (hipStream_t)stream);
    return check_launch("vtx_vertex_forces");
}

int vtx_cell_geometry(vtx_tissue t, int32_t mode, const void *X, double *A_dev, double *P_dev,
                      void *stream) {
    if (!t || !X || !mode_ok(mode)) return fail(VTX_E_ARG, "bad argument");
    launch_cell_exact(t->d, mode, X, A_dev, P_dev, (hipStream_t)stream);
    return check_launch("vtx_cell_geometry");
}

int vtx_edge_lengths(vtx_tissue t, int32_t mode, const void *X, double *len_dev, void *stream) {
    if (!t || !X || !len_dev || !mode_ok(mode)) return fail(VTX_E_ARG, "bad argument");
    launch_edge_len(t->d, mode, X, len_dev, (hipStream_t)stream);
    return check_launch("vtx_edge_lengths");
}

int vtx_relax(vtx_tissue t, int32_t mode, void *X, const vtx_params *p, const vtx_relax_opts *o,
              vtx_relax_result *res, void *stream) {
    if (!t || !X || !p || !o || !mode_ok(mode)) return fail(VTX_E_ARG, "bad argument");
    return relax_impl(t, mode, X, p, o, res, (hipStream_t)stream);
}

int vtx_t1(vtx_tissue t, int32_t mode, void *X, const vtx_params *p, double l_min, double l_new,
           int64_t *n_swap, int64_t *n_stretch, void *stream) {
    if (!t || !X || !p || !mode_ok(mode)) return fail(VTX_E_ARG, "bad argument");
    if (!(l_min > 0) || !(l_new > 0)) return fail(VTX_E_ARG, "l_min and l_new must be > 0");
    hipStream_t s = (hipStream_t)stream;
    LoopCtl z{};
    int rc = reset_ctl(t, 1, z, s);
    if (rc) return rc;
    launch_t1(t->d, t->w, mode, X, raw(p), l_min, l_new, s);
    if ((rc = check_launch("vtx_t1"))) return rc;
    if ((rc = vtx::tissue_topology_changed(t, s))) return rc;
    if ((rc = read_ctl(t, 1, s))) return rc;
    const LoopCtl h = t->w.ctl_host[1];
    if (n_swap) *n_swap = h.n_t1;
    if (n_stretch) *n_stretch = h.n_stretch;
    LoopCtl z2{};  // the evaluation control block must never stay `done`
    if ((rc = reset_ctl(t, 1, z2, s))) return rc;
    if (h.t1_overflow) return fail(VTX_E_CAPACITY, "T1 pass overflow (%d)", h.t1_overflow);
    return VTX_OK;
}

int vtx_hvp(vtx_tissue t, int32_t mode, const void *X, const vtx_params *p, const double *v,
            double *Hv, void *stream) {
    if (!t || !X || !p || !v || !Hv || !mode_ok(mode)) return fail(VTX_E_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    launch_cell_coeffs(t->d, t->w, mode, X, raw(p), s);
    launch_hvp(t->d, t->w, mode, X, raw(p), v, Hv, nullptr, nullptr, s);
    return check_launch("vtx_hvp");
}

int vtx_v2v(vtx_tissue t, int32_t mode, const void *X, const void *X_target, double *C_dev,
            double *grad, void *stream) {
    if (!t || !X || !X_target || !mode_ok(mode)) return fail(VTX_E_ARG, "bad argument");
    launch_v2v(t->d, t->w, mode, X, X_target, C_dev, grad, (hipStream_t)stream);
    return check_launch("vtx_v2v");
}

// Solves H x = P b at X (H restricted to the zero-mean subspace) by CG or
// MINRES on the device, x left projected in the first workspace vector.
static int solve_hessian(vtx_tissue t, int mode, const void *X, const vtx_params *p,
                         const double *b, bool minres, double tol, int64_t max_iter,
                         hipStream_t s, vtx_grad_result *r) {
    const int nv = (int)t->n_vert;
    launch_cell_coeffs(t->d, t->w, mode, X, raw(p), s);
    LoopCtl c{};
    c.status = VTX_CG_MAXITER;
    c.tol = tol;
    c.max_iter = max_iter;
    c.solver = minres ? 1 : 0;
    int rc;
    if ((rc = reset_ctl(t, 0, c, s))) return rc;
    if (minres) launch_minres_init(t->w, nv, b, s);
    else launch_cg_init(t->w, nv, b, s);
    if ((rc = check_launch("Krylov init"))) return rc;
    if ((rc = read_ctl(t, 0, s))) return rc;
    if (!t->w.ctl_host[0].done) {
        rc = run_loop(t, 32, max_iter, s, [&](int, hipStream_t cs) {
            if (minres) launch_minres_iter(t->d, t->w, mode, X, raw(p), cs);
            else launch_cg_iter(t->d, t->w, mode, X, raw(p), cs);
        });
        if (rc) return rc;
    }
    const LoopCtl &h = t->w.ctl_host[0];
    launch_project(t->w, nv, t->w.cg, s);
    r->cg_iters = h.cg_iter;
    r->cg_rel_res = h.rel_res;
    r->status = h.status;
    return check_launch("Krylov solve");
}

int vtx_param_grad(vtx_tissue t, int32_t mode, const void *X_star, const vtx_params *p,
                   const double *dC_dX, const void *X_target, const vtx_grad_opts *o,
                   double *dC_dtheta, vtx_grad_result *res, void *stream) {
    if (!t || !X_star || !p || !o || !dC_dtheta || !mode_ok(mode))
        return fail(VTX_E_ARG, "bad argument");
    if (o->theta != VTX_THETA_LAMBDA && o->theta != VTX_THETA_P0)
        return fail(VTX_E_ARG, "unknown theta selector");
    hipStream_t s = (hipStream_t)stream;
    vtx_grad_result r{};
    int rc;
    if (o->method == VTX_GRAD_ADJOINT || o->method == VTX_GRAD_ADJOINT_MINRES) {
        if (!dC_dX) return fail(VTX_E_ARG, "the adjoint needs dC_dX");
        if (!(o->cg_tol > 0) || o->cg_max_iter < 1) return fail(VTX_E_ARG, "bad Krylov options");
        if ((rc = solve_hessian(t, mode, X_star, p, dC_dX, o->method == VTX_GRAD_ADJOINT_MINRES,
                                o->cg_tol, o->cg_max_iter, s, &r)))
            return rc;
        launch_contract(t->d, mode, X_star, raw(p), o->theta, t->w.cg, dC_dtheta, s);
        if ((rc = check_launch("adjoint contraction"))) return rc;
        HIPCHK(hipStreamSynchronize(s));
    } else if (o->method == VTX_GRAD_EP_CENTRED || o->method == VTX_GRAD_EP_FORWARD) {
        const bool centred = o->method == VTX_GRAD_EP_CENTRED;
        if (!(o->beta != 0.0)) return fail(VTX_E_ARG, "EP needs beta != 0");
        if (o->ep_relax.t1_enable) return fail(VTX_E_ARG, "EP relaxations cannot use T1");
        if (!X_target && !dC_dX) return fail(VTX_E_ARG, "EP needs X_target or dC_dX");
        const size_t pb = pos_bytes(t, mode);
        char *Xp = (char *)t->ep_buf, *Xm = Xp + 16 * (size_t)t->n_vert;
        HIPCHK(hipMemcpyAsync(Xp, X_star, pb, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(Xm, X_star, pb, hipMemcpyDeviceToDevice, s));
        vtx_relax_opts ro = o->ep_relax;
        ro.X_target = X_target;
        ro.g_lin = X_target ? nullptr : dC_dX;
        ro.beta = centred ? 0.5 * o->beta : o->beta;
        if ((rc = relax_impl(t, mode, Xp, p, &ro, &r.ep_plus, s))) return rc;
        if (centred) {
            ro.beta = -0.5 * o->beta;
            if ((rc = relax_impl(t, mode, Xm, p, &ro, &r.ep_minus, s))) return rc;
        }
        launch_ep(t->d, mode, Xp, Xm, raw(p), o->theta, o->beta, dC_dtheta, s);
        if ((rc = check_launch("EP estimate"))) return rc;
        HIPCHK(hipStreamSynchronize(s));
        r.status = combine_status(r.ep_plus.status, r.ep_minus.status);
    } else {
        return fail(VTX_E_ARG, "unknown hypergradient method");
    }
    if (res) *res = r;
    return VTX_OK;
}

int vtx_param_sens(vtx_tissue t, int32_t mode, const void *X_star, const vtx_params *p,
                   const double *d, const double *dC_dX, const vtx_grad_opts *o, double *dC_dd,
                   double *dX_dd, vtx_grad_result *res, void *stream) {
    if (!t || !X_star || !p || !d || !dC_dX || !o || !dC_dd || !mode_ok(mode))
        return fail(VTX_E_ARG, "bad argument");
    if (mode == VTX_F32) return fail(VTX_E_ARG, "sensitivities need double positions");
    if (o->theta != VTX_THETA_LAMBDA && o->theta != VTX_THETA_P0)
        return fail(VTX_E_ARG, "unknown theta selector");
    if (!(o->cg_tol > 0) || o->cg_max_iter < 1) return fail(VTX_E_ARG, "bad CG options");
    hipStream_t s = (hipStream_t)stream;
    const int nv = (int)t->n_vert;
    double *rhs = t->ep_buf;  // [n_vert][2]
    launch_sens_rhs(t->d, t->w, X_star, raw(p), o->theta, d, rhs, s);
    vtx_grad_result r{};
    int rc = solve_hessian(t, mode, X_star, p, rhs, o->method == VTX_GRAD_ADJOINT_MINRES,
                           o->cg_tol, o->cg_max_iter, s, &r);
    if (rc) return rc;
    launch_dot_pos(t->w, VTX_F64, nv, dC_dX, t->w.cg, dC_dd, s);
    if (dX_dd)
        HIPCHK(hipMemcpyAsync(dX_dd, t->w.cg, 16 * (size_t)nv, hipMemcpyDeviceToDevice, s));
    if ((rc = check_launch("sensitivity"))) return rc;
    HIPCHK(hipStreamSynchronize(s));
    if (res) *res = r;
    return VTX_OK;
}

}  // extern "C"
