// Host side of libiblb: the C ABI declared in include/iblb.h.
//
// Responsibilities: argument and mesh validation, device memory layout
// (one workspace carved into 256-byte aligned arrays), per-face reference data
// and the vertex -> (face, corner) table, step scheduling (plain launches,
// a captured hipGraph of one step, or launches bracketed by hipEvents), the
// FP64 solves behind the shape and contact-angle queries, and checkpoints.
// All arithmetic of the step itself runs in the kernels of iblb_kernels.hip.
#include "iblb.h"
#include "iblb_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

using namespace iblb;

namespace {

constexpr char kMagic[8] = {'I', 'B', 'L', 'B', 'S', 'T', '0', '1'};
constexpr int kNumKernels = 5;
constexpr int kGraphSteps = 16;  // steps per captured graph (even)
const char *const kKernelNames[kNumKernels] = {"forces", "spread", "moments", "move", "lb"};
enum { K_FORCES = 0, K_SPREAD = 1, K_MOMENTS = 2, K_MOVE = 3, K_LB = 4 };

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct Layout {
    // byte offsets into the workspace; domain part then mesh part
    size_t f, F, stamp, ctr, err, scratch, dom_end;
    size_t q, Xref, faces, fref, inc4, U, phiSW, gV, base, wts, partials, mask, act, acnt, alist, mesh_end;
};

size_t pop_bytes(int precision) { return precision == IBLB_FP64 ? 8 : (precision == IBLB_FP32_DEV ? 4 : 2); }

// Population pitch: each population's array rounded up to 256 bytes plus
// 3 KB, so that the 19 arrays do not start at addresses that agree modulo a
// large power of two.  Measured on k_lb beyond the Infinity Cache (median of
// three, GB/s, pad 0 / 1 / 2 / 3 KB / 256 KB + 128 B / 256 KB + 1 KB), FP32:
// 256^3 with walls 3946 / 4813 / 4613 / 5056 / 4792 / 5026, 128x512x256
// 3810 / 5078 / 5225 / 5233 / 5033 / 4911, 512x256x128 4787 / 5177 / 4753 /
// 5123 / 4889 / 5118; FP16 256^3 3710 / 4351 / 4251 / 4389 / 4816 / 4432;
// the 128x128x96 lattice, inside the cache, is unchanged (7628 / 7593 at 3 KB).
long long population_pitch(long long n, size_t ps)
{
    const long long bytes = (n * (long long)ps + 255) / 256 * 256 + 3072;
    return bytes / (long long)ps;
}

Grid make_grid(const iblb_domain_desc &d)
{
    Grid g;
    g.nx = d.nx;
    g.ny = d.ny;
    g.nz = d.nz;
    g.walls = d.wall_mode == IBLB_WALLS_Z ? 1 : 0;
    g.zoff = g.walls;
    g.nzf = g.walls ? d.nz - 2 : d.nz;
    g.n = (long long)g.nx * g.ny * g.nzf;
    g.ntx = (g.nx + kTileX - 1) >> kTileLX;
    g.nty = (g.ny + kTileY - 1) >> kTileLY;
    g.ntz = (g.nzf + kTileZ - 1) >> kTileLZ;
    g.nt = g.ntx * g.nty * g.ntz;
    g.pp = population_pitch(g.n, pop_bytes(d.precision));
    return g;
}

// Incidence slots per vertex: 8 x ceil(max valence / 8), so that the eight
// lanes of a vertex in the force kernel find its entries at fixed positions.
int incidence_slots(const iblb_mesh_desc *m)
{
    if (!m || !m->faces || m->n_vertices <= 0 || m->n_faces <= 0) return 8;
    std::vector<int> val((size_t)m->n_vertices, 0);
    int mx = 0;
    for (int j = 0; j < 3 * m->n_faces; ++j) {
        const int v = m->faces[j];
        if (v >= 0 && v < m->n_vertices) mx = std::max(mx, ++val[v]);
    }
    return 8 * std::max(1, (mx + 7) / 8);
}

// ps: bytes per stored population; ts: bytes per value of the other
// per-node and per-vertex fields (F, U, vertex forces and weights)
Layout make_layout(const Grid &g, size_t ps, size_t ts, int nv, int nf, int slots)
{
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.f = take(19 * (size_t)g.pp * ps);
    L.F = take(3 * (size_t)g.n * ts);
    L.stamp = take((size_t)g.nt * 4);
    L.ctr = take(2 * 4);
    L.err = take(4);
    L.scratch = take(64 * 8);
    L.dom_end = o;
    const int nparts = (nv + 31) / 32;
    L.q = take((size_t)3 * nv * 8);
    L.Xref = take((size_t)3 * nv * 8);
    L.faces = take((size_t)3 * nf * 4);
    L.fref = take((size_t)5 * nf * 8);
    L.inc4 = take((size_t)nv * slots * 16);
    L.U = take(nv ? (size_t)4 * g.n * ts : 0);
    L.phiSW = take((size_t)3 * nv * ts);
    L.gV = take((size_t)3 * nv * ts);
    L.base = take((size_t)nv * sizeof(Base));
    L.wts = take((size_t)12 * nv * ts);
    L.partials = take((size_t)nparts * 8);
    L.mask = take((size_t)g.nt * ((nv + 63) / 64) * 8);
    L.act = take((size_t)(g.nt + 4095) / 4096 * 4096);
    L.acnt = take(2 * 4);
    L.alist = take((size_t)g.nt * 4);
    L.mesh_end = o;
    return L;
}

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }


}  // namespace

struct iblb_ctx {
    iblb_domain_desc dom;
    int prec = 0;
    size_t ps = 8;  // bytes per stored population
    size_t ts = 8;  // bytes per value of the other fields
    Grid g;
    LBArgs lb;
    MeshArgs m;
    Dev d;
    Layout L;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;  // the device current at creation, which holds the workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    bool has_mesh = false;
    int nv = 0, nf = 0;
    double V0 = 0.0;
    long long t = 0;
    bool use_graph = true;
    // captured steps: [start parity][0: kGraphSteps steps, 1: one step]
    hipGraph_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    bool timing = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> pool;
    double ktime[kNumKernels] = {0, 0, 0, 0, 0};
    long long kcount[kNumKernels] = {0, 0, 0, 0, 0};
    void *fext_alloc = nullptr;
    void *mesh_alloc = nullptr;
    struct AdjState *adj = nullptr;  // recorded window of the adjoint, if any
    std::string err;
};

namespace {
void free_adjoint(iblb_ctx *c);

int fail(iblb_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

int hip_fail(iblb_ctx *c, hipError_t e, const char *what)
{
    return fail(c, IBLB_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(c, expr)                                   \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_fail(c, e_, #expr); \
    } while (0)

int check_domain(const iblb_domain_desc *d, std::string &why)
{
    if (!d) { why = "null domain"; return IBLB_E_INVAL; }
    if (d->nx < 8 || d->ny < 8 || d->nz < 8) { why = "nx, ny, nz must be >= 8"; return IBLB_E_INVAL; }
    if ((long long)d->nx * d->ny * d->nz > (1ll << 31)) { why = "lattice too large"; return IBLB_E_INVAL; }
    if (19ll * population_pitch((long long)d->nx * d->ny * d->nz, pop_bytes(d->precision)) *
            (long long)pop_bytes(d->precision) >= (1ll << 32)) {
        why = "lattice too large: the populations must fit in 4 GiB (19 x nodes x bytes per population)";
        return IBLB_E_INVAL;
    }
    if (d->wall_mode != IBLB_WALLS_Z && d->wall_mode != IBLB_PERIODIC_ALL) { why = "bad wall_mode"; return IBLB_E_INVAL; }
    if (d->precision < IBLB_FP64 || d->precision > IBLB_BF16_DEV) { why = "bad precision"; return IBLB_E_INVAL; }
    if (!(d->tau > 0.5) || !std::isfinite(d->tau)) { why = "tau must be > 1/2"; return IBLB_E_INVAL; }
    if (!(d->rho0 > 0.0) || !std::isfinite(d->rho0)) { why = "rho0 must be > 0"; return IBLB_E_INVAL; }
    if (!finite3(d->u_wall_lo) || !finite3(d->u_wall_hi) || !finite3(d->body_force)) {
        why = "non-finite wall velocity or body force";
        return IBLB_E_INVAL;
    }
    if (d->u_wall_lo[2] != 0.0 || d->u_wall_hi[2] != 0.0) { why = "wall velocities must be tangential"; return IBLB_E_INVAL; }
    return IBLB_OK;
}

int check_mesh(const iblb_mesh_desc *m, std::string &why)
{
    if (!m || !m->vertices || !m->faces) { why = "null mesh arrays"; return IBLB_E_INVAL; }
    if (m->n_vertices < 4 || m->n_faces < 4) { why = "mesh too small"; return IBLB_E_MESH; }
    if (m->n_vertices > kMaxVertices || m->n_faces > (1 << 28)) { why = "mesh too large (at most 65536 vertices)"; return IBLB_E_INVAL; }
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(m->alpha[k])) { why = "non-finite alpha"; return IBLB_E_INVAL; }
    if (!std::isfinite(m->k_v) || !std::isfinite(m->eps_wall_lo) || !std::isfinite(m->eps_wall_hi) ||
        !(m->xi_wall > 0.0) || !std::isfinite(m->r_cut_wall)) {
        why = "bad volume or wall parameters";
        return IBLB_E_INVAL;
    }
    const int nv = m->n_vertices, nf = m->n_faces;
    for (int i = 0; i < nv; ++i) {
        if (!finite3(m->vertices + 3 * i) || std::fabs(m->vertices[3 * i]) > 1e6 ||
            std::fabs(m->vertices[3 * i + 1]) > 1e6 || std::fabs(m->vertices[3 * i + 2]) > 1e6) {
            why = "vertex " + std::to_string(i) + " not finite or beyond 1e6";
            return IBLB_E_INVAL;
        }
        if (m->ref_vertices && !finite3(m->ref_vertices + 3 * i)) { why = "non-finite reference vertex"; return IBLB_E_INVAL; }
    }
    // closed, consistently oriented 2-manifold: each directed edge once, with its reverse
    std::unordered_map<unsigned long long, int> edges;
    edges.reserve((size_t)nf * 4);
    for (int j = 0; j < nf; ++j) {
        const int *f = m->faces + 3 * j;
        for (int c = 0; c < 3; ++c)
            if (f[c] < 0 || f[c] >= nv) { why = "face " + std::to_string(j) + " index out of range"; return IBLB_E_MESH; }
        if (f[0] == f[1] || f[1] == f[2] || f[0] == f[2]) { why = "degenerate face " + std::to_string(j); return IBLB_E_MESH; }
        for (int c = 0; c < 3; ++c) {
            const unsigned long long key = ((unsigned long long)f[c] << 32) | (unsigned)f[(c + 1) % 3];
            if (++edges[key] > 1) { why = "edge used twice in the same direction (orientation)"; return IBLB_E_MESH; }
        }
    }
    for (const auto &kv : edges) {
        const unsigned long long rev = ((kv.first & 0xffffffffull) << 32) | (kv.first >> 32);
        if (edges.find(rev) == edges.end()) { why = "mesh is not closed"; return IBLB_E_MESH; }
    }
    return IBLB_OK;
}

void lb_args(iblb_ctx *c)
{
    LBArgs &a = c->lb;
    a.g = c->g;
    a.tau_inv = 1.0 / c->dom.tau;
    a.guo = 1.0 - 1.0 / (2.0 * c->dom.tau);
    a.rho0 = c->dom.rho0;
    for (int k = 0; k < 3; ++k) {
        a.body[k] = c->dom.body_force[k];
        a.ulo[k] = c->dom.u_wall_lo[k];
        a.uhi[k] = c->dom.u_wall_hi[k];
    }
    a.has_fext = c->d.Fext != nullptr;
}

void drop_graph(iblb_ctx *c)
{
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k < 2; ++k) {
            if (c->gexec[p][k]) (void)hipGraphExecDestroy(c->gexec[p][k]);
            if (c->graph[p][k]) (void)hipGraphDestroy(c->graph[p][k]);
            c->gexec[p][k] = nullptr;
            c->graph[p][k] = nullptr;
        }
}

hipEvent_t get_event(iblb_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

hipError_t launch_kernel(iblb_ctx *c, int which, int p, hipStream_t st)
{
    const Dev &d = c->d;
    switch (which) {
    case K_FORCES: return launch_forces(c->prec, d, c->lb, c->m, p, 1, st);
    case K_SPREAD: return launch_spread(c->prec, d, c->lb, c->m, p, 1, st);
    case K_MOMENTS: return launch_moments(c->prec, d, c->lb, c->m, p, st);
    case K_MOVE: return launch_move(c->prec, d, c->lb, c->m, p, st);
    default: return launch_lb(c->prec, d, c->lb, p, 0, st);
    }
}

// One step of parity p.  With a mesh, four dispatches: the interface forces
// and the list of active tiles; the spreading onto the active tiles (force +
// their LB); the moments of the active tiles; the interpolation and move.
// The LB of all other nodes runs in the first two, split between them.
// Without a mesh, the LB alone.  Timed steps bracket each dispatch with
// hipEvents (the same launches otherwise).
hipError_t enqueue_step(iblb_ctx *c, int p, bool timed)
{
    static const int with_mesh[4] = {K_FORCES, K_SPREAD, K_MOMENTS, K_MOVE};
    static const int no_mesh[1] = {K_LB};
    const int *seq = c->has_mesh ? with_mesh : no_mesh;
    const int ns = c->has_mesh ? 4 : 1;
    for (int k = 0; k < ns; ++k) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timed) {
            e0 = get_event(c);
            e1 = get_event(c);
            (void)hipEventRecord(e0, c->stream);
        }
        hipError_t e = launch_kernel(c, seq[k], p, c->stream);
        if (e != hipSuccess) return e;
        if (timed) {
            (void)hipEventRecord(e1, c->stream);
            c->pending.push_back({seq[k], {e0, e1}});
        }
    }
    return hipSuccess;
}

// Captures the graph of kGraphSteps steps (which = 0) or of one step
// (which = 1) from a time of parity p, if not yet captured: every kernel
// reads the step from the device counter, so a graph replays at any later
// time of the same parity.
int capture_steps(iblb_ctx *c, int p, int which)
{
    if (c->gexec[p][which]) return IBLB_OK;
    const int steps = which == 0 ? kGraphSteps : 1;
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < steps && e == hipSuccess; ++k) e = enqueue_step(c, (p + k) & 1, false);
    hipGraph_t gr = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->stream, &gr);
    if (e != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return hip_fail(c, e, "step capture");
    }
    if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
    c->graph[p][which] = gr;
    HIP_TRY(c, hipGraphInstantiate(&c->gexec[p][which], gr, nullptr, nullptr, 0));
    return IBLB_OK;
}

int capture_all(iblb_ctx *c)
{
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k < 2; ++k) {
            int rc = capture_steps(c, p, k);
            if (rc) return rc;
        }
    return IBLB_OK;
}

int collect_timing(iblb_ctx *c)
{
    if (c->pending.empty()) return IBLB_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto &p : c->pending) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, p.second.first, p.second.second);
        c->ktime[p.first] += ms;
        c->kcount[p.first] += 1;
        c->pool.push_back(p.second.first);
        c->pool.push_back(p.second.second);
    }
    c->pending.clear();
    return IBLB_OK;
}

std::string err_text(int e)
{
    std::string why = "device reported:";
    if (e & kErrNonFinite) why += " non-finite vertex position;";
    if (e & kErrOverflow) why += " tile list overflow (vertex pile-up);";
    if (e & kErrDensity) why += " density out of range or non-finite;";
    if (e & kErrMach) why += " |u| above 0.3;";
    if (e & kErrList) why += " invalid vertex index in a tile list;";
    return why;
}

int read_err(iblb_ctx *c)
{
    int e = 0;
    HIP_TRY(c, hipMemcpy(&e, c->d.err, sizeof(int), hipMemcpyDeviceToHost));
    if (e) return fail(c, IBLB_E_UNSTABLE, err_text(e));
    return IBLB_OK;
}

int sync_ctx(iblb_ctx *c)
{
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return read_err(c);
}

// temporary device buffer for debug / query copies
struct TmpDev {
    void *p = nullptr;
    ~TmpDev() { if (p) (void)hipFree(p); }
};

// Tiles holding a fluid node of some vertex's 4^3 stencil at the stored
// positions: sizes the moments launch (the kernels do not depend on it).
int count_active_tiles(iblb_ctx *c, int *out)
{
    std::vector<double> q((size_t)3 * c->nv);
    HIP_TRY(c, hipMemcpyAsync(q.data(), c->d.q, q.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const Grid &g = c->g;
    std::vector<char> on((size_t)g.nt, 0);
    auto wrap = [](long long a, int n) { long long r = a % n; return (int)(r < 0 ? r + n : r); };
    for (int v = 0; v < c->nv; ++v) {
        const double p[3] = {q[v], q[(size_t)c->nv + v], q[(size_t)2 * c->nv + v]};
        if (!(std::fabs(p[0]) < 1e6 && std::fabs(p[1]) < 1e6 && std::fabs(p[2]) < 1e6)) continue;
        const long long b[3] = {(long long)std::floor(p[0]) - 1, (long long)std::floor(p[1]) - 1,
                                (long long)std::floor(p[2]) - 1};
        for (int k = 0; k < 64; ++k) {
            const int x = wrap(b[0] + (k & 3), g.nx), y = wrap(b[1] + ((k >> 2) & 3), g.ny);
            long long zf = b[2] + (k >> 4);
            if (g.walls) {
                zf -= g.zoff;
                if (zf < 0 || zf >= g.nzf) continue;
            } else {
                zf = wrap(zf, g.nz);
            }
            on[((size_t)(zf >> kTileLZ) * g.nty + (y >> kTileLY)) * g.ntx + (x >> kTileLX)] = 1;
        }
    }
    int n = 0;
    for (char x : on) n += x;
    *out = n;
    return IBLB_OK;
}

// Clears the vertex masks and activity stamps, then sets both for the current
// step from the stored positions (each step sets them for the next one).
int rebuild_lists(iblb_ctx *c)
{
    int rc = count_active_tiles(c, &c->m.tiles_hint);
    if (rc) return rc;
    HIP_TRY(c, hipMemsetAsync(c->d.mask, 0, (size_t)c->g.nt * c->m.nwords * 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->d.act, 0, (size_t)(c->g.nt + 4095) / 4096 * 4096, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->d.acnt, 0, 2 * 4, c->stream));
    HIP_TRY(c, launch_stamp(c->d, c->g, c->m, (int)(c->t & 1), c->stream));
    return IBLB_OK;
}

int mesh_ok(iblb_ctx *c, int32_t mesh_id)
{
    if (!c) return IBLB_E_INVAL;
    if (!c->has_mesh) return fail(c, IBLB_E_STATE, "no mesh attached");
    if (mesh_id != 0) return fail(c, IBLB_E_INVAL, "mesh_id must be 0");
    return IBLB_OK;
}

}  // namespace

namespace iblb {
int get_fields_staged(iblb_ctx *c, double *staging, double *rho, double *u)
{
    int rc = sync_ctx(c);
    if (rc == IBLB_E_DEVICE) return rc;
    const size_t n = (size_t)c->g.n;
    double *dr = staging, *du = staging + n;
    HIP_TRY(c, launch_get_fields(c->prec, c->d, c->lb, (int)(c->t & 1), dr, du, c->stream));
    HIP_TRY(c, hipMemcpyAsync(rho, dr, n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(u, du, 3 * n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return rc;
}

long long ctx_fluid_nodes(const iblb_ctx *c) { return (long long)c->g.n; }
int ctx_device(const iblb_ctx *c) { return c->device; }
int ctx_fail(iblb_ctx *c, int code, const char *msg) { return fail(c, code, msg); }
}  // namespace iblb

extern "C" {

int iblb_workspace_bytes(const iblb_domain_desc *dom, const iblb_mesh_desc *mesh, size_t *bytes)
{
    std::string why;
    if (!bytes) return IBLB_E_INVAL;
    int rc = check_domain(dom, why);
    if (rc) return rc;
    const Grid g = make_grid(*dom);
    const size_t ts = dom->precision == IBLB_FP64 ? 8 : 4;
    const size_t ps = pop_bytes(dom->precision);
    if (mesh && (mesh->n_vertices < 0 || mesh->n_faces < 0 || (mesh->n_faces > 0 && !mesh->faces))) return IBLB_E_INVAL;
    const Layout L = make_layout(g, ps, ts, mesh ? mesh->n_vertices : 0, mesh ? mesh->n_faces : 0,
                                 incidence_slots(mesh));
    *bytes = mesh ? L.mesh_end : L.dom_end;
    return IBLB_OK;
}

int iblb_create(const iblb_domain_desc *dom, void *dev_workspace, size_t workspace_bytes, void *hip_stream,
                iblb_ctx **out)
{
    if (!out) return IBLB_E_INVAL;
    *out = nullptr;
    std::string why;
    int rc = check_domain(dom, why);
    if (rc) return rc;
    iblb_ctx *c = new iblb_ctx();
    c->dom = *dom;
    c->prec = dom->precision;
    c->ts = c->prec == IBLB_FP64 ? 8 : 4;
    c->ps = pop_bytes(c->prec);
    c->g = make_grid(*dom);
    c->L = make_layout(c->g, c->ps, c->ts, 0, 0, 8);
    auto bail = [&](int code) {
        iblb_destroy(c);
        return code;
    };
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return bail(IBLB_E_DEVICE);
        c->own_stream = true;
    }

    if (dev_workspace) {
        if (workspace_bytes < c->L.dom_end) return bail(IBLB_E_INVAL);
        c->ws = (char *)dev_workspace;
        c->ws_bytes = workspace_bytes;
    } else {
        void *p = nullptr;
        if (hipMalloc(&p, c->L.dom_end) != hipSuccess) return bail(IBLB_E_DEVICE);
        c->ws = (char *)p;
        c->ws_bytes = c->L.dom_end;
        c->own_ws = true;
    }
    Dev &d = c->d;
    std::memset(&d, 0, sizeof(d));
    d.f = c->ws + c->L.f;
    d.F = c->ws + c->L.F;
    d.stamp = (uint32_t *)(c->ws + c->L.stamp);
    d.ctr = (uint32_t *)(c->ws + c->L.ctr);
    d.err = (int *)(c->ws + c->L.err);
    d.scratch = (double *)(c->ws + c->L.scratch);
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            return bail(IBLB_E_DEVICE);
        d.num_cus = cus;
        c->device = dev;
        noalloc_setup(dev);
    }
    lb_args(c);
    if (hipMemsetAsync(c->ws + c->L.stamp, 0, c->L.dom_end - c->L.stamp, c->stream) != hipSuccess ||
        hipMemsetAsync(d.F, 0, 3 * (size_t)c->g.n * c->ts, c->stream) != hipSuccess ||
        launch_init(c->prec, d, c->lb, dom->init_couette, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return bail(IBLB_E_DEVICE);
    *out = c;
    return IBLB_OK;
}

int iblb_add_mesh(iblb_ctx *c, const iblb_mesh_desc *mesh, int32_t *mesh_id)
{
    if (!c) return IBLB_E_INVAL;
    if (c->has_mesh) return fail(c, IBLB_E_STATE, "a mesh is already attached (one per context)");
    if (c->d.Fext) return fail(c, IBLB_E_STATE, "debug force field set: no mesh allowed");
    std::string why;
    int rc = check_mesh(mesh, why);
    if (rc) return fail(c, rc, why);
    const int nv = mesh->n_vertices, nf = mesh->n_faces;
    const double *X = mesh->ref_vertices ? mesh->ref_vertices : mesh->vertices;

    // reference geometry in FP64
    double o[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < nv; ++i)
        for (int k = 0; k < 3; ++k) o[k] += X[3 * i + k];
    for (int k = 0; k < 3; ++k) o[k] /= nv;
    std::vector<double> fref((size_t)5 * nf);
    double V0 = 0.0;
    for (int j = 0; j < nf; ++j) {
        const int *f = mesh->faces + 3 * j;
        const double *a = X + 3 * f[0], *b = X + 3 * f[1], *cc = X + 3 * f[2];
        double E1[3], E2[3];
        for (int k = 0; k < 3; ++k) {
            E1[k] = b[k] - a[k];
            E2[k] = cc[k] - a[k];
        }
        const double G11 = E1[0] * E1[0] + E1[1] * E1[1] + E1[2] * E1[2];
        const double G12 = E1[0] * E2[0] + E1[1] * E2[1] + E1[2] * E2[2];
        const double G22 = E2[0] * E2[0] + E2[1] * E2[1] + E2[2] * E2[2];
        const double det = G11 * G22 - G12 * G12;
        if (!(det > 0.0) || !std::isfinite(det)) return fail(c, IBLB_E_MESH, "degenerate reference face " + std::to_string(j));
        fref[j] = G22 / det;
        fref[(size_t)nf + j] = -G12 / det;
        fref[(size_t)2 * nf + j] = G11 / det;
        fref[(size_t)3 * nf + j] = 0.5 * std::sqrt(det);
        fref[(size_t)4 * nf + j] = 1.0 / det;
        const double A[3] = {a[0] - o[0], a[1] - o[1], a[2] - o[2]};
        const double B[3] = {b[0] - o[0], b[1] - o[1], b[2] - o[2]};
        const double C[3] = {cc[0] - o[0], cc[1] - o[1], cc[2] - o[2]};
        const double Vj = (A[0] * (B[1] * C[2] - B[2] * C[1]) + A[1] * (B[2] * C[0] - B[0] * C[2]) +
                           A[2] * (B[0] * C[1] - B[1] * C[0])) / 6.0;
        V0 += Vj;
    }
    if (!(V0 > 0.0)) return fail(c, IBLB_E_MESH, "reference volume not positive (faces must point outward)");

    // vertex -> (face, corner), faces ascending, in `slots` fixed slots per
    // vertex; unused slots carry w = -1
    const int slots = incidence_slots(mesh);
    std::vector<int4> inc((size_t)nv * slots, make_int4(0, 0, 0, -1));
    {
        std::vector<int> fill((size_t)nv, 0);
        for (int j = 0; j < nf; ++j)
            for (int k = 0; k < 3; ++k) {
                const int *f = mesh->faces + 3 * j;
                inc[(size_t)f[k] * slots + fill[f[k]]++] = make_int4(f[0], f[1], f[2], (j << 2) | k);
            }
    }
    // structure-of-arrays copies
    std::vector<double> qs((size_t)3 * nv), Xs((size_t)3 * nv);
    for (int i = 0; i < nv; ++i)
        for (int k = 0; k < 3; ++k) {
            qs[(size_t)k * nv + i] = mesh->vertices[3 * i + k];
            Xs[(size_t)k * nv + i] = X[3 * i + k];
        }
    std::vector<int> fs((size_t)3 * nf);
    for (int j = 0; j < nf; ++j)
        for (int k = 0; k < 3; ++k) fs[(size_t)k * nf + j] = mesh->faces[3 * j + k];

    // device memory for the mesh part
    const Layout L = make_layout(c->g, c->ps, c->ts, nv, nf, slots);
    char *mb = nullptr;
    if (c->own_ws || c->ws_bytes < L.mesh_end) {
        // the mesh block is not covered by a caller's workspace: allocate it here
        void *p = nullptr;
        HIP_TRY(c, hipMalloc(&p, L.mesh_end - L.dom_end));
        c->mesh_alloc = p;
        mb = (char *)p - L.dom_end;  // the offsets below are workspace-relative
    } else {
        mb = c->ws;
    }
    c->L = L;
    Dev &d = c->d;
    d.q = (double *)(mb + L.q);
    d.Xref = (double *)(mb + L.Xref);
    d.faces = (int *)(mb + L.faces);
    d.fref = (double *)(mb + L.fref);
    d.inc4 = (int4 *)(mb + L.inc4);
    d.U = mb + L.U;
    d.phiSW = mb + L.phiSW;
    d.gV = mb + L.gV;
    d.base = (Base *)(mb + L.base);
    d.wts = mb + L.wts;
    d.partials = (double *)(mb + L.partials);
    d.mask = (uint64_t *)(mb + L.mask);
    d.act = (uint8_t *)(mb + L.act);
    d.acnt = (uint32_t *)(mb + L.acnt);
    d.alist = (int *)(mb + L.alist);
    HIP_TRY(c, hipMemcpyAsync(d.q, qs.data(), qs.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d.Xref, Xs.data(), Xs.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d.faces, fs.data(), fs.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d.fref, fref.data(), fref.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d.inc4, inc.data(), inc.size() * 16, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemsetAsync(d.partials, 0, (size_t)((nv + 31) / 32) * 8, c->stream));

    MeshArgs &m = c->m;
    m.nv = nv;
    m.nf = nf;
    for (int k = 0; k < 3; ++k) {
        m.alpha[k] = mesh->alpha[k];
        m.origin[k] = o[k];
    }
    m.eps_lo = mesh->eps_wall_lo;
    m.eps_hi = mesh->eps_wall_hi;
    m.xi = mesh->xi_wall;
    m.rc = mesh->r_cut_wall;
    m.z_lo = 0.5;
    m.z_hi = c->dom.nz - 1.5;
    m.kv_over_V0 = mesh->k_v / V0;
    m.nparts = (nv + 31) / 32;
    m.nwords = (nv + 63) / 64;
    m.slots = slots;
    c->V0 = V0;
    c->nv = nv;
    c->nf = nf;
    c->has_mesh = true;
    drop_graph(c);
    rc = rebuild_lists(c);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (mesh_id) *mesh_id = 0;
    return IBLB_OK;
}

int iblb_step(iblb_ctx *c, int32_t n_steps)
{
    if (!c || n_steps < 0) return IBLB_E_INVAL;
    // Captured graphs of kGraphSteps steps, then of one step, from the
    // current parity; launched directly when graphs are off or when timing.
    int left = n_steps;
    while (left > 0) {
        const int p = (int)(c->t & 1);
        if (!c->timing && c->use_graph) {
            const int which = left >= kGraphSteps ? 0 : 1;
            int rc = capture_steps(c, p, which);
            if (rc) return rc;
            HIP_TRY(c, hipGraphLaunch(c->gexec[p][which], c->stream));
            const int k = which == 0 ? kGraphSteps : 1;
            c->t += k;
            left -= k;
        } else {
            hipError_t e = enqueue_step(c, p, c->timing);
            if (e != hipSuccess) return hip_fail(c, e, "step launch");
            c->t += 1;
            left -= 1;
        }
    }
    if (c->timing) return collect_timing(c);
    return IBLB_OK;
}

int iblb_sync(iblb_ctx *c)
{
    if (!c) return IBLB_E_INVAL;
    return sync_ctx(c);
}

int iblb_step_count(const iblb_ctx *c, int64_t *t)
{
    if (!c || !t) return IBLB_E_INVAL;
    *t = c->t;
    return IBLB_OK;
}

int iblb_get_vertices(iblb_ctx *c, int32_t mesh_id, double *host_out)
{
    int rc = mesh_ok(c, mesh_id);
    if (rc) return rc;
    if (!host_out) return IBLB_E_INVAL;
    rc = sync_ctx(c);
    std::vector<double> qs((size_t)3 * c->nv);
    HIP_TRY(c, hipMemcpy(qs.data(), c->d.q, qs.size() * 8, hipMemcpyDeviceToHost));
    for (int i = 0; i < c->nv; ++i)
        for (int k = 0; k < 3; ++k) host_out[3 * i + k] = qs[(size_t)k * c->nv + i];
    return rc;
}

int iblb_vertices_device(iblb_ctx *c, int32_t mesh_id, const double **dev_ptr)
{
    int rc = mesh_ok(c, mesh_id);
    if (rc) return rc;
    if (!dev_ptr) return IBLB_E_INVAL;
    *dev_ptr = c->d.q;
    return IBLB_OK;
}

static int mesh_moments(iblb_ctx *c, double *mom)
{
    int rc = sync_ctx(c);
    HIP_TRY(c, launch_mesh_moments(c->d, c->m, c->d.scratch, c->stream));
    HIP_TRY(c, hipMemcpyAsync(mom, c->d.scratch, 11 * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return rc;
}

int iblb_volume(iblb_ctx *c, int32_t mesh_id, double *V, double *A)
{
    int rc = mesh_ok(c, mesh_id);
    if (rc) return rc;
    double mom[11];
    rc = mesh_moments(c, mom);
    if (rc == IBLB_E_DEVICE) return rc;
    if (V) *V = mom[0];
    if (A) *A = mom[1];
    return rc;
}

int iblb_shape(iblb_ctx *c, int32_t mesh_id, double *D, double *Theta, double centroid[3])
{
    int rc = mesh_ok(c, mesh_id);
    if (rc) return rc;
    double mom[11];
    rc = mesh_moments(c, mom);
    if (rc == IBLB_E_DEVICE) return rc;
    const double V = mom[0];
    if (!(V > 0.0)) return fail(c, IBLB_E_UNSTABLE, "non-positive enclosed volume");
    const double xc[3] = {mom[2] / V, mom[3] / V, mom[4] / V};
    // central second moments, x-z block
    const double a = mom[5] - V * xc[0] * xc[0];  // xx
    const double cz = mom[7] - V * xc[2] * xc[2]; // zz
    const double b = mom[9] - V * xc[0] * xc[2];  // xz
    const double mean = 0.5 * (a + cz), hd = 0.5 * (a - cz);
    const double rad = std::sqrt(hd * hd + b * b);
    const double l1 = mean + rad, l3 = mean - rad;
    const double r1 = std::sqrt(5.0 * std::max(l1, 0.0) / V), r3 = std::sqrt(5.0 * std::max(l3, 0.0) / V);
    double th = 0.5 * std::atan2(2.0 * b, a - cz);
    if (th > M_PI / 2) th -= M_PI;
    if (th <= -M_PI / 2) th += M_PI;
    if (D) *D = (r1 - r3) / (r1 + r3);
    if (Theta) *Theta = th;
    if (centroid)
        for (int k = 0; k < 3; ++k) centroid[k] = c->m.origin[k] + xc[k];
    return rc;
}

// Solves the n x n (n <= 4) symmetric normal equations N s = r of an algebraic
// least-squares fit, N given as its packed upper triangle (row by row), by
// Gaussian elimination with partial pivoting.  False when N is singular.
static bool solve_normal(int n, const double *packed, const double *r, double *s)
{
    double N[4][5];
    int k = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) {
            N[i][j] = packed[k];
            N[j][i] = packed[k];
            ++k;
        }
    for (int i = 0; i < n; ++i) N[i][n] = r[i];
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int row = col + 1; row < n; ++row)
            if (std::fabs(N[row][col]) > std::fabs(N[piv][col])) piv = row;
        if (!(std::fabs(N[piv][col]) > 0.0)) return false;
        for (int cc = 0; cc <= n; ++cc) std::swap(N[col][cc], N[piv][cc]);
        for (int row = col + 1; row < n; ++row) {
            const double fct = N[row][col] / N[col][col];
            for (int cc = col; cc <= n; ++cc) N[row][cc] -= fct * N[col][cc];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double acc = N[i][n];
        for (int j = i + 1; j < n; ++j) acc -= N[i][j] * s[j];
        s[i] = acc / N[i][i];
    }
    return true;
}

// Nodes of the paper's fitting slice, (4 / 3^(1/4)) sqrt(pi N_f) rounded
// (appendix on the resolution test), at most the vertex count.
static int slice_count(int nf, int nv)
{
    const int K = (int)std::floor(4.0 / std::pow(3.0, 0.25) * std::sqrt(M_PI * nf) + 0.5);
    return std::max(1, std::min(nv, K));
}

int iblb_contact_angle(iblb_ctx *c, int32_t mesh_id, int32_t wall, int32_t method, double *theta_deg,
                       double *contact_radius, double *height)
{
    int rc = mesh_ok(c, mesh_id);
    if (rc) return rc;
    if (wall != 0 && wall != 1) return fail(c, IBLB_E_INVAL, "wall must be 0 (lower) or 1 (upper)");
    if (method != 0 && method != 1) return fail(c, IBLB_E_INVAL, "method must be 0 (sphere) or 1 (slice circle)");
    if (!c->g.walls) return fail(c, IBLB_E_STATE, "no walls in a periodic domain");
    rc = sync_ctx(c);
    const double zw = wall ? c->dom.nz - 1.5 : 0.5;
    const double shift[3] = {c->m.origin[0], c->m.origin[1], zw};
    double R, hc;
    if (method == 0) {
        double mom[15], s[4];
        HIP_TRY(c, launch_sphere_moments(c->d, c->m, wall, zw, 2.0, shift, c->d.scratch, c->stream));
        HIP_TRY(c, hipMemcpyAsync(mom, c->d.scratch, 15 * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (mom[14] < 4.0) return fail(c, IBLB_E_STATE, "fewer than 4 vertices away from the wall");
        if (!solve_normal(4, mom, mom + 10, s)) return fail(c, IBLB_E_STATE, "singular sphere fit");
        R = std::sqrt(s[3] + s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        hc = wall ? -s[2] : s[2];  // centre height above the wall plane (into the fluid)
    } else {
        // mesh moments (for the centroid plane) into scratch[0..10], the slice's
        // normal equations into scratch[16..25]
        double mom[10], s[3];
        const double sh2[2] = {shift[0], zw};
        HIP_TRY(c, launch_mesh_moments(c->d, c->m, c->d.scratch, c->stream));
        HIP_TRY(c, launch_slice_moments(c->d, c->m, c->d.scratch, slice_count(c->m.nf, c->m.nv), wall, zw, 2.0,
                                        sh2, c->d.scratch + 16, c->stream));
        HIP_TRY(c, hipMemcpyAsync(mom, c->d.scratch + 16, 10 * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (mom[9] < 3.0) return fail(c, IBLB_E_STATE, "fewer than 3 slice vertices away from the wall");
        if (!solve_normal(3, mom, mom + 6, s)) return fail(c, IBLB_E_STATE, "singular circle fit");
        R = std::sqrt(s[2] + s[0] * s[0] + s[1] * s[1]);
        hc = wall ? -s[1] : s[1];
    }
    const double cth = std::max(-1.0, std::min(1.0, -hc / R));
    if (theta_deg) *theta_deg = std::acos(cth) * 180.0 / M_PI;
    if (contact_radius) *contact_radius = std::sqrt(std::max(0.0, R * R - hc * hc));
    if (height) *height = hc + R;
    return rc;
}

int iblb_get_fields(iblb_ctx *c, double *rho, double *u)
{
    if (!c || !rho || !u) return IBLB_E_INVAL;
    TmpDev tmp;
    HIP_TRY(c, hipMalloc(&tmp.p, 4 * (size_t)c->g.n * 8));
    return get_fields_staged(c, (double *)tmp.p, rho, u);
}

int iblb_debug_set_force(iblb_ctx *c, const double *F)
{
    if (!c || !F) return IBLB_E_INVAL;
    if (c->has_mesh) return fail(c, IBLB_E_STATE, "debug force field only without a mesh");
    const size_t n = (size_t)c->g.n;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (!c->d.Fext) {
        HIP_TRY(c, hipMalloc(&c->fext_alloc, 3 * n * c->ts));
        c->d.Fext = c->fext_alloc;
    }
    if (c->prec == IBLB_FP64) {
        HIP_TRY(c, hipMemcpy(c->d.Fext, F, 3 * n * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> tmp(3 * n);
        for (size_t i = 0; i < 3 * n; ++i) tmp[i] = (float)F[i];
        HIP_TRY(c, hipMemcpy(c->d.Fext, tmp.data(), 3 * n * 4, hipMemcpyHostToDevice));
    }
    lb_args(c);
    drop_graph(c);
    return IBLB_OK;
}

int iblb_debug_get_force(iblb_ctx *c, double *F)
{
    if (!c || !F) return IBLB_E_INVAL;
    int rc = sync_ctx(c);
    const size_t n = (size_t)c->g.n;
    TmpDev tmp;
    HIP_TRY(c, hipMalloc(&tmp.p, 3 * n * 8));
    HIP_TRY(c, launch_get_force(c->prec, c->d, c->lb, (int)(c->t & 1), (double *)tmp.p, c->stream));
    HIP_TRY(c, hipMemcpyAsync(F, tmp.p, 3 * n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return rc;
}

int iblb_debug_get_populations(iblb_ctx *c, double *f)
{
    if (!c || !f) return IBLB_E_INVAL;
    int rc = sync_ctx(c);
    const size_t n = (size_t)c->g.n;
    TmpDev tmp;
    HIP_TRY(c, hipMalloc(&tmp.p, 19 * n * 8));
    HIP_TRY(c, launch_get_pops(c->prec, c->d, c->g, (int)(c->t & 1), (double *)tmp.p, c->stream));
    HIP_TRY(c, hipMemcpyAsync(f, tmp.p, 19 * n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return rc;
}

int iblb_debug_set_populations(iblb_ctx *c, const double *f)
{
    if (!c || !f) return IBLB_E_INVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const size_t n = (size_t)c->g.n;
    TmpDev tmp;
    HIP_TRY(c, hipMalloc(&tmp.p, 19 * n * 8));
    HIP_TRY(c, hipMemcpyAsync(tmp.p, f, 19 * n * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, launch_set_pops(c->prec, c->d, c->g, (int)(c->t & 1), (const double *)tmp.p, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return IBLB_OK;
}

int iblb_debug_get_nodal_forces(iblb_ctx *c, int32_t mesh_id, double *phi)
{
    int rc = mesh_ok(c, mesh_id);
    if (rc) return rc;
    if (!phi) return IBLB_E_INVAL;
    rc = sync_ctx(c);
    TmpDev tmp;
    HIP_TRY(c, hipMalloc(&tmp.p, (size_t)3 * c->nv * 8));
    HIP_TRY(c, launch_nodal_forces(c->prec, c->d, c->m, (double *)tmp.p, c->stream));
    HIP_TRY(c, hipMemcpyAsync(phi, tmp.p, (size_t)3 * c->nv * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return rc;
}

namespace {
struct StateHeader {
    char magic[8];
    int32_t precision, nx, ny, nz, wall_mode, nv;
    int64_t t;
    int32_t err, pad;
};
}  // namespace

int iblb_save_state(iblb_ctx *c, void *host_buf, size_t *bytes)
{
    if (!c || !bytes) return IBLB_E_INVAL;
    const size_t n = (size_t)c->g.n;
    const size_t need = sizeof(StateHeader) + 19 * n * c->ps + 3 * n * c->ts + (size_t)c->g.nt * 4 +
                        (size_t)3 * c->nv * 8;
    if (!host_buf) {
        *bytes = need;
        return IBLB_OK;
    }
    if (*bytes < need) return fail(c, IBLB_E_INVAL, "state buffer too small");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    StateHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, kMagic, 8);
    h.precision = c->prec;
    h.nx = c->g.nx;
    h.ny = c->g.ny;
    h.nz = c->g.nz;
    h.wall_mode = c->dom.wall_mode;
    h.nv = c->nv;
    h.t = c->t;
    HIP_TRY(c, hipMemcpy(&h.err, c->d.err, 4, hipMemcpyDeviceToHost));
    char *p = (char *)host_buf;
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    HIP_TRY(c, hipMemcpy2D(p, n * c->ps, c->d.f, (size_t)c->g.pp * c->ps, n * c->ps, 19, hipMemcpyDeviceToHost));
    p += 19 * n * c->ps;
    HIP_TRY(c, hipMemcpy(p, c->d.F, 3 * n * c->ts, hipMemcpyDeviceToHost));
    p += 3 * n * c->ts;
    HIP_TRY(c, hipMemcpy(p, c->d.stamp, (size_t)c->g.nt * 4, hipMemcpyDeviceToHost));
    p += (size_t)c->g.nt * 4;
    if (c->nv) HIP_TRY(c, hipMemcpy(p, c->d.q, (size_t)3 * c->nv * 8, hipMemcpyDeviceToHost));
    *bytes = need;
    return IBLB_OK;
}

int iblb_load_state(iblb_ctx *c, const void *host_buf, size_t bytes)
{
    if (!c || !host_buf) return IBLB_E_INVAL;
    const size_t n = (size_t)c->g.n;
    const size_t need = sizeof(StateHeader) + 19 * n * c->ps + 3 * n * c->ts + (size_t)c->g.nt * 4 +
                        (size_t)3 * c->nv * 8;
    if (bytes < need) return fail(c, IBLB_E_INVAL, "state buffer too small");
    StateHeader h;
    std::memcpy(&h, host_buf, sizeof(h));
    if (std::memcmp(h.magic, kMagic, 8) != 0) return fail(c, IBLB_E_INVAL, "not an iblb state buffer");
    if (h.precision != c->prec || h.nx != c->g.nx || h.ny != c->g.ny || h.nz != c->g.nz ||
        h.wall_mode != c->dom.wall_mode || h.nv != c->nv || h.t < 0 || h.t > 0xffffffffll)
        return fail(c, IBLB_E_INVAL, "state buffer does not match this context");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const char *p = (const char *)host_buf + sizeof(h);
    HIP_TRY(c, hipMemcpy2D(c->d.f, (size_t)c->g.pp * c->ps, p, n * c->ps, n * c->ps, 19, hipMemcpyHostToDevice));
    p += 19 * n * c->ps;
    HIP_TRY(c, hipMemcpy(c->d.F, p, 3 * n * c->ts, hipMemcpyHostToDevice));
    p += 3 * n * c->ts;
    HIP_TRY(c, hipMemcpy(c->d.stamp, p, (size_t)c->g.nt * 4, hipMemcpyHostToDevice));
    p += (size_t)c->g.nt * 4;
    if (c->nv) HIP_TRY(c, hipMemcpy(c->d.q, p, (size_t)3 * c->nv * 8, hipMemcpyHostToDevice));
    uint32_t ctr[2];
    ctr[h.t & 1] = (uint32_t)h.t;
    ctr[1 - (h.t & 1)] = (uint32_t)h.t;  // not read before it is written
    HIP_TRY(c, hipMemcpy(c->d.ctr, ctr, 8, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d.err, &h.err, 4, hipMemcpyHostToDevice));
    c->t = h.t;
    if (c->has_mesh) {
        int rc = rebuild_lists(c);
        if (rc) return rc;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return IBLB_OK;
}

int iblb_set_graph(iblb_ctx *c, int32_t graph)
{
    if (!c) return IBLB_E_INVAL;
    c->use_graph = graph != 0;
    if (!c->use_graph) {
        drop_graph(c);
        return IBLB_OK;
    }
    return capture_all(c);
}

int iblb_get_lb_split(const iblb_ctx *c, int32_t *block_x, double *share_forces)
{
    if (!c) return IBLB_E_INVAL;
    if (block_x) *block_x = lb_block_width(c->g);
    if (share_forces) *share_forces = lb_share_with_forces();
    return IBLB_OK;
}

int iblb_set_timing(iblb_ctx *c, int32_t timing)
{
    if (!c) return IBLB_E_INVAL;
    c->timing = timing != 0;
    return IBLB_OK;
}

int iblb_kernel_time(iblb_ctx *c, const char *name, double *total_ms, int64_t *launches)
{
    if (!c || !name) return IBLB_E_INVAL;
    int rc = collect_timing(c);
    if (rc) return rc;
    for (int k = 0; k < kNumKernels; ++k)
        if (std::strcmp(name, kKernelNames[k]) == 0) {
            if (total_ms) *total_ms = c->ktime[k];
            if (launches) *launches = c->kcount[k];
            return IBLB_OK;
        }
    return fail(c, IBLB_E_INVAL, std::string("unknown kernel name ") + name);
}

void iblb_tile_shape(int32_t *tx, int32_t *ty, int32_t *tz)
{
    if (tx) *tx = kTileX;
    if (ty) *ty = kTileY;
    if (tz) *tz = kTileZ;
}

int iblb_active_nodes(iblb_ctx *c, int64_t *n)
{
    if (!c || !n) return IBLB_E_INVAL;
    *n = 0;
    if (!c->has_mesh) return IBLB_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->t == 0) return IBLB_OK;
    // the count of the last completed step t - 1 (its move cleared the other
    // parity's counter for the next step)
    uint32_t na = 0;
    HIP_TRY(c, hipMemcpy(&na, c->d.acnt + ((c->t - 1) & 1), 4, hipMemcpyDeviceToHost));
    if (na > (uint32_t)c->g.nt) return fail(c, IBLB_E_STATE, "active tile count out of range");
    std::vector<int> tiles(na);
    if (na) HIP_TRY(c, hipMemcpy(tiles.data(), c->d.alist, (size_t)na * 4, hipMemcpyDeviceToHost));
    const Grid &g = c->g;
    int64_t total = 0;
    for (int tile : tiles) {
        if (tile < 0 || tile >= g.nt) return fail(c, IBLB_E_STATE, "active tile index out of range");
        const int tz = tile / (g.ntx * g.nty), rem = tile % (g.ntx * g.nty);
        const int ty = rem / g.ntx, tx = rem % g.ntx;
        total += (int64_t)std::min(kTileX, g.nx - kTileX * tx) * std::min(kTileY, g.ny - kTileY * ty) *
                 std::min(kTileZ, g.nzf - kTileZ * tz);
    }
    *n = total;
    return IBLB_OK;
}

int iblb_reset_timing(iblb_ctx *c)
{
    if (!c) return IBLB_E_INVAL;
    int rc = collect_timing(c);
    for (int k = 0; k < kNumKernels; ++k) {
        c->ktime[k] = 0.0;
        c->kcount[k] = 0;
    }
    return rc;
}

const char *iblb_last_error(const iblb_ctx *c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

int iblb_destroy(iblb_ctx *c)
{
    if (!c) return IBLB_E_INVAL;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto &p : c->pending) {
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    drop_graph(c);
    free_adjoint(c);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    if (c->mesh_alloc) (void)hipFree(c->mesh_alloc);
    if (c->fext_alloc) (void)hipFree(c->fext_alloc);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return IBLB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: independent contexts advanced together, one launch of each step
// kernel per step for all of them
// ---------------------------------------------------------------------------
namespace {

// Share of each member's LB blocks in the forces dispatch before tuning (the
// single-context value).
constexpr double kBatchLbShare = 0.6;

// Launch shape of a batch; zero fields take the defaults resolved by `resolved`.
struct BatchCfg {
    int lb_bx = 0;
    int spread_per_cu = 0;
    int vpw = 0;
    double lb_share = kBatchLbShare;
};

}  // namespace

struct iblb_batch {
    std::vector<iblb_ctx *> mem;
    std::vector<int> status;        // IBLB_OK while stepped; the code that froze the member otherwise
    std::vector<std::string> why;
    int prec = 0;
    int num_cus = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t ev = nullptr;        // end of the batch's work, waited for by the members' streams
    std::vector<hipEvent_t> mev;    // end of each member's own work, waited for by the batch stream
    DomRec *recs = nullptr;         // device: one record per member
    uint32_t *tabs = nullptr;       // device: the four dispatch tables, back to back
    int *errs = nullptr;            // device: the members' error bits
    size_t tab_cap = 0;             // entries allocated in tabs
    int off[4] = {0, 0, 0, 0}, cnt[4] = {0, 0, 0, 0};
    BatchCfg cfg;
    int vpw_used = 1;
    int nw_used = 4;                // wavefronts per spreading block
    bool dirty = true;              // tables to rebuild before the next launch
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::string err;
};

namespace {

int bfail(iblb_batch *b, int code, const std::string &msg)
{
    if (b) b->err = msg;
    return code;
}

#define BHIP_TRY(b, expr)                                                                                  \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess) return bfail(b, IBLB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

void bdrop_graph(iblb_batch *b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
}

// the single-context LB block width for a lattice of width nx
int lb_width_rule(int nx) { return nx >= 64 ? 64 : (nx >= 32 ? 32 : 16); }

// Wavefronts per spreading block of a batch: two while every stepped member's
// vertex mask fits four words per thread of them (at most 32768 vertices),
// else four, as for a single context.
int spread_nw(const iblb_batch *b)
{
    for (size_t k = 0; k < b->mem.size(); ++k)
        if (b->status[k] == IBLB_OK && b->mem[k]->m.nwords > 4 * 128) return 4;
    return 2;
}

BatchCfg resolved(const iblb_batch *b)
{
    BatchCfg c = b->cfg;
    // default: eight spreading wavefronts per CU (four with FP64)
    if (c.spread_per_cu == 0) c.spread_per_cu = (b->prec == IBLB_FP64 ? 4 : 8) / spread_nw(b);
    if (c.vpw == 0) {
        long long nv = 0;
        for (size_t k = 0; k < b->mem.size(); ++k)
            if (b->status[k] == IBLB_OK) nv += b->mem[k]->nv;
        c.vpw = nv <= 32ll * b->num_cus ? 1 : 2;
    }
    return c;
}

// Per-member records and the four dispatch tables.  The latency-bound blocks
// of every member (forces and list scan; spreading) come first in their
// dispatch and the LB blocks of the nodes outside the active tiles after
// them, so that the hardware starts the former first.
int build_tables(iblb_batch *b)
{
    // launches already queued read the current records and tables
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    const BatchCfg cfg = resolved(b);
    const int nw = spread_nw(b), nsub = 4 / nw;
    const int n = (int)b->mem.size();
    std::vector<DomRec> recs((size_t)n);
    std::vector<uint32_t> tab[4];
    long long hint_sum = 0;
    for (int k = 0; k < n; ++k)
        if (b->status[(size_t)k] == IBLB_OK) hint_sum += std::max(1, b->mem[(size_t)k]->m.tiles_hint);
    const double budget = (double)cfg.spread_per_cu * b->num_cus;
    std::vector<int> nlb((size_t)n, 0);
    for (int k = 0; k < n; ++k) {
        const iblb_ctx *c = b->mem[(size_t)k];
        DomRec &r = recs[(size_t)k];
        std::memset(&r, 0, sizeof(r));
        r.d = c->d;
        r.a = c->lb;
        r.m = c->m;
        const int bx = cfg.lb_bx ? std::min(cfg.lb_bx, lb_width_rule(c->g.nx)) : lb_width_rule(c->g.nx);
        r.bxw = bx;
        r.nbx = (c->g.nx + bx - 1) / bx;
        r.nby = (c->g.ny + 256 / bx - 1) / (256 / bx);
        nlb[(size_t)k] = r.nbx * r.nby * c->g.nzf;
        r.lb0 = (int)(cfg.lb_share * nlb[(size_t)k] + 0.5);
        const int hint = std::max(1, c->m.tiles_hint);
        const long long want = hint_sum > 0 ? std::llround(budget * hint / (double)hint_sum) : 1;
        r.nsp = (int)std::max(1ll, std::min(want, (long long)c->g.nt));
        r.mblocks = std::max(1, moments_blocks(c->g, c->m, 4));
        if ((long long)c->m.nparts + scan_block_count(c->g) + nlb[(size_t)k] >= (1ll << 24) ||
            (long long)r.nsp + (long long)nsub * nlb[(size_t)k] >= (1ll << 24))
            return bfail(b, IBLB_E_INVAL, "member " + std::to_string(k) + " has too many blocks for a batch");
    }
    auto entry = [](int k, int blk) { return (uint32_t)k | ((uint32_t)blk << 8); };
    auto on = [&](int k) { return b->status[(size_t)k] == IBLB_OK; };
    for (int k = 0; k < n; ++k)
        if (on(k)) {
            const int nf = recs[(size_t)k].m.nparts + scan_block_count(recs[(size_t)k].a.g);
            for (int j = 0; j < nf; ++j) tab[B_FORCES].push_back(entry(k, j));
        }
    for (int k = 0; k < n; ++k)
        if (on(k)) {
            const int nf = recs[(size_t)k].m.nparts + scan_block_count(recs[(size_t)k].a.g);
            for (int j = 0; j < recs[(size_t)k].lb0; ++j) tab[B_FORCES].push_back(entry(k, nf + j));
        }
    for (int k = 0; k < n; ++k)
        if (on(k))
            for (int j = 0; j < recs[(size_t)k].nsp; ++j) tab[B_SPREAD].push_back(entry(k, j));
    for (int k = 0; k < n; ++k)
        if (on(k))
            for (int j = 0; j < nsub * (nlb[(size_t)k] - recs[(size_t)k].lb0); ++j)
                tab[B_SPREAD].push_back(entry(k, recs[(size_t)k].nsp + j));
    for (int k = 0; k < n; ++k)
        if (on(k))
            for (int j = 0; j < recs[(size_t)k].mblocks; ++j) tab[B_MOMENTS].push_back(entry(k, j));
    for (int k = 0; k < n; ++k)
        if (on(k)) {
            const int nv = recs[(size_t)k].m.nv;
            const int blocks = cfg.vpw == 2 ? (nv + 7) / 8 : (nv + 3) / 4;
            for (int j = 0; j < blocks; ++j) tab[B_MOVE].push_back(entry(k, j));
        }
    size_t total = 0;
    for (int w = 0; w < 4; ++w) {
        b->off[w] = (int)total;
        b->cnt[w] = (int)tab[w].size();
        total += tab[w].size();
    }
    bdrop_graph(b);
    if (total > b->tab_cap) {
        if (b->tabs) (void)hipFree(b->tabs);
        b->tabs = nullptr;
        b->tab_cap = 0;
        BHIP_TRY(b, hipMalloc(&b->tabs, total * 4));
        b->tab_cap = total;
    }
    std::vector<uint32_t> all;
    all.reserve(total);
    for (int w = 0; w < 4; ++w) all.insert(all.end(), tab[w].begin(), tab[w].end());
    BHIP_TRY(b, hipMemcpyAsync(b->recs, recs.data(), recs.size() * sizeof(DomRec), hipMemcpyHostToDevice, b->stream));
    if (total) BHIP_TRY(b, hipMemcpyAsync(b->tabs, all.data(), total * 4, hipMemcpyHostToDevice, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    b->vpw_used = cfg.vpw;
    b->nw_used = nw;
    b->dirty = false;
    return IBLB_OK;
}

hipError_t batch_enqueue(iblb_batch *b, int p)
{
    for (int w = 0; w < 4; ++w) {
        hipError_t e = launch_batch(b->prec, w, b->recs, b->tabs + b->off[w], b->cnt[w], p, b->vpw_used, b->nw_used,
                                    b->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// n steps of every stepped member from a time of parity t0 & 1 (the members'
// host step counters are the caller's): graphs of kGraphSteps steps from even
// times, single launches otherwise.
int batch_advance(iblb_batch *b, long long t0, int n)
{
    if (b->dirty) {
        int rc = build_tables(b);
        if (rc) return rc;
    }
    if (b->cnt[B_FORCES] == 0) return IBLB_OK;  // every member frozen
    long long t = t0;
    int left = n;
    while (left > 0) {
        const int p = (int)(t & 1);
        if (p == 0 && left >= kGraphSteps) {
            if (!b->gexec) {
                BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
                hipError_t e = hipSuccess;
                for (int k = 0; k < kGraphSteps && e == hipSuccess; ++k) e = batch_enqueue(b, k & 1);
                hipGraph_t gr = nullptr;
                hipError_t e2 = hipStreamEndCapture(b->stream, &gr);
                if (e != hipSuccess) {
                    if (gr) (void)hipGraphDestroy(gr);
                    return bfail(b, IBLB_E_DEVICE, std::string("batch step capture: ") + hipGetErrorString(e));
                }
                BHIP_TRY(b, e2);
                b->graph = gr;
                BHIP_TRY(b, hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
            }
            BHIP_TRY(b, hipGraphLaunch(b->gexec, b->stream));
            t += kGraphSteps;
            left -= kGraphSteps;
        } else {
            BHIP_TRY(b, batch_enqueue(b, p));
            t += 1;
            left -= 1;
        }
    }
    return IBLB_OK;
}

// the batch stream waits for the work already queued on each stepped member's stream
int order_after_members(iblb_batch *b)
{
    for (size_t k = 0; k < b->mem.size(); ++k) {
        if (b->status[k] != IBLB_OK) continue;
        BHIP_TRY(b, hipEventRecord(b->mev[k], b->mem[k]->stream));
        BHIP_TRY(b, hipStreamWaitEvent(b->stream, b->mev[k], 0));
    }
    return IBLB_OK;
}

// each member's stream waits for the batch's work queued so far
int order_members_after(iblb_batch *b)
{
    BHIP_TRY(b, hipEventRecord(b->ev, b->stream));
    for (size_t k = 0; k < b->mem.size(); ++k) BHIP_TRY(b, hipStreamWaitEvent(b->mem[k]->stream, b->ev, 0));
    return IBLB_OK;
}

// a step counter of the stepped members (whose parities must agree)
int batch_time(iblb_batch *b, long long *t0)
{
    bool have = false;
    *t0 = 0;
    for (size_t k = 0; k < b->mem.size(); ++k) {
        if (b->status[k] != IBLB_OK) continue;
        const long long t = b->mem[k]->t;
        if (!have) {
            *t0 = t;
            have = true;
        } else if ((t & 1) != (*t0 & 1)) {
            return bfail(b, IBLB_E_STATE, "member " + std::to_string(k) +
                                              " was stepped on its own: the members' step parities differ");
        }
    }
    return IBLB_OK;
}

// device byte ranges holding a member's whole state (workspace and mesh block)
void state_regions(const iblb_ctx *c, std::vector<std::pair<char *, size_t>> &out)
{
    if (c->mesh_alloc) {
        out.push_back({c->ws, c->L.dom_end});
        out.push_back({(char *)c->mesh_alloc, c->L.mesh_end - c->L.dom_end});
    } else {
        out.push_back({c->ws, c->L.mesh_end});
    }
}

}  // namespace

extern "C" {

int iblb_batch_create(iblb_ctx *const *members, int32_t n, void *hip_stream, iblb_batch **out)
{
    if (!out) return IBLB_E_INVAL;
    *out = nullptr;
    if (!members || n < 1 || n > kMaxBatch) return IBLB_E_INVAL;
    for (int k = 0; k < n; ++k) {
        const iblb_ctx *c = members[k];
        if (!c) return IBLB_E_INVAL;
        for (int j = 0; j < k; ++j)
            if (members[j] == c) return IBLB_E_INVAL;
        if (!c->has_mesh || c->prec != members[0]->prec || ((c->t ^ members[0]->t) & 1)) return IBLB_E_STATE;
    }
    iblb_batch *b = new iblb_batch();
    b->mem.assign(members, members + n);
    b->status.assign((size_t)n, IBLB_OK);
    b->why.assign((size_t)n, std::string());
    b->prec = members[0]->prec;
    b->num_cus = members[0]->d.num_cus;
    auto bail = [&](int code) {
        iblb_batch_destroy(b);
        return code;
    };
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) return bail(IBLB_E_DEVICE);
        b->own_stream = true;
    }
    if (hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) return bail(IBLB_E_DEVICE);
    b->mev.assign((size_t)n, nullptr);
    for (int k = 0; k < n; ++k)
        if (hipEventCreateWithFlags(&b->mev[(size_t)k], hipEventDisableTiming) != hipSuccess) return bail(IBLB_E_DEVICE);
    if (hipMalloc(&b->recs, (size_t)n * sizeof(DomRec)) != hipSuccess ||
        hipMalloc(&b->errs, (size_t)n * sizeof(int)) != hipSuccess)
        return bail(IBLB_E_DEVICE);
    if (order_after_members(b) || build_tables(b)) return bail(IBLB_E_DEVICE);
    *out = b;
    return IBLB_OK;
}

int iblb_batch_step(iblb_batch *b, int32_t n_steps)
{
    if (!b || n_steps < 0) return IBLB_E_INVAL;
    long long t0 = 0;
    int rc = batch_time(b, &t0);
    if (!rc) rc = order_after_members(b);
    if (!rc) rc = batch_advance(b, t0, n_steps);
    if (!rc) rc = order_members_after(b);
    if (rc) return rc;
    for (size_t k = 0; k < b->mem.size(); ++k)
        if (b->status[k] == IBLB_OK) b->mem[k]->t += n_steps;
    return IBLB_OK;
}

int iblb_batch_sync(iblb_batch *b)
{
    if (!b) return IBLB_E_INVAL;
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    return IBLB_OK;
}

int iblb_batch_check(iblb_batch *b, int32_t *status, int32_t *n_frozen)
{
    if (!b) return IBLB_E_INVAL;
    const int n = (int)b->mem.size();
    std::vector<int> e((size_t)n, 0);
    BHIP_TRY(b, launch_batch_errors(b->recs, n, b->errs, b->stream));
    BHIP_TRY(b, hipMemcpyAsync(e.data(), b->errs, (size_t)n * 4, hipMemcpyDeviceToHost, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    int frozen = 0;
    for (int k = 0; k < n; ++k) {
        if (b->status[(size_t)k] == IBLB_OK && e[(size_t)k] != 0) {
            b->status[(size_t)k] = IBLB_E_UNSTABLE;
            b->why[(size_t)k] = err_text(e[(size_t)k]);
            b->dirty = true;
        }
        if (status) status[k] = b->status[(size_t)k];
        frozen += b->status[(size_t)k] != IBLB_OK;
    }
    if (n_frozen) *n_frozen = frozen;
    return IBLB_OK;
}

const char *iblb_batch_member_error(const iblb_batch *b, int32_t member)
{
    if (!b || member < 0 || member >= (int)b->mem.size()) return "bad batch or member index";
    return b->why[(size_t)member].c_str();
}

int iblb_batch_get_config(const iblb_batch *b, iblb_batch_config *cfg)
{
    if (!b || !cfg) return IBLB_E_INVAL;
    const BatchCfg c = resolved(b);
    cfg->lb_block_x = c.lb_bx;
    cfg->spread_blocks_per_cu = c.spread_per_cu;
    cfg->vertices_per_wave = c.vpw;
    cfg->reserved = 0;
    cfg->lb_share_forces = c.lb_share;
    return IBLB_OK;
}

int iblb_batch_set_config(iblb_batch *b, const iblb_batch_config *cfg)
{
    if (!b || !cfg) return IBLB_E_INVAL;
    if ((cfg->lb_block_x != 0 && cfg->lb_block_x != 16 && cfg->lb_block_x != 32 && cfg->lb_block_x != 64) ||
        cfg->spread_blocks_per_cu < 0 || cfg->spread_blocks_per_cu > 8 || cfg->vertices_per_wave < 0 ||
        cfg->vertices_per_wave > 2 || !(cfg->lb_share_forces >= 0.0 && cfg->lb_share_forces <= 1.0))
        return bfail(b, IBLB_E_INVAL, "bad batch configuration");
    b->cfg.lb_bx = cfg->lb_block_x;
    b->cfg.spread_per_cu = cfg->spread_blocks_per_cu;
    b->cfg.vpw = cfg->vertices_per_wave;
    b->cfg.lb_share = cfg->lb_share_forces;
    b->dirty = true;
    return IBLB_OK;
}

int iblb_batch_tune(iblb_batch *b, int32_t trial_steps, double *best_ms_per_step)
{
    if (!b || trial_steps < 1) return IBLB_E_INVAL;
    const int trial = (trial_steps + kGraphSteps - 1) / kGraphSteps * kGraphSteps;
    long long t0 = 0;
    int rc = batch_time(b, &t0);
    if (!rc) rc = order_after_members(b);
    if (rc) return rc;
    // a copy of every stepped member's device state, put back afterwards
    std::vector<std::pair<char *, size_t>> regs;
    for (size_t k = 0; k < b->mem.size(); ++k)
        if (b->status[k] == IBLB_OK) state_regions(b->mem[k], regs);
    size_t total = 0;
    for (auto &r : regs) total += align256(r.second);
    struct Owned {
        char *p = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Owned()
        {
            if (p) (void)hipFree(p);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } own;
    BHIP_TRY(b, hipMalloc(&own.p, std::max<size_t>(total, 256)));
    BHIP_TRY(b, hipEventCreate(&own.e0));
    BHIP_TRY(b, hipEventCreate(&own.e1));
    size_t o = 0;
    for (auto &r : regs) {
        BHIP_TRY(b, hipMemcpyAsync(own.p + o, r.first, r.second, hipMemcpyDeviceToDevice, b->stream));
        o += align256(r.second);
    }
    long long t = t0;
    auto run = [&](const BatchCfg &cfg, double *ms) -> int {
        b->cfg = cfg;
        b->dirty = true;
        const int warm = kGraphSteps + (int)(t & 1);  // graph capture included; ends at an even time
        int r = batch_advance(b, t, warm);
        if (r) return r;
        t += warm;
        BHIP_TRY(b, hipEventRecord(own.e0, b->stream));
        r = batch_advance(b, t, trial);
        if (r) return r;
        t += trial;
        BHIP_TRY(b, hipEventRecord(own.e1, b->stream));
        BHIP_TRY(b, hipEventSynchronize(own.e1));
        float f = 0.f;
        BHIP_TRY(b, hipEventElapsedTime(&f, own.e0, own.e1));
        *ms = (double)f / trial;
        return IBLB_OK;
    };
    const BatchCfg start = b->cfg;
    BatchCfg best = resolved(b);
    if (best.lb_bx == 0) best.lb_bx = 64;
    double best_ms = 0.0;
    rc = run(best, &best_ms);
    // coordinate descent: two passes over the four launch parameters
    for (int pass = 0; pass < 2 && !rc; ++pass) {
        for (int dim = 0; dim < 4 && !rc; ++dim) {
            std::vector<BatchCfg> cands;
            BatchCfg c = best;
            if (dim == 0)
                for (int v : {16, 32, 64}) { c.lb_bx = v; cands.push_back(c); }
            if (dim == 1)
                for (double v : {0.3, 0.45, 0.6, 0.75, 0.9}) { c.lb_share = v; cands.push_back(c); }
            // spreading wavefronts per CU: 4, 8, 12 (the most the register
            // budget holds at once with FP32)
            if (dim == 2)
                for (int v : {4, 8, 12}) { c.spread_per_cu = v / spread_nw(b); cands.push_back(c); }
            if (dim == 3)
                for (int v : {1, 2}) { c.vpw = v; cands.push_back(c); }
            const BatchCfg cur = best;
            for (const BatchCfg &cand : cands) {
                if (cand.lb_bx == cur.lb_bx && cand.lb_share == cur.lb_share &&
                    cand.spread_per_cu == cur.spread_per_cu && cand.vpw == cur.vpw)
                    continue;
                double ms = 0.0;
                rc = run(cand, &ms);
                if (rc) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = cand;
                }
            }
        }
    }
    o = 0;
    for (auto &r : regs) {
        BHIP_TRY(b, hipMemcpyAsync(r.first, own.p + o, r.second, hipMemcpyDeviceToDevice, b->stream));
        o += align256(r.second);
    }
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    b->cfg = rc ? start : best;
    b->dirty = true;
    if (rc) return rc;
    rc = build_tables(b);
    if (!rc) rc = order_members_after(b);
    if (rc) return rc;
    if (best_ms_per_step) *best_ms_per_step = best_ms;
    return IBLB_OK;
}

const char *iblb_batch_last_error(const iblb_batch *b)
{
    if (!b) return "null batch";
    return b->err.c_str();
}

int iblb_batch_destroy(iblb_batch *b)
{
    if (!b) return IBLB_E_INVAL;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    bdrop_graph(b);
    if (b->recs) (void)hipFree(b->recs);
    if (b->tabs) (void)hipFree(b->tabs);
    if (b->errs) (void)hipFree(b->errs);
    if (b->ev) (void)hipEventDestroy(b->ev);
    for (hipEvent_t e : b->mev)
        if (e) (void)hipEventDestroy(e);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return IBLB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Adjoint: a recorded window of steps and its reverse sweep
// ---------------------------------------------------------------------------
// Time levels of a recorded window (or of one checkpoint segment) and the
// forward's own fields of the steps between them.
struct Recording {
    void *store = nullptr;                // [levels][19][n] populations (element size es)
    double *qs = nullptr;                 // [levels][3][nv] positions
    uint64_t *mask_s = nullptr;           // [levels][tiles][nwords] tile vertex masks of the positions
    int *alist_s = nullptr;               // [steps][tiles] active tiles of each step
    uint32_t *acnt_s = nullptr;           // [steps] and their count
    void *Fs = nullptr, *Us = nullptr;    // [steps][3][n_nodes] force density (active tiles), u(t+1)
    void *phs = nullptr, *gvs = nullptr;  // [steps][3][nv] phi_S + phi_W, dV/dq
    double *dVs = nullptr;                // [steps] V - V0
};

struct AdjState {
    long long t0 = 0;                  // time at the start of the recorded window
    int n = 0, every = 0;              // steps recorded; steps per checkpoint, 0 = every level kept
    std::vector<char *> ck;            // checkpoint mode: device states at t0, t0 + every, ..., t0 + n
    size_t snap = 0;                   // bytes of one checkpoint
    size_t es = 8;                     // bytes per stored population: the step's arithmetic precision
    Recording rec[2];                  // every level of the window; or two segments, one being
                                       // recorded while the sweep reads the other
    hipStream_t rs = nullptr;          // checkpoint mode: the reverse sweep's stream
    hipEvent_t recorded[2] = {nullptr, nullptr}, swept[2] = {nullptr, nullptr};  // per recording
    double *lam[2] = {nullptr, nullptr};  // ping-pong adjoints of the populations: [1] is t+1
    double *qb[2] = {nullptr, nullptr};   // and of the positions
    double *lam_buf[2] = {nullptr, nullptr}, *qb_buf[2] = {nullptr, nullptr};  // their allocations
    double *Fb = nullptr, *ub = nullptr, *phib = nullptr;
    double *grads = nullptr;           // [6]
    double *tpart = nullptr;           // per-block sums of the tau derivative
    double *vpart = nullptr;           // per-block shares of grad V . phib
    double *serr = nullptr;            // the reverse sweep's error bits (one int): apart from the
                                       // context's, which the checkpoint restores overwrite
};

namespace {

void free_sweep(AdjState *a);

void free_adjoint(iblb_ctx *c)
{
    AdjState *a = c->adj;
    if (!a) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (a->rs) (void)hipStreamSynchronize(a->rs);
    for (char *p : a->ck) (void)hipFree(p);
    free_sweep(a);
    for (int k = 0; k < 2; ++k) {
        if (a->recorded[k]) (void)hipEventDestroy(a->recorded[k]);
        if (a->swept[k]) (void)hipEventDestroy(a->swept[k]);
    }
    if (a->rs) (void)hipStreamDestroy(a->rs);
    delete a;
    c->adj = nullptr;
}

// device copy of the whole state of a context into / out of a checkpoint
int checkpoint(iblb_ctx *c, char *dst, bool save)
{
    std::vector<std::pair<char *, size_t>> regs;
    state_regions(c, regs);
    size_t o = 0;
    for (auto &r : regs) {
        if (save)
            HIP_TRY(c, hipMemcpyAsync(dst + o, r.first, r.second, hipMemcpyDeviceToDevice, c->stream));
        else
            HIP_TRY(c, hipMemcpyAsync(r.first, dst + o, r.second, hipMemcpyDeviceToDevice, c->stream));
        o += align256(r.second);
    }
    return IBLB_OK;
}

size_t checkpoint_bytes(const iblb_ctx *c)
{
    std::vector<std::pair<char *, size_t>> regs;
    state_regions(c, regs);
    size_t o = 0;
    for (auto &r : regs) o += align256(r.second);
    return o;
}

AdjArgs adj_args(const iblb_ctx *c)
{
    AdjArgs A;
    std::memset(&A, 0, sizeof(A));
    A.g = c->g;
    A.nv = c->nv;
    A.nf = c->nf;
    A.slots = c->m.slots;
    A.rho0 = c->dom.rho0;
    A.omega = 1.0 / c->dom.tau;
    for (int k = 0; k < 3; ++k) {
        A.body[k] = c->dom.body_force[k];
        A.ulo[k] = c->dom.u_wall_lo[k];
        A.uhi[k] = c->dom.u_wall_hi[k];
        A.alpha[k] = c->m.alpha[k];
        A.origin[k] = c->m.origin[k];
    }
    A.kv_over_V0 = c->m.kv_over_V0;
    A.V0 = c->V0;
    A.eps_lo = c->m.eps_lo;
    A.eps_hi = c->m.eps_hi;
    A.xi = c->m.xi;
    A.rc = c->m.rc;
    A.z_lo = c->m.z_lo;
    A.z_hi = c->m.z_hi;
    const int hint = std::max(1, c->m.tiles_hint);
    A.tile_blocks = std::min(c->g.nt, hint + hint / 4 + 16);
    return A;
}

void *level(const AdjState *a, const Recording &r, size_t n, int k)
{
    return (char *)r.store + (size_t)k * 19 * n * a->es;
}

// Frees the recording buffers and working arrays of the reverse sweep (not
// the checkpoints).
void free_sweep(AdjState *a)
{
    for (Recording &r : a->rec)
        for (void **p : {&r.store, &r.Fs, &r.Us, &r.phs, &r.gvs, (void **)&r.mask_s, (void **)&r.alist_s,
                         (void **)&r.acnt_s, (void **)&r.qs, (void **)&r.dVs}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
    for (double **p : {&a->lam_buf[0], &a->lam_buf[1], &a->qb_buf[0], &a->qb_buf[1], &a->Fb, &a->ub,
                       &a->phib, &a->grads, &a->tpart, &a->vpart, &a->serr}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
}

// Device memory for `nrec` recordings of `levels` time levels (populations,
// positions) and the fields of the levels - 1 steps between them, and the
// reverse sweep's working arrays; on failure nothing stays allocated.
int alloc_sweep(iblb_ctx *c, AdjState *a, size_t levels, int nrec)
{
    const size_t n = (size_t)c->g.n, nv = (size_t)c->nv, L = levels - 1, es = a->es;
    auto getb = [](void **p, size_t bytes) {
        if (hipMalloc(p, std::max<size_t>(bytes, 1)) == hipSuccess) return true;
        *p = nullptr;
        return false;
    };
    auto get = [&](double **p, size_t count) { return getb((void **)p, count * 8); };
    for (int k = 0; k < nrec; ++k) {
        Recording &r = a->rec[k];
        if (!getb(&r.store, levels * 19 * n * es) || !getb(&r.Fs, L * 3 * n * es) || !getb(&r.Us, L * 3 * n * es) ||
            !getb(&r.phs, L * 3 * nv * es) || !getb(&r.gvs, L * 3 * nv * es) || !get(&r.dVs, L) ||
            !get(&r.qs, levels * 3 * nv) ||
            !getb((void **)&r.mask_s, levels * (size_t)c->g.nt * (size_t)c->m.nwords * 8) ||
            !getb((void **)&r.alist_s, L * (size_t)c->g.nt * 4) || !getb((void **)&r.acnt_s, L * 4)) {
            free_sweep(a);
            return fail(c, IBLB_E_DEVICE, "no device memory for " + std::to_string(levels) +
                                              " recorded time levels (record with a checkpoint interval instead)");
        }
    }
    if (!get(&a->lam_buf[0], 19 * n) || !get(&a->lam_buf[1], 19 * n) || !get(&a->qb_buf[0], 3 * nv) ||
        !get(&a->qb_buf[1], 3 * nv) || !get(&a->Fb, 3 * n) || !get(&a->ub, 3 * n) || !get(&a->phib, 3 * nv) ||
        !get(&a->grads, 6) || !get(&a->tpart, (size_t)adj_lb_blocks((long long)n)) ||
        !get(&a->vpart, (size_t)adj_vertex_blocks((long long)nv)) || !get(&a->serr, 1)) {
        free_sweep(a);
        return fail(c, IBLB_E_DEVICE, "no device memory for the reverse sweep");
    }
    return IBLB_OK;
}

// Steps the context `len` times from its current time t0, recording time
// levels 0 .. len (populations in the step's arithmetic precision, positions)
// and the forward's own fields of each step (launch_record; the level index
// comes from the device step counter).  With use_graph, full runs of
// kGraphSteps steps from even times replay one captured graph.
int record_steps(iblb_ctx *c, AdjState *a, Recording &r, int len, bool use_graph)
{
    const uint32_t t0 = (uint32_t)c->t, maxl = (uint32_t)len;
    const uint32_t maxf = (uint32_t)len - 1u;  // field levels: the steps recorded
    hipGraphExec_t gx = nullptr;
    hipGraph_t gr = nullptr;
    auto record = [&](int p) {
        return launch_record(c->prec, c->d, c->g, c->m, p, t0, maxl, maxf, r.store, r.qs, r.Fs, r.Us, r.phs, r.gvs,
                             r.dVs, r.mask_s, r.alist_s, r.acnt_s, c->stream);
    };
    auto one = [&](int p) {
        hipError_t e = record(p);
        return e == hipSuccess ? enqueue_step(c, p, false) : e;
    };
    int rc = IBLB_OK, left = len;
    while (!rc && left > 0) {
        const int p = (int)(c->t & 1);
        hipError_t e = hipSuccess;
        if (p == 0 && left >= kGraphSteps && use_graph && c->use_graph) {
            if (!gx) {
                e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
                hipError_t e1 = hipSuccess;
                for (int k = 0; k < kGraphSteps && e == hipSuccess && e1 == hipSuccess; ++k) e1 = one(k & 1);
                if (e == hipSuccess) e = hipStreamEndCapture(c->stream, &gr);
                if (e == hipSuccess) e = e1;
                if (e == hipSuccess) e = hipGraphInstantiate(&gx, gr, nullptr, nullptr, 0);
            }
            if (e == hipSuccess) e = hipGraphLaunch(gx, c->stream);
            c->t += kGraphSteps;
            left -= kGraphSteps;
        } else {
            e = one(p);
            c->t += 1;
            left -= 1;
        }
        if (e != hipSuccess) rc = hip_fail(c, e, "recording the window");
    }
    if (!rc) {
        hipError_t e = record((int)(c->t & 1));
        if (e != hipSuccess) rc = hip_fail(c, e, "storing the last level");
    }
    if (gx || gr) {
        if (c->stream) (void)hipStreamSynchronize(c->stream);
        if (gx) (void)hipGraphExecDestroy(gx);
        if (gr) (void)hipGraphDestroy(gr);
    }
    return rc;
}

// One reverse step, at level k of a recording, on stream s: (lam[1], qb[1])
// of time k + 1 to (lam[0], qb[0]) of time k, then the two swap roles.
hipError_t reverse_step(iblb_ctx *c, AdjState *a, const Recording &r, const AdjArgs &A, int k, hipStream_t s)
{
    const size_t n = (size_t)c->g.n, nv = (size_t)c->nv;
    const size_t fl = 3 * n * a->es, vl = 3 * nv * a->es;
    AdjLevel L;
    L.f0 = level(a, r, n, k);
    L.f1 = level(a, r, n, k + 1);
    L.F = (const char *)r.Fs + (size_t)k * fl;
    L.U = (const char *)r.Us + (size_t)k * fl;
    L.phs = (const char *)r.phs + (size_t)k * vl;
    L.gvs = (const char *)r.gvs + (size_t)k * vl;
    L.dV = r.dVs + k;
    L.q = r.qs + (size_t)k * 3 * nv;
    const size_t nw = (size_t)c->g.nt * (size_t)c->m.nwords;
    L.mask = r.mask_s + (size_t)k * nw;
    L.alist = r.alist_s + (size_t)k * c->g.nt;
    L.acnt = r.acnt_s + k;
    L.Xref = c->d.Xref;
    L.faces = c->d.faces;
    L.inc4 = c->d.inc4;
    L.fref = c->d.fref;
    const AdjWork W{a->ub,    a->lam[1], a->lam[0], a->Fb,    a->phib,
                    a->qb[1], a->qb[0],  a->grads,  a->tpart, a->vpart, (int *)a->serr};
    const hipError_t e = adj_reverse_kept(A, a->es == 8, L, W, s);
    std::swap(a->lam[0], a->lam[1]);
    std::swap(a->qb[0], a->qb[1]);
    return e;
}

// Checkpoint mode: segments from the last.  Each is recorded again from its
// checkpoint on the context's stream (which owns the state) into one of two
// recordings, while the reverse sweep of the segment after it runs from the
// other recording on a stream of its own; the launches of the two alternate
// step by step.  Events order each recording before its sweep, and each
// sweep before the recording that reuses its buffers.  Both streams are
// latency-bound at these sizes, so they share the device.
int sweep_segments(iblb_ctx *c, AdjState *a, const AdjArgs &A)
{
    const int every = a->every, nseg = (a->n + every - 1) / every;
    auto seg_len = [&](int sgm) { return std::min(every, a->n - sgm * every); };
    // the stream and events, created at the first sweep (each one that is
    // still missing, should an earlier attempt have failed part-way)
    if (!a->rs && hipStreamCreateWithFlags(&a->rs, hipStreamNonBlocking) != hipSuccess) {
        a->rs = nullptr;
        return fail(c, IBLB_E_DEVICE, "cannot create the reverse sweep's stream");
    }
    for (hipEvent_t *ev : {&a->recorded[0], &a->recorded[1], &a->swept[0], &a->swept[1]})
        if (!*ev && hipEventCreateWithFlags(ev, hipEventDisableTiming) != hipSuccess) {
            *ev = nullptr;
            return fail(c, IBLB_E_DEVICE, "cannot create the reverse sweep's events");
        }
    int rc = checkpoint(c, a->ck[(size_t)nseg - 1], false);
    if (rc) return rc;
    c->t = a->t0 + (long long)(nseg - 1) * every;
    rc = record_steps(c, a, a->rec[0], seg_len(nseg - 1), false);
    if (rc) return rc;
    HIP_TRY(c, hipEventRecord(a->recorded[0], c->stream));
    for (int sgm = nseg - 1; sgm >= 0; --sgm) {
        const int b = (nseg - 1 - sgm) & 1;  // this segment's recording; the one before it takes 1 - b
        const int lv = seg_len(sgm), lr = sgm > 0 ? seg_len(sgm - 1) : 0;
        HIP_TRY(c, hipStreamWaitEvent(a->rs, a->recorded[b], 0));
        Recording &next = a->rec[1 - b];
        uint32_t t0 = 0;
        if (lr) {
            if (sgm + 1 < nseg)  // rec[1 - b] was read by the sweep of segment sgm + 1
                HIP_TRY(c, hipStreamWaitEvent(c->stream, a->swept[1 - b], 0));
            rc = checkpoint(c, a->ck[(size_t)sgm - 1], false);
            if (rc) return rc;
            c->t = a->t0 + (long long)(sgm - 1) * every;
            t0 = (uint32_t)c->t;
        }
        auto record = [&](int p) {
            return launch_record(c->prec, c->d, c->g, c->m, p, t0, (uint32_t)lr, (uint32_t)lr - 1u, next.store,
                                 next.qs, next.Fs, next.Us, next.phs, next.gvs, next.dVs, next.mask_s, next.alist_s,
                                 next.acnt_s, c->stream);
        };
        for (int j = 0; j < std::max(lr, lv); ++j) {
            if (j < lr) {
                const int p = (int)(c->t & 1);
                hipError_t e = record(p);
                if (e == hipSuccess) e = enqueue_step(c, p, false);
                if (e != hipSuccess) return hip_fail(c, e, "recording a segment");
                c->t += 1;
            }
            if (j < lv) {
                const hipError_t e = reverse_step(c, a, a->rec[b], A, lv - 1 - j, a->rs);
                if (e != hipSuccess) return hip_fail(c, e, "reverse sweep");
            }
        }
        if (lr) {
            const hipError_t e = record((int)(c->t & 1));
            if (e != hipSuccess) return hip_fail(c, e, "storing the last level");
            HIP_TRY(c, hipEventRecord(a->recorded[1 - b], c->stream));
        }
        HIP_TRY(c, hipEventRecord(a->swept[b], a->rs));
    }
    // the results are read on the context's stream, after the last sweep
    HIP_TRY(c, hipStreamWaitEvent(c->stream, a->swept[(nseg - 1) & 1], 0));
    return IBLB_OK;
}

}  // namespace

extern "C" {

int iblb_adjoint_record(iblb_ctx *c, int32_t n_steps, int32_t every)
{
    if (!c || n_steps < 1 || every < 0) return IBLB_E_INVAL;
    if (!c->has_mesh) return fail(c, IBLB_E_STATE, "the adjoint needs a mesh");
    free_adjoint(c);
    AdjState *a = new AdjState();
    c->adj = a;
    a->t0 = c->t;
    a->n = n_steps;
    a->every = every;
    a->es = c->prec == IBLB_FP64 ? 8 : 4;
    int rc = IBLB_OK;
    if (every == 0) {
        // every time level kept: the reverse sweep needs no recompute
        rc = alloc_sweep(c, a, (size_t)n_steps + 1, 1);
        if (!rc) rc = record_steps(c, a, a->rec[0], n_steps, true);
        if (c->stream) (void)hipStreamSynchronize(c->stream);
    } else {
        // a device copy of the whole state every `every` steps; the sweep
        // records each segment again from its checkpoint
        a->snap = checkpoint_bytes(c);
        const int nseg = (n_steps + every - 1) / every;
        for (int k = 0; !rc && k <= nseg; ++k) {
            char *p = nullptr;
            if (hipMalloc(&p, a->snap) != hipSuccess)
                rc = fail(c, IBLB_E_DEVICE, "no device memory for the adjoint checkpoints");
            else
                a->ck.push_back(p);
        }
        for (int sgm = 0; !rc && sgm < nseg; ++sgm) {
            rc = checkpoint(c, a->ck[(size_t)sgm], true);
            if (!rc) rc = iblb_step(c, std::min(every, n_steps - sgm * every));
        }
        if (!rc) rc = checkpoint(c, a->ck[(size_t)nseg], true);
    }
    if (rc) free_adjoint(c);
    return rc;
}

int iblb_adjoint_backward(iblb_ctx *c, const double *dJdq, double *grads, double *dJdq0)
{
    if (!c || !dJdq || !grads) return IBLB_E_INVAL;
    AdjState *a = c->adj;
    if (!a) return fail(c, IBLB_E_STATE, "no recorded window (iblb_adjoint_record)");
    if (c->t != a->t0 + a->n) return fail(c, IBLB_E_STATE, "the context was stepped after the recorded window");
    int rc = sync_ctx(c);
    if (rc) return rc;
    const size_t n = (size_t)c->g.n, nv = (size_t)c->nv;
    if (!a->lam_buf[0]) {  // checkpoint mode: buffers for two segments, allocated at the first sweep
        rc = alloc_sweep(c, a, (size_t)std::min(a->every, a->n) + 1, a->n > a->every ? 2 : 1);
        if (rc) return rc;
    }
    // the same buffer roles at the start of every call
    for (int k = 0; k < 2; ++k) {
        a->lam[k] = a->lam_buf[k];
        a->qb[k] = a->qb_buf[k];
    }
    const AdjArgs A = adj_args(c);
    std::vector<double> soa(3 * nv);
    for (size_t i = 0; i < nv; ++i)
        for (int k = 0; k < 3; ++k) soa[(size_t)k * nv + i] = dJdq[3 * i + k];
    HIP_TRY(c, hipMemcpyAsync(a->qb[1], soa.data(), 3 * nv * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemsetAsync(a->lam[1], 0, 19 * n * 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(a->grads, 0, 6 * 8, c->stream));
    // the sweep clears ub itself after this first zeroing; the tau
    // derivative collects in per-block slots, added up below
    HIP_TRY(c, hipMemsetAsync(a->ub, 0, 3 * n * 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(a->tpart, 0, (size_t)adj_lb_blocks((long long)n) * 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(a->serr, 0, 8, c->stream));
    if (a->every == 0) {
        for (int k = a->n - 1; k >= 0; --k) HIP_TRY(c, reverse_step(c, a, a->rec[0], A, k, c->stream));
    } else {
        rc = sweep_segments(c, a, A);
        if (rc && a->rs) (void)hipStreamSynchronize(a->rs);
        // back to the end of the window
        const int nseg = (a->n + a->every - 1) / a->every;
        const int rc2 = checkpoint(c, a->ck[(size_t)nseg], false);
        c->t = a->t0 + a->n;
        if (rc) return rc;
        if (rc2) return rc2;
    }
    HIP_TRY(c, hipMemcpyAsync(grads, a->grads, 6 * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(soa.data(), a->qb[1], 3 * nv * 8, hipMemcpyDeviceToHost, c->stream));
    std::vector<double> tp((size_t)adj_lb_blocks((long long)n));
    HIP_TRY(c, hipMemcpyAsync(tp.data(), a->tpart, tp.size() * 8, hipMemcpyDeviceToHost, c->stream));
    int serr = 0;
    HIP_TRY(c, hipMemcpyAsync(&serr, a->serr, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (serr) {  // the sweep's errors join the context's
        int e = 0;
        HIP_TRY(c, hipMemcpy(&e, c->d.err, sizeof(int), hipMemcpyDeviceToHost));
        e |= serr;
        HIP_TRY(c, hipMemcpy(c->d.err, &e, sizeof(int), hipMemcpyHostToDevice));
    }
    for (double v : tp) grads[5] += v;  // the tau derivative, by blocks
    if (dJdq0)
        for (size_t i = 0; i < nv; ++i)
            for (int k = 0; k < 3; ++k) dJdq0[3 * i + k] = soa[(size_t)k * nv + i];
    return read_err(c);
}

int iblb_adjoint_release(iblb_ctx *c)
{
    if (!c) return IBLB_E_INVAL;
    free_adjoint(c);
    return IBLB_OK;
}

int iblb_sphere_fit_grad(int32_t nv, const double *q, int32_t wall, double z_wall, double exclude, double *h,
                         double *r2, double *dh_dq, double *dr2_dq)
{
    if (nv < 4 || !q || (wall != 0 && wall != 1) || !std::isfinite(z_wall) || !std::isfinite(exclude))
        return IBLB_E_INVAL;
    // vertices at least `exclude` from the wall plane, coordinates relative to
    // their centroid in x, y and to the wall plane in z
    std::vector<int> sel;
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < nv; ++i) {
        const double dz = wall ? z_wall - q[3 * i + 2] : q[3 * i + 2] - z_wall;
        if (dz >= exclude) {
            sel.push_back(i);
            sx += q[3 * i];
            sy += q[3 * i + 1];
        }
    }
    const int m = (int)sel.size();
    if (m < 4) return IBLB_E_STATE;
    sx /= m;
    sy /= m;
    auto row = [&](int i, double *p, double *Arow, double *b) {
        p[0] = q[3 * i] - sx;
        p[1] = q[3 * i + 1] - sy;
        p[2] = q[3 * i + 2] - z_wall;
        Arow[0] = 2.0 * p[0];
        Arow[1] = 2.0 * p[1];
        Arow[2] = 2.0 * p[2];
        Arow[3] = 1.0;
        *b = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    };
    // normal equations M s = A^T b of |p|^2 = 2 c.p + k
    double M[4][4] = {{0}}, r[4] = {0, 0, 0, 0};
    for (int i : sel) {
        double p[3], Ar[4], b;
        row(i, p, Ar, &b);
        for (int u = 0; u < 4; ++u) {
            r[u] += Ar[u] * b;
            for (int v = 0; v < 4; ++v) M[u][v] += Ar[u] * Ar[v];
        }
    }
    // inverse of M (symmetric positive definite) by Gauss-Jordan with pivoting
    double Mi[4][8];
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 8; ++v) Mi[u][v] = v < 4 ? M[u][v] : (v - 4 == u ? 1.0 : 0.0);
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int u = col + 1; u < 4; ++u)
            if (std::fabs(Mi[u][col]) > std::fabs(Mi[piv][col])) piv = u;
        if (!(std::fabs(Mi[piv][col]) > 0.0)) return IBLB_E_STATE;
        for (int v = 0; v < 8; ++v) std::swap(Mi[col][v], Mi[piv][v]);
        const double dgn = Mi[col][col];
        for (int v = 0; v < 8; ++v) Mi[col][v] /= dgn;
        for (int u = 0; u < 4; ++u)
            if (u != col) {
                const double f = Mi[u][col];
                for (int v = 0; v < 8; ++v) Mi[u][v] -= f * Mi[col][v];
            }
    }
    double s[4];
    for (int u = 0; u < 4; ++u) {
        s[u] = 0.0;
        for (int v = 0; v < 4; ++v) s[u] += Mi[u][4 + v] * r[v];
    }
    const double R = std::sqrt(s[3] + s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    const double hc = wall ? -s[2] : s[2];
    if (h) *h = hc + R;
    if (r2) *r2 = s[3] + s[0] * s[0] + s[1] * s[1];  // R^2 - hc^2
    // d(observable)/ds, then through the least-squares solution: with
    // w = M^-1 ds and e_i = b_i - A_i.s, dL/dA_i = e_i w - (A_i.w) s and
    // dL/db_i = A_i.w; A_i = (2 p_i, 1), b_i = |p_i|^2
    const double dh[4] = {s[0] / R, s[1] / R, (wall ? -1.0 : 1.0) + s[2] / R, 0.5 / R};
    const double dr[4] = {2.0 * s[0], 2.0 * s[1], 0.0, 1.0};
    for (int which = 0; which < 2; ++which) {
        double *out = which == 0 ? dh_dq : dr2_dq;
        if (!out) continue;
        const double *ds = which == 0 ? dh : dr;
        double w[4];
        for (int u = 0; u < 4; ++u) {
            w[u] = 0.0;
            for (int v = 0; v < 4; ++v) w[u] += Mi[u][4 + v] * ds[v];
        }
        for (int i = 0; i < 3 * nv; ++i) out[i] = 0.0;
        for (int i : sel) {
            double p[3], Ar[4], b;
            row(i, p, Ar, &b);
            const double e = b - (Ar[0] * s[0] + Ar[1] * s[1] + Ar[2] * s[2] + Ar[3] * s[3]);
            const double Aw = Ar[0] * w[0] + Ar[1] * w[1] + Ar[2] * w[2] + Ar[3] * w[3];
            for (int k = 0; k < 3; ++k) out[3 * i + k] = 2.0 * (e * w[k] - Aw * s[k]) + 2.0 * p[k] * Aw;
        }
    }
    return IBLB_OK;
}

}  // extern "C"
