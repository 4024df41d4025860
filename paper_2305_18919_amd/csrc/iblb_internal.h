// Internal interface between the host side of libiblb (iblb_api.cpp) and its
// HIP kernels (iblb_kernels.hip).  Not installed, not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct iblb_ctx;

namespace iblb {

// Force-density tiles: kTileX x kTileY x kTileZ fluid nodes (x fastest), the
// 64 lanes of one wavefront; the extents are powers of two, given as log2.
// An x-row of a tile is 8 consecutive nodes, 32 bytes of an FP32 population
// array: the spreading and moments gather the populations of the active tiles
// row by row, and rows of 4 nodes used a quarter of each 64-byte fetch.
constexpr int kTileLX = 3, kTileLY = 1, kTileLZ = 2;
constexpr int kTileX = 1 << kTileLX, kTileY = 1 << kTileLY, kTileZ = 1 << kTileLZ;
// one-dimensional stencil weights staged per listed vertex: one per tile coordinate
constexpr int kTileW = kTileX + kTileY + kTileZ;
static_assert(kTileX * kTileY * kTileZ == 64, "a tile is one wavefront");
static_assert(kTileX >= 1 && kTileY >= 1 && kTileZ >= 1, "tile extents");
// Maximum vertices whose stencil reaches one tile.
constexpr int kTileCap = 512;
// Maximum mesh vertices: the per-tile vertex masks hold nv bits in at most
// 1024 64-bit words (four per thread of a 256-thread spreading block).
constexpr int kMaxVertices = 65536;
// Device error bits.
constexpr int kErrNonFinite = 1;   // a vertex position left the finite range
constexpr int kErrOverflow = 2;    // a tile list overflowed kTileCap
constexpr int kErrDensity = 4;     // a node density became non-finite or left (0.5, 2)
constexpr int kErrMach = 8;        // |u| above 0.3 somewhere
constexpr int kErrList = 16;       // a tile list held an invalid vertex index

// Index of the r-th set bit (counted from 0, r < popcount(x)) of x, by halving.
__host__ __device__ inline int select_bit(uint64_t x, int r)
{
    int pos = 0;
    uint32_t v = (uint32_t)x;
    int c = __builtin_popcount(v);
    if (r >= c) {
        r -= c;
        pos = 32;
        v = (uint32_t)(x >> 32);
    }
    c = __builtin_popcount(v & 0xffffu);
    if (r >= c) {
        r -= c;
        pos += 16;
        v >>= 16;
    }
    c = __builtin_popcount(v & 0xffu);
    if (r >= c) {
        r -= c;
        pos += 8;
        v >>= 8;
    }
    c = __builtin_popcount(v & 0xfu);
    if (r >= c) {
        r -= c;
        pos += 4;
        v >>= 4;
    }
    c = __builtin_popcount(v & 0x3u);
    if (r >= c) {
        r -= c;
        pos += 2;
        v >>= 2;
    }
    return pos + (r >= (int)(v & 1u) ? 1 : 0);
}

struct alignas(16) Base {
    int x, y, z, ok;  // stencil corner floor(q)-1 (x, y wrapped; z absolute, wrapped if periodic); ok = 1 if finite
};

struct Grid {
    int nx, ny, nz;       // lattice
    int nzf, zoff;        // fluid layers, first fluid z
    int walls;            // 1: solid z layers, 0: periodic z
    long long n;          // fluid nodes
    int ntx, nty, ntz;    // tiles over fluid nodes
    int nt;
    long long pp;         // population pitch: population i of node k is f[i * pp + k]
};

struct LBArgs {
    Grid g;
    double tau_inv;       // 1/tau
    double guo;           // 1 - 1/(2 tau)
    double rho0;
    double body[3];
    double ulo[3], uhi[3];
    int has_fext;
};

struct MeshArgs {
    int nv, nf;
    double alpha[3];
    double eps_lo, eps_hi, xi, rc;
    double z_lo, z_hi;
    double origin[3];
    double kv_over_V0;    // k_V / V0
    int nparts;           // force-kernel blocks (32 vertices each) = number of volume partials
    int nwords;           // 64-bit words of one tile's vertex mask, ceil(nv / 64)
    int slots;            // incidence slots per vertex (a multiple of 8)
    int tiles_hint;       // active tiles counted at set-up (launch sizing only)
};

// Device buffers of one context (typed as void* where the precision varies).
struct Dev {
    void *f;              // [19][pp] populations (deviation; FP16/BF16: deviation / w_i, scaled), AA
                          // layout; entries n..pp-1 of each population are padding
    void *F;              // [3][n] IB force density of the step stamped in `stamp`
    void *Fext;           // [3][n] or null
    uint32_t *stamp;      // [nt] step+1 for which F of the tile is valid
    uint32_t *ctr;        // [2] step counter, ctr[t & 1] = t
    int *err;             // error bits
    // mesh
    double *q;            // [3][nv] FP64 positions
    double *Xref;         // [3][nv] FP64 reference (stress-free) positions
    int *faces;           // [3][nf]
    double *fref;         // [5][nf]: Ginv11, Ginv12, Ginv22, A0, 1/detG
    int4 *inc4;           // [nv][slots]: (a, b, c, face*4 + corner), faces ascending; unused slots w = -1
    void *U;              // [n][4] u(t+1) (x, y, z, unused) on the nodes of the active tiles
    void *phiSW;          // [3][nv] elastic + wall force
    void *gV;             // [3][nv] dV/dq
    Base *base;           // [nv]
    void *wts;            // [nv][12] phi4 weights (x 0..3, y 0..3, z 0..3)
    double *partials;     // [nparts]: sum (V_j - V0_j) per force block
    uint64_t *mask;       // [nt][nwords] bit v: vertex v's stencil reaches the tile (set by the
                          // move, read and cleared by the next step's spreading)
    uint8_t *act;         // [nt, padded to 4096] act_stamp(t) of the step t at which the tile is
                          // active (written by the previous move; 0 = never)
    uint32_t *acnt;       // [2] acnt[t & 1]: active tiles of step t (cleared by the move of step
                          // t - 1, counted up by the scan blocks of step t)
    int *alist;           // [nt] active tile indices of the step (in the order the scan found them)
    double *scratch;      // small FP64 scratch for queries (64 doubles)
    int num_cus;          // compute units of the device (launch sizing)
};

// One domain of a batch: its arrays, arguments and launch shape, read by every
// block of a batched dispatch that works on it.
struct DomRec {
    Dev d;
    LBArgs a;
    MeshArgs m;
    int bxw, nbx, nby;    // LB blocks: bxw x (256 / bxw) nodes of one z layer, nbx x nby per layer
    int nsp;              // spreading blocks
    int lb0;              // LB blocks run by the forces dispatch (the spreading dispatch runs the rest)
    int mblocks;          // moments blocks
};
// Domains per batch: a batched dispatch names a block's domain in 8 bits.
constexpr int kMaxBatch = 256;
// Batched dispatches of one step, in launch order.
enum { B_FORCES = 0, B_SPREAD = 1, B_MOMENTS = 2, B_MOVE = 3 };

// launchers (iblb_kernels.hip); precision 0 = FP64, 1 = FP32, 2 = FP16 and
// 3 = BF16 population storage (the last three compute in FP32)
hipError_t launch_init(int prec, const Dev &d, const LBArgs &a, int couette, hipStream_t s);
// p = t & 1 of the step (or of the current time for the debug kernels)
// bulk != 0: only the nodes outside this step's active tiles (mesh present);
// bulk == 0: every node, and the kernel advances the step counter (no mesh)
hipError_t launch_lb(int prec, const Dev &d, const LBArgs &a, int p, int bulk, hipStream_t s);
// interface forces and the step's list of active tiles; with_lb != 0: the same
// dispatch also runs its share of the LB of the nodes outside the active tiles
hipError_t launch_forces(int prec, const Dev &d, const LBArgs &a, const MeshArgs &m, int p, int with_lb,
                         hipStream_t s);
// spreading of the active tiles followed by their LB update; with_lb != 0:
// the same dispatch also runs its share of the LB of the nodes outside the
// active tiles
hipError_t launch_spread(int prec, const Dev &d, const LBArgs &a, const MeshArgs &m, int p, int with_lb,
                         hipStream_t s);
// u(t+1) on the nodes of the active tiles
hipError_t launch_moments(int prec, const Dev &d, const LBArgs &a, const MeshArgs &m, int p, hipStream_t s);
// interpolation, move, and the next step's act stamps and vertex masks
hipError_t launch_move(int prec, const Dev &d, const LBArgs &a, const MeshArgs &m, int p, hipStream_t s);
// the LB blocks of the nodes outside the active tiles: width (nodes along x;
// 256 / width rows of one z layer) and the share run by the forces dispatch
// (the spreading dispatch runs the rest)
int lb_block_width(const Grid &g);
double lb_share_with_forces();
// blocks of the moments dispatch of `waves` wavefronts each (launch sizing)
int moments_blocks(const Grid &g, const MeshArgs &m, int waves);
// blocks that list the active tiles in the forces dispatch
inline int scan_block_count(const Grid &g) { return (g.nt + 4095) / 4096; }
// act stamps and vertex masks of the current step from the stored positions
// (masks and stamps cleared beforehand)
hipError_t launch_stamp(const Dev &d, const Grid &g, const MeshArgs &m, int p, hipStream_t s);
// One batched dispatch `which` over `nblocks` blocks: entry k of `tab` is block
// k's domain (low 8 bits) and its block index within the single-domain
// dispatch of that domain (upper 24 bits).  vpw: vertices per wavefront of the
// move (1 or 2); spread_nw: wavefronts per block of the spreading dispatch (2
// or 4; its LB blocks of 256 nodes then span 4 / spread_nw table entries).
hipError_t launch_batch(int prec, int which, const DomRec *recs, const uint32_t *tab, int nblocks, int p, int vpw,
                        int spread_nw, hipStream_t s);
// err[k] = *recs[k].d.err for k < n
hipError_t launch_batch_errors(const DomRec *recs, int n, int *err, hipStream_t s);
// Discrete adjoint of the step (iblb_adjoint.hip), FP64 arithmetic: the
// constants of one context's step.  Fields are canonical [19][n] / [3][n]
// arrays (deviations f - w rho0, in the step's own precision), vertex arrays
// SoA [3][nv].
struct AdjArgs {
    Grid g;
    int nv, nf, slots;
    double rho0, omega;         // omega = 1/tau
    double body[3], ulo[3], uhi[3];
    double alpha[3], kv_over_V0, V0, eps_lo, eps_hi, xi, rc, z_lo, z_hi;
    double origin[3];
    int tile_blocks;            // blocks of the reverse spread over the active tiles (launch sizing)
};
// One reverse step from a recording (launch_record; every level of the
// window, or of one checkpoint segment): the level's arrays, element type
// double (fp64 != 0) or float, and the working arrays of the sweep.
struct AdjLevel {
    const void *f0, *f1;          // populations of time t and t + 1
    const void *F, *U;            // force density of step t (zero off its active tiles), u(t+1)
    const void *phs, *gvs;        // phi_S + phi_W and dV/dq of step t
    const double *dV;             // V - V0 of step t
    const double *q;              // positions of time t
    const uint64_t *mask;         // tile vertex masks of these positions, [tiles][ceil(nv / 64)]
    const int *alist;             // active tiles of step t and their count
    const uint32_t *acnt;
    const double *Xref;
    const int *faces;
    const int4 *inc4;
    const double *fref;
};
struct AdjWork {
    double *ub;     // [3][n] adjoint of u' over 2 rho(t+1) (element type of the level), zero at the step's start (ka_lb_adj clears it)
    double *lam1, *lam0;      // [19][n] adjoint populations at t + 1 and t (element type of the level)
    double *Fb;               // [3][n]
    double *phib, *qb1, *qb0; // [3][nv]
    double *grads;            // [6]: grads[0..4] accumulate here

    double *tpart;  // [adj_lb_blocks(n)] per-block running sums of the tau derivative
    double *vpart;  // [adj_vertex_blocks(nv)] per-block shares of grad V . phib
    int *err;         // the sweep's error bits (a tile list overflow), added to the context's
                      // once the sweep is done
};
// Blocks of the LB adjoint over n nodes and of the 64-lanes-per-vertex
// kernels over nv vertices (256 threads per block): the sizes of tpart, vpart.
inline int adj_lb_blocks(long long n) { return (int)((n + 255) / 256); }
inline int adj_vertex_blocks(long long nv) { return (int)((64 * nv + 255) / 256); }
hipError_t adj_reverse_kept(const AdjArgs &A, int fp64, const AdjLevel &L, const AdjWork &w, hipStream_t s);
// debug / query kernels
hipError_t launch_get_pops(int prec, const Dev &d, const Grid &g, int p, double *out, hipStream_t s);
// One step of an adjoint recording (device step counter t = ctr[p]): the
// populations (double for FP64 storage, else float) and positions of time t
// into level t - t0 (at most maxl) of [level][19][n] and [level][3][nv]; the
// fields of the step just taken into level t - 1 - t0 (at most maxf): force
// density on its active tiles (zero elsewhere) and u (on those tiles only) into [level][3][n], the
// nodal force parts phi_S + phi_W and dV/dq into [level][3][nv], V - V0 into
// [level]; the tiles' vertex masks of time t into [level][tiles][nwords], the
// step's active tile list and count into [level][tiles] and [level].
hipError_t launch_record(int prec, const Dev &d, const Grid &g, const MeshArgs &m, int p, uint32_t t0, uint32_t maxl,
                         uint32_t maxf, void *store, double *qs, void *Fs, void *Us, void *phs, void *gvs,
                         double *dVs, uint64_t *mask_s, int *alist_s, uint32_t *acnt_s, hipStream_t s);

hipError_t launch_set_pops(int prec, const Dev &d, const Grid &g, int p, const double *in, hipStream_t s);
hipError_t launch_get_fields(int prec, const Dev &d, const LBArgs &a, int p, double *rho, double *u, hipStream_t s);
hipError_t launch_get_force(int prec, const Dev &d, const LBArgs &a, int p, double *F, hipStream_t s);
hipError_t launch_nodal_forces(int prec, const Dev &d, const MeshArgs &m, double *phi, hipStream_t s);
hipError_t launch_mesh_moments(const Dev &d, const MeshArgs &m, double *out, hipStream_t s);
hipError_t launch_sphere_moments(const Dev &d, const MeshArgs &m, int wall_hi, double z_wall, double excl,
                                 const double *shift, double *out, hipStream_t s);
// circle fit on the mesh slice of the K vertices nearest the centroid plane;
// mom = the output of launch_mesh_moments (device), shift = (x, z)
hipError_t launch_slice_moments(const Dev &d, const MeshArgs &m, const double *mom, int K, int wall_hi,
                                double z_wall, double excl, const double *shift, double *out, hipStream_t s);

// Context accessors for entry points outside iblb_api.cpp.
long long ctx_fluid_nodes(const iblb_ctx *c);
int ctx_device(const iblb_ctx *c);
int ctx_fail(iblb_ctx *c, int code, const char *msg);  // records msg, returns code
// iblb_get_fields through a caller-chosen device staging buffer of 4 n doubles
// (rho [n], then u [3][n]); allocates nothing.
int get_fields_staged(iblb_ctx *c, double *staging, double *rho, double *u);
// Per-device set-up of the fixed staging array of iblb_get_fields_noalloc; run
// by iblb_create with `device` current, once per device.
void noalloc_setup(int device);

}  // namespace iblb
