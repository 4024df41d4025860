// HIP kernels of libiblb for gfx950 (MI355X): one IB-LB time step of
// arXiv:2305.18919 (the enumerated algorithm of the "Numerical
// implementation" section), plus the debug and query reductions.
//
// Per step, in stream order:
//   k_forces  eight lanes per vertex, one incident face each: elastic force
//             -dW/dq (Eqs. generalised_energy1, nodal_force_S), dV/dq (Eq.
//             nodal_force_V), wall force (Eq. LJ_interaction), FP64 block
//             partials of V - V0, and the vertex's phi4 stencil weights; one
//             more block compacts the step's active tiles
//   k_spread  one block per active tile (kTileX x kTileY x kTileZ nodes, one
//             lane each): gathers phi_i w_i(x) of the
//             vertices whose stencil reaches the tile, in ascending vertex order
//             (Eq. ibm-governing_eq2), no floating-point atomics, then the LB
//             update of the tile's nodes with that force; further blocks of the
//             same dispatch run the LB of every other fluid node (Eqs. LBeq, feq)
//   k_moments u(t+1) on the nodes of the active tiles, with F(t)/2
//   k_move    one or two vertices per wavefront, one lane per stencil node:
//             interpolation (Eq. ibm-governing_eq1), Euler update (Eq.
//             ibm_update_pos), the stamps and vertex masks of the tiles the
//             vertex reaches at t + 1, and the device step counter.
// Without a mesh the step is k_lb alone, over every fluid node.
//
// Step counter: ctr[2] in device memory, ctr[t & 1] = t.  Every kernel of
// step t is launched with p = t & 1 and reads t from ctr[p]; the last kernel
// of the step writes t + 1 into ctr[1 - p], which no kernel of step t reads.
// So a captured graph of two steps (p = 0, then p = 1) replays correctly
// without atomics, and the AA parity is a compile-time property of each
// launch.
//
// Data layout (all structure-of-arrays, x fastest):
//   populations f[19][pp] (N fluid nodes, row pitch pp >= N), deviations f_i - w_i rho0, in place
//   with the AA pattern: at even times slot (i, x) holds f_i(x); at odd times
//   slot (opp(i), x - c_i) holds f_i(x) (slot (i, x) when x - c_i is solid).
//   force density F[3][N], valid on a tile when stamp[tile] == step + 1.
#include "iblb_internal.h"

#include <math.h>

namespace iblb {
namespace {

// D3Q19 velocities in the canonical order of the ABI: rest, +-x, +-y, +-z,
// +-(1,1,0), +-(1,-1,0), +-(1,0,1), +-(1,0,-1), +-(0,1,1), +-(0,1,-1).
__device__ __forceinline__ constexpr int cx(int i)
{
    constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return t[i];
}
__device__ __forceinline__ constexpr int cy(int i)
{
    constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return t[i];
}
__device__ __forceinline__ constexpr int cz(int i)
{
    constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return t[i];
}
__device__ __forceinline__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// The ten populations that move along x (c_x != 0): their indices, and the
// place of population i among them.
__device__ __forceinline__ constexpr int xpop(int k)
{
    constexpr int t[10] = {1, 2, 7, 8, 9, 10, 11, 12, 13, 14};
    return t[k];
}
__device__ __forceinline__ constexpr int xslot(int i)
{
    constexpr int t[19] = {-1, 0, 1, -1, -1, -1, -1, 2, 3, 4, 5, 6, 7, 8, 9, -1, -1, -1, -1};
    return t[i];
}
template <typename T>
__device__ __forceinline__ constexpr T wgt(int i)
{
    return i == 0 ? T(1.0 / 3.0) : (i <= 6 ? T(1.0 / 18.0) : T(1.0 / 36.0));
}
// c_i . (x, y, z) with only the nonzero components of c_i (a product with a
// zero component is not folded away in IEEE arithmetic).
template <typename T>
__device__ __forceinline__ T cdot(int i, T x, T y, T z)
{
    T r = T(0);
    bool any = false;
    if (cx(i) != 0) { r = cx(i) > 0 ? x : -x; any = true; }
    if (cy(i) != 0) { const T t = cy(i) > 0 ? y : -y; r = any ? r + t : t; any = true; }
    if (cz(i) != 0) { const T t = cz(i) > 0 ? z : -z; r = any ? r + t : t; any = true; }
    return r;
}
// The collision pairs population i (odd) with i + 1: opposite velocities,
// equal weights.
__device__ constexpr bool pairs_opposite()
{
    for (int i = 1; i < 19; i += 2)
        if (cx(i + 1) != -cx(i) || cy(i + 1) != -cy(i) || cz(i + 1) != -cz(i) || opp(i) != i + 1 ||
            wgt<double>(i) != wgt<double>(i + 1))
            return false;
    return true;
}
static_assert(pairs_opposite(), "populations i and i + 1 (i odd) must be opposite");

// Population storage.  FP64 and FP32 hold the deviation f_i - w_i rho0 as
// it is.  FP16 and BF16 hold it relative to w_i (h_i = (f_i - w_i rho0) / w_i),
// FP16 scaled by 2^12 so that the deviations of slow flows (~1e-6) stay in its
// normal range (|h_i| up to 16 fits); the arithmetic on them is FP32 (C).  The
// conversions round to nearest even.  w_i = w_opp(i), so a population keeps
// its scale wherever the AA pattern stores it.
__device__ __forceinline__ constexpr float inv_w(int i) { return i == 0 ? 3.0f : (i <= 6 ? 18.0f : 36.0f); }

template <typename S>
struct Pop {
    using C = S;
    static __device__ __forceinline__ C get(S v, int) { return v; }
    static __device__ __forceinline__ S put(C v, int) { return v; }
};
template <>
struct Pop<_Float16> {
    using C = float;
    static __device__ __forceinline__ C get(_Float16 v, int i)
    {
        return float(v) * (i == 0 ? float(1.0 / 12288.0) : (i <= 6 ? float(1.0 / 73728.0) : float(1.0 / 147456.0)));
    }
    static __device__ __forceinline__ _Float16 put(C v, int i) { return (_Float16)(v * (4096.0f * inv_w(i))); }
};
template <>
struct Pop<__bf16> {
    using C = float;
    static __device__ __forceinline__ C get(__bf16 v, int i) { return float(v) * wgt<float>(i); }
    static __device__ __forceinline__ __bf16 put(C v, int i) { return (__bf16)(v * inv_w(i)); }
};

// Activity stamp of step t: one byte, (t mod 255) + 1, never 0, so a tile
// that was never marked (0) never matches.  A tile last marked a multiple of
// 255 steps ago matches again; it is then treated as active with an empty
// vertex mask, which gives the same LB update (zero interface force) at the
// cost of a little extra work.
__host__ __device__ __forceinline__ uint8_t act_stamp(uint32_t t) { return (uint8_t)(t % 255u + 1u); }

// Four values loaded or stored as one vector (16 bytes in FP32).
template <typename T>
struct alignas(4 * sizeof(T)) Quad {
    T v[4];
};

// a modulo n in [0, n); the common case, a already in range, skips the
// integer division
__device__ __forceinline__ int wrapi(int a, int n)
{
    if ((unsigned)a < (unsigned)n)
        return a;
    int r = a % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ long long nidx(const Grid &g, int x, int y, int zf)
{
    return ((long long)zf * g.ny + y) * g.nx + x;
}

__device__ __forceinline__ int tile_of(const Grid &g, int x, int y, int zf)
{
    return ((zf >> kTileLZ) * g.nty + (y >> kTileLY)) * g.ntx + (x >> kTileLX);
}

// 4-point stencil phi4, Eq. ibm-interpolation_stencil.
template <typename T>
__device__ __forceinline__ T phi4(T r)
{
    const T a = fabs(r);
    if (a <= T(1))
        return T(0.125) * (T(3) - T(2) * a + sqrt(T(1) + T(4) * a - T(4) * a * a));
    if (a <= T(2))
        return T(0.125) * (T(5) - T(2) * a - sqrt(T(-7) + T(12) * a - T(4) * a * a));
    return T(0);
}

// Wall force magnitude along the wall normal at centroid distance d,
// Eq. LJ_interaction: 48 eps [(xi/d)^12 - (xi/d)^6/2] / d, cut at rc, d >= xi/2.
template <typename T>
__device__ __forceinline__ T lj(T eps, T xi, T rc, T d)
{
    if (eps == T(0) || !(d < rc))
        return T(0);
    if (d < T(0.5) * xi)
        d = T(0.5) * xi;
    const T rd = T(1) / d;
    const T s = xi * rd;
    const T s2 = s * s;
    const T s6 = s2 * s2 * s2;
    return T(48) * eps * (s6 * s6 - T(0.5) * s6) * rd;
}

// Store that writes through the L2 of the issuing XCD to memory (system-scope
// coherence bits on a plain vector store).  Used for the populations: every
// kernel boundary writes back and invalidates the per-XCD L2s, and data
// written through leaves nothing dirty there, which shortens the boundary;
// the LB streams its output anyway.
template <typename T>
__device__ __forceinline__ void store_through(T *p, T v)
{
    if constexpr (sizeof(T) == 2)
        __hip_atomic_store(reinterpret_cast<unsigned short *>(p), __builtin_bit_cast(unsigned short, v),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    else
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Populations at time t in canonical order, for either AA layout.
// swapped = (t odd): f_i(x) is at slot (opp(i), x - c_i), or at (i, x) when
// x - c_i is not a fluid node.
// ---------------------------------------------------------------------------
// A node's index and the index offsets (modulo 2^32, periodic wrap applied)
// to its neighbours one step up and down each axis: a shifted node's index is
// then two or three 32-bit adds (node indices stay below 2^32).
struct Nbr {
    uint32_t me;
    uint32_t xp, xm, yp, ym, zp, zm;
    bool zp_ok, zm_ok;
};

__device__ __forceinline__ Nbr neighbours(const Grid &g, int x, int y, int zf)
{
    Nbr b;
    const uint32_t nx = (uint32_t)g.nx, sxy = nx * (uint32_t)g.ny;
    b.me = (uint32_t)nidx(g, x, y, zf);
    b.xp = (x + 1 == g.nx) ? 1u - nx : 1u;
    b.xm = (x == 0) ? nx - 1u : 0u - 1u;
    b.yp = (y + 1 == g.ny) ? nx - sxy : nx;
    b.ym = (y == 0) ? sxy - nx : 0u - nx;
    b.zp = sxy;
    b.zm = 0u - sxy;
    if (g.walls) {
        b.zp_ok = zf + 1 < g.nzf;
        b.zm_ok = zf - 1 >= 0;
    } else {
        b.zp_ok = b.zm_ok = true;
        const uint32_t all = sxy * (uint32_t)g.nzf;
        if (zf + 1 == g.nzf) b.zp = sxy - all;
        if (zf == 0) b.zm = all - sxy;
    }
    return b;
}

// node x + s*c_i (s = +1 destination, -1 source); returns false if not fluid
__device__ __forceinline__ bool shifted(const Nbr &b, int i, int s, uint32_t &out)
{
    const int ddx = s * cx(i), ddy = s * cy(i), ddz = s * cz(i);
    uint32_t o = b.me;
    if (ddx != 0) o += ddx > 0 ? b.xp : b.xm;
    if (ddy != 0) o += ddy > 0 ? b.yp : b.ym;
    bool ok = true;
    if (ddz > 0) { o += b.zp; ok = b.zp_ok; }
    if (ddz < 0) { o += b.zm; ok = b.zm_ok; }
    out = o;
    return ok;
}

// Population slot `idx` (= i * n + node) of f.  The byte offset is formed in
// 32 bits (the domain check keeps 19 n sizeof(S) below 2^32), which lets the
// compiler address from a uniform base with one register per access.
template <typename S>
__device__ __forceinline__ const S *pop_at(const S *f, uint32_t idx)
{
    return reinterpret_cast<const S *>(reinterpret_cast<const char *>(f) + idx * (uint32_t)sizeof(S));
}
template <typename S>
__device__ __forceinline__ S *pop_at(S *f, uint32_t idx)
{
    return reinterpret_cast<S *>(reinterpret_cast<char *>(f) + idx * (uint32_t)sizeof(S));
}

template <typename S, bool SWAPPED>
__device__ __forceinline__ void load_pops(const S *__restrict__ f, const Grid &g, int x, int y, int zf,
                                          typename Pop<S>::C *d)
{
    const uint32_t me = (uint32_t)nidx(g, x, y, zf);
    const uint32_t n = (uint32_t)g.pp;
    if (!SWAPPED) {
#pragma unroll
        for (int i = 0; i < 19; ++i)
            d[i] = Pop<S>::get(*pop_at(f, i * n + me), i);
    } else {
        const Nbr b = neighbours(g, x, y, zf);
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            uint32_t src;
            const bool ok = shifted(b, i, -1, src);
            d[i] = Pop<S>::get(*pop_at(f, ok ? opp(i) * n + src : i * n + me), i);
        }
    }
}

// ---------------------------------------------------------------------------
// LB: AA-pattern stream + collide
// ---------------------------------------------------------------------------
// Value v of the lane CTRL names (a DPP wave shift or rotation by one lane).
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_move(T v)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
    } else {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
        const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
        return __builtin_bit_cast(T, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    }
}

// Odd-step stores of the ten populations that move along x, for LB rows held
// whole by consecutive lanes: RW = 1, a row is one wavefront (64 nodes);
// RW = 2, a row is two consecutive wavefronts (128 nodes).  Node x's value
// belongs at x + c_x; each lane instead stores, at its own x (in the
// destination row), the value of node x - c_x, taken from the neighbouring
// lane by a wave shift (across the two halves of a row through LDS, and
// around the row's periodic seam).  Each wavefront then writes whole lines
// instead of lines offset by one node.  xv, xa, xf: per population the value,
// the aligned slot and whether the destination row is fluid (the same for the
// whole row); own: the node is this thread's to update.  Every lane of the
// block must get here.
template <typename S, int RW, typename T>
__device__ __forceinline__ void aligned_x_stores(S *__restrict__ f, const T *xv, const uint32_t *xa, const bool *xf,
                                                 bool own)
{
    constexpr int BACK = RW == 1 ? 0x13c : 0x138;  // lane k takes lane k - 1 (wave_ror:1 / wave_shr:1)
    constexpr int FWD = RW == 1 ? 0x134 : 0x130;   // lane k takes lane k + 1 (wave_rol:1 / wave_shl:1)
    // the block's linear thread index (k_lb runs two-dimensional blocks)
    const int tid = (int)(threadIdx.y * blockDim.x + threadIdx.x);
    const int lane = tid & 63, wave = tid >> 6;
    const int ow = own ? 1 : 0;
    T vs[10];
    int os[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        if (cx(xpop(k)) > 0) {
            vs[k] = dpp_move<BACK>(xv[k]);
            os[k] = dpp_move<BACK>(ow);
        } else {
            vs[k] = dpp_move<FWD>(xv[k]);
            os[k] = dpp_move<FWD>(ow);
        }
    }
    if constexpr (RW == 2) {
        // the value leaving one half of the row enters the other half (the
        // second half's last node wraps to the first half's first)
        __shared__ T ev[16][10];
        __shared__ int eo[16][10];
#pragma unroll
        for (int k = 0; k < 10; ++k)
            if (lane == (cx(xpop(k)) > 0 ? 63 : 0)) {
                ev[wave][k] = xv[k];
                eo[wave][k] = ow;
            }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 10; ++k)
            if (lane == (cx(xpop(k)) > 0 ? 0 : 63)) {
                vs[k] = ev[wave ^ 1][k];
                os[k] = eo[wave ^ 1][k];
            }
    }
#pragma unroll
    for (int k = 0; k < 10; ++k)
        if (xf[k] && os[k])
            store_through(pop_at(f, xa[k]), Pop<S>::put(vs[k], xpop(k)));
}

// Collision of node (x, y, zf) whose populations d (canonical order, time t)
// are in hand, with the immersed-boundary force density (fx, fy, fz) of this
// step (body force and external field are added here), and the AA write-back.
// RW > 0: whole LB rows per lane group, odd steps store the x-moving
// populations aligned (aligned_x_stores); write == false: the node is not
// this thread's, nothing is stored or flagged (its lanes still take part).
template <typename S, bool ODD, int RW = 0, typename T = typename Pop<S>::C>
__device__ __forceinline__ void lb_collide(S *__restrict__ f, const T *__restrict__ Fext, int *err,
                                           const LBArgs &a, int x, int y, int zf, const T *d, T fx, T fy, T fz,
                                           bool write = true)
{
    const Grid &g = a.g;
    const long long n = g.n;
    const long long me = nidx(g, x, y, zf);
    const Nbr b = neighbours(g, x, y, zf);

    // force density: body force + IB force + external
    T Fx = T(a.body[0]) + fx, Fy = T(a.body[1]) + fy, Fz = T(a.body[2]) + fz;
    if (a.has_fext) {
        Fx += Fext[me];
        Fy += Fext[n + me];
        Fz += Fext[2 * n + me];
    }

    // density and momentum from the sums and differences of opposite pairs
    T drho = d[0], mx = T(0), my = T(0), mz = T(0);
#pragma unroll
    for (int i = 1; i < 19; i += 2) {
        const T dif = d[i] - d[i + 1];
        drho += d[i] + d[i + 1];
        if (cx(i) != 0) mx += T(cx(i)) * dif;
        if (cy(i) != 0) my += T(cy(i)) * dif;
        if (cz(i) != 0) mz += T(cz(i)) * dif;
    }
    const T rho = T(a.rho0) + drho;
    // three divisions, not one reciprocal: the reciprocal's rounding is the
    // same for neighbouring nodes of equal density and biased the FP32
    // velocities of a sheared run (4x the error after 2000 steps)
    const T ux = (mx + T(0.5) * Fx) / rho;
    const T uy = (my + T(0.5) * Fy) / rho;
    const T uz = (mz + T(0.5) * Fz) / rho;
    const T uu = ux * ux + uy * uy + uz * uz;
    if (write && !(fabs(drho) < T(0.5)))
        atomicOr(err, kErrDensity);
    if (write && uu > T(0.09))
        atomicOr(err, kErrMach);

    const T tinv = T(a.tau_inv), guo = T(a.guo);
    const T uF = ux * Fx + uy * Fy + uz * Fz;
    constexpr bool AL = ODD && RW > 0;
    T xv[10] = {};
    uint32_t xa[10] = {};
    bool xf[10] = {};
    // post-collision value of population i: write-back, bounce-back off a wall
    auto emit = [&](int i, T post) {
        const T w = wgt<T>(i);
        uint32_t dst;
        const bool fluid = shifted(b, i, +1, dst);
        if (!fluid) {
            // half-way bounce-back off a (moving) wall: -2 w rho (c.u_w)/c_s^2
            const double *uw = cz(i) < 0 ? a.ulo : a.uhi;
            const T cuw = T(cx(i)) * T(uw[0]) + T(cy(i)) * T(uw[1]) + T(cz(i)) * T(uw[2]);
            post -= T(6) * w * rho * cuw;
        }
        const uint32_t n32 = (uint32_t)g.pp, me32 = (uint32_t)me;
        if (AL && cx(i) != 0)
            xf[xslot(i)] = fluid;
        if (AL && cx(i) != 0 && fluid) {
            xv[xslot(i)] = post;
            xa[xslot(i)] = i * n32 + dst - (cx(i) > 0 ? b.xp : b.xm);
        } else if (write) {
            if (!ODD || !fluid)
                store_through(pop_at(f, opp(i) * n32 + me32), Pop<S>::put(post, i));
            else
                store_through(pop_at(f, i * n32 + dst), Pop<S>::put(post, i));
        }
    };
    // BGK with Guo's source: post_i = d_i - (d_i - deq_i) / tau + S_i, with
    // deq_i = w_i drho + w_i rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u) and
    // S_i = w_i (1 - 1/(2 tau)) (3 (c_i - u).F + 9 (c.F)(c.u)).  Populations
    // i and i + 1 (i odd) have c_{i+1} = -c_i and the same weight: the parts
    // of deq and S even in c are computed once for both, the odd parts with
    // both signs.  The relaxation keeps the form d - (d - deq) / tau, whose
    // rounding scales with the (small) non-equilibrium part.
    {
        const T w = wgt<T>(0);
        const T deq = w * drho - w * rho * (T(1.5) * uu);
        const T src = w * guo * (T(-3) * uF);
        emit(0, d[0] - (d[0] - deq) * tinv + src);
    }
#pragma unroll
    for (int i = 1; i < 19; i += 2) {
        const T w = wgt<T>(i);
        const T cu = cdot<T>(i, ux, uy, uz);
        const T cF = cdot<T>(i, Fx, Fy, Fz);
        const T wr = w * rho, wg = w * guo;
        const T qe = w * drho + wr * (T(4.5) * cu * cu - T(1.5) * uu), qo = T(3) * wr * cu;
        const T se = wg * (T(9) * cF * cu - T(3) * uF), so = (T(3) * wg) * cF;
        const T dp = qe + qo, dm = qe - qo;
        emit(i, d[i] - (d[i] - dp) * tinv + (se + so));
        emit(i + 1, d[i + 1] - (d[i + 1] - dm) * tinv + (se - so));
    }
    if constexpr (AL)
        aligned_x_stores<S, RW>(f, xv, xa, xf, write);
}

// LB update of node (x, y, zf): load its populations, collide, write back.
template <typename S, bool ODD, typename T = typename Pop<S>::C>
__device__ __forceinline__ void lb_node(S *__restrict__ f, const T *__restrict__ Fext, int *err, const LBArgs &a,
                                        int x, int y, int zf, T fx, T fy, T fz)
{
    T d[19];
    load_pops<S, ODD>(f, a.g, x, y, zf, d);
    lb_collide<S, ODD>(f, Fext, err, a, x, y, zf, d, fx, fy, fz);
}

// LB of one node of the LB tiling (blocks of bxw x (256 / bxw) nodes in one
// z layer, numbered x fastest), unless its tile is active at step t (those
// nodes are updated by the spreading, with their force).
// A block of NT < 256 threads runs part `sub` of the 256-node LB block b (its
// consecutive rows NT / bxw at a time).
template <typename S, bool ODD, int NT = 256, typename T = typename Pop<S>::C>
__device__ __forceinline__ void bulk_lb_block(int b, S *__restrict__ f, const T *__restrict__ Fext,
                                              const uint8_t *__restrict__ act, uint32_t t, int *err, const LBArgs &a,
                                              int bxw, int nbx, int nby, int sub = 0)
{
    const int zf = b / (nbx * nby);
    const int rem = b - zf * nbx * nby;
    const int byi = rem / nbx, bxi = rem - byi * nbx;
    const int x = bxi * bxw + (int)(threadIdx.x % (unsigned)bxw);
    const int y = byi * (256 / bxw) + sub * (NT / bxw) + (int)(threadIdx.x / (unsigned)bxw);
    if (x >= a.g.nx || y >= a.g.ny)
        return;
    if (act[tile_of(a.g, x, y, zf)] == act_stamp(t))
        return;
    lb_node<S, ODD>(f, Fext, err, a, x, y, zf, T(0), T(0), T(0));
}

// LB over the fluid nodes.  Without a mesh (act == null) every node, and the
// kernel advances the step counter.  With a mesh only the nodes outside this
// step's active tiles (act[tile] != act_stamp(t)): it runs concurrently with the
// force and spreading kernels, which update the active tiles themselves.
// In the AA pattern each node reads and writes only its own 19 slots, so the
// two node sets never touch the same memory.
// RW > 0 (the block's rows are the lattice's whole rows of 64 or 128 nodes):
// odd steps store the x-moving populations aligned; every lane takes part,
// rows beyond the lattice on copies of its last row that store nothing.
template <typename S, bool ODD, int RW>
__global__ __launch_bounds__(1024) void k_lb(S *__restrict__ f, const typename Pop<S>::C *__restrict__ Fext,
                                            const uint8_t *__restrict__ act, uint32_t *ctr, int *err, LBArgs a)
{
    using T = typename Pop<S>::C;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int zf = blockIdx.z;
    if constexpr (ODD && RW > 0) {
        const int tid = threadIdx.y * blockDim.x + threadIdx.x;
        if (act == nullptr && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && tid == 0)
            ctr[0] = ctr[1] + 1u;
        const bool in = y < a.g.ny;
        const int yc = in ? y : a.g.ny - 1;
        bool own = in;
        if (act != nullptr)
            own = own && act[tile_of(a.g, x, yc, zf)] != act_stamp(ctr[1]);
        T d[19];
        load_pops<S, ODD>(f, a.g, x, yc, zf, d);
        lb_collide<S, ODD, RW>(f, Fext, err, a, x, yc, zf, d, T(0), T(0), T(0), own);
        return;
    }
    if (act == nullptr) {
        // only the thread that advances the counter reads it: the other
        // wavefronts go straight to their populations
        if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0 && threadIdx.y == 0)
            ctr[ODD ? 0 : 1] = ctr[ODD ? 1 : 0] + 1u;
    } else {
        if (x >= a.g.nx || y >= a.g.ny)
            return;
        if (act[tile_of(a.g, x, y, zf)] == act_stamp(ctr[ODD ? 1 : 0]))
            return;
    }
    if (x >= a.g.nx || y >= a.g.ny)
        return;
    lb_node<S, ODD>(f, Fext, err, a, x, y, zf, T(0), T(0), T(0));
}

template <typename S>
__global__ __launch_bounds__(256) void k_init(S *__restrict__ f, LBArgs a, int couette)
{
    using T = typename Pop<S>::C;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int zf = blockIdx.z;
    if (x >= a.g.nx || y >= a.g.ny)
        return;
    const Grid &g = a.g;
    const long long me = nidx(g, x, y, zf);
    double u[3] = {0.0, 0.0, 0.0};
    if (couette && g.walls) {
        const double z = zf + g.zoff, zlo = 0.5, zhi = g.nz - 1.5;
        for (int k = 0; k < 3; ++k)
            u[k] = a.ulo[k] + (a.uhi[k] - a.ulo[k]) * (z - zlo) / (zhi - zlo);
    }
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
        const double w = wgt<double>(i);
        f[i * g.pp + me] = Pop<S>::put(T(w * a.rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu)), i);
    }
}

// ---------------------------------------------------------------------------
// Active tiles.  A vertex at q touches every tile that holds a fluid node of
// its 4^3 stencil, floor(q) - 1 + {0..3} along each axis (x, y wrapped; z
// wrapped if periodic, clipped to the fluid layers between walls).  Along an
// axis the stencil's nodes form runs of consecutive nodes in one tile; a run
// opens at offset k when node k is in the fluid and node k - 1 is not, or lies
// in another tile: bit k of the mask is set when offset k opens a run (at
// most three per axis).  The openings name every touched tile; a periodic axis
// whose last tile is partial can name one twice, which the marks (a stamp and
// an OR) absorb.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned runs_wrapped(int b, int n, int sh)
{
    unsigned mask = 1u;
    int prev = wrapi(b, n) >> sh;
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        const int tl = wrapi(b + k, n) >> sh;
        mask |= tl != prev ? 1u << k : 0u;
        prev = tl;
    }
    return mask;
}

// b = first stencil layer counted in fluid layers (may be outside [0, nzf))
__device__ __forceinline__ unsigned runs_clipped(int b, int nzf, int sh)
{
    unsigned mask = 0u;
    int prev = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int zf = b + k;
        const bool in = zf >= 0 && zf < nzf;
        const int tl = in ? zf >> sh : -1;
        mask |= (in && tl != prev) ? 1u << k : 0u;
        prev = tl;
    }
    return mask;
}

struct StencilRuns {
    int bx, by, bz;          // stencil corner floor(q) - 1
    unsigned mx, my, mz;     // run openings per axis
};

__device__ __forceinline__ StencilRuns stencil_runs(const Grid &g, double qx, double qy, double qz)
{
    StencilRuns r;
    r.bx = (int)floor(qx) - 1;
    r.by = (int)floor(qy) - 1;
    r.bz = (int)floor(qz) - 1;
    r.mx = runs_wrapped(r.bx, g.nx, kTileLX);
    r.my = runs_wrapped(r.by, g.ny, kTileLY);
    r.mz = g.walls ? runs_clipped(r.bz - g.zoff, g.nzf, kTileLZ) : runs_wrapped(r.bz, g.nz, kTileLZ);
    return r;
}

// tile of the stencil node at offsets (kx, ky, kz)
__device__ __forceinline__ int stencil_tile(const Grid &g, const StencilRuns &r, int kx, int ky, int kz)
{
    const int x = wrapi(r.bx + kx, g.nx), y = wrapi(r.by + ky, g.ny);
    const int zf = g.walls ? r.bz + kz - g.zoff : wrapi(r.bz + kz, g.nz);
    return tile_of(g, x, y, zf);
}

// Inclusive sum over the 64 lanes of a wavefront, in lane order, with DPP
// lane moves: shifts by 1, 2, 4 and 8 lanes within each row of 16, then the
// last lane of row 0 added to row 1 and of row 2 to row 3 (row_bcast:15), and
// the last lane of row 1 to rows 2 and 3 (row_bcast:31).  A lane whose source
// lies outside its row, or whose row the mask leaves out, adds 0.
__device__ __forceinline__ int wave_incl_scan(int c)
{
    c += __builtin_amdgcn_update_dpp(0, c, 0x111, 0xf, 0xf, false);  // row_shr:1
    c += __builtin_amdgcn_update_dpp(0, c, 0x112, 0xf, 0xf, false);  // row_shr:2
    c += __builtin_amdgcn_update_dpp(0, c, 0x114, 0xf, 0xf, false);  // row_shr:4
    c += __builtin_amdgcn_update_dpp(0, c, 0x118, 0xf, 0xf, false);  // row_shr:8
    c += __builtin_amdgcn_update_dpp(0, c, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    c += __builtin_amdgcn_update_dpp(0, c, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    return c;
}

// The step's active tiles, those stamped act[tile] == act_stamp(t) by the
// previous move, compacted into alist: one 256-thread block per chunk of 4096
// tiles, 16 per thread (one 16-byte load each; the array is padded to whole
// chunks).  A block-wide prefix sum of the per-thread counts orders the
// chunk's tiles, and one atomic add on the step's counter (cleared by the
// previous move) reserves their place in the list.  Chunks therefore land in
// the order their blocks finish; every consumer of the list treats its tiles
// independently, so nothing computed depends on that order.
constexpr int kScanChunk = 4096;

__device__ __forceinline__ int scan_blocks(const Grid &g) { return (g.nt + kScanChunk - 1) / kScanChunk; }

__device__ __forceinline__ void scan_block(int chunk, const uint8_t *__restrict__ act, uint32_t *acnt, int *alist,
                                           uint32_t t)
{
    __shared__ int swt[4];
    __shared__ uint32_t sbase;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t st = act_stamp(t);
    const uint4 v = reinterpret_cast<const uint4 *>(act)[chunk * (kScanChunk / 16) + tid];
    // bit b: the b-th of this thread's 16 tiles carries the stamp
    uint32_t msk = 0u;
    const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            msk |= ((w4[q] >> (8 * b)) & 0xffu) == st ? 1u << (4 * q + b) : 0u;
    const int c = __popc(msk);
    const int incl = wave_incl_scan(c);
    if (lane == 63)
        swt[wave] = incl;
    __syncthreads();
    if (tid == 0) {
        const int tot = swt[0] + swt[1] + swt[2] + swt[3];
        sbase = tot ? atomicAdd(acnt, (uint32_t)tot) : 0u;
    }
    __syncthreads();
    int o = (int)sbase + incl - c;
    for (int w = 0; w < wave; ++w)
        o += swt[w];
    const int k0 = chunk * kScanChunk + tid * 16;
    while (msk != 0u) {
        alist[o++] = k0 + __builtin_ctz(msk);
        msk &= msk - 1u;
    }
}

// ---------------------------------------------------------------------------
// Interface forces, one thread per vertex
// ---------------------------------------------------------------------------
constexpr double kSixth = 1.0 / 6.0;

__device__ __forceinline__ void cross6(double ux, double uy, double uz, double vx, double vy, double vz, double *o)
{
    o[0] = (uy * vz - uz * vy) * kSixth;
    o[1] = (uz * vx - ux * vz) * kSixth;
    o[2] = (ux * vy - uy * vx) * kSixth;
}

__device__ __forceinline__ double triple(double ax, double ay, double az, double bx, double by, double bz, double cx_,
                                         double cy_, double cz_)
{
    return ax * (by * cz_ - bz * cy_) + ay * (bz * cx_ - bx * cz_) + az * (bx * cy_ - by * cx_);
}

// V_j(q) - V_j(X) of the tetrahedron (o, a, b, c), expanded exactly in the
// displacements from the reference vertices X: the seven triple products that
// contain at least one displacement (the triple product is trilinear).  Each
// term is as small as the change itself, so it survives FP64 rounding.
__device__ __forceinline__ double volume_change(const double *__restrict__ X, int nv, int ia, int ib, int ic,
                                                double ax, double ay, double az, double bx, double by,
                                                double bz, double cxv, double cyv, double czv, const double *o)
{
    const double Ax = X[ia] - o[0], Ay = X[nv + ia] - o[1], Az = X[2 * nv + ia] - o[2];
    const double Bx = X[ib] - o[0], By = X[nv + ib] - o[1], Bz = X[2 * nv + ib] - o[2];
    const double Cx = X[ic] - o[0], Cy = X[nv + ic] - o[1], Cz = X[2 * nv + ic] - o[2];
    const double dax = ax - X[ia], day = ay - X[nv + ia], daz = az - X[2 * nv + ia];
    const double dbx = bx - X[ib], dby = by - X[nv + ib], dbz = bz - X[2 * nv + ib];
    const double dcx = cxv - X[ic], dcy = cyv - X[nv + ic], dcz = czv - X[2 * nv + ic];
    const double t = triple(dax, day, daz, Bx, By, Bz, Cx, Cy, Cz) + triple(Ax, Ay, Az, dbx, dby, dbz, Cx, Cy, Cz) +
                     triple(Ax, Ay, Az, Bx, By, Bz, dcx, dcy, dcz) + triple(dax, day, daz, dbx, dby, dbz, Cx, Cy, Cz) +
                     triple(dax, day, daz, Bx, By, Bz, dcx, dcy, dcz) + triple(Ax, Ay, Az, dbx, dby, dbz, dcx, dcy, dcz) +
                     triple(dax, day, daz, dbx, dby, dbz, dcx, dcy, dcz);
    return t * kSixth;
}

// Eight lanes per vertex (32 vertices per 256-thread block); lane k of a
// vertex handles its incident faces k, k + 8, ... (fixed incidence slots, so
// the first entry is read without a lookup); the group sums by butterfly.
template <typename T>
__device__ __forceinline__ void forces_block(int blk, const double *__restrict__ q, const double *__restrict__ Xref,
                                             const int4 *__restrict__ inc4,
                                             const double *__restrict__ fref, T *__restrict__ phiSW,
                                             T *__restrict__ gVout, Base *__restrict__ base, T *__restrict__ wts,
                                             double *__restrict__ partials, int *err, const Grid &g,
                                             const MeshArgs &m)
{
    __shared__ double red[4];
    const int sub = threadIdx.x & 7;
    const int v = blk * 32 + (threadIdx.x >> 3);
    const int nv = m.nv, nf = m.nf;
    double dvol = 0.0;
    T fs[3] = {T(0), T(0), T(0)};
    T gv[3] = {T(0), T(0), T(0)};
    if (v < nv) {
        const T a1 = T(m.alpha[0]), a2 = T(m.alpha[1]), a3 = T(m.alpha[2]);
        const int4 *ev = inc4 + (long long)v * m.slots;
        for (int k = sub; k < m.slots; k += 8) {
            const int4 e = ev[k];
            if (e.w < 0)
                break;  // the vertex's entries come first, unused slots last
            const int ia = e.x, ib = e.y, ic = e.z, j = e.w >> 2, corner = e.w & 3;
            const double ax = q[ia], ay = q[nv + ia], az = q[2 * nv + ia];
            const double bx = q[ib], by = q[nv + ib], bz = q[2 * nv + ib];
            const double cxv = q[ic], cyv = q[nv + ic], czv = q[2 * nv + ic];
            // elastic corner forces of the face: dW/de1 = 2(S11 e1 + S12 e2), dW/de2 = 2(S12 e1 + S22 e2)
            const T e1x = T(bx - ax), e1y = T(by - ay), e1z = T(bz - az);
            const T e2x = T(cxv - ax), e2y = T(cyv - ay), e2z = T(czv - az);
            const T g11 = e1x * e1x + e1y * e1y + e1z * e1z;
            const T g12 = e1x * e2x + e1y * e2y + e1z * e2z;
            const T g22 = e2x * e2x + e2y * e2y + e2z * e2z;
            const T detg = g11 * g22 - g12 * g12;
            const T Gi11 = T(fref[j]), Gi12 = T(fref[nf + j]), Gi22 = T(fref[2 * nf + j]);
            const T A0 = T(fref[3 * nf + j]), idetG = T(fref[4 * nf + j]);
            const T J = detg * idetG;
            const T lnJ = log(J);
            const T w1 = T(0.5) * a3;
            // w2 adj(g) / det G, with w2 = [(a1 - a3)/2 + (a1 + a2)/4 ln J] / J
            const T w2g = (T(0.5) * (a1 - a3) + T(0.25) * (a1 + a2) * lnJ) / J * idetG;
            const T S11 = A0 * (w1 * Gi11 + w2g * g22);
            const T S12 = A0 * (w1 * Gi12 - w2g * g12);
            const T S22 = A0 * (w1 * Gi22 + w2g * g11);
            const T Fb[3] = {T(-2) * (S11 * e1x + S12 * e2x), T(-2) * (S11 * e1y + S12 * e2y),
                             T(-2) * (S11 * e1z + S12 * e2z)};
            const T Fc[3] = {T(-2) * (S12 * e1x + S22 * e2x), T(-2) * (S12 * e1y + S22 * e2y),
                             T(-2) * (S12 * e1z + S22 * e2z)};
            // volume gradient of this face at this corner, relative to the origin
            const double Ax = ax - m.origin[0], Ay = ay - m.origin[1], Az = az - m.origin[2];
            const double Bx = bx - m.origin[0], By = by - m.origin[1], Bz = bz - m.origin[2];
            const double Cx = cxv - m.origin[0], Cy = cyv - m.origin[1], Cz = czv - m.origin[2];
            double dv[3];
            if (corner == 0) {
                fs[0] += -Fb[0] - Fc[0];
                fs[1] += -Fb[1] - Fc[1];
                fs[2] += -Fb[2] - Fc[2];
                cross6(Bx, By, Bz, Cx, Cy, Cz, dv);
                // owner of the face: accumulate V_j - V0_j in FP64
                dvol += volume_change(Xref, nv, ia, ib, ic, ax, ay, az, bx, by, bz, cxv, cyv, czv, m.origin);
            } else if (corner == 1) {
                fs[0] += Fb[0];
                fs[1] += Fb[1];
                fs[2] += Fb[2];
                cross6(Cx, Cy, Cz, Ax, Ay, Az, dv);
            } else {
                fs[0] += Fc[0];
                fs[1] += Fc[1];
                fs[2] += Fc[2];
                cross6(Ax, Ay, Az, Bx, By, Bz, dv);
            }
            gv[0] += T(dv[0]);
            gv[1] += T(dv[1]);
            gv[2] += T(dv[2]);
            if (g.walls) {
                const double cz3 = (az + bz + czv) / 3.0;
                const T fzw = lj<T>(T(m.eps_lo), T(m.xi), T(m.rc), T(cz3 - m.z_lo)) -
                              lj<T>(T(m.eps_hi), T(m.xi), T(m.rc), T(m.z_hi - cz3));
                fs[2] += fzw / T(3);
            }
        }
    }
#pragma unroll
    for (int off = 1; off < 8; off <<= 1)
        for (int c = 0; c < 3; ++c) {
            fs[c] += __shfl_xor(fs[c], off, 64);
            gv[c] += __shfl_xor(gv[c], off, 64);
        }
    if (v < nv && sub == 0) {
        phiSW[v] = fs[0];
        phiSW[nv + v] = fs[1];
        phiSW[2 * nv + v] = fs[2];
        gVout[v] = gv[0];
        gVout[nv + v] = gv[1];
        gVout[2 * nv + v] = gv[2];
    }
    // stencil corner and phi4 weights of this vertex for the spreading:
    // sub-lanes 0..3 compute the x, y, z weights of offset `sub`, sub-lane 4 the corner
    if (v < nv && sub < 5) {
        const double qx = q[v], qy = q[nv + v], qz = q[2 * nv + v];
        if (fabs(qx) < 1e6 && fabs(qy) < 1e6 && fabs(qz) < 1e6) {
            const int fx = (int)floor(qx) - 1, fy = (int)floor(qy) - 1, fz = (int)floor(qz) - 1;
            if (sub < 4) {
                wts[v * 12 + sub] = phi4<T>(T((double)(fx + sub) - qx));
                wts[v * 12 + 4 + sub] = phi4<T>(T((double)(fy + sub) - qy));
                wts[v * 12 + 8 + sub] = phi4<T>(T((double)(fz + sub) - qz));
            } else {
                Base bs;
                bs.x = wrapi(fx, g.nx);
                bs.y = wrapi(fy, g.ny);
                bs.z = g.walls ? fz : wrapi(fz, g.nz);
                bs.ok = 1;
                base[v] = bs;
            }
        } else if (sub == 4) {
            Base bs;
            bs.x = bs.y = bs.z = 0;
            bs.ok = 0;
            base[v] = bs;
            atomicOr(err, kErrNonFinite);
        }
    }
    // FP64 block partial of V - V0: a butterfly in each wavefront, then the
    // four wavefront sums in order (a fixed order)
    dvol = wave_sum<double>(dvol);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = dvol;
    __syncthreads();
    if (threadIdx.x == 0)
        partials[blk] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Block b of n renumbered so that the blocks the hardware dispatches to one
// XCD (b mod 8, round-robin) take a contiguous range: the force blocks of one
// XCD then read neighbouring vertices, whose positions share its L2.  A
// permutation of [0, n), so results do not change.
__device__ __forceinline__ int xcd_block(int b, int n)
{
    const int q = n / 8, r = n % 8, x = b % 8, k = b / 8;
    return x * q + (x < r ? x : r) + k;
}

// Blocks [0, nparts) compute the interface forces, the next scan_blocks
// blocks list the step's active tiles, and the blocks after them (if any) run
// the first LB blocks of the nodes outside the active tiles (the spreading
// dispatch runs the rest).
template <typename S, int P, typename T = typename Pop<S>::C>
__device__ __forceinline__ void forces_dispatch(int blk, const double *__restrict__ q,
                                                const double *__restrict__ Xref, const int4 *__restrict__ inc4,
                                                const double *__restrict__ fref, T *__restrict__ phiSW,
                                                T *__restrict__ gVout, Base *__restrict__ base,
                                                T *__restrict__ wts, double *__restrict__ partials,
                                                const uint8_t *__restrict__ act, uint32_t *acnt, int *alist,
                                                const uint32_t *__restrict__ ctr, S *__restrict__ f,
                                                const T *__restrict__ Fext, int *err, const LBArgs &a,
                                                const MeshArgs &m, int bxw, int nbx, int nby)
{
    const int nscan = scan_blocks(a.g);
    if (blk < m.nparts)
        forces_block<T>(xcd_block(blk, m.nparts), q, Xref, inc4, fref, phiSW, gVout, base, wts, partials, err, a.g, m);
    else if (blk < m.nparts + nscan)
        scan_block(blk - m.nparts, act, acnt + P, alist, ctr[P]);
    else
        bulk_lb_block<S, P == 1>(blk - m.nparts - nscan, f, Fext, act, ctr[P], err, a, bxw, nbx, nby);
}

template <typename S, int P, typename T = typename Pop<S>::C>
__global__ __launch_bounds__(256) void k_forces(const double *__restrict__ q, const double *__restrict__ Xref,
                                                const int4 *__restrict__ inc4,
                                                const double *__restrict__ fref, T *__restrict__ phiSW,
                                                T *__restrict__ gVout, Base *__restrict__ base,
                                                T *__restrict__ wts, double *__restrict__ partials,
                                                const uint8_t *__restrict__ act, uint32_t *acnt, int *alist,
                                                const uint32_t *__restrict__ ctr, S *__restrict__ f,
                                                const T *__restrict__ Fext, int *err, LBArgs a, MeshArgs m, int bxw,
                                                int nbx, int nby)
{
    forces_dispatch<S, P, T>((int)blockIdx.x, q, Xref, inc4, fref, phiSW, gVout, base, wts, partials, act, acnt,
                             alist, ctr, f, Fext, err, a, m, bxw, nbx, nby);
}

// k_V (V - V0)/V0 from the force-kernel partials, summed by one wavefront in a
// fixed order (lane-strided, then a butterfly); the loads of a lane are issued
// in groups of eight before any of them is added.
__device__ __forceinline__ double volume_factor(const double *__restrict__ partials, const MeshArgs &m, int lane)
{
    double s = 0.0;
    for (int k0 = lane; k0 < m.nparts; k0 += 64 * 8) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            v[j] = k0 + 64 * j < m.nparts ? partials[k0 + 64 * j] : 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            s += v[j];
    }
    s = wave_sum<double>(s);
    return m.kv_over_V0 * s;
}

// ---------------------------------------------------------------------------
// Spreading, one block per active tile (gather form, no FP atomics)
// ---------------------------------------------------------------------------
// A listed vertex as the gather needs it: its phi4 weight at each of the
// tile's local coordinates per axis (kTileX, then kTileY, then kTileZ of
// them; zero where the stencil misses that coordinate), and phi_S + phi_W and
// dV/dq.
template <typename T>
struct Staged {
    T w[kTileW];
    T ph[3], gv[3];
};

// Weights of one axis at the tile's TW local coordinates origin + 0..TW-1: the
// stencil of corner b covers node b + k, k = 0..3 (wrapped with period n when
// n > 0).
template <int TW, typename T>
__device__ __forceinline__ void local_weights(const T *sw, int b, int origin, int n, T *out)
{
#pragma unroll
    for (int l = 0; l < TW; ++l) {
        int k = origin + l - b;
        if (n > 0 && k < 0)
            k += n;
        out[l] = (unsigned)k < 4u ? sw[k & 3] : T(0);
    }
}

template <typename T>
__device__ __forceinline__ Staged<T> stage_load(int v, const Base *__restrict__ base, const T *__restrict__ wts,
                                                const T *__restrict__ phiSW, const T *__restrict__ gV, int nv,
                                                int *err, const Grid &g, int x0, int y0, int z0)
{
    Staged<T> s;
    // a corrupt list entry is never used as an index: it weighs zero everywhere
    const bool ok = (unsigned)v < (unsigned)nv;
    if (!ok)
        atomicOr(err, kErrList);
    const int u = ok ? v : 0;
    const Base bs = base[u];
    T w[12];
    if constexpr (sizeof(T) == 4) {
        const float4 *pw = reinterpret_cast<const float4 *>(wts) + 3 * u;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float4 w4 = pw[k];
            w[4 * k] = w4.x;
            w[4 * k + 1] = w4.y;
            w[4 * k + 2] = w4.z;
            w[4 * k + 3] = w4.w;
        }
    } else {
        const double2 *pw = reinterpret_cast<const double2 *>(wts) + 6 * u;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double2 w2 = pw[k];
            w[2 * k] = w2.x;
            w[2 * k + 1] = w2.y;
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        s.ph[c] = phiSW[c * nv + u];
        s.gv[c] = gV[c * nv + u];
    }
    local_weights<kTileX>(w, bs.x, x0, g.nx, s.w);
    local_weights<kTileY>(w + 4, bs.y, y0, g.ny, s.w + kTileX);
    local_weights<kTileZ>(w + 8, bs.z, z0, g.walls ? 0 : g.nz, s.w + kTileX + kTileY);
    if (!ok || !bs.ok) {
#pragma unroll
        for (int k = 0; k < kTileW; ++k)
            s.w[k] = T(0);
    }
    return s;
}

// Entries of a tile's vertex list staged in LDS per pass of the spreading.
constexpr int kStageChunk = 128;
// Staged entries are summed in groups of four: one 4-wide LDS read per axis
// gives the group's weights at the lane's local coordinate.
constexpr int kGroup = 4;

// A staged entry e: sw[r][e] is its phi4 weight at tile coordinate r (x
// coordinates first, then y, then z, as in Staged); sph[e] its
// phi_S + phi_W - k dV/dq.
template <typename T>
__device__ __forceinline__ void stage_store(const Staged<T> &s, int e, T kf, T (*sw)[kStageChunk], T (*sph)[4])
{
#pragma unroll
    for (int r = 0; r < kTileW; ++r)
        sw[r][e] = s.w[r];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        sph[e][c] = s.ph[c] - kf * s.gv[c];
    sph[e][3] = T(0);
}

// A padding entry: zero weight and a finite (zero) force.
template <typename T>
__device__ __forceinline__ void stage_zero(int e, T (*sw)[kStageChunk], T (*sph)[4])
{
#pragma unroll
    for (int r = 0; r < kTileW; ++r)
        sw[r][e] = T(0);
#pragma unroll
    for (int c = 0; c < 4; ++c)
        sph[e][c] = T(0);
}


// Wavefronts per SIMD the spreading's register budget aims at (the second
// launch bound): three with FP32 arithmetic; FP64 needs the whole register
// file of one.
template <typename S>
constexpr int kSpreadWaves = sizeof(typename Pop<S>::C) == 8 ? 1 : 3;

// Blocks [0, nsp) spread: one block of NW wavefronts per active tile,
// striding over the list.  Blocks from nsp on (if any) run the LB of the
// nodes outside the active tiles: it is bandwidth-bound, the spreading is
// latency-bound, and the two touch disjoint nodes (in the AA pattern each node
// reads and writes only its own 19 slots), so they share the dispatch.
//
// Spreading: the tile's vertex mask (bit v set when vertex v's stencil
// reaches the tile) is read whole, thread k taking the k-th contiguous run of
// words, and copied to LDS with each thread's first list position (a prefix
// sum of the words' bit counts), so the list is in ascending vertex order.
// List entry e is then found by the thread that stages it: a binary search
// over the positions names the thread holding it and a halving search its
// bit, with no serial walk over the bits.  The list is staged in LDS in passes
// of kStageChunk entries (one pass for all but the most crowded tiles);
// wavefront w sums the w-th contiguous part of each pass's groups of four
// entries for the 64 nodes of the tile (one per lane), and the partial sums are
// added in wavefront order, so every node's sum has a fixed order.  Wavefront
// 0 fetches its node's populations once it has counted its mask words (so
// that waiting for the words does not wait for them) and finishes with the
// LB update of the tile's nodes.  Block indices map to these roles through
// spread_role (part of the LB blocks come first).
template <typename S, int P, int NW, typename T = typename Pop<S>::C>
__device__ __forceinline__ void spread_dispatch(int blk, const Base *__restrict__ base, const T *__restrict__ wts,
                                                const T *__restrict__ phiSW, const T *__restrict__ gV,
                                                const double *__restrict__ partials, const uint32_t *__restrict__ ctr,
                                                uint64_t *__restrict__ mask, const uint32_t *__restrict__ acnt,
                                                const int *__restrict__ alist, T *__restrict__ F,
                                                uint32_t *__restrict__ stamp, S *__restrict__ f,
                                                const T *__restrict__ Fext, int *err, const LBArgs &a, const MeshArgs &m,
                                                const uint8_t *__restrict__ act, int nsp, int lb0, int bxw, int nbx,
                                                int nby)
{
    constexpr int NT = 64 * NW;  // threads per block
    constexpr int NSUB = 256 / NT;
    static_assert(NW == 2 || NW == 4, "two or four wavefronts per block");
    static_assert(kStageChunk <= NT && kStageChunk % kGroup == 0, "one staged entry per thread and pass");
    const Grid &g = a.g;
    if (blk >= nsp) {
        const int j = blk - nsp;
        bulk_lb_block<S, P == 1, NT>(lb0 + j / NSUB, f, Fext, act, ctr[P], err, a, bxw, nbx, nby, j % NSUB);
        return;
    }
    __shared__ uint64_t swd[4 * NT];  // the tile's mask words
    __shared__ int spre[NT];          // each thread's first list position within its wavefront
    __shared__ __align__(32) T sw[kTileW][kStageChunk];
    __shared__ __align__(32) T sph[kStageChunk][4];
    __shared__ T part[NW - 1][3][64];
    __shared__ T spop[19][64];  // wavefront 0's prefetched populations
    __shared__ int swt[NW];
    __shared__ T skfac;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nv = m.nv, W = m.nwords;
    const int J = (W + NT - 1) / NT;  // words per thread, at most 4 (the launch keeps W <= 4 NT)
    // the count of active tiles and the block's first tile are read together
    // (block index < nsp <= tile count, so the slot exists); the volatile
    // read keeps the compiler from deferring it past the test on the count
    const uint32_t na = acnt[P];
    int tile = ((const volatile int *)alist)[(uint32_t)blk];
    const uint32_t t = ctr[P];
    const int w0 = tid * J;
    uint64_t wv[4];  // this thread's mask words of the current tile
    for (uint32_t ai = (uint32_t)blk; ai < na; ai += nsp) {
        const uint32_t an = ai + nsp;
        const int next = alist[an < na ? an : ai];
        // this lane's node (wavefront 0 updates it once the force is known)
        const int tz = tile / (g.ntx * g.nty);
        const int rem = tile - tz * g.ntx * g.nty;
        const int ty = rem / g.ntx, tx = rem - ty * g.ntx;
        const int lx = lane & (kTileX - 1), ly = (lane >> kTileLX) & (kTileY - 1), lz = lane >> (kTileLX + kTileLY);
        const int x0 = tx << kTileLX, y0 = ty << kTileLY, zt = tz << kTileLZ;
        const int x = x0 + lx, y = y0 + ly, zf = zt + lz;
        const bool node = x < g.nx && y < g.ny && zf < g.nzf;
        uint64_t *mw = mask + (long long)tile * W;
        if (ai == (uint32_t)blk) {
            // the first tile's words; later tiles' words were fetched during
            // the previous tile
#pragma unroll
            for (int j = 0; j < 4; ++j)
                wv[j] = (j < J && w0 + j < W) ? mw[w0 + j] : 0ull;
        }
        // wavefront 1 sums the volume partials (their loads overlap those of
        // the words)
        if (wave == 1 && ai == (uint32_t)blk) {
            const T kfac = T(volume_factor(partials, m, lane));
            if (lane == 0)
                skfac = kfac;
        }
        // set bits of this thread's words
        int c = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            c += __popcll(wv[j]);
        // wavefront 0 fetches its node's populations now, once the words are
        // in: issued earlier, they would be waited for with the words (a wait
        // after a branch holding loads covers every load issued before it).
        // The test on an opaque copy of c (never negative) keeps the loads
        // behind the count.
        T d[19];
        int ck = c;
        asm volatile("" : "+v"(ck));
        if (wave == 0 && node && ck >= 0)
            load_pops<S, P == 1>(f, g, x, y, zf, d);
        const int incl = wave_incl_scan(c);
        if (lane == 63)
            swt[wave] = incl;
        spre[tid] = incl - c;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < J)
                swd[w0 + j] = wv[j];
        __syncthreads();
        // the next tile's words (its index has arrived by now)
        uint64_t wn[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            wn[j] = (an < na && j < J && w0 + j < W) ? mask[(long long)next * W + w0 + j] : 0ull;
        int sb[NW];  // list position of each wavefront's first entry
        int nent = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            sb[w] = nent;
            nent += swt[w];
        }
        if (nent > kTileCap) {
            if (tid == 0)
                atomicOr(err, kErrOverflow);
            nent = kTileCap;
        }
        const int z0 = zt + g.zoff;
        const T kf = skfac;
        T Fx = T(0), Fy = T(0), Fz = T(0);
        // Entry e of the list: the thread k holding it is the last one whose
        // first position is <= e; the entry is the r-th set bit of its words.
        auto entry = [&](int e) {
            int k = 0;
#pragma unroll
            for (int step = NT / 2; step > 0; step >>= 1) {
                const int kk = k + step;
                int pk = spre[kk];
#pragma unroll
                for (int w = 1; w < NW; ++w)
                    pk += kk >= 64 * w ? sb[w] - sb[w - 1] : 0;
                if (pk <= e)
                    k = kk;
            }
            int r = e - spre[k];
#pragma unroll
            for (int w = 1; w < NW; ++w)
                r -= k >= 64 * w ? sb[w] - sb[w - 1] : 0;
            int v = -1;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j < J && v < 0) {
                    const uint64_t word = swd[k * J + j];
                    const int cnt = __popcll(word);
                    if (r < cnt)
                        v = (k * J + j) * 64 + select_bit(word, r);
                    else
                        r -= cnt;
                }
            }
            return v;
        };
        // pass [c0, c0 + cn), padded with zero entries to whole groups
        auto stage = [&](int c0, int cn) {
            const int cp = (cn + kGroup - 1) / kGroup * kGroup;
            if (tid < cn) {
                const Staged<T> st = stage_load<T>(entry(c0 + tid), base, wts, phiSW, gV, nv, err, g, x0, y0, z0);
                stage_store<T>(st, tid, kf, sw, sph);
            } else if (tid < cp) {
                stage_zero<T>(tid, sw, sph);
            }
        };
        auto accumulate = [&](int cn) {
            const int ng = (cn + kGroup - 1) / kGroup;
            const int gq = (ng + NW - 1) / NW;
            const int g0 = wave * gq, g1 = min(ng, g0 + gq);
#pragma unroll 2
            for (int gi = g0; gi < g1; ++gi) {
                const int e = gi * kGroup;
                const Quad<T> wx = *reinterpret_cast<const Quad<T> *>(&sw[lx][e]);
                const Quad<T> wy = *reinterpret_cast<const Quad<T> *>(&sw[kTileX + ly][e]);
                const Quad<T> wz = *reinterpret_cast<const Quad<T> *>(&sw[kTileX + kTileY + lz][e]);
#pragma unroll
                for (int j = 0; j < kGroup; ++j) {
                    const Quad<T> ph = *reinterpret_cast<const Quad<T> *>(&sph[e + j][0]);
                    const T w = wx.v[j] * wy.v[j] * wz.v[j];
                    Fx += ph.v[0] * w;
                    Fy += ph.v[1] * w;
                    Fz += ph.v[2] * w;
                }
            }
        };
        // the first pass; wavefront 0 parks its populations in LDS with it
        const int cn0 = min(kStageChunk, nent);
        stage(0, cn0);
        if (wave == 0 && node) {
#pragma unroll
            for (int i = 0; i < 19; ++i)
                spop[i][lane] = d[i];
        }
        __syncthreads();
        accumulate(cn0);
        // further passes (tiles listing more than kStageChunk vertices)
        for (int c0 = kStageChunk; c0 < nent; c0 += kStageChunk) {
            const int cn = min(kStageChunk, nent - c0);
            __syncthreads();  // the previous pass is done with sw and sph
            stage(c0, cn);
            __syncthreads();
            accumulate(cn);
        }
        if (wave > 0) {
            part[wave - 1][0][lane] = Fx;
            part[wave - 1][1][lane] = Fy;
            part[wave - 1][2][lane] = Fz;
        }
        __syncthreads();
        // the mask words are cleared for the next step (stores are not waited
        // for by the barriers)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (wv[j] != 0ull)
                mw[w0 + j] = 0ull;
        // LDS is not written again before every wavefront has passed the next
        // iteration's first barrier, which wavefront 0 reaches only after this
        if (wave == 0) {
            for (int w = 0; w < NW - 1; ++w) {
                Fx += part[w][0][lane];
                Fy += part[w][1][lane];
                Fz += part[w][2][lane];
            }
            if (node) {
                const long long me = nidx(g, x, y, zf);
                F[me] = Fx;
                F[g.n + me] = Fy;
                F[2 * g.n + me] = Fz;
                // the LB update of this active node, with its force in hand
                T dd[19];
#pragma unroll
                for (int i = 0; i < 19; ++i)
                    dd[i] = spop[i][lane];
                lb_collide<S, P == 1>(f, Fext, err, a, x, y, zf, dd, Fx, Fy, Fz);
            }
            if (lane == 0)
                stamp[tile] = t + 1u;
        }
        tile = next;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            wv[j] = wn[j];
    }
}

// Role of block b of the spreading dispatch: its first `pre` blocks run LB
// blocks (those from nsp on), the next nsp spread, the rest run the remaining
// LB blocks.  LB blocks dispatched ahead of the spreading keep the memory
// system busy while the spreading's first dependent loads are in flight.
__device__ __forceinline__ int spread_role(int b, int nsp, int pre)
{
    return b < pre ? nsp + b : (b < pre + nsp ? b - pre : b);
}

template <typename S, int P, int NW, typename T = typename Pop<S>::C>
__global__ __launch_bounds__(64 * NW, kSpreadWaves<S>) void k_spread(const Base *__restrict__ base, const T *__restrict__ wts,
                                                const T *__restrict__ phiSW, const T *__restrict__ gV,
                                                const double *__restrict__ partials, const uint32_t *__restrict__ ctr,
                                                uint64_t *__restrict__ mask, const uint32_t *__restrict__ acnt,
                                                const int *__restrict__ alist, T *__restrict__ F,
                                                uint32_t *__restrict__ stamp, S *__restrict__ f,
                                                const T *__restrict__ Fext, int *err, LBArgs a, MeshArgs m,
                                                const uint8_t *__restrict__ act, int nsp, int lb0, int bxw, int nbx,
                                                int nby, int pre)
{
    spread_dispatch<S, P, NW, T>(spread_role((int)blockIdx.x, nsp, pre), base, wts, phiSW, gV, partials, ctr, mask, acnt, alist, F, stamp,
                                 f, Fext, err, a, m, act, nsp, lb0, bxw, nbx, nby);
}

// u(t+1) = (sum c f(t+1) + F(t)/2) / rho(t+1) once per node of the active
// tiles (one wavefront per tile, one lane per node), for the interpolation.
// P = t & 1: after this step's LB the populations of time t + 1 sit in the
// swapped layout exactly when P == 0.
template <typename S, int P, typename T = typename Pop<S>::C>
__device__ __forceinline__ void moments_dispatch(int blk, int nblk, const S *__restrict__ f, const T *__restrict__ Fib,
                                                 const T *__restrict__ Fext, const uint32_t *__restrict__ acnt,
                                                 const int *__restrict__ alist, T *__restrict__ U, const LBArgs &a)
{
    const Grid &g = a.g;
    const int lane = threadIdx.x & 63;
    const uint32_t na = acnt[P];
    const uint32_t wpb = blockDim.x >> 6;  // wavefronts (tiles) per block
    const uint32_t first = (uint32_t)blk * wpb + (threadIdx.x >> 6);
    // the first tile is read together with the count (clamped into the list;
    // volatile, so that it is not deferred past the test on the count)
    int tile = ((const volatile int *)alist)[first < (uint32_t)g.nt ? first : 0u];
    for (uint32_t ai = first; ai < na; ai += (uint32_t)nblk * wpb) {
        const uint32_t an = ai + (uint32_t)nblk * wpb;
        const int next = alist[an < na ? an : ai];
        const int tz = tile / (g.ntx * g.nty);
        const int rem = tile - tz * g.ntx * g.nty;
        const int ty = rem / g.ntx, tx = rem - ty * g.ntx;
        const int x = (tx << kTileLX) + (lane & (kTileX - 1)), y = (ty << kTileLY) + ((lane >> kTileLX) & (kTileY - 1)),
                  zf = (tz << kTileLZ) + (lane >> (kTileLX + kTileLY));
        tile = next;
        if (x >= g.nx || y >= g.ny || zf >= g.nzf)
            continue;
        T d[19];
        load_pops<S, P == 0>(f, g, x, y, zf, d);
        const long long me = nidx(g, x, y, zf);
        T Fx = T(a.body[0]) + Fib[me], Fy = T(a.body[1]) + Fib[g.n + me], Fz = T(a.body[2]) + Fib[2 * g.n + me];
        if (a.has_fext) {
            Fx += Fext[me];
            Fy += Fext[g.n + me];
            Fz += Fext[2 * g.n + me];
        }
        T drho = T(0), mx = T(0), my = T(0), mz = T(0);
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            drho += d[i];
            if (cx(i) != 0) mx += T(cx(i)) * d[i];
            if (cy(i) != 0) my += T(cy(i)) * d[i];
            if (cz(i) != 0) mz += T(cz(i)) * d[i];
        }
        const T rho = T(a.rho0) + drho;
        Quad<T> u;
        u.v[0] = (mx + T(0.5) * Fx) / rho;
        u.v[1] = (my + T(0.5) * Fy) / rho;
        u.v[2] = (mz + T(0.5) * Fz) / rho;
        u.v[3] = T(0);
        reinterpret_cast<Quad<T> *>(U)[me] = u;
    }
}

template <typename S, int P, typename T = typename Pop<S>::C>
__global__ __launch_bounds__(512) void k_moments(const S *__restrict__ f, const T *__restrict__ Fib,
                                                 const T *__restrict__ Fext, const uint32_t *__restrict__ acnt,
                                                 const int *__restrict__ alist, T *__restrict__ U, LBArgs a)
{
    moments_dispatch<S, P, T>((int)blockIdx.x, (int)gridDim.x, f, Fib, Fext, acnt, alist, U, a);
}

// Marks the tiles of vertex v's stencil for the step `step`: act[tile] =
// act_stamp(step) and bit v of the tile's vertex mask (called for each of the
// 64 stencil offsets k; each tile is marked by the offset at the opening of
// its runs).  The mask update is an atomic OR whose result is not waited for.
__device__ __forceinline__ void mark_vertex(int v, const StencilRuns &r, int k, const Grid &g, uint8_t *act,
                                            uint64_t *mask, int nwords, uint32_t step)
{
    const int kx = k & 3, ky = (k >> 2) & 3, kz = k >> 4;
    if ((r.mx >> kx) & (r.my >> ky) & (r.mz >> kz) & 1u) {
        const int tile = stencil_tile(g, r, kx, ky, kz);
        act[tile] = act_stamp(step);
        atomicOr((unsigned long long *)&mask[(long long)tile * nwords + (v >> 6)], 1ull << (v & 63));
    }
}

// VPW vertices per wavefront (1: one lane per stencil node; 2: lanes 0-31
// and 32-63, two stencil nodes per lane, offsets k and k + 32): interpolation
// of u(t+1) (from k_moments on fluid nodes, the wall velocity beyond the
// walls), Euler update, and the marks of the tiles the vertex reaches at
// t + 1.  Two per wavefront halves the wavefronts when there are more than
// the GPU holds at once.
template <typename T>
__device__ __forceinline__ void stencil_velocity(const T *__restrict__ U, const uint32_t *__restrict__ stamp,
                                                 uint32_t t, const LBArgs &a, int bx, int by, int bz, double qx,
                                                 double qy, double qz, int k, T &sx, T &sy, T &sz)
{
    const Grid &g = a.g;
    const int kx = k & 3, ky = (k >> 2) & 3, kz = k >> 4;
    const T w = phi4<T>(T((double)(bx + kx) - qx)) * phi4<T>(T((double)(by + ky) - qy)) *
                phi4<T>(T((double)(bz + kz) - qz));
    const int x = wrapi(bx + kx, g.nx), y = wrapi(by + ky, g.ny);
    int z = bz + kz;
    T ux, uy, uz;
    if (g.walls && z < 1) {
        ux = T(a.ulo[0]); uy = T(a.ulo[1]); uz = T(a.ulo[2]);
    } else if (g.walls && z > g.nz - 2) {
        ux = T(a.uhi[0]); uy = T(a.uhi[1]); uz = T(a.uhi[2]);
    } else {
        if (!g.walls)
            z = wrapi(z, g.nz);
        const int zf = z - g.zoff;
        const long long me = nidx(g, x, y, zf);
        // every fluid stencil node lies in an active tile of this step; U is
        // read unconditionally and used if the tile carries this step's stamp
        const Quad<T> u = reinterpret_cast<const Quad<T> *>(U)[me];
        const bool fresh = stamp[tile_of(g, x, y, zf)] == t + 1u;
        ux = fresh ? u.v[0] : T(0);
        uy = fresh ? u.v[1] : T(0);
        uz = fresh ? u.v[2] : T(0);
    }
    sx += ux * w;
    sy += uy * w;
    sz += uz * w;
}

// sum over the 64 / VPW lanes of a vertex
template <typename T, int VPW>
__device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int off = 32 / VPW; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// The first thread also advances the step counter and clears the next step's
// active-tile counter acnt[1 - P] (no kernel of this step reads it).
template <typename T, int P, int VPW>
__device__ __forceinline__ void move_dispatch(int blk, double *__restrict__ q, const T *__restrict__ U,
                                              const uint32_t *__restrict__ stamp, uint32_t *ctr, uint32_t *acnt,
                                              uint8_t *act, uint64_t *mask, int *err, const LBArgs &a,
                                              const MeshArgs &m)
{
    const Grid &g = a.g;
    constexpr int L = 64 / VPW;  // lanes per vertex
    const int sl = threadIdx.x & (L - 1);
    const int v = (blk * 256 + (int)threadIdx.x) / L;
    const uint32_t t = ctr[P];
    if (blk == 0 && threadIdx.x == 0) {
        ctr[1 - P] = t + 1u;
        acnt[1 - P] = 0u;
    }
    if (v >= m.nv)
        return;
    const int nv = m.nv;
    const double qx = q[v], qy = q[nv + v], qz = q[2 * nv + v];
    if (!(fabs(qx) < 1e6 && fabs(qy) < 1e6 && fabs(qz) < 1e6)) {
        if (sl == 0)
            atomicOr(err, kErrNonFinite);
        return;
    }
    const int bx = (int)floor(qx) - 1, by = (int)floor(qy) - 1, bz = (int)floor(qz) - 1;
    T sx = T(0), sy = T(0), sz = T(0);
#pragma unroll
    for (int r = 0; r < VPW; ++r)
        stencil_velocity<T>(U, stamp, t, a, bx, by, bz, qx, qy, qz, sl + r * L, sx, sy, sz);
    sx = group_sum<T, VPW>(sx);
    sy = group_sum<T, VPW>(sy);
    sz = group_sum<T, VPW>(sz);
    const double nqx = qx + double(sx), nqy = qy + double(sy), nqz = qz + double(sz);
    if (sl == 0) {
        q[v] = nqx;
        q[nv + v] = nqy;
        q[2 * nv + v] = nqz;
    }
    if (fabs(nqx) < 1e6 && fabs(nqy) < 1e6 && fabs(nqz) < 1e6) {
        const StencilRuns rn = stencil_runs(g, nqx, nqy, nqz);
#pragma unroll
        for (int r = 0; r < VPW; ++r)
            mark_vertex(v, rn, sl + r * L, g, act, mask, m.nwords, t + 1u);
    } else if (sl == 0) {
        atomicOr(err, kErrNonFinite);
    }
}

template <typename T, int P, int VPW>
__global__ __launch_bounds__(256) void k_move(double *__restrict__ q, const T *__restrict__ U,
                                              const uint32_t *__restrict__ stamp, uint32_t *ctr, uint32_t *acnt,
                                              uint8_t *act, uint64_t *mask, int *err, LBArgs a, MeshArgs m)
{
    move_dispatch<T, P, VPW>((int)blockIdx.x, q, U, stamp, ctr, acnt, act, mask, err, a, m);
}

// marks of the current step t = ctr[p] from the stored positions (after a
// reset of the positions or the state; masks cleared beforehand)
__global__ __launch_bounds__(256) void k_stamp(const double *__restrict__ q, uint8_t *act, uint64_t *mask,
                                               const uint32_t *__restrict__ ctr, int *err, Grid g, MeshArgs m, int p)
{
    const int lane = threadIdx.x & 63;
    const int v = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (v >= m.nv)
        return;
    const double qx = q[v], qy = q[m.nv + v], qz = q[2 * m.nv + v];
    if (fabs(qx) < 1e6 && fabs(qy) < 1e6 && fabs(qz) < 1e6)
        mark_vertex(v, stencil_runs(g, qx, qy, qz), lane, g, act, mask, m.nwords, ctr[p]);
    else if (lane == 0)
        atomicOr(err, kErrNonFinite);
}

// ---------------------------------------------------------------------------
// Batched dispatches: one launch of each step kernel advances every domain of
// a batch.  Block k reads its domain and its block index within that domain's
// dispatch from tab[k], then that domain's record, and runs exactly the code
// of the single-domain dispatch; the ordering of the table (latency-bound
// blocks of every domain first, LB blocks after) is the host's.
// ---------------------------------------------------------------------------
template <typename S, int P, typename T = typename Pop<S>::C>
__global__ __launch_bounds__(256) void kb_forces(const DomRec *__restrict__ R, const uint32_t *__restrict__ tab)
{
    const uint32_t e = tab[blockIdx.x];
    const DomRec &r = R[e & 0xffu];
    const Dev &d = r.d;
    if (*d.err != 0)
        return;  // the member turned unstable: its blocks stop until the check freezes it
    forces_dispatch<S, P, T>((int)(e >> 8), d.q, d.Xref, d.inc4, d.fref, (T *)d.phiSW, (T *)d.gV, d.base,
                             (T *)d.wts, d.partials, d.act, d.acnt, d.alist, d.ctr, (S *)d.f, (const T *)d.Fext,
                             d.err, r.a, r.m, r.bxw, r.nbx, r.nby);
}

template <typename S, int P, int NW, typename T = typename Pop<S>::C>
__global__ __launch_bounds__(64 * NW, kSpreadWaves<S>) void kb_spread(const DomRec *__restrict__ R,
                                                                     const uint32_t *__restrict__ tab)
{
    const uint32_t e = tab[blockIdx.x];
    const DomRec &r = R[e & 0xffu];
    const Dev &d = r.d;
    if (*d.err != 0)
        return;  // the member turned unstable: its blocks stop until the check freezes it
    spread_dispatch<S, P, NW, T>((int)(e >> 8), d.base, (const T *)d.wts, (const T *)d.phiSW, (const T *)d.gV,
                             d.partials, d.ctr, d.mask, d.acnt, d.alist, (T *)d.F, d.stamp, (S *)d.f,
                             (const T *)d.Fext, d.err, r.a, r.m, d.act, r.nsp, r.lb0, r.bxw, r.nbx, r.nby);
}

template <typename S, int P, typename T = typename Pop<S>::C>
__global__ __launch_bounds__(256) void kb_moments(const DomRec *__restrict__ R, const uint32_t *__restrict__ tab)
{
    const uint32_t e = tab[blockIdx.x];
    const DomRec &r = R[e & 0xffu];
    const Dev &d = r.d;
    if (*d.err != 0)
        return;  // the member turned unstable: its blocks stop until the check freezes it
    moments_dispatch<S, P, T>((int)(e >> 8), r.mblocks, (const S *)d.f, (const T *)d.F, (const T *)d.Fext, d.acnt,
                              d.alist, (T *)d.U, r.a);
}

template <typename T, int P, int VPW>
__global__ __launch_bounds__(256) void kb_move(const DomRec *__restrict__ R, const uint32_t *__restrict__ tab)
{
    const uint32_t e = tab[blockIdx.x];
    const DomRec &r = R[e & 0xffu];
    const Dev &d = r.d;
    if (*d.err != 0)
        return;  // the member turned unstable: its blocks stop until the check freezes it
    move_dispatch<T, P, VPW>((int)(e >> 8), d.q, (const T *)d.U, d.stamp, d.ctr, d.acnt, d.act, d.mask, d.err, r.a,
                             r.m);
}

__global__ __launch_bounds__(256) void kb_errors(const DomRec *__restrict__ R, int n, int *__restrict__ err)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n)
        err[k] = *R[k].d.err;
}

// ---------------------------------------------------------------------------
// Debug and query kernels (not on the per-step path)
// ---------------------------------------------------------------------------
template <typename S, typename O = double>
__global__ __launch_bounds__(256) void k_get_pops(const S *__restrict__ f, int p, O *__restrict__ out, Grid g)
{
    using T = typename Pop<S>::C;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int zf = blockIdx.z;
    if (x >= g.nx || y >= g.ny)
        return;
    T d[19];
    if (p)
        load_pops<S, true>(f, g, x, y, zf, d);
    else
        load_pops<S, false>(f, g, x, y, zf, d);
    const long long me = nidx(g, x, y, zf);
    for (int i = 0; i < 19; ++i)
        out[i * g.n + me] = O(d[i]);
}

// One step of an adjoint recording, from the device step counter t = ctr[p]
// (so that a captured graph of several steps records a new level at every
// step):
//  - level t - t0 (at most maxl) of the time levels: the populations of time
//    t in canonical order, converted to O, the positions, and the tiles'
//    vertex masks of these positions (set by the previous move, not yet read
//    by this step's spreading);
//  - level t - 1 - t0 (at most maxf; the wrapped -1 before the window's
//    first step is skipped) of the fields of the step just taken: its force
//    density on its active tiles (stamp == t) and zero elsewhere, u(t) as it
//    left it in U, on the active tiles (the only nodes where it is valid
//    and the adjoint reads it; the rest of the level is not written), the
//    nodal force parts phi_S + phi_W and dV/dq, and V - V0.
// O is the step's arithmetic type (double for FP64 storage, else float).
template <typename S, typename O>
__global__ __launch_bounds__(256) void k_record(const S *__restrict__ f, const O *__restrict__ F,
                                                const O *__restrict__ U, const uint32_t *__restrict__ stamp,
                                                const uint32_t *__restrict__ ctr, int p, uint32_t t0, uint32_t maxl,
                                                uint32_t maxf, O *__restrict__ store, double *__restrict__ qs,
                                                O *__restrict__ Fs, O *__restrict__ Us, const double *__restrict__ q,
                                                const O *__restrict__ phiSW, const O *__restrict__ gV,
                                                const double *__restrict__ partials, int nparts, int nv,
                                                O *__restrict__ phs, O *__restrict__ gvs, double *__restrict__ dVs,
                                                const uint64_t *__restrict__ mask, const int *__restrict__ alist,
                                                const uint32_t *__restrict__ acnt, int nwords,
                                                uint64_t *__restrict__ mask_s, int *__restrict__ alist_s,
                                                uint32_t *__restrict__ acnt_s, Grid g)
{
    using T = typename Pop<S>::C;
    const long long n = g.n;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    // the node's populations, fields and stamp are loaded before the step
    // counter is known (they are the live state, whatever the level), so
    // that the wavefront waits for one round of loads; the counter decides
    // only which stores happen
    T d[19];
    O Fv[3], Uv[3];
    uint32_t st = 0;
    if (i < n) {
        // n < 2^31: 32-bit index arithmetic
        const uint32_t ui = (uint32_t)i, row = ui / (uint32_t)g.nx, zr = row / (uint32_t)g.ny;
        const int x = (int)(ui - row * (uint32_t)g.nx), y = (int)(row - zr * (uint32_t)g.ny), zf = (int)zr;
        if (p)
            load_pops<S, true>(f, g, x, y, zf, d);
        else
            load_pops<S, false>(f, g, x, y, zf, d);
        st = stamp[tile_of(g, x, y, zf)];
        for (int c = 0; c < 3; ++c) {
            Fv[c] = F[(size_t)c * n + i];
            Uv[c] = U[(size_t)4 * i + c];
        }
    }
    const uint32_t t = ctr[p];
    const uint32_t lev = t - t0, levf = t - 1u - t0;
    const bool rec = lev <= maxl, recf = levf <= maxf;
    if (i < n) {
        // the levels are written once here and read once, in reverse order,
        // by the sweep: non-temporal stores keep them from displacing the
        // step's own arrays in the caches
        if (rec) {
            O *out = store + (size_t)lev * 19 * (size_t)n;
            for (int k = 0; k < 19; ++k)
                __builtin_nontemporal_store(O(d[k]), &out[(size_t)k * n + i]);
        }
        if (recf) {
            // U is valid, and read by the sweep, on the step's active tiles only
            const bool on = st == t;
            O *Fo = Fs + (size_t)levf * 3 * (size_t)n;
            O *Uo = Us + (size_t)levf * 3 * (size_t)n;
            for (int c = 0; c < 3; ++c) {
                __builtin_nontemporal_store(on ? Fv[c] : O(0), &Fo[(size_t)c * n + i]);
                if (on)
                    __builtin_nontemporal_store(Uv[c], &Uo[(size_t)c * n + i]);
            }
        }
    }
    if (i < 3ll * nv) {
        if (rec)
            qs[(size_t)lev * 3 * nv + i] = q[i];
        if (recf) {
            phs[(size_t)levf * 3 * nv + i] = phiSW[i];
            gvs[(size_t)levf * 3 * nv + i] = gV[i];
        }
    }
    const long long nw = (long long)g.nt * nwords;
    if (rec && i < nw)
        mask_s[(size_t)lev * (size_t)nw + i] = mask[i];
    if (recf && i < g.nt)
        alist_s[(size_t)levf * g.nt + i] = alist[i];
    if (recf && blockIdx.x == 0 && threadIdx.x < 64) {
        double sum = 0.0;
        for (int k = threadIdx.x; k < nparts; k += 64)
            sum += partials[k];
        sum = wave_sum<double>(sum);
        if (threadIdx.x == 0) {
            dVs[levf] = sum;
            acnt_s[levf] = acnt[1 - p];
        }
    }
}

template <typename S>
__global__ __launch_bounds__(256) void k_set_pops(S *__restrict__ f, int p, const double *__restrict__ in, Grid g)
{
    using T = typename Pop<S>::C;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int zf = blockIdx.z;
    if (x >= g.nx || y >= g.ny)
        return;
    const long long me = nidx(g, x, y, zf);
    const long long n = g.n;
    if (p) {
        const Nbr b = neighbours(g, x, y, zf);
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            uint32_t src;
            const bool ok = shifted(b, i, -1, src);
            if (ok)
                f[opp(i) * g.pp + src] = Pop<S>::put(T(in[i * n + me]), i);
            else
                f[i * g.pp + me] = Pop<S>::put(T(in[i * n + me]), i);
        }
    } else {
        for (int i = 0; i < 19; ++i)
            f[i * g.pp + me] = Pop<S>::put(T(in[i * n + me]), i);
    }
}

// force density of the last step (t-1) at node me, zero before the first step
template <typename T>
__device__ __forceinline__ void last_force(const T *Fib, const T *Fext, const uint32_t *stamp, uint32_t t,
                                           const LBArgs &a, int x, int y, int zf, long long me, double *F)
{
    F[0] = F[1] = F[2] = 0.0;
    if (t == 0u)
        return;
    F[0] = a.body[0];
    F[1] = a.body[1];
    F[2] = a.body[2];
    if (stamp != nullptr && stamp[tile_of(a.g, x, y, zf)] == t) {
        F[0] += double(Fib[me]);
        F[1] += double(Fib[a.g.n + me]);
        F[2] += double(Fib[2 * a.g.n + me]);
    }
    if (a.has_fext) {
        F[0] += double(Fext[me]);
        F[1] += double(Fext[a.g.n + me]);
        F[2] += double(Fext[2 * a.g.n + me]);
    }
}

template <typename S, typename T = typename Pop<S>::C>
__global__ __launch_bounds__(256) void k_get_fields(const S *__restrict__ f, const T *__restrict__ Fib,
                                                    const T *__restrict__ Fext, const uint32_t *__restrict__ stamp,
                                                    const uint32_t *__restrict__ ctr, int p, double *__restrict__ rho_out,
                                                    double *__restrict__ u_out, double *__restrict__ F_out, LBArgs a)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int zf = blockIdx.z;
    const Grid &g = a.g;
    if (x >= g.nx || y >= g.ny)
        return;
    const uint32_t t = ctr[p];
    const long long me = nidx(g, x, y, zf);
    double F[3];
    last_force<T>(Fib, Fext, stamp, t, a, x, y, zf, me, F);
    if (F_out != nullptr) {
        F_out[me] = F[0];
        F_out[g.n + me] = F[1];
        F_out[2 * g.n + me] = F[2];
    }
    if (rho_out == nullptr)
        return;
    T d[19];
    if (p)
        load_pops<S, true>(f, g, x, y, zf, d);
    else
        load_pops<S, false>(f, g, x, y, zf, d);
    double drho = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; ++i) {
        const double di = double(d[i]);
        drho += di;
        m[0] += cx(i) * di;
        m[1] += cy(i) * di;
        m[2] += cz(i) * di;
    }
    const double rho = a.rho0 + drho;
    rho_out[me] = rho;
    for (int k = 0; k < 3; ++k)
        u_out[k * g.n + me] = (m[k] + 0.5 * F[k]) / rho;
}

template <typename T>
__global__ __launch_bounds__(256) void k_nodal_forces(const T *__restrict__ phiSW, const T *__restrict__ gV,
                                                      const double *__restrict__ partials, double *__restrict__ out,
                                                      MeshArgs m)
{
    __shared__ double kf;
    if (threadIdx.x < 64) {
        const double s = volume_factor(partials, m, threadIdx.x);
        if (threadIdx.x == 0)
            kf = s;
    }
    __syncthreads();
    const T kfac = T(kf);
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= m.nv)
        return;
    for (int c = 0; c < 3; ++c)
        out[3 * v + c] = double(phiSW[c * m.nv + v] - kfac * gV[c * m.nv + v]);
}

// FP64 block reduction of K values per thread, fixed tree order, 1024 threads
template <int K>
__device__ __forceinline__ void block_reduce_store(double (&acc)[K], double *out)
{
    __shared__ double sh[1024];
    for (int k = 0; k < K; ++k) {
        sh[threadIdx.x] = acc[k];
        __syncthreads();
        for (int s = 512; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s)
                sh[threadIdx.x] += sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            out[k] = sh[0];
        __syncthreads();
    }
}

// V, A, volume first moments, volume second moments (about the origin)
__global__ __launch_bounds__(1024) void k_mesh_moments(const double *__restrict__ q, const int *__restrict__ faces,
                                                       double *__restrict__ out, MeshArgs m)
{
    double acc[11];
    for (int k = 0; k < 11; ++k)
        acc[k] = 0.0;
    const int nv = m.nv, nf = m.nf;
    for (int j = threadIdx.x; j < nf; j += blockDim.x) {
        const int ia = faces[j], ib = faces[nf + j], ic = faces[2 * nf + j];
        double A[3], B[3], C[3], S[3];
        for (int k = 0; k < 3; ++k) {
            A[k] = q[k * nv + ia] - m.origin[k];
            B[k] = q[k * nv + ib] - m.origin[k];
            C[k] = q[k * nv + ic] - m.origin[k];
            S[k] = A[k] + B[k] + C[k];
        }
        const double vt = (A[0] * (B[1] * C[2] - B[2] * C[1]) + A[1] * (B[2] * C[0] - B[0] * C[2]) +
                           A[2] * (B[0] * C[1] - B[1] * C[0])) / 6.0;
        const double e[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        const double f2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
        const double n[3] = {e[1] * f2[2] - e[2] * f2[1], e[2] * f2[0] - e[0] * f2[2], e[0] * f2[1] - e[1] * f2[0]};
        acc[0] += vt;
        acc[1] += 0.5 * sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int k = 0; k < 3; ++k)
            acc[2 + k] += vt * S[k] / 4.0;
        const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
        for (int p = 0; p < 6; ++p) {
            const int r = ii[p], c = jj[p];
            acc[5 + p] += vt / 20.0 * (A[r] * A[c] + B[r] * B[c] + C[r] * C[c] + S[r] * S[c]);
        }
    }
    block_reduce_store<11>(acc, out);
}

// normal equations of the algebraic sphere fit |p|^2 = 2 c.p + k over vertices
// at least excl away from the chosen wall plane; p shifted by `shift`
__global__ __launch_bounds__(1024) void k_sphere_moments(const double *__restrict__ q, double *__restrict__ out,
                                                         MeshArgs m, int wall_hi, double z_wall, double excl,
                                                         double sx, double sy, double sz)
{
    double acc[15];
    for (int k = 0; k < 15; ++k)
        acc[k] = 0.0;
    const int nv = m.nv;
    for (int v = threadIdx.x; v < nv; v += blockDim.x) {
        const double zq = q[2 * nv + v];
        const double dist = wall_hi ? z_wall - zq : zq - z_wall;
        if (!(dist >= excl))
            continue;
        const double p[3] = {q[v] - sx, q[nv + v] - sy, zq - sz};
        const double r[4] = {2.0 * p[0], 2.0 * p[1], 2.0 * p[2], 1.0};
        const double b = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
        int k = 0;
        for (int i = 0; i < 4; ++i)
            for (int j = i; j < 4; ++j)
                acc[k++] += r[i] * r[j];
        for (int i = 0; i < 4; ++i)
            acc[10 + i] += r[i] * b;
        acc[14] += 1.0;
    }
    block_reduce_store<15>(acc, out);
}

// The paper's contact-angle measurement (appendix on the resolution test): a
// circle cut by the wall chord fitted to a slice of the mesh.  The slice is the
// K vertices nearest the plane, normal to y, through the volume centroid (ties
// to the lower vertex index).  One block: a radix select over the 64-bit
// patterns of |y - y_c| (non-negative doubles order as their bit patterns)
// finds the K-th key T; the vertices below T and the lowest-indexed ones equal
// to T make the slice.  Those at least excl from the wall plane add to the
// normal equations of x^2 + z^2 = 2 c.p + k in the (x, z) plane, p shifted by
// (sx, sz): packed upper triangle (6), right side (3), count.  mom holds the
// mesh moments of k_mesh_moments (V at 0, the volume y moment about m.origin
// at 3).
__global__ __launch_bounds__(1024) void k_slice_moments(const double *__restrict__ q, const double *__restrict__ mom,
                                                        double *__restrict__ out, MeshArgs m, int K, int wall_hi,
                                                        double z_wall, double excl, double sx, double sz)
{
    __shared__ unsigned hist[256];
    __shared__ unsigned wave_ties[16];
    __shared__ unsigned long long s_prefix;
    __shared__ unsigned s_need;
    const int nv = m.nv, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double yc = m.origin[1] + mom[3] / mom[0];
    auto key_of = [&](int v) { return (unsigned long long)__double_as_longlong(fabs(q[nv + v] - yc)); };

    unsigned long long prefix = 0, mask = 0;
    unsigned need = (unsigned)K;
    for (int shift = 56; shift >= 0; shift -= 8) {
        if (tid < 256)
            hist[tid] = 0;
        __syncthreads();
        for (int v = tid; v < nv; v += blockDim.x) {
            const unsigned long long key = key_of(v);
            if ((key & mask) == prefix)
                atomicAdd(&hist[(key >> shift) & 255], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            unsigned cum = 0;
            int b = 0;
            for (; b < 255 && cum + hist[b] < need; ++b)
                cum += hist[b];
            s_prefix = prefix | ((unsigned long long)b << shift);
            s_need = need - cum;
        }
        __syncthreads();
        prefix = s_prefix;
        need = s_need;
        mask |= 255ull << shift;
    }

    // prefix is T; `need` vertices with key T belong to the slice, in index order
    double acc[10];
    for (int k = 0; k < 10; ++k)
        acc[k] = 0.0;
    unsigned base = 0;
    for (int c0 = 0; c0 < nv; c0 += blockDim.x) {
        const int v = c0 + tid;
        const unsigned long long key = v < nv ? key_of(v) : ~0ull;
        const bool tie = v < nv && key == prefix;
        const unsigned long long bal = __ballot(tie);
        if (lane == 0)
            wave_ties[wv] = (unsigned)__popcll(bal);
        __syncthreads();
        unsigned rank = base + (unsigned)__popcll(bal & ((1ull << lane) - 1ull)), total = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            rank += w < wv ? wave_ties[w] : 0u;
            total += wave_ties[w];
        }
        __syncthreads();
        base += total;
        if (v < nv && (key < prefix || (tie && rank < need))) {
            const double zq = q[2 * nv + v];
            const double dist = wall_hi ? z_wall - zq : zq - z_wall;
            if (dist >= excl) {
                const double px = q[v] - sx, pz = zq - sz;
                const double r[3] = {2.0 * px, 2.0 * pz, 1.0};
                const double b = px * px + pz * pz;
                int k = 0;
                for (int i = 0; i < 3; ++i)
                    for (int j = i; j < 3; ++j)
                        acc[k++] += r[i] * r[j];
                for (int i = 0; i < 3; ++i)
                    acc[6 + i] += r[i] * b;
                acc[9] += 1.0;
            }
        }
    }
    block_reduce_store<10>(acc, out);
}

// LB blocks of 256 nodes, rows as long as the lattice allows up to 128 nodes
// (at most 128, so that a 128-thread block of the spreading dispatch runs
// whole rows): on odd steps a row's populations are read and written one node
// off in x, and each row costs one extra line at each end.  128-node rows
// took the 128x128x96 droplet's FP32 step from 67.0 to 64.5 us.
dim3 lb_block(const Grid &g)
{
    const int bx = g.nx >= 128 ? 128 : (g.nx >= 64 ? 64 : (g.nx >= 32 ? 32 : 16));
    return dim3(bx, 256 / bx, 1);
}
dim3 lb_grid(const Grid &g)
{
    const dim3 b = lb_block(g);
    return dim3((g.nx + b.x - 1) / b.x, (g.ny + b.y - 1) / b.y, g.nzf);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Calls fn with a value of the population storage type of `prec` (0 FP64,
// 1 FP32, 2 FP16, 3 BF16).
template <typename Fn>
static hipError_t with_pop_type(int prec, Fn &&fn)
{
    switch (prec) {
    case 0: fn(double{}); break;
    case 1: fn(float{}); break;
    case 2: fn(_Float16{}); break;
    default: fn(__bf16{}); break;
    }
    return hipGetLastError();
}

hipError_t launch_init(int prec, const Dev &d, const LBArgs &a, int couette, hipStream_t s)
{
    return with_pop_type(prec, [&](auto tag) {
        using S = decltype(tag);
        k_init<S><<<lb_grid(a.g), lb_block(a.g), 0, s>>>((S *)d.f, a, couette);
    });
}

// The LB-only kernel runs 1024-thread blocks, 128 nodes wide where the rows
// are that long (else the x-width of lb_block), 1024 / width rows.  Measured
// on MI355X, FP32, us per launch: on the 128x128x96 lattice 64x16 blocks took
// 33.2 against 33.3 (64x8) and 34.0 (64x4), and 128x8 blocks 32.6; x-widths
// below a 64-node row were 13 % slower.  128-wide blocks also gave 485 us
// against 576 (64-wide) and 497 (256-wide) on 512x256x128, 507 against 530
// on 250^3, and 647 against 640 on 256^3.
template <typename S, bool ODD>
static void lb_launch(const Dev &d, const LBArgs &a, bool bulk, hipStream_t s)
{
    using T = typename Pop<S>::C;
    const int bx = a.g.nx >= 128 ? 128 : (int)lb_block(a.g).x;
    // whole rows of 128 or 64 nodes per block: aligned odd-step x stores;
    // rows of 128 in blocks of two rows, so that the exchange between a row's
    // halves waits for four wavefronts, not sixteen
    const int rw = a.g.nx == bx ? (bx == 128 ? 2 : (bx == 64 ? 1 : 0)) : 0;
    const int by = rw == 2 ? 2 : 1024 / bx;
    const dim3 blk(bx, by, 1), grd((a.g.nx + bx - 1) / bx, (a.g.ny + by - 1) / by, a.g.nzf);
    const uint8_t *ac = bulk ? d.act : nullptr;
    if (rw == 2)
        k_lb<S, ODD, 2><<<grd, blk, 0, s>>>((S *)d.f, (const T *)d.Fext, ac, d.ctr, d.err, a);
    else if (rw == 1)
        k_lb<S, ODD, 1><<<grd, blk, 0, s>>>((S *)d.f, (const T *)d.Fext, ac, d.ctr, d.err, a);
    else
        k_lb<S, ODD, 0><<<grd, blk, 0, s>>>((S *)d.f, (const T *)d.Fext, ac, d.ctr, d.err, a);
}

hipError_t launch_lb(int prec, const Dev &d, const LBArgs &a, int p, int bulk, hipStream_t s)
{
    return with_pop_type(prec, [&](auto tag) {
        using S = decltype(tag);
        p ? lb_launch<S, true>(d, a, bulk, s) : lb_launch<S, false>(d, a, bulk, s);
    });
}

// Share of the LB blocks of the nodes outside the active tiles that runs in
// the forces dispatch (the rest runs in the spreading dispatch), balancing the
// two latency-bound kernels.  Measured (FP32, us per step): on the 64^3
// sheared capsule shares 0 / 0.2 / 0.35 / 0.5 / 0.6 / 0.7 / 0.8 gave 29.1 /
// 28.6 / 28.6 / 28.5 / 28.7 / 29.8 / 29.8; shares 0.45 / 0.6 / 0.75 gave
// 28.8 / 28.2 / 28.9 there and 82.4 / 81.5 / 83.8 on the 128x128x96 wetting
// droplet.  With the spreading's population fetch next to its staged loads,
// 0.4 / 0.5 / 0.6 / 0.7 gave 28.01 / 28.00 / 28.42 / 29.40 at 64^3 and
// 77.3 / 77.4 / 77.3 / 79.0 on the wetting droplet.
constexpr double kLbShareWithForces = 0.5;
// Share of the spreading dispatch's LB blocks dispatched ahead of its
// spreading blocks.  Measured on the 128x128x96 droplet (FP32, us per step):
// 0 / 0.25 / 0.375 / 0.5 / 0.625 / 0.75 / 1 gave 69.3 / 68.2 / 67.4 / 67.6 /
// 67.1 / 67.4 / 69.8.
constexpr double kLbAheadOfSpread = 0.625;

int lb_block_width(const Grid &g) { return (int)lb_block(g).x; }
double lb_share_with_forces() { return kLbShareWithForces; }

int lb_blocks_with_forces(const Grid &g)
{
    const dim3 gr = lb_grid(g);
    const int nlb = (int)(gr.x * gr.y * gr.z);
    return (int)(kLbShareWithForces * nlb + 0.5);
}

template <typename S, int P>
static void forces_launch(const Dev &d, const LBArgs &a, const MeshArgs &m, int nlb, hipStream_t s)
{
    using T = typename Pop<S>::C;
    const dim3 bl = lb_block(a.g), gr = lb_grid(a.g);
    k_forces<S, P><<<m.nparts + (a.g.nt + kScanChunk - 1) / kScanChunk + nlb, 256, 0, s>>>(d.q, d.Xref, d.inc4, d.fref, (T *)d.phiSW, (T *)d.gV, d.base,
                                                       (T *)d.wts, d.partials, d.act, d.acnt, d.alist, d.ctr,
                                                       (S *)d.f, (const T *)d.Fext, d.err, a, m, (int)bl.x,
                                                       (int)gr.x, (int)gr.y);
}

hipError_t launch_forces(int prec, const Dev &d, const LBArgs &a, const MeshArgs &m, int p, int with_lb,
                         hipStream_t s)
{
    const int nlb = with_lb ? lb_blocks_with_forces(a.g) : 0;
    return with_pop_type(prec, [&](auto tag) {
        using S = decltype(tag);
        p ? forces_launch<S, 1>(d, a, m, nlb, s) : forces_launch<S, 0>(d, a, m, nlb, s);
    });
}

// Spreading blocks of NW wavefronts one CU holds at once (limited by
// registers and LDS).
template <typename S, int P, int NW>
static int spread_blocks_per_cu()
{
    using T = typename Pop<S>::C;
    static int n = 0;
    if (n == 0) {
        int k = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, k_spread<S, P, NW, T>, 64 * NW, 0) != hipSuccess ||
            k < 1)
            k = 1;
        n = k;
    }
    return n;
}

// The spreading dispatch with blocks of NW wavefronts: as many spreading
// blocks as the CUs hold at once, striding over the active tiles (one each
// while the list is no longer than that), then the LB blocks from lb0 on,
// each 256-node LB block split over 4 / NW blocks.
template <typename S, int P, int NW>
static void spread_launch(const Dev &d, const LBArgs &a, const MeshArgs &m, int with_lb, hipStream_t s)
{
    using T = typename Pop<S>::C;
    const dim3 bl = lb_block(a.g), gr = lb_grid(a.g);
    const int fit = d.num_cus * spread_blocks_per_cu<S, P, NW>();
    const int nsp = a.g.nt < fit ? a.g.nt : fit;
    const int lb0 = lb_blocks_with_forces(a.g);
    const int nlb = with_lb ? ((int)(gr.x * gr.y * gr.z) - lb0) * (4 / NW) : 0;
    const int pre = (int)(kLbAheadOfSpread * nlb);
    k_spread<S, P, NW><<<nsp + nlb, 64 * NW, 0, s>>>(d.base, (const T *)d.wts, (const T *)d.phiSW,
                                                     (const T *)d.gV, d.partials, d.ctr, d.mask, d.acnt, d.alist,
                                                     (T *)d.F, d.stamp, (S *)d.f, (const T *)d.Fext, d.err, a, m,
                                                     d.act, nsp, lb0, (int)bl.x, (int)gr.x, (int)gr.y, pre);
}

hipError_t launch_spread(int prec, const Dev &d, const LBArgs &a, const MeshArgs &m, int p, int with_lb,
                         hipStream_t s)
{
    // two-wavefront blocks (twice as many resident, so that each active tile
    // of a large mesh gets a block of its own) while a tile's vertex mask fits
    // four words per thread of them; four-wavefront blocks beyond that
    const bool two = m.nwords <= 4 * 128;
    return with_pop_type(prec, [&](auto tag) {
        using S = decltype(tag);
        if (two)
            p ? spread_launch<S, 1, 2>(d, a, m, with_lb, s) : spread_launch<S, 0, 2>(d, a, m, with_lb, s);
        else
            p ? spread_launch<S, 1, 4>(d, a, m, with_lb, s) : spread_launch<S, 0, 4>(d, a, m, with_lb, s);
    });
}

// Blocks of `waves` active tiles (one per wavefront) for the active-tile
// count expected at set-up with a quarter in reserve; the blocks stride over
// the list if it grows beyond that.
int moments_blocks(const Grid &g, const MeshArgs &m, int waves)
{
    const int want = (m.tiles_hint + m.tiles_hint / 4 + waves - 1) / waves + 1;
    const int cap = (g.nt + waves - 1) / waves;
    return want < cap ? want : cap;
}

// The moments dispatch runs 512-thread blocks: on the 128x128x96 FP32 step
// blocks of 64 / 256 / 512 / 1024 threads took 64.1 / 62.9 / 62.55 / 63.25 us
// per step (fewer, larger blocks launch faster; 1024 leave CUs idle).
constexpr int kMomentsThreads = 512;

template <typename S, int P>
static void moments_launch(const Dev &d, const LBArgs &a, const MeshArgs &m, hipStream_t s)
{
    using T = typename Pop<S>::C;
    k_moments<S, P><<<moments_blocks(a.g, m, kMomentsThreads / 64), kMomentsThreads, 0, s>>>(
        (const S *)d.f, (const T *)d.F, (const T *)d.Fext, d.acnt, d.alist, (T *)d.U, a);
}

hipError_t launch_moments(int prec, const Dev &d, const LBArgs &a, const MeshArgs &m, int p, hipStream_t s)
{
    return with_pop_type(prec, [&](auto tag) {
        using S = decltype(tag);
        p ? moments_launch<S, 1>(d, a, m, s) : moments_launch<S, 0>(d, a, m, s);
    });
}

template <typename S, int P>
static void move_launch(const Dev &d, const LBArgs &a, const MeshArgs &m, hipStream_t s)
{
    using T = typename Pop<S>::C;
    // one vertex per wavefront while the GPU holds all of them at once (about
    // 32 wavefronts per CU at this kernel's register count), else two
    if (m.nv <= 32 * d.num_cus)
        k_move<T, P, 1><<<(m.nv + 3) / 4, 256, 0, s>>>(d.q, (const T *)d.U, d.stamp, d.ctr, d.acnt, d.act, d.mask,
                                                        d.err, a, m);
    else
        k_move<T, P, 2><<<(m.nv + 7) / 8, 256, 0, s>>>(d.q, (const T *)d.U, d.stamp, d.ctr, d.acnt, d.act, d.mask,
                                                        d.err, a, m);
}

hipError_t launch_move(int prec, const Dev &d, const LBArgs &a, const MeshArgs &m, int p, hipStream_t s)
{
    return with_pop_type(prec, [&](auto tag) {
        using S = decltype(tag);
        p ? move_launch<S, 1>(d, a, m, s) : move_launch<S, 0>(d, a, m, s);
    });
}

template <typename S, int P>
static void batch_launch(int which, const DomRec *R, const uint32_t *tab, int nb, int vpw, int nw, hipStream_t s)
{
    using T = typename Pop<S>::C;
    switch (which) {
    case B_FORCES: kb_forces<S, P><<<nb, 256, 0, s>>>(R, tab); break;
    case B_SPREAD:
        if (nw == 2)
            kb_spread<S, P, 2><<<nb, 128, 0, s>>>(R, tab);
        else
            kb_spread<S, P, 4><<<nb, 256, 0, s>>>(R, tab);
        break;
    case B_MOMENTS: kb_moments<S, P><<<nb, 256, 0, s>>>(R, tab); break;
    default:
        if (vpw == 2)
            kb_move<T, P, 2><<<nb, 256, 0, s>>>(R, tab);
        else
            kb_move<T, P, 1><<<nb, 256, 0, s>>>(R, tab);
    }
}

hipError_t launch_batch(int prec, int which, const DomRec *recs, const uint32_t *tab, int nblocks, int p, int vpw,
                        int spread_nw, hipStream_t s)
{
    if (nblocks <= 0)
        return hipSuccess;
    return with_pop_type(prec, [&](auto tag) {
        using S = decltype(tag);
        p ? batch_launch<S, 1>(which, recs, tab, nblocks, vpw, spread_nw, s)
          : batch_launch<S, 0>(which, recs, tab, nblocks, vpw, spread_nw, s);
    });
}

hipError_t launch_batch_errors(const DomRec *recs, int n, int *err, hipStream_t s)
{
    kb_errors<<<(n + 255) / 256, 256, 0, s>>>(recs, n, err);
    return hipGetLastError();
}

hipError_t launch_stamp(const Dev &d, const Grid &g, const MeshArgs &m, int p, hipStream_t s)
{
    k_stamp<<<(m.nv + 3) / 4, 256, 0, s>>>(d.q, d.act, d.mask, d.ctr, d.err, g, m, p);
    return hipGetLastError();
}

hipError_t launch_record(int prec, const Dev &d, const Grid &g, const MeshArgs &m, int p, uint32_t t0, uint32_t maxl,
                         uint32_t maxf, void *store, double *qs, void *Fs, void *Us, void *phs, void *gvs,
                         double *dVs, uint64_t *mask_s, int *alist_s, uint32_t *acnt_s, hipStream_t s)
{
    long long work = g.n > 3ll * m.nv ? g.n : 3ll * m.nv;
    if ((long long)g.nt * m.nwords > work)
        work = (long long)g.nt * m.nwords;
    const int blocks = (int)((work + 255) / 256);
    return with_pop_type(prec, [&](auto tag) {
        using S = decltype(tag);
        using O = typename Pop<S>::C;
        k_record<S, O><<<blocks, 256, 0, s>>>((const S *)d.f, (const O *)d.F, (const O *)d.U, d.stamp, d.ctr, p, t0,
                                             maxl, maxf, (O *)store, qs, (O *)Fs, (O *)Us, d.q, (const O *)d.phiSW,
                                             (const O *)d.gV, d.partials, m.nparts, m.nv, (O *)phs, (O *)gvs, dVs,
                                             d.mask, d.alist, d.acnt, m.nwords, mask_s, alist_s, acnt_s, g);
    });
}

hipError_t launch_get_pops(int prec, const Dev &d, const Grid &g, int p, double *out, hipStream_t s)
{
    return with_pop_type(prec, [&](auto tag) {
        using S = decltype(tag);
        k_get_pops<S><<<lb_grid(g), lb_block(g), 0, s>>>((const S *)d.f, p, out, g);
    });
}

hipError_t launch_set_pops(int prec, const Dev &d, const Grid &g, int p, const double *in, hipStream_t s)
{
    return with_pop_type(prec, [&](auto tag) {
        using S = decltype(tag);
        k_set_pops<S><<<lb_grid(g), lb_block(g), 0, s>>>((S *)d.f, p, in, g);
    });
}

static hipError_t fields_launch(int prec, const Dev &d, const LBArgs &a, int p, double *rho, double *u, double *F,
                                hipStream_t s)
{
    const uint32_t *stamp = d.q ? d.stamp : nullptr;
    return with_pop_type(prec, [&](auto tag) {
        using S = decltype(tag);
        using T = typename Pop<S>::C;
        k_get_fields<S><<<lb_grid(a.g), lb_block(a.g), 0, s>>>((const S *)d.f, (const T *)d.F, (const T *)d.Fext,
                                                               stamp, d.ctr, p, rho, u, F, a);
    });
}

hipError_t launch_get_fields(int prec, const Dev &d, const LBArgs &a, int p, double *rho, double *u, hipStream_t s)
{
    return fields_launch(prec, d, a, p, rho, u, nullptr, s);
}

hipError_t launch_get_force(int prec, const Dev &d, const LBArgs &a, int p, double *F, hipStream_t s)
{
    return fields_launch(prec, d, a, p, nullptr, nullptr, F, s);
}

hipError_t launch_nodal_forces(int prec, const Dev &d, const MeshArgs &m, double *phi, hipStream_t s)
{
    const int blocks = (m.nv + 255) / 256;
    if (prec == 0)
        k_nodal_forces<double><<<blocks, 256, 0, s>>>((const double *)d.phiSW, (const double *)d.gV, d.partials,
                                                      phi, m);
    else
        k_nodal_forces<float><<<blocks, 256, 0, s>>>((const float *)d.phiSW, (const float *)d.gV, d.partials,
                                                     phi, m);
    return hipGetLastError();
}

hipError_t launch_mesh_moments(const Dev &d, const MeshArgs &m, double *out, hipStream_t s)
{
    k_mesh_moments<<<1, 1024, 0, s>>>(d.q, d.faces, out, m);
    return hipGetLastError();
}

hipError_t launch_sphere_moments(const Dev &d, const MeshArgs &m, int wall_hi, double z_wall, double excl,
                                 const double *shift, double *out, hipStream_t s)
{
    k_sphere_moments<<<1, 1024, 0, s>>>(d.q, out, m, wall_hi, z_wall, excl, shift[0], shift[1], shift[2]);
    return hipGetLastError();
}

hipError_t launch_slice_moments(const Dev &d, const MeshArgs &m, const double *mom, int K, int wall_hi,
                                double z_wall, double excl, const double *shift, double *out, hipStream_t s)
{
    k_slice_moments<<<1, 1024, 0, s>>>(d.q, mom, out, m, K, wall_hi, z_wall, excl, shift[0], shift[1]);
    return hipGetLastError();
}

}  // namespace iblb
