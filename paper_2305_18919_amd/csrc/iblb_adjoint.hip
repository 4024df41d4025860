// Discrete adjoint of one IB-LB step (reverse mode), in FP64 arithmetic.
//
// The forward step maps (f(t), q(t)) to (f(t+1), q(t+1)):
//   phi = Phi(q)                              nodal forces (Eqs. generalised_energy1,
//                                             nodal_force_S, nodal_force_V, LJ_interaction)
//   F   = sum_i phi_i delta(x - q_i)          spreading (Eq. ibm-governing_eq2)
//   f*  = f - (f - f^eq(rho, u)) / tau + S(u, F),  rho u = sum c f + F/2   (Eqs. LBeq, feq)
//   f(t+1) = propagation of f*, half-way bounce-back with the moving-wall term
//   u'  = (sum c f(t+1) + F/2) / rho(t+1)
//   q(t+1) = q + sum_x u'(x) delta(x - q)     interpolation (Eq. ibm-governing_eq1)
// Given the adjoints lam(t+1) of f(t+1) and qb(t+1) of q(t+1), the kernels
// below produce lam(t), qb(t) and add this step's share of the parameter
// derivatives, in the reverse order of the forward operations:
//   ka_spread_tiles      ub(x) = sum_i delta(x - q_i) qb_i (the adjoint of u'),
//                        gathered per tile, and lam(t+1) += d u'/d f(t+1)^T ub;
//                        keeps ub / (2 rho') for the next kernel
//   ka_lb_adj            lam(t) from lam(t+1): propagation reversed (a pull),
//                        then the transposed Jacobian of the collision;
//                        Fb = d f*/d F^T Lam + ub / (2 rho'), tau derivative
//   ka_interp_adj        phib_i = sum_x Fb delta, qb(t) = qb(t+1) + sum_x
//                        (Fb . phi_i + u'(x) . qb(t+1)) grad_q delta, and the
//                        shares of Vdot = grad V . phib
//   ka_force_jvp         qb += (d Phi / d q)^T phib and the alpha, k_V, eps
//                        derivatives.
// Every nodal force is minus the gradient of an energy (W_S, k_V (V - V0)^2 /
// (2 V0) and the LJ potential of each face centroid), so d Phi / d q is
// symmetric and its transpose product is the directional derivative of Phi
// along phib, computed with dual numbers.  The forward's own force density,
// u(t+1) and nodal force parts of each step are read back from the recording
// (every level of the window, or of one checkpoint segment at a time), so
// nothing of the forward is recomputed here, and the adjoints lam and ub are
// stored in the step's own precision (FP32 for an FP32 step).
#include "iblb_internal.h"

#include <hip/hip_runtime.h>

namespace iblb {
namespace {

// D3Q19 velocities
constexpr int kCx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

__device__ __forceinline__ double wq(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
__device__ __forceinline__ int oppq(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

__device__ __forceinline__ int wrapn(int a, int n)
{
    if ((unsigned)a < (unsigned)n)  // the usual case: no division
        return a;
    int r = a % n;
    return r < 0 ? r + n : r;
}

// ---------------------------------------------------------------- dual numbers
struct Dual {
    double v, d;
};
__device__ __forceinline__ Dual mk(double v, double d = 0.0) { return Dual{v, d}; }
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual{a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual{a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return Dual{-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual{a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator*(double s, Dual a) { return Dual{s * a.v, s * a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, double s) { return Dual{s * a.v, s * a.d}; }
__device__ __forceinline__ Dual operator+(Dual a, double s) { return Dual{a.v + s, a.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) { return Dual{a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
__device__ __forceinline__ Dual operator/(Dual a, double s) { return Dual{a.v / s, a.d / s}; }
__device__ __forceinline__ Dual operator/(double s, Dual b) { return Dual{s / b.v, -s * b.d / (b.v * b.v)}; }
__device__ __forceinline__ Dual dlog(Dual a) { return Dual{log(a.v), a.d / a.v}; }
__device__ __forceinline__ double dlog(double a) { return log(a); }
__device__ __forceinline__ double val(double a) { return a; }
__device__ __forceinline__ double val(Dual a) { return a.v; }

// ---------------------------------------------------------------- face mechanics
// Corner `corner` of a face (a, b, c): the two parts of the elastic force,
// F = w1 FG + w2 Fadj with w1 = alpha3/2 and w2 = dw_S/dI2, where FG comes
// from the G^-1 term and Fadj from the adj(g)/det G term of
// S = A0 [w1 G^-1 + w2 adj(g)/det G] (Fb = -2 (S11 e1 + S12 e2),
// Fc = -2 (S12 e1 + S22 e2), Fa = -Fb - Fc), and J = det g / det G.
template <typename T>
struct FaceParts {
    T FG[3], Fadj[3];
    T J, lnJ;
};

template <typename T>
__device__ __forceinline__ FaceParts<T> face_parts(const T *a, const T *b, const T *c, const double *fr, int corner)
{
    // fr: Ginv11, Ginv12, Ginv22, A0, 1/det G
    T e1[3], e2[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = b[k] - a[k];
        e2[k] = c[k] - a[k];
    }
    const T g11 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
    const T g12 = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
    const T g22 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
    const T detg = g11 * g22 - g12 * g12;
    FaceParts<T> p;
    p.J = detg * fr[4];
    p.lnJ = dlog(p.J);
    const double A0 = fr[3];
    // G^-1 part: S = A0 G^-1 (constant); adj part: S = A0 adj(g) / det G
    const double G11 = A0 * fr[0], G12 = A0 * fr[1], G22 = A0 * fr[2];
    const T H11 = g22 * (A0 * fr[4]), H12 = -(g12 * (A0 * fr[4])), H22 = g11 * (A0 * fr[4]);
    T fbG[3], fcG[3], fbH[3], fcH[3];
    for (int k = 0; k < 3; ++k) {
        fbG[k] = -2.0 * (G11 * e1[k] + G12 * e2[k]);
        fcG[k] = -2.0 * (G12 * e1[k] + G22 * e2[k]);
        fbH[k] = -2.0 * (H11 * e1[k] + H12 * e2[k]);
        fcH[k] = -2.0 * (H12 * e1[k] + H22 * e2[k]);
    }
    for (int k = 0; k < 3; ++k) {
        if (corner == 0) {
            p.FG[k] = -(fbG[k] + fcG[k]);
            p.Fadj[k] = -(fbH[k] + fcH[k]);
        } else if (corner == 1) {
            p.FG[k] = fbG[k];
            p.Fadj[k] = fbH[k];
        } else {
            p.FG[k] = fcG[k];
            p.Fadj[k] = fcH[k];
        }
    }
    return p;
}

// dV/d(corner) of the tetrahedron (o, a, b, c): (b-o)x(c-o)/6 for a, and cyclically
template <typename T>
__device__ __forceinline__ void volume_corner(const T *a, const T *b, const T *c, const double *o, int corner, T *g)
{
    const T *u = corner == 0 ? b : (corner == 1 ? c : a);
    const T *w = corner == 0 ? c : (corner == 1 ? a : b);
    T U[3], Wv[3];
    for (int k = 0; k < 3; ++k) {
        U[k] = u[k] + (-o[k]);
        Wv[k] = w[k] + (-o[k]);
    }
    constexpr double sixth = 1.0 / 6.0;
    g[0] = (U[1] * Wv[2] - U[2] * Wv[1]) * sixth;
    g[1] = (U[2] * Wv[0] - U[0] * Wv[2]) * sixth;
    g[2] = (U[0] * Wv[1] - U[1] * Wv[0]) * sixth;
}

// LJ force magnitude per unit eps along the wall normal at distance d
// (Eq. LJ_interaction): 48 [(xi/d)^12 - (xi/d)^6 / 2] / d, 0 from rc on, d >= xi/2
__device__ __forceinline__ double lj_unit(double xi, double rc, double d)
{
    if (!(d < rc)) return 0.0;
    const double dd = d < 0.5 * xi ? 0.5 * xi : d;
    const double r = xi / dd, r2 = r * r, r6 = r2 * r2 * r2;
    return 48.0 * (r6 * r6 - 0.5 * r6) / dd;
}

__device__ __forceinline__ Dual lj_unit(double xi, double rc, Dual d)
{
    if (!(d.v < rc)) return mk(0.0);
    const Dual dd = d.v < 0.5 * xi ? mk(0.5 * xi) : d;
    // one reciprocal for both quotients: r = xi / dd and the result / dd
    const double id = 1.0 / dd.v;
    const Dual r = Dual{xi * id, -xi * dd.d * id * id};
    const Dual r2 = r * r;
    const Dual r6 = r2 * r2 * r2;
    const Dual g = 48.0 * (r6 * r6 - 0.5 * r6);
    return Dual{g.v * id, (g.d - g.v * id * dd.d) * id};
}

// ---------------------------------------------------------------- 4-point stencil
__device__ __forceinline__ double phi4d(double r)
{
    const double a = fabs(r);
    if (a <= 1.0) return 0.125 * (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a));
    if (a <= 2.0) return 0.125 * (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a));
    return 0.0;
}

// d phi4 / d r
__device__ __forceinline__ double dphi4d(double r)
{
    const double a = fabs(r), s = r < 0.0 ? -1.0 : 1.0;
    if (a <= 1.0) return s * 0.125 * (-2.0 + (2.0 - 4.0 * a) / sqrt(1.0 + 4.0 * a - 4.0 * a * a));
    if (a <= 2.0) return s * 0.125 * (-2.0 - (6.0 - 4.0 * a) / sqrt(-7.0 + 12.0 * a - 4.0 * a * a));
    return 0.0;
}

__device__ __forceinline__ bool finite_pos(double x, double y, double z)
{
    return fabs(x) < 1e6 && fabs(y) < 1e6 && fabs(z) < 1e6;
}

// Stencil node k (0..63, x fastest) of a vertex at (qx, qy, qz): its fluid
// index (or -1 outside the fluid, then side = 0 below / 1 above), weight and
// weight gradient with respect to the vertex position.
struct Node {
    long long id;
    int side;
    double w, gw[3];
};

// Called by all 64 lanes of a wavefront for one vertex, k = the lane: the 12
// one-dimensional weights and derivatives (axis l / 4, offset l % 4) are
// evaluated once, by lanes l < 12, and every lane takes its three by shuffle.
__device__ __forceinline__ Node stencil_node(const AdjArgs &A, double qx, double qy, double qz, int k)
{
    const Grid &g = A.g;
    const int bx = (int)floor(qx) - 1, by = (int)floor(qy) - 1, bz = (int)floor(qz) - 1;
    const int nxk = bx + (k & 3), nyk = by + ((k >> 2) & 3), nzk = bz + (k >> 4);
    const int ax = k >> 2, off = k & 3;
    const double r = k < 12 ? double((ax == 0 ? bx : (ax == 1 ? by : bz)) + off) - (ax == 0 ? qx : (ax == 1 ? qy : qz))
                            : 0.0;
    const double w1 = phi4d(r), d1 = dphi4d(r);
    const int lx = k & 3, ly = 4 + ((k >> 2) & 3), lz = 8 + (k >> 4);
    const double px = __shfl(w1, lx, 64), py = __shfl(w1, ly, 64), pz = __shfl(w1, lz, 64);
    const double dx = __shfl(d1, lx, 64), dy = __shfl(d1, ly, 64), dz = __shfl(d1, lz, 64);
    Node nd;
    nd.w = px * py * pz;
    // d/dq of phi4(node - q) = -phi4'(node - q)
    nd.gw[0] = -dx * py * pz;
    nd.gw[1] = -px * dy * pz;
    nd.gw[2] = -px * py * dz;
    nd.side = 0;
    int zf;
    if (g.walls) {
        if (nzk < 1 || nzk > g.nz - 2) {
            nd.id = -1;
            nd.side = nzk < 1 ? 0 : 1;
            return nd;
        }
        zf = nzk - 1;
    } else {
        zf = wrapn(nzk, g.nz);
    }
    nd.id = ((long long)zf * g.ny + wrapn(nyk, g.ny)) * g.nx + wrapn(nxk, g.nx);
    return nd;
}

__device__ __forceinline__ double wave_sum64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sum over the aligned group of 8 lanes
__device__ __forceinline__ double group8_sum(double v)
{
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 1, 64);
    return v;
}

template <int K>
__device__ __forceinline__ void block_atomic_add(double (&v)[K], double *out)
{
    __shared__ double red[K][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double s = wave_sum64(v[k]);
        if (lane == 0) red[k][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        const int k = threadIdx.x;
        atomicAdd(out + k, red[k][0] + red[k][1] + red[k][2] + red[k][3]);
    }
}

// Sums of the block (256 threads) into thread 0's v[]: for partial sums kept
// per block, which avoid many blocks' atomics on one address
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K])
{
    __shared__ double red[K][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double s = wave_sum64(v[k]);
        if (lane == 0) red[k][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < K; ++k) v[k] = red[k][0] + red[k][1] + red[k][2] + red[k][3];
}

// ---------------------------------------------------------------- kernels
// Collision and propagation reversed at node x: Lam_i = lam1_i(x + c_i), or
// lam1_opp(i)(x) for a link that bounces back at a wall (whose moving-wall
// term -6 w_i rho (c_i . u_w) adds to the density adjoint); then
//   lam0_j = (1 - 1/tau) Lam_j + a + b . (c_j - u) / rho,
//   a = sum_i Lam_i d f*_i / d rho |u,   b = sum_i Lam_i d f*_i / d u,
//   Fb = sum_i Lam_i d S_i / d F + b / (2 rho) + ub / (2 rho1)  (the last term
//        the force share of the interpolated velocity's adjoint, which the
//        spread adjoint leaves in ub already divided by 2 rho1),
//   d/dtau: sum_i Lam_i [(f_i - f^eq_i) + s_i / 2] / tau^2  with S_i = (1 - 1/(2 tau)) s_i.
// Lam, the populations, F and ub are all loaded before any is used.  ub is
// zeroed where it was read (this kernel is its last reader in the step).  The tau derivative goes to tslot[block], a running
// sum per block that the caller adds up at the end of the sweep.  P is the
// element type of the kept populations, force density and of lam.
// element at a 32-bit byte offset from a base pointer (a uniform base and
// one address register per access)
template <typename T>
__device__ __forceinline__ T ld32(const T *base, uint32_t byte_off)
{
    return *(const T *)((const char *)base + byte_off);
}
// the same for a recorded level, read once by the sweep
template <typename T>
__device__ __forceinline__ T ld32_once(const T *base, uint32_t byte_off)
{
    return __builtin_nontemporal_load((const T *)((const char *)base + byte_off));
}

template <typename P>
__global__ __launch_bounds__(256) void ka_lb_adj(AdjArgs A, const P *__restrict__ f0,
                                                 const P *__restrict__ F, P *__restrict__ ub,
                                                 double *__restrict__ tslot, const P *__restrict__ lam1,
                                                 P *__restrict__ lam0, double *__restrict__ Fb)
{
    const Grid &g = A.g;
    const long long n = g.n;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double tb[1] = {0.0};
    if (id < n) {
        // node coordinates and the row/plane offsets of its neighbours (no
        // division per link): index 0, 1, 2 for the offsets -1, 0, +1
        const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny, nxy = nx * ny, uid = (uint32_t)id;
        const uint32_t row = uid / nx, x = uid - row * nx, zf = row / ny, y = row - zf * ny;
        const uint32_t xo[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
        const uint32_t yo[3] = {(y == 0 ? ny - 1 : y - 1) * nx, y * nx, (y == ny - 1 ? 0 : y + 1) * nx};
        const uint32_t nzf = (uint32_t)g.nzf;
        const uint32_t zo[3] = {(zf == 0 ? nzf - 1 : zf - 1) * nxy, zf * nxy, (zf == nzf - 1 ? 0 : zf + 1) * nxy};
        // a link whose source lies in a solid wall layer bounces back at x
        const bool wlo = g.walls && zf == 0, whi = g.walls && zf == nzf - 1;
        // byte offsets of this node in a [19][n] array of P and of doubles
        const uint32_t oP = uid * (uint32_t)sizeof(P);
        // the node's populations and Lam_i, the adjoint of post-collision
        // population i at x, gathered before any is used (all loads in
        // flight together)
        P fv[19];
        P lt[19];
        const P ubv[3] = {ld32(ub, oP), ld32(ub + n, oP), ld32(ub + 2 * n, oP)};
#pragma unroll
        for (int i = 0; i < 19; ++i) fv[i] = ld32_once(f0 + (size_t)i * n, oP);
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const bool wall = (kCz[i] < 0 && wlo) || (kCz[i] > 0 && whi);
            const uint32_t to = zo[kCz[i] + 1] + yo[kCy[i] + 1] + xo[kCx[i] + 1];
            lt[i] = wall ? ld32(lam1 + (size_t)oppq(i) * n, oP) : ld32(lam1 + (size_t)i * n, to * (uint32_t)sizeof(P));
        }
        double dr = 0.0, m[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const double d = double(fv[i]);
            dr += d;
            if (kCx[i] != 0) m[0] += kCx[i] > 0 ? d : -d;
            if (kCy[i] != 0) m[1] += kCy[i] > 0 ? d : -d;
            if (kCz[i] != 0) m[2] += kCz[i] > 0 ? d : -d;
        }
        const double rho = A.rho0 + dr;
        const double Fx = double(ld32_once(F, oP)) + A.body[0], Fy = double(ld32_once(F + n, oP)) + A.body[1],
                     Fz = double(ld32_once(F + 2 * n, oP)) + A.body[2];
        const double u0 = (m[0] + 0.5 * Fx) / rho, u1 = (m[1] + 0.5 * Fy) / rho, u2 = (m[2] + 0.5 * Fz) / rho;
        const double uu = u0 * u0 + u1 * u1 + u2 * u2;
        const double uF = u0 * Fx + u1 * Fy + u2 * Fz;
        const double om = A.omega, guo = 1.0 - 0.5 * om;
        // Every sum over i of Lam_i times a polynomial of degree <= 2 in c_i
        // (the transposed Jacobians of f^eq and of the Guo source) is a
        // combination of the moments of w_i Lam_i: M0, M1_a = sum w Lam c_a,
        // M2_ab = sum w Lam c_a c_b.  Lf = sum Lam_i f_i for the tau
        // derivative; aw collects the moving-wall terms of the wall links.
        double M0 = 0.0, M1[3] = {0.0, 0.0, 0.0}, Mxx = 0.0, Myy = 0.0, Mzz = 0.0, Mxy = 0.0, Mxz = 0.0,
               Myz = 0.0, Lf = 0.0, aw = 0.0;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const double L = double(lt[i]);
            const double wl = wq(i) * L;
            Lf += L * double(fv[i]);
            M0 += wl;
            if (kCx[i] != 0) {
                M1[0] += kCx[i] > 0 ? wl : -wl;
                Mxx += wl;
            }
            if (kCy[i] != 0) {
                M1[1] += kCy[i] > 0 ? wl : -wl;
                Myy += wl;
            }
            if (kCz[i] != 0) {
                M1[2] += kCz[i] > 0 ? wl : -wl;
                Mzz += wl;
            }
            if (kCx[i] * kCy[i] != 0) Mxy += kCx[i] * kCy[i] > 0 ? wl : -wl;
            if (kCx[i] * kCz[i] != 0) Mxz += kCx[i] * kCz[i] > 0 ? wl : -wl;
            if (kCy[i] * kCz[i] != 0) Myz += kCy[i] * kCz[i] > 0 ? wl : -wl;
            if ((kCz[i] < 0 && wlo) || (kCz[i] > 0 && whi)) {
                // wall velocities are tangential
                const double uwx = kCz[i] < 0 ? A.ulo[0] : A.uhi[0], uwy = kCz[i] < 0 ? A.ulo[1] : A.uhi[1];
                aw += -6.0 * wl * (kCx[i] * uwx + kCy[i] * uwy);
            }
        }
        const double M2u0 = Mxx * u0 + Mxy * u1 + Mxz * u2, M2u1 = Mxy * u0 + Myy * u1 + Myz * u2,
                     M2u2 = Mxz * u0 + Myz * u1 + Mzz * u2;
        const double M2F0 = Mxx * Fx + Mxy * Fy + Mxz * Fz, M2F1 = Mxy * Fx + Myy * Fy + Myz * Fz,
                     M2F2 = Mxz * Fx + Myz * Fy + Mzz * Fz;
        const double uM1 = u0 * M1[0] + u1 * M1[1] + u2 * M1[2];
        const double uM2u = u0 * M2u0 + u1 * M2u1 + u2 * M2u2;
        const double FM1 = Fx * M1[0] + Fy * M1[1] + Fz * M1[2];
        const double FM2u = Fx * M2u0 + Fy * M2u1 + Fz * M2u2;
        // f*_i = d_i - om (d_i - deq_i) + guo s_i: the density adjoint a, the
        // velocity adjoint b and the force adjoint g
        const double a = aw + om * (M0 + 3.0 * uM1 + 4.5 * uM2u - 1.5 * uu * M0);
        const double orho = om * rho;
        const double b0 = orho * (3.0 * M1[0] + 9.0 * M2u0 - 3.0 * u0 * M0) + guo * (-3.0 * Fx * M0 + 9.0 * M2F0);
        const double b1 = orho * (3.0 * M1[1] + 9.0 * M2u1 - 3.0 * u1 * M0) + guo * (-3.0 * Fy * M0 + 9.0 * M2F1);
        const double b2 = orho * (3.0 * M1[2] + 9.0 * M2u2 - 3.0 * u2 * M0) + guo * (-3.0 * Fz * M0 + 9.0 * M2F2);
        const double g0 = guo * (3.0 * (M1[0] - u0 * M0) + 9.0 * M2u0);
        const double g1 = guo * (3.0 * (M1[1] - u1 * M0) + 9.0 * M2u1);
        const double g2 = guo * (3.0 * (M1[2] - u2 * M0) + 9.0 * M2u2);
        // tau derivative: sum_j Lam_j om^2 (f_j - deq_j + s_j / 2)
        const double Ldeq = dr * M0 + rho * (3.0 * uM1 + 4.5 * uM2u - 1.5 * uu * M0);
        const double Lsrc = 3.0 * FM1 - 3.0 * uF * M0 + 9.0 * FM2u;
        const double tt = om * om * (Lf - Ldeq + 0.5 * Lsrc);
        // lam(t)_j = (1 - om) Lam_j + a + b . (c_j - u) / rho
        const double ir = 1.0 / rho;
        const double bi0 = b0 * ir, bi1 = b1 * ir, bi2 = b2 * ir;
        const double a0 = a - (bi0 * u0 + bi1 * u1 + bi2 * u2);
#pragma unroll
        for (int j = 0; j < 19; ++j) {
            double v = (1.0 - om) * double(lt[j]) + a0;
            if (kCx[j] != 0) v += kCx[j] > 0 ? bi0 : -bi0;
            if (kCy[j] != 0) v += kCy[j] > 0 ? bi1 : -bi1;
            if (kCz[j] != 0) v += kCz[j] > 0 ? bi2 : -bi2;
            *(P *)((char *)(lam0 + (size_t)j * n) + oP) = P(v);
        }
        tb[0] = tt;
        double fb0 = g0 + 0.5 * b0 * ir, fb1 = g1 + 0.5 * b1 * ir, fb2 = g2 + 0.5 * b2 * ir;
        const double ub0 = double(ubv[0]), ub1 = double(ubv[1]), ub2 = double(ubv[2]);
        if (ub0 != 0.0 || ub1 != 0.0 || ub2 != 0.0) {
            // ub / (2 rho1), as the spread adjoint left it
            fb0 += ub0;
            fb1 += ub1;
            fb2 += ub2;
            // this thread was its last reader: zero for the next step's spread
            ub[id] = P(0);
            ub[n + id] = P(0);
            ub[2 * n + id] = P(0);
        }
        Fb[id] = fb0;
        Fb[n + id] = fb1;
        Fb[2 * n + id] = fb2;
    }
    block_sum<1>(tb);  // this block's running sum over the sweep, in its own slot
    if (threadIdx.x == 0)
        tslot[blockIdx.x] += tb[0];
}

// qb0_i += (d Phi / d q phib)_i (the directional derivative of the nodal
// forces along phib, with dVp[0] = V - V0 and grad V . phib the sum of
// vparts[0 .. nvp)), and the
// parameter derivatives phib . dPhi/dalpha_m (m = 1..3), phib . dPhi/dk_V,
// phib . dPhi/deps_lo into grads[0..4].  8 lanes per vertex, one incident
// face each.
template <typename G>
__global__ __launch_bounds__(256) void ka_force_jvp(AdjArgs A, const double *__restrict__ q,
                                                    const int4 *__restrict__ inc4, const double *__restrict__ fref,
                                                    const double *__restrict__ phib, const G *__restrict__ gV,
                                                    const double *__restrict__ dVp, const double *__restrict__ vparts,
                                                    int nvp, double *__restrict__ qb0, double *grads)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = t >> 3, lane = t & 7;
    const int nv = A.nv, nf = A.nf;
    // the vertex's own phib, dV/dq and qb0 so far, read by lane 0 at the
    // end: loaded first, so that they arrive with the face data
    double pbv[3] = {0.0, 0.0, 0.0}, gvv[3] = {0.0, 0.0, 0.0}, qbv[3] = {0.0, 0.0, 0.0};
    if (v < nv && lane == 0)
        for (int k = 0; k < 3; ++k) {
            pbv[k] = phib[k * nv + v];
            gvv[k] = double(gV[k * nv + v]);
            qbv[k] = qb0[k * nv + v];
        }
    double pg[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double jv[3] = {0.0, 0.0, 0.0}, dgv[3] = {0.0, 0.0, 0.0}, dS[3][3] = {{0}}, ljz = 0.0;
    if (v < nv) {  // whole groups of 8 take the same branch
        const double w1 = 0.5 * A.alpha[2];
        for (int s = lane; s < A.slots; s += 8) {
            const int4 e = inc4[(long long)v * A.slots + s];
            if (e.w < 0) continue;
            const int j = e.w >> 2, corner = e.w & 3;
            Dual a[3], b[3], c[3];
            double fr[5];
            for (int k = 0; k < 3; ++k) {
                a[k] = mk(q[k * nv + e.x], phib[k * nv + e.x]);
                b[k] = mk(q[k * nv + e.y], phib[k * nv + e.y]);
                c[k] = mk(q[k * nv + e.z], phib[k * nv + e.z]);
            }
            for (int k = 0; k < 5; ++k) fr[k] = fref[k * nf + j];
            const FaceParts<Dual> p = face_parts<Dual>(a, b, c, fr, corner);
            // w2 = num / J, with one reciprocal of J for it and its derivatives
            const Dual num = mk(0.5 * (A.alpha[0] - A.alpha[2])) + 0.25 * (A.alpha[0] + A.alpha[1]) * p.lnJ;
            const double iJ = 1.0 / p.J.v;
            const Dual w2 = Dual{num.v * iJ, (num.d - num.v * iJ * p.J.d) * iJ};
            // derivatives of w2 with respect to alpha_1..3 (w1 = alpha3/2)
            const double lnJ = p.lnJ.v;
            const double dw2[3] = {(0.5 + 0.25 * lnJ) * iJ, 0.25 * lnJ * iJ, -0.5 * iJ};
            Dual gc[3];
            volume_corner<Dual>(a, b, c, A.origin, corner, gc);
            for (int k = 0; k < 3; ++k) {
                jv[k] += (w1 * p.FG[k] + w2 * p.Fadj[k]).d;
                dgv[k] += gc[k].d;
                for (int m = 0; m < 3; ++m) dS[m][k] += dw2[m] * p.Fadj[k].v + (m == 2 ? 0.5 * p.FG[k].v : 0.0);
            }
            if (A.g.walls) {
                constexpr double third = 1.0 / 3.0;
                const Dual cz = (a[2] + b[2] + c[2]) * third;
                const Dual flo = lj_unit(A.xi, A.rc, cz + (-A.z_lo));
                const Dual fhi = lj_unit(A.xi, A.rc, (-1.0) * cz + A.z_hi);
                jv[2] += (A.eps_lo * flo.d - A.eps_hi * fhi.d) * third;
                ljz += flo.v * third;
            }
        }
        for (int k = 0; k < 3; ++k) {
            jv[k] = group8_sum(jv[k]);
            dgv[k] = group8_sum(dgv[k]);
            for (int m = 0; m < 3; ++m) dS[m][k] = group8_sum(dS[m][k]);
        }
        ljz = group8_sum(ljz);
    }
    // Vdot = grad V . phib, the sum of nvp partial sums (after the face work,
    // which does not need it)
    __shared__ double s_vdot;
    {
        double vs[1] = {0.0};
        for (int k = threadIdx.x; k < nvp; k += 256) vs[0] += vparts[k];
        block_sum<1>(vs);
        if (threadIdx.x == 0) s_vdot = vs[0];
        __syncthreads();
    }
    if (v < nv) {
        if (lane == 0) {
            const double dV = dVp[0], Vdot = s_vdot;
            for (int k = 0; k < 3; ++k) {
                const double gvk = gvv[k];
                qb0[k * nv + v] = qbv[k] + (jv[k] - A.kv_over_V0 * (Vdot * gvk + dV * dgv[k]));
                for (int m = 0; m < 3; ++m) pg[m] += pbv[k] * dS[m][k];
                pg[3] += pbv[k] * (-dV / A.V0) * gvk;
            }
            pg[4] = pbv[2] * ljz;
        }
    }
    block_atomic_add<5>(pg, grads);
}

// ---- variants for a window whose every level was kept by the forward run:
// the force density F, u(t+1) in U, the nodal force parts and V - V0 of each
// step come from the forward itself (element type P), so nothing is recomputed

__device__ __forceinline__ int wave_incl_scan(int c, int lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(c, off, 64);
        c += lane >= off ? y : 0;
    }
    return c;
}

// Tile blocks (lane = node), striding over the forward step's list of active
// tiles: the adjoint of u' gathered from the vertices whose stencil reaches
// the tile (the tile's vertex mask as the forward spread it), ub(x) =
// sum_i delta(x - q_i) qb1_i, written for every node of the tile; then, where
// ub != 0, the adjoint of u' = (sum c f1 + F/2) / rho1 with respect to f1:
// lam_j += (c_j - u') . ub / rho1, u' from U; ub / (2 rho1), its force share,
// is what stays in ub for the LB adjoint.  The list is in ascending vertex
// order (entry e found by a binary search over the threads' first list
// positions, as in the forward spreading) and four wavefronts each sum a
// quarter of its groups of four entries (one 4-wide LDS read per axis and
// group), so the sums have a fixed order (no atomics).  The listed
// vertices' positions and qb1 are loaded in one round and their
// one-dimensional weights at the tile's coordinates (kTileW per vertex) are
// evaluated one per thread; wavefront 0 fetches its nodes' f1, U and lam
// while the sums run.
// Four values read from LDS as one vector.
template <typename T>
struct alignas(4 * sizeof(T)) Quad4 {
    T v[4];
};

template <typename P>
__global__ __launch_bounds__(256) void ka_spread_tiles(AdjArgs A, const double *__restrict__ q,
                                                       const double *__restrict__ qb1, const P *__restrict__ f1,
                                                       const P *__restrict__ U, const uint64_t *__restrict__ mask,
                                                       const int *__restrict__ alist, const uint32_t *__restrict__ acnt,
                                                       int ntb, P *__restrict__ ub, P *__restrict__ lam, int *err)
{
    const Grid &g = A.g;
    const int nv = A.nv;
    const long long n = g.n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ uint64_t swd[4 * 256];  // the tile's mask words
    __shared__ int spre[256];          // each thread's first list position within its wavefront
    // per listed vertex e its weight at tile coordinate r (x coordinates, then
    // y, then z) in sw[r][e], so that one 4-wide read per axis gives four
    // entries' weights
    __shared__ __align__(32) P sw[kTileW][kTileCap];
    __shared__ double sqb[kTileCap * 3];  // and qb1
    __shared__ double sq[kTileCap * 3];   // and q
    __shared__ int swt[4];
    __shared__ double part[3][3][64];
    const int W = (nv + 63) >> 6, J = (W + 255) >> 8;  // mask words per thread: at most 4 (65536 vertices)
    // the first tile is read together with the count (clamped into the list;
    // volatile, so that it is not deferred past the test on the count)
    int tile = ((const volatile int *)alist)[(int)blockIdx.x < g.nt ? (int)blockIdx.x : 0];
    const uint32_t na = acnt[0];
    for (uint32_t ai = blockIdx.x; ai < na; ai += (uint32_t)ntb) {
        if (ai != blockIdx.x)
            tile = alist[ai];
        const uint64_t *mw = mask + (long long)tile * W;
        // wavefront 0: its node of the tile, and that node's f1, U and lam
        const int tz = tile / (g.ntx * g.nty);
        const int rem = tile - tz * g.ntx * g.nty;
        const int ty = rem / g.ntx, tx = rem - ty * g.ntx;
        const int lx = lane & (kTileX - 1), ly = (lane >> kTileLX) & (kTileY - 1), lz = lane >> (kTileLX + kTileLY);
        const int x = (tx << kTileLX) + lx, y = (ty << kTileLY) + ly, zf = (tz << kTileLZ) + lz;
        const bool node = wave == 0 && x < g.nx && y < g.ny && zf < g.nzf;
        const long long id = ((long long)zf * g.ny + y) * g.nx + x;
        const int w0 = tid * J;
        uint64_t wv[4];
        int c = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            wv[j] = (j < J && w0 + j < W) ? mw[w0 + j] : 0ull;
            c += __popcll(wv[j]);
        }
        const int incl = wave_incl_scan(c, lane);
        if (lane == 63)
            swt[wave] = incl;
        spre[tid] = incl - c;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < J)
                swd[w0 + j] = wv[j];
        __syncthreads();
        // list position of each wavefront's first entry
        const int sb1 = swt[0], sb2 = sb1 + swt[1], sb3 = sb2 + swt[2];
        const int tot = sb3 + swt[3];
        const int nent = tot < kTileCap ? tot : kTileCap;
        if (tot > kTileCap && tid == 0)
            atomicOr(err, kErrOverflow);
        // entry e of the list (ascending vertex order): the thread k holding it
        // is the last one whose first position is <= e (binary search), the
        // entry the r-th set bit of its words
        auto entry = [&](int e) {
            auto first = [&](int k) {
                return spre[k] + (k >= 192 ? sb3 : (k >= 128 ? sb2 : (k >= 64 ? sb1 : 0)));
            };
            int k = 0;
#pragma unroll
            for (int step = 128; step > 0; step >>= 1)
                if (first(k + step) <= e)
                    k += step;
            int r = e - first(k), v = -1;
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
        // lattice coordinates of the tile's first node
        const int x0 = tx << kTileLX, y0 = ty << kTileLY, z0 = (tz << kTileLZ) + g.zoff;
        // the listed vertices' positions and qb1, all loads in flight together
        for (int e = tid; e < nent; e += 256) {
            const int ve = entry(e);
            const int v = (unsigned)ve < (unsigned)nv ? ve : 0;  // (marks name vertices below nv only)
            double a[6];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                a[k] = q[k * nv + v];
                a[3 + k] = qb1[k * nv + v];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                sq[e * 3 + k] = a[k];
                sqb[e * 3 + k] = a[3 + k];
            }
        }
        __syncthreads();
        // their 1D weights at the tile's x, y and z coordinates, one per
        // thread (kTileW per vertex), so that the evaluations run side by side
        for (int it = tid; it < nent * kTileW; it += 256) {
            const int e = it / kTileW, r = it - e * kTileW;
            const int ax = r < kTileX ? 0 : (r < kTileX + kTileY ? 1 : 2);
            const int l = r - (ax == 0 ? 0 : (ax == 1 ? kTileX : kTileX + kTileY));
            const double qa = sq[e * 3 + ax];
            const int b = (int)floor(qa) - 1;
            // offset of the tile's node in the vertex's stencil (0..3 inside)
            int o;
            if (ax == 0)
                o = wrapn(x0 + l - b, g.nx);
            else if (ax == 1)
                o = wrapn(y0 + l - b, g.ny);
            else
                o = g.walls ? z0 + l - b : wrapn(z0 + l - b, g.nz);
            sw[r][e] = P(o >= 0 && o <= 3 ? phi4d(double(b + o) - qa) : 0.0);
        }
        // the list padded to whole groups of four with zero entries
        const int npad = (nent + 3) & ~3;
        for (int it = tid; it < (npad - nent) * kTileW; it += 256)
            sw[it % kTileW][nent + it / kTileW] = P(0);
        for (int it = tid; it < (npad - nent) * 3; it += 256)
            sqb[nent * 3 + it] = 0.0;
        __syncthreads();
        // wavefront 0 fetches its node's f1, U and lam now: the loads overlap
        // the sums below, which read LDS only
        P fv[19], lv[19], uv[3];
        if (node) {
#pragma unroll
            for (int k = 0; k < 19; ++k) {
                fv[k] = f1[k * n + id];
                lv[k] = lam[k * n + id];
            }
            for (int k = 0; k < 3; ++k) uv[k] = U[k * n + id];
        }
        // wavefront w sums the w-th contiguous quarter of the groups of four
        const int ng = npad >> 2, gq = (ng + 3) >> 2;
        const int g0 = wave * gq, g1 = min(ng, g0 + gq);
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int gi = g0; gi < g1; ++gi) {
            const int e = gi * 4;
            const Quad4<P> wx = *reinterpret_cast<const Quad4<P> *>(&sw[lx][e]);
            const Quad4<P> wy = *reinterpret_cast<const Quad4<P> *>(&sw[kTileX + ly][e]);
            const Quad4<P> wz = *reinterpret_cast<const Quad4<P> *>(&sw[kTileX + kTileY + lz][e]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double w = double(wx.v[j]) * double(wy.v[j]) * double(wz.v[j]);
                s0 += sqb[(e + j) * 3] * w;
                s1 += sqb[(e + j) * 3 + 1] * w;
                s2 += sqb[(e + j) * 3 + 2] * w;
            }
        }
        if (wave > 0) {
            part[wave - 1][0][lane] = s0;
            part[wave - 1][1][lane] = s1;
            part[wave - 1][2][lane] = s2;
        }
        __syncthreads();
        // wavefront 0 finishes the tile; the others go on to the next, whose
        // first barrier wavefront 0 reaches only after this
        if (wave == 0) {
            for (int w = 0; w < 3; ++w) {
                s0 += part[w][0][lane];
                s1 += part[w][1][lane];
                s2 += part[w][2][lane];
            }
            if (node) {
                const double b[3] = {double(P(s0)), double(P(s1)), double(P(s2))};
                // the force share of u' = (sum c f1 + F/2) / rho1 needs
                // ub / (2 rho1): kept in ub for the LB adjoint
                double h = 0.0;
                if (b[0] != 0.0 || b[1] != 0.0 || b[2] != 0.0) {
                    double dr = 0.0;
#pragma unroll
                    for (int k = 0; k < 19; ++k) dr += double(fv[k]);
                    const double ir = 1.0 / (A.rho0 + dr);
                    h = 0.5 * ir;
                    const double ub_u = b[0] * double(uv[0]) + b[1] * double(uv[1]) + b[2] * double(uv[2]);
#pragma unroll
                    for (int j = 0; j < 19; ++j)
                        lam[j * n + id] = P(double(lv[j]) + (kCx[j] * b[0] + kCy[j] * b[1] + kCz[j] * b[2] - ub_u) * ir);
                }
                ub[id] = P(b[0] * h);
                ub[n + id] = P(b[1] * h);
                ub[2 * n + id] = P(b[2] * h);
            }
        }
    }
}

// The adjoints of both interpolations, one wavefront per vertex, one lane
// per stencil node, sharing the stencil weights:
//  - of the force spreading: phib_i = sum_x Fb delta(x - q_i), and
//    sum_x (Fb . phi_i) grad_q delta, with phi_i = (phi_S + phi_W)_i -
//    k_V (V - V0) / V0 (dV/dq)_i from the kept parts;
//  - of the velocity interpolation of the move: sum_x (u'(x) . qb1_i)
//    grad_q delta, u' from U (the wall velocity at a wall node);
// qb0_i = qb1_i + both sums (the force Jacobian's share is added after), and
// vpart[block] = this block's share of grad V . phib.
template <typename P>
__global__ __launch_bounds__(256) void ka_interp_adj(AdjArgs A, const double *__restrict__ q,
                                                     const double *__restrict__ qb1, const P *__restrict__ U,
                                                     const P *__restrict__ phs, const P *__restrict__ gvs,
                                                     const double *__restrict__ dV, const double *__restrict__ Fb,
                                                     double *__restrict__ phib, double *__restrict__ qb0,
                                                     double *__restrict__ vpart)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = (int)(t >> 6), k = (int)(t & 63);
    const int nv = A.nv;
    const long long n = A.g.n;
    double vd[1] = {0.0};
    if (v < nv) {  // whole wavefronts take the same branch
        // every load of the vertex's own data first; each is waited for only
        // where it is used
        const double qx = q[v], qy = q[nv + v], qz = q[2 * nv + v];
        const double b[3] = {qb1[v], qb1[nv + v], qb1[2 * nv + v]};
        const P gvr[3] = {gvs[v], gvs[nv + v], gvs[2 * nv + v]};
        const P phr[3] = {phs[v], phs[nv + v], phs[2 * nv + v]};
        const double dVv = dV[0];
        double pb[3] = {0.0, 0.0, 0.0}, s[3] = {0.0, 0.0, 0.0};
        if (finite_pos(qx, qy, qz)) {
            const Node nd = stencil_node(A, qx, qy, qz, k);
            double sw;  // the weight of grad_q delta at this node
            if (nd.id >= 0) {
                const double fb[3] = {Fb[nd.id], Fb[n + nd.id], Fb[2 * n + nd.id]};
                const double u[3] = {double(U[nd.id]), double(U[n + nd.id]), double(U[2 * n + nd.id])};
                const double kf = A.kv_over_V0 * dVv;
                sw = u[0] * b[0] + u[1] * b[1] + u[2] * b[2];
                for (int c = 0; c < 3; ++c) {
                    sw += fb[c] * (double(phr[c]) - kf * double(gvr[c]));
                    pb[c] = fb[c] * nd.w;
                }
            } else {
                // beyond a wall u' is the wall velocity: its products with
                // qb1 are uniform values, so no lane indexes the arguments
                const double blo = A.ulo[0] * b[0] + A.ulo[1] * b[1] + A.ulo[2] * b[2];
                const double bhi = A.uhi[0] * b[0] + A.uhi[1] * b[1] + A.uhi[2] * b[2];
                sw = nd.side ? bhi : blo;
            }
            for (int c = 0; c < 3; ++c) s[c] = sw * nd.gw[c];
        }
        for (int c = 0; c < 3; ++c) {
            pb[c] = wave_sum64(pb[c]);
            s[c] = wave_sum64(s[c]);
        }
        if (k == 0) {
            for (int c = 0; c < 3; ++c) {
                phib[c * nv + v] = pb[c];
                qb0[c * nv + v] = b[c] + s[c];
            }
            vd[0] = double(gvr[0]) * pb[0] + double(gvr[1]) * pb[1] + double(gvr[2]) * pb[2];
        }
    }
    block_sum<1>(vd);  // grad V . phib = sum_i (dV/dq)_i . phib_i, by blocks
    if (threadIdx.x == 0)
        vpart[blockIdx.x] = vd[0];
}

int blocks_for(long long threads) { return (int)((threads + 255) / 256); }

}  // namespace

template <typename P>
static hipError_t reverse_kept(const AdjArgs &A, const AdjLevel &L, const AdjWork &w, hipStream_t s)
{
    const long long n = A.g.n;
    const P *f0 = (const P *)L.f0, *f1 = (const P *)L.f1, *F = (const P *)L.F, *U = (const P *)L.U;
    const P *phs = (const P *)L.phs, *gvs = (const P *)L.gvs;
    // ub starts at zero (cleared by the sweep's caller, then by ka_lb_adj of
    // every step); grad V . phib goes through per-block partial sums
    P *ub = (P *)w.ub;
    // tile blocks for the active-tile count expected at set-up, with a
    // quarter in reserve; they stride over the list if it grows beyond that
    const int ntb = A.tile_blocks;
    ka_spread_tiles<P><<<ntb, 256, 0, s>>>(A, L.q, w.qb1, f1, U, L.mask, L.alist, L.acnt, ntb, ub, (P *)w.lam1,
                                           w.err);
    ka_lb_adj<P><<<blocks_for(n), 256, 0, s>>>(A, f0, F, ub, w.tpart, (const P *)w.lam1, (P *)w.lam0, w.Fb);
    const int nvp = blocks_for(64ll * A.nv);
    ka_interp_adj<P><<<nvp, 256, 0, s>>>(A, L.q, w.qb1, U, phs, gvs, L.dV, w.Fb, w.phib, w.qb0, w.vpart);
    ka_force_jvp<P><<<blocks_for(8ll * A.nv), 256, 0, s>>>(A, L.q, L.inc4, L.fref, w.phib, gvs, L.dV, w.vpart, nvp,
                                                          w.qb0, w.grads);
    return hipGetLastError();
}

hipError_t adj_reverse_kept(const AdjArgs &A, int fp64, const AdjLevel &L, const AdjWork &w, hipStream_t s)
{
    return fp64 ? reverse_kept<double>(A, L, w, s) : reverse_kept<float>(A, L, w, s);
}

}  // namespace iblb
