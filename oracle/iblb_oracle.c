/*
 * iblb_oracle.c -- plain FP64 CPU oracle of one immersed-boundary / lattice
 * Boltzmann (IB-LB) time step, after Pelusi, Guglietta, Sega, Aouane, Harting,
 * "A sharp interface approach for wetting dynamics of hydrophobic coated
 * droplets and soft particles" (arXiv:2305.18919).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no source with the GPU library (no headers, tables or helpers) and calls
 * nothing in it.
 *
 * Every floating-point operation is IEEE binary64.  Loops follow the order of
 * the paper's algorithm (Sec. "Numerical implementation", the enumerated list
 * of the IB-LB algorithm):
 *   1. nodal forces phi_i = phi^S + phi^V + phi^W      (Eq. total_nodal_force)
 *   2. spreading F(x) = sum_i phi_i delta(x - q_i)     (Eq. ibm-governing_eq2)
 *   3. BGK collision with Guo forcing, propagation      (Eqs. LBeq, feq)
 *   4. fluid velocity from the populations              (Guo velocity, footnote)
 *   5. interpolation qdot_i = sum_x u(x) delta(x - q_i) (Eq. ibm-governing_eq1)
 *   6. q_i += qdot_i                                    (Eq. ibm_update_pos)
 *
 * Readings taken where the paper is silent or garbled (each one is listed in
 * the design notes of the repository):
 *  - equilibrium: the second-order term is divided by 2 c_s^4 (the printed
 *    denominator 2 c_s^2 would not give the Navier-Stokes stress);
 *  - populations are held as deviations d_i = f_i - w_i rho0, an exact change
 *    of variables that keeps small velocity signals above FP64 rounding;
 *  - phi4: first branch for |r| <= 1, second for 1 <= |r| <= 2, zero beyond;
 *  - walls: solid layers z = 0 and z = nz-1, half-way planes at 0.5 and
 *    nz-1.5, moving-wall bounce-back f_opp = f*_i - 2 w_i rho (c_i.u_w)/c_s^2
 *    with rho the local density;
 *  - interpolation uses u(t+1) = (sum c f(t+1) + F(t)/2)/rho(t+1), with F(t)
 *    the force that drove this step's collision; stencil nodes outside the
 *    fluid are dropped when spreading and carry the wall velocity when
 *    interpolating;
 *  - elastic force: constant-strain linear triangles, I1 = tr(G^-1 g) - 2,
 *    I2 = det g / det G - 1, energy A0 * w_S summed over faces, reference
 *    shape = the unperturbed mesh;
 *  - volume: V_j is the signed tetrahedron volume of face j with apex at the
 *    centroid o of the reference vertices; V0 = volume of the reference mesh;
 *    V - V0 is accumulated as sum_j (V_j - V0_j), each difference expanded
 *    exactly in the vertex displacements from the reference shape, which keeps
 *    the small volume change out of the rounding of O(1) tetrahedron volumes;
 *  - wall force: d = distance of the face centroid to the wall plane along its
 *    normal, cut off at r_cut, d clamped to >= xi/2, one third per vertex.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* D3Q19 velocity set: rest, the 6 axis directions, the 12 face diagonals.
 * Opposite directions are adjacent (odd i, i+1).  Weights from the footnote on
 * the D3Q19 model: 1/3 (rest), 1/18 (axis), 1/36 (diagonals). */
static const int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

static double weight(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
static int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

/* ------------------------------------------------------------------ */
/* point formulas                                                       */
/* ------------------------------------------------------------------ */

void oracle_lattice(int *c, double *w, int *opp)
{
    for (int i = 0; i < Q; ++i) {
        c[3 * i + 0] = CX[i];
        c[3 * i + 1] = CY[i];
        c[3 * i + 2] = CZ[i];
        w[i] = weight(i);
        opp[i] = opposite(i);
    }
}

/* Eq. feq as printed, with c_s^2 = 1/3 and the quadratic term over 2 c_s^4:
 * f_i^eq = w_i rho [1 + c.u/c_s^2 + u_k u_j (c_k c_j - c_s^2 delta_kj)/(2 c_s^4)]. */
void oracle_feq(double rho, const double *u, double *feq)
{
    const double cs2 = 1.0 / 3.0;
    for (int i = 0; i < Q; ++i) {
        const double c[3] = {CX[i], CY[i], CZ[i]};
        double lin = 0.0, quad = 0.0;
        for (int k = 0; k < 3; ++k) {
            lin += u[k] * c[k];
            for (int j = 0; j < 3; ++j)
                quad += u[k] * u[j] * (c[k] * c[j] - (k == j ? cs2 : 0.0));
        }
        feq[i] = weight(i) * rho * (1.0 + lin / cs2 + quad / (2.0 * cs2 * cs2));
    }
}

/* The same equilibrium minus the rest value w_i rho0, written so that every
 * term is small:  f_i^eq - w_i rho0 = w_i (rho - rho0)
 *                   + w_i rho [3 c.u + 9/2 (c.u)^2 - 3/2 u.u]. */
void oracle_feq_dev(double rho0, double drho, const double *u, double *deq)
{
    const double rho = rho0 + drho;
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        const double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
        deq[i] = weight(i) * drho + weight(i) * rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* Guo source of Eq. LBeq (dt = 1):
 * S_i = w_i (1 - 1/(2 tau)) [ (c_i - u).F / c_s^2 + (c_i.F)(c_i.u) / c_s^4 ]. */
void oracle_guo(double tau, const double *u, const double *F, double *S)
{
    const double cs2 = 1.0 / 3.0;
    for (int i = 0; i < Q; ++i) {
        const double c[3] = {CX[i], CY[i], CZ[i]};
        double cmuF = 0.0, cF = 0.0, cu = 0.0;
        for (int k = 0; k < 3; ++k) {
            cmuF += (c[k] - u[k]) * F[k];
            cF += c[k] * F[k];
            cu += c[k] * u[k];
        }
        S[i] = weight(i) * (1.0 - 1.0 / (2.0 * tau)) * (cmuF / cs2 + cF * cu / (cs2 * cs2));
    }
}

/* 4-point stencil phi4 of Eq. ibm-interpolation_stencil (lattice spacing 1). */
double oracle_phi4(double r)
{
    const double a = fabs(r);
    if (a <= 1.0)
        return 0.125 * (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a));
    if (a <= 2.0)
        return 0.125 * (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a));
    return 0.0;
}

/* Wall-particle force of Eq. LJ_interaction along the wall normal for a
 * centroid at distance d from the wall plane:
 * 48 eps [(xi/d)^12 - (xi/d)^6 / 2] / d  (the vector d/d^2 has length 1/d).
 * Zero at or beyond r_cut, d clamped from below at xi/2. */
double oracle_lj(double eps, double xi, double r_cut, double d)
{
    if (eps == 0.0 || !(d < r_cut))
        return 0.0;
    if (d < 0.5 * xi)
        d = 0.5 * xi;
    const double s6 = pow(xi / d, 6.0);
    return 48.0 * eps * (s6 * s6 - 0.5 * s6) / d;
}

/* ------------------------------------------------------------------ */
/* interface mechanics on a whole mesh                                  */
/* ------------------------------------------------------------------ */

/* Reference data of face j from the stress-free vertices X:
 * G_kl = E_k . E_l with E1 = X_b - X_a, E2 = X_c - X_a; A0 = sqrt(det G)/2. */
static void face_reference(const double *X, const int *f, double *Ginv, double *A0, double *detG)
{
    const double *a = X + 3 * f[0], *b = X + 3 * f[1], *c = X + 3 * f[2];
    double E1[3], E2[3];
    for (int k = 0; k < 3; ++k) {
        E1[k] = b[k] - a[k];
        E2[k] = c[k] - a[k];
    }
    const double G11 = E1[0] * E1[0] + E1[1] * E1[1] + E1[2] * E1[2];
    const double G12 = E1[0] * E2[0] + E1[1] * E2[1] + E1[2] * E2[2];
    const double G22 = E2[0] * E2[0] + E2[1] * E2[1] + E2[2] * E2[2];
    const double det = G11 * G22 - G12 * G12;
    Ginv[0] = G22 / det;
    Ginv[1] = -G12 / det;
    Ginv[2] = G11 / det;
    *detG = det;
    *A0 = 0.5 * sqrt(det);
}

/* Signed volume of the tetrahedron (o, a, b, c): (a-o).((b-o)x(c-o))/6. */
static double tet_volume(const double *a, const double *b, const double *c, const double *o)
{
    const double A[3] = {a[0] - o[0], a[1] - o[1], a[2] - o[2]};
    const double B[3] = {b[0] - o[0], b[1] - o[1], b[2] - o[2]};
    const double C[3] = {c[0] - o[0], c[1] - o[1], c[2] - o[2]};
    const double x[3] = {B[1] * C[2] - B[2] * C[1], B[2] * C[0] - B[0] * C[2], B[0] * C[1] - B[1] * C[0]};
    return (A[0] * x[0] + A[1] * x[1] + A[2] * x[2]) / 6.0;
}

/* T(a, b, c) = a . (b x c) */
static double triple(const double *a, const double *b, const double *c)
{
    return a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) + a[2] * (b[0] * c[1] - b[1] * c[0]);
}

/* V(a,b,c) - V(A,B,C) for the tetrahedra with apex o, expanded exactly in the
 * displacements da = a - A, db = b - B, dc = c - C: with T trilinear,
 * T(A+da, B+db, C+dc) - T(A, B, C) is the sum of the seven terms that contain
 * at least one displacement.  Every term is as small as the volume change
 * itself, so the difference is not lost to the rounding of O(1) volumes. */
static double tet_volume_change(const double *A, const double *B, const double *C, const double *a,
                                const double *b, const double *c, const double *o)
{
    double Ar[3], Br[3], Cr[3], da[3], db[3], dc[3];
    for (int k = 0; k < 3; ++k) {
        Ar[k] = A[k] - o[k];
        Br[k] = B[k] - o[k];
        Cr[k] = C[k] - o[k];
        da[k] = a[k] - A[k];
        db[k] = b[k] - B[k];
        dc[k] = c[k] - C[k];
    }
    const double t = triple(da, Br, Cr) + triple(Ar, db, Cr) + triple(Ar, Br, dc) + triple(da, db, Cr) +
                     triple(da, Br, dc) + triple(Ar, db, dc) + triple(da, db, dc);
    return t / 6.0;
}

/* (u - o) x (v - o) / 6 */
static void cross6(const double *u, const double *v, const double *o, double *out)
{
    const double U[3] = {u[0] - o[0], u[1] - o[1], u[2] - o[2]};
    const double V[3] = {v[0] - o[0], v[1] - o[1], v[2] - o[2]};
    out[0] = (U[1] * V[2] - U[2] * V[1]) / 6.0;
    out[1] = (U[2] * V[0] - U[0] * V[2]) / 6.0;
    out[2] = (U[0] * V[1] - U[1] * V[0]) / 6.0;
}

/* Elastic corner forces of one face, -dW/dq for W = A0 w_S(I1, I2)
 * (Eqs. generalised_energy1 and nodal_force_S).  With g_kl = e_k . e_l:
 *   dI1/dg = G^-1 (g12 counted twice),  d(det g)/dg = adj(g),
 *   dw_S/dI1 = alpha3/2,
 *   dw_S/dI2 = [(alpha1-alpha3)/2 + (alpha1+alpha2)/4 ln(I2+1)] / (I2+1),
 * so that dW/de1 = 2 (S11 e1 + S12 e2), dW/de2 = 2 (S12 e1 + S22 e2) with
 * S = A0 [w1 G^-1 + w2 adj(g)/det G].  Force on b is -dW/de1, on c -dW/de2,
 * on a the negative of their sum.  Returns the face energy A0 w_S - A0 w_S0. */
static double face_elastic(const double *q, const int *f, const double *Ginv, double A0, double detG,
                           const double *alpha, double *Fa, double *Fb, double *Fc)
{
    const double *a = q + 3 * f[0], *b = q + 3 * f[1], *c = q + 3 * f[2];
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = b[k] - a[k];
        e2[k] = c[k] - a[k];
    }
    const double g11 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
    const double g12 = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
    const double g22 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
    const double detg = g11 * g22 - g12 * g12;
    const double I1 = Ginv[0] * g11 + 2.0 * Ginv[1] * g12 + Ginv[2] * g22 - 2.0;
    const double J = detg / detG; /* I2 + 1 */
    const double lnJ = log(J);
    const double a1 = alpha[0], a2 = alpha[1], a3 = alpha[2];
    const double w1 = 0.5 * a3;
    const double w2 = (0.5 * (a1 - a3) + 0.25 * (a1 + a2) * lnJ) / J;
    const double S11 = A0 * (w1 * Ginv[0] + w2 * g22 / detG);
    const double S12 = A0 * (w1 * Ginv[1] - w2 * g12 / detG);
    const double S22 = A0 * (w1 * Ginv[2] + w2 * g11 / detG);
    for (int k = 0; k < 3; ++k) {
        Fb[k] = -2.0 * (S11 * e1[k] + S12 * e2[k]);
        Fc[k] = -2.0 * (S12 * e1[k] + S22 * e2[k]);
        Fa[k] = -Fb[k] - Fc[k];
    }
    const double wS = 0.5 * (a1 - a3) * lnJ + 0.125 * (a1 + a2) * lnJ * lnJ + a3 * (0.5 * (I1 + 2.0) - 1.0);
    return A0 * wS;
}

/* Mesh-level forces, exposed for the pins.
 *  q, X      : current and reference vertices [nv*3]
 *  faces     : [nf*3]
 *  alpha     : (alpha1, alpha2, alpha3)
 *  kv        : volume stiffness of w_V = kv (V - V0)^2 / (2 V0)
 *  walls     : nonzero => LJ planes at z_lo and z_hi act
 * Outputs (may be NULL): phiS, phiV, phiW [nv*3]; energy = sum A0 w_S (w_S0 = 0);
 * out_V = V, out_dV = V - V0 (as sum_j (V_j - V0_j)), out_V0 = V0, out_A = area. */
void oracle_mesh_forces(int nv, int nf, const double *q, const double *X, const int *faces,
                        const double *alpha, double kv, int walls, double z_lo, double z_hi,
                        double eps_lo, double eps_hi, double xi, double r_cut,
                        double *phiS, double *phiV, double *phiW, double *energy,
                        double *out_V, double *out_dV, double *out_V0, double *out_A)
{
    double o[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < nv; ++i)
        for (int k = 0; k < 3; ++k)
            o[k] += X[3 * i + k];
    for (int k = 0; k < 3; ++k)
        o[k] /= nv;

    double *gS = calloc((size_t)nv * 3, sizeof(double));
    double *gV = calloc((size_t)nv * 3, sizeof(double));
    double *gW = calloc((size_t)nv * 3, sizeof(double));
    double W = 0.0, V = 0.0, V0 = 0.0, dV = 0.0, A = 0.0;
    for (int j = 0; j < nf; ++j) {
        const int *f = faces + 3 * j;
        double Ginv[3], A0, detG;
        face_reference(X, f, Ginv, &A0, &detG);
        double Fa[3], Fb[3], Fc[3];
        W += face_elastic(q, f, Ginv, A0, detG, alpha, Fa, Fb, Fc);
        for (int k = 0; k < 3; ++k) {
            gS[3 * f[0] + k] += Fa[k];
            gS[3 * f[1] + k] += Fb[k];
            gS[3 * f[2] + k] += Fc[k];
        }
        const double *a = q + 3 * f[0], *b = q + 3 * f[1], *c = q + 3 * f[2];
        const double Vj = tet_volume(a, b, c, o);
        const double V0j = tet_volume(X + 3 * f[0], X + 3 * f[1], X + 3 * f[2], o);
        V += Vj;
        V0 += V0j;
        dV += tet_volume_change(X + 3 * f[0], X + 3 * f[1], X + 3 * f[2], a, b, c, o);
        double da[3], db[3], dc[3];
        cross6(b, c, o, da);
        cross6(c, a, o, db);
        cross6(a, b, o, dc);
        for (int k = 0; k < 3; ++k) {
            gV[3 * f[0] + k] += da[k];
            gV[3 * f[1] + k] += db[k];
            gV[3 * f[2] + k] += dc[k];
        }
        double e1[3], e2[3];
        for (int k = 0; k < 3; ++k) {
            e1[k] = b[k] - a[k];
            e2[k] = c[k] - a[k];
        }
        const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
        A += 0.5 * sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (walls) {
            const double cz = (a[2] + b[2] + c[2]) / 3.0;
            const double fz = oracle_lj(eps_lo, xi, r_cut, cz - z_lo) - oracle_lj(eps_hi, xi, r_cut, z_hi - cz);
            for (int m = 0; m < 3; ++m)
                gW[3 * f[m] + 2] += fz / 3.0;
        }
    }
    for (int i = 0; i < 3 * nv; ++i) {
        if (phiS) phiS[i] = gS[i];
        if (phiV) phiV[i] = -kv * dV / V0 * gV[i];
        if (phiW) phiW[i] = gW[i];
    }
    if (energy) *energy = W;
    if (out_V) *out_V = V;
    if (out_dV) *out_dV = dV;
    if (out_V0) *out_V0 = V0;
    if (out_A) *out_A = A;
    free(gS);
    free(gV);
    free(gW);
}

/* ------------------------------------------------------------------ */
/* the coupled simulation                                               */
/* ------------------------------------------------------------------ */

typedef struct {
    int nx, ny, nz, nzf, zoff, walls;
    long n;
    double tau, rho0, ulo[3], uhi[3], g[3];
    double *d, *dn; /* [Q][n] deviations d_i = f_i - w_i rho0, pre-collision at time t */
    double *F;      /* [3][n] force density used by the last step */
    double *Fext;   /* [3][n] optional fixed force, NULL if unset */
    int has_F;      /* a step has been taken */
    /* mesh */
    int nv, nf;
    double *q, *X, *phi, *qdot;
    int *faces;
    double alpha[3], kv, eps_lo, eps_hi, xi, rc;
    long step;
    int unstable;
} oracle_sim;

static long node(const oracle_sim *s, int x, int y, int zf) { return ((long)zf * s->ny + y) * s->nx + x; }
static int wrap(int a, int n) { a %= n; return a < 0 ? a + n : a; }

/* nx, ny, nz: lattice size; walls != 0: solid layers z = 0 and nz-1 (fluid
 * z = 1..nz-2), else periodic in z as well.  init_couette: f = f^eq(rho0,
 * linear wall profile) instead of rest. */
oracle_sim *oracle_create(int nx, int ny, int nz, int walls, double tau, double rho0, const double *u_lo,
                          const double *u_hi, const double *g, int init_couette)
{
    oracle_sim *s = calloc(1, sizeof(oracle_sim));
    s->nx = nx; s->ny = ny; s->nz = nz;
    s->walls = walls ? 1 : 0;
    s->zoff = s->walls;
    s->nzf = s->walls ? nz - 2 : nz;
    s->n = (long)nx * ny * s->nzf;
    s->tau = tau;
    s->rho0 = rho0;
    for (int k = 0; k < 3; ++k) {
        s->ulo[k] = u_lo ? u_lo[k] : 0.0;
        s->uhi[k] = u_hi ? u_hi[k] : 0.0;
        s->g[k] = g ? g[k] : 0.0;
    }
    s->d = calloc((size_t)Q * s->n, sizeof(double));
    s->dn = calloc((size_t)Q * s->n, sizeof(double));
    s->F = calloc((size_t)3 * s->n, sizeof(double));
    if (init_couette && s->walls) {
        const double zlo = 0.5, zhi = nz - 1.5;
        for (int zf = 0; zf < s->nzf; ++zf) {
            const double z = zf + s->zoff;
            double u[3], deq[Q];
            for (int k = 0; k < 3; ++k)
                u[k] = s->ulo[k] + (s->uhi[k] - s->ulo[k]) * (z - zlo) / (zhi - zlo);
            oracle_feq_dev(rho0, 0.0, u, deq);
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    for (int i = 0; i < Q; ++i)
                        s->d[(long)i * s->n + node(s, x, y, zf)] = deq[i];
        }
    }
    return s;
}

void oracle_destroy(oracle_sim *s)
{
    if (!s) return;
    free(s->d); free(s->dn); free(s->F); free(s->Fext);
    free(s->q); free(s->X); free(s->phi); free(s->qdot); free(s->faces);
    free(s);
}

int oracle_add_mesh(oracle_sim *s, int nv, int nf, const double *q, const double *X, const int *faces,
                    const double *alpha, double kv, double eps_lo, double eps_hi, double xi, double r_cut)
{
    if (s->nv) return -1;
    s->nv = nv; s->nf = nf;
    s->q = malloc(sizeof(double) * 3 * nv);
    s->X = malloc(sizeof(double) * 3 * nv);
    s->phi = calloc((size_t)3 * nv, sizeof(double));
    s->qdot = calloc((size_t)3 * nv, sizeof(double));
    s->faces = malloc(sizeof(int) * 3 * nf);
    memcpy(s->q, q, sizeof(double) * 3 * nv);
    memcpy(s->X, X ? X : q, sizeof(double) * 3 * nv);
    memcpy(s->faces, faces, sizeof(int) * 3 * nf);
    for (int k = 0; k < 3; ++k) s->alpha[k] = alpha[k];
    s->kv = kv; s->eps_lo = eps_lo; s->eps_hi = eps_hi; s->xi = xi; s->rc = r_cut;
    return 0;
}

void oracle_set_force(oracle_sim *s, const double *F)
{
    if (!s->Fext) s->Fext = malloc(sizeof(double) * 3 * s->n);
    memcpy(s->Fext, F, sizeof(double) * 3 * s->n);
}

/* rho and u at fluid node id from the current populations and the force
 * density F of the step that produced them (Guo velocity, footnote on
 * forcing: rho u = sum c_i f_i + F/2). */
static void moments(const oracle_sim *s, long id, double *rho, double *u)
{
    double drho = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        const double di = s->d[(long)i * s->n + id];
        drho += di;
        m[0] += CX[i] * di;
        m[1] += CY[i] * di;
        m[2] += CZ[i] * di;
    }
    *rho = s->rho0 + drho;
    for (int k = 0; k < 3; ++k)
        u[k] = (m[k] + 0.5 * s->F[(long)k * s->n + id]) / *rho;
}

/* Step 1: phi_i = phi^S + phi^V + phi^W. */
static void nodal_forces(oracle_sim *s)
{
    double *pS = malloc(sizeof(double) * 3 * s->nv);
    double *pV = malloc(sizeof(double) * 3 * s->nv);
    double *pW = malloc(sizeof(double) * 3 * s->nv);
    oracle_mesh_forces(s->nv, s->nf, s->q, s->X, s->faces, s->alpha, s->kv, s->walls, 0.5, s->nz - 1.5,
                       s->eps_lo, s->eps_hi, s->xi, s->rc, pS, pV, pW, NULL, NULL, NULL, NULL, NULL);
    for (int i = 0; i < 3 * s->nv; ++i)
        s->phi[i] = pS[i] + pV[i] + pW[i];
    free(pS); free(pV); free(pW);
}

static int finite_vertex(const double *q)
{
    for (int k = 0; k < 3; ++k)
        if (!(fabs(q[k]) < 1e9)) return 0;
    return 1;
}

/* Geometry of the lattice seen by the delta-kernel operations. */
typedef struct {
    int nx, ny, nz, nzf, zoff, walls;
    long n;
} grid_t;

static grid_t grid_of(int nx, int ny, int nz, int walls)
{
    grid_t g;
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.walls = walls ? 1 : 0;
    g.zoff = g.walls;
    g.nzf = g.walls ? nz - 2 : nz;
    g.n = (long)nx * ny * g.nzf;
    return g;
}

static long gnode(const grid_t *g, int x, int y, int z) { return ((long)(z - g->zoff) * g->ny + y) * g->nx + x; }

/* Spreading, Eq. ibm-governing_eq2: F(x) += sum_i phi_i phi4(x-qx) phi4(y-qy)
 * phi4(z-qz) over the 4x4x4 nodes floor(q)-1 .. floor(q)+2 of each vertex.
 * x and y wrap; with walls, nodes outside the fluid layers are dropped.
 * Vertices are visited in index order.  F is [3][n], accumulated into.
 * Returns the number of skipped non-finite vertices. */
int oracle_spread(int nx, int ny, int nz, int walls, int nv, const double *q, const double *phi, double *F)
{
    const grid_t g = grid_of(nx, ny, nz, walls);
    int bad = 0;
    for (int v = 0; v < nv; ++v) {
        const double *qv = q + 3 * v;
        if (!finite_vertex(qv)) { ++bad; continue; }
        const int bx = (int)floor(qv[0]) - 1, by = (int)floor(qv[1]) - 1, bz = (int)floor(qv[2]) - 1;
        for (int kz = 0; kz < 4; ++kz)
            for (int ky = 0; ky < 4; ++ky)
                for (int kx = 0; kx < 4; ++kx) {
                    int z = bz + kz;
                    if (g.walls) {
                        if (z < 1 || z > nz - 2) continue;
                    } else {
                        z = wrap(z, nz);
                    }
                    const double w = oracle_phi4(bx + kx - qv[0]) * oracle_phi4(by + ky - qv[1]) *
                                     oracle_phi4(bz + kz - qv[2]);
                    const long id = gnode(&g, wrap(bx + kx, nx), wrap(by + ky, ny), z);
                    for (int k = 0; k < 3; ++k)
                        F[(long)k * g.n + id] += phi[3 * v + k] * w;
                }
    }
    return bad;
}

/* Interpolation, Eq. ibm-governing_eq1: qdot_i = sum_x u(x) phi4 phi4 phi4
 * over the same 64 nodes.  u is [3][n] on the fluid nodes; with walls, nodes
 * below / above the fluid carry u_lo / u_hi.  Non-finite vertices get 0. */
void oracle_interp(int nx, int ny, int nz, int walls, int nv, const double *q, const double *u,
                   const double *u_lo, const double *u_hi, double *qdot)
{
    const grid_t g = grid_of(nx, ny, nz, walls);
#pragma omp parallel for schedule(static)
    for (int v = 0; v < nv; ++v) {
        const double *qv = q + 3 * v;
        double acc[3] = {0.0, 0.0, 0.0};
        if (finite_vertex(qv)) {
            const int bx = (int)floor(qv[0]) - 1, by = (int)floor(qv[1]) - 1, bz = (int)floor(qv[2]) - 1;
            for (int kz = 0; kz < 4; ++kz)
                for (int ky = 0; ky < 4; ++ky)
                    for (int kx = 0; kx < 4; ++kx) {
                        const double w = oracle_phi4(bx + kx - qv[0]) * oracle_phi4(by + ky - qv[1]) *
                                         oracle_phi4(bz + kz - qv[2]);
                        int z = bz + kz;
                        double un[3];
                        if (g.walls && z < 1) {
                            for (int k = 0; k < 3; ++k) un[k] = u_lo[k];
                        } else if (g.walls && z > nz - 2) {
                            for (int k = 0; k < 3; ++k) un[k] = u_hi[k];
                        } else {
                            if (!g.walls) z = wrap(z, nz);
                            const long id = gnode(&g, wrap(bx + kx, nx), wrap(by + ky, ny), z);
                            for (int k = 0; k < 3; ++k) un[k] = u[(long)k * g.n + id];
                        }
                        for (int k = 0; k < 3; ++k) acc[k] += un[k] * w;
                    }
        }
        for (int k = 0; k < 3; ++k) qdot[3 * v + k] = acc[k];
    }
}

/* Step 3: BGK collision with Guo forcing (Eq. LBeq, dt = 1), propagation to
 * x + c_i (periodic in x, y), half-way bounce-back on the z walls with the
 * moving-wall term -2 w_i rho (c_i.u_w) / c_s^2, rho the local density. */
static void lb_collide_stream(oracle_sim *s)
{
    const long n = s->n;
#pragma omp parallel for schedule(static)
    for (int zf = 0; zf < s->nzf; ++zf)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                const long id = node(s, x, y, zf);
                double dloc[Q], drho = 0.0, m[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < Q; ++i) {
                    dloc[i] = s->d[(long)i * n + id];
                    drho += dloc[i];
                    m[0] += CX[i] * dloc[i];
                    m[1] += CY[i] * dloc[i];
                    m[2] += CZ[i] * dloc[i];
                }
                const double rho = s->rho0 + drho;
                const double F[3] = {s->F[id], s->F[n + id], s->F[2 * n + id]};
                double u[3], deq[Q], S[Q];
                for (int k = 0; k < 3; ++k) u[k] = (m[k] + 0.5 * F[k]) / rho;
                oracle_feq_dev(s->rho0, drho, u, deq);
                oracle_guo(s->tau, u, F, S);
                for (int i = 0; i < Q; ++i) {
                    const double post = dloc[i] - (dloc[i] - deq[i]) / s->tau + S[i];
                    const int tx = wrap(x + CX[i], s->nx), ty = wrap(y + CY[i], s->ny);
                    int tz = zf + s->zoff + CZ[i];
                    if (s->walls && (tz < 1 || tz > s->nz - 2)) {
                        const double *uw = tz < 1 ? s->ulo : s->uhi;
                        const double cuw = CX[i] * uw[0] + CY[i] * uw[1] + CZ[i] * uw[2];
                        s->dn[(long)opposite(i) * n + id] = post - 6.0 * weight(i) * rho * cuw;
                    } else {
                        if (!s->walls) tz = wrap(tz, s->nz);
                        s->dn[(long)i * n + node(s, tx, ty, tz - s->zoff)] = post;
                    }
                }
            }
    double *t = s->d; s->d = s->dn; s->dn = t;
}

/* Steps 4-6: u(t+1) on every fluid node, qdot_i by interpolation, then
 * q_i += qdot_i once every vertex has its velocity. */
static void interpolate_move(oracle_sim *s)
{
    double *u = malloc(sizeof(double) * 3 * s->n);
#pragma omp parallel for schedule(static)
    for (long id = 0; id < s->n; ++id) {
        double rho, uu[3];
        moments(s, id, &rho, uu);
        for (int k = 0; k < 3; ++k) u[(long)k * s->n + id] = uu[k];
    }
    oracle_interp(s->nx, s->ny, s->nz, s->walls, s->nv, s->q, u, s->ulo, s->uhi, s->qdot);
    free(u);
    for (int i = 0; i < 3 * s->nv; ++i)
        s->q[i] += s->qdot[i];
}

/* Advance n steps.  Returns 0, or -4 once a vertex has left the finite range. */
int oracle_step(oracle_sim *s, int nsteps)
{
    for (int it = 0; it < nsteps; ++it) {
        if (s->nv) nodal_forces(s);
        for (long id = 0; id < s->n; ++id)
            for (int k = 0; k < 3; ++k)
                s->F[(long)k * s->n + id] = s->g[k] + (s->Fext ? s->Fext[(long)k * s->n + id] : 0.0);
        if (s->nv && oracle_spread(s->nx, s->ny, s->nz, s->walls, s->nv, s->q, s->phi, s->F))
            s->unstable = 1;
        lb_collide_stream(s);
        if (s->nv) interpolate_move(s);
        s->has_F = 1;
        s->step++;
    }
    return s->unstable ? -4 : 0;
}

long oracle_n_fluid(const oracle_sim *s) { return s->n; }
long oracle_step_count(const oracle_sim *s) { return s->step; }

void oracle_get_vertices(const oracle_sim *s, double *out) { memcpy(out, s->q, sizeof(double) * 3 * s->nv); }
void oracle_set_vertices(oracle_sim *s, const double *in) { memcpy(s->q, in, sizeof(double) * 3 * s->nv); }
void oracle_get_nodal_forces(const oracle_sim *s, double *out) { memcpy(out, s->phi, sizeof(double) * 3 * s->nv); }

/* Population deviations d_i = f_i - w_i rho0, [19][nz_f][ny][nx]. */
void oracle_get_populations(const oracle_sim *s, double *out) { memcpy(out, s->d, sizeof(double) * Q * s->n); }
void oracle_set_populations(oracle_sim *s, const double *in) { memcpy(s->d, in, sizeof(double) * Q * s->n); }

/* Force density of the last step [3][n] (zero before the first step). */
void oracle_get_force(const oracle_sim *s, double *out)
{
    if (s->has_F) memcpy(out, s->F, sizeof(double) * 3 * s->n);
    else memset(out, 0, sizeof(double) * 3 * s->n);
}

/* rho [n] and u [3][n] at the current time, with the last step's force. */
void oracle_get_fields(const oracle_sim *s, double *rho, double *u)
{
    for (long id = 0; id < s->n; ++id) {
        double r, uu[3];
        if (s->has_F) {
            moments(s, id, &r, uu);
        } else {
            double drho = 0.0, m[3] = {0, 0, 0};
            for (int i = 0; i < Q; ++i) {
                const double di = s->d[(long)i * s->n + id];
                drho += di; m[0] += CX[i] * di; m[1] += CY[i] * di; m[2] += CZ[i] * di;
            }
            r = s->rho0 + drho;
            for (int k = 0; k < 3; ++k) uu[k] = m[k] / r;
        }
        rho[id] = r;
        for (int k = 0; k < 3; ++k) u[(long)k * s->n + id] = uu[k];
    }
}
