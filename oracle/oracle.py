"""Python face of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  It loads ``liboracle.so`` built from ``iblb_oracle.c``
with plain gcc (no GPU code, nothing shared with the GPU library) and adds the
query-time observables in numpy:

* volume, area and volume centroid of the closed mesh (signed tetrahedra);
* Taylor deformation D = (r1 - r3)/(r1 + r3) and inclination Theta in the
  shear plane (Eq. taylor_deform) from the central second-moment tensor of the
  enclosed polyhedron, read as an ellipsoid with M = V/5 diag(r^2);
* equilibrium contact angle from an algebraic least-squares sphere fit of the
  vertices away from the wall, and the paper's own measurement (appendix on the
  resolution test): a circle cut by the wall chord, fitted to a slice of the
  mesh holding about (4 / 3^(1/4)) sqrt(pi N_f) nodes;
* the small-deformation theory of a particle in shear the paper compares its
  shear runs with (Eqs. evJK, L_M, deformation_J), integrated in time.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "iblb_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 -fopenmp (no fast-math, no FMA target)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        L.oracle_phi4.restype = C.c_double
        L.oracle_phi4.argtypes = [C.c_double]
        L.oracle_lj.restype = C.c_double
        L.oracle_lj.argtypes = [C.c_double] * 4
        L.oracle_feq.argtypes = [C.c_double, _dp, _dp]
        L.oracle_feq_dev.argtypes = [C.c_double, C.c_double, _dp, _dp]
        L.oracle_guo.argtypes = [C.c_double, _dp, _dp, _dp]
        L.oracle_lattice.argtypes = [_ip, _dp, _ip]
        L.oracle_mesh_forces.argtypes = ([C.c_int, C.c_int, _dp, _dp, _ip, _dp, C.c_double, C.c_int]
                                         + [C.c_double] * 6 + [_dp] * 8)
        L.oracle_create.restype = C.c_void_p
        L.oracle_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                    _dp, _dp, _dp, C.c_int]
        L.oracle_destroy.argtypes = [C.c_void_p]
        L.oracle_add_mesh.argtypes = ([C.c_void_p, C.c_int, C.c_int, _dp, _dp, _ip, _dp]
                                      + [C.c_double] * 5)
        L.oracle_set_force.argtypes = [C.c_void_p, _dp]
        L.oracle_step.argtypes = [C.c_void_p, C.c_int]
        L.oracle_n_fluid.restype = C.c_long
        L.oracle_n_fluid.argtypes = [C.c_void_p]
        L.oracle_step_count.restype = C.c_long
        L.oracle_step_count.argtypes = [C.c_void_p]
        for name in ("oracle_get_vertices", "oracle_set_vertices", "oracle_get_nodal_forces",
                     "oracle_get_populations", "oracle_set_populations", "oracle_get_force"):
            getattr(L, name).argtypes = [C.c_void_p, _dp]
        L.oracle_get_fields.argtypes = [C.c_void_p, _dp, _dp]
        L.oracle_spread.restype = C.c_int
        L.oracle_spread.argtypes = [C.c_int] * 5 + [_dp, _dp, _dp]
        L.oracle_interp.argtypes = [C.c_int] * 5 + [_dp] * 5
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------- point formulas

def lattice():
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, dtype=np.int32)
    lib().oracle_lattice(c.ctypes.data_as(_ip), _p(w), opp.ctypes.data_as(_ip))
    return c, w, opp


def phi4(r: float) -> float:
    return lib().oracle_phi4(float(r))


def lj(eps: float, xi: float, r_cut: float, d: float) -> float:
    return lib().oracle_lj(float(eps), float(xi), float(r_cut), float(d))


def feq(rho: float, u) -> np.ndarray:
    out = np.zeros(19)
    lib().oracle_feq(float(rho), _p(_f64(u)), _p(out))
    return out


def feq_dev(rho0: float, drho: float, u) -> np.ndarray:
    out = np.zeros(19)
    lib().oracle_feq_dev(float(rho0), float(drho), _p(_f64(u)), _p(out))
    return out


def guo(tau: float, u, F) -> np.ndarray:
    out = np.zeros(19)
    lib().oracle_guo(float(tau), _p(_f64(u)), _p(_f64(F)), _p(out))
    return out


def mesh_forces(q, X, faces, alpha, kv=1.0, walls=False, z_lo=0.5, z_hi=1e30,
                eps_lo=0.0, eps_hi=0.0, xi=0.5, r_cut=2.0) -> dict:
    """Nodal force parts phi^S, phi^V, phi^W and the scalars W, V, V-V0, V0, A."""
    q = _f64(q)
    X = _f64(X)
    faces = np.ascontiguousarray(np.asarray(faces, dtype=np.int32))
    nv, nf = q.shape[0], faces.shape[0]
    pS, pV, pW = np.zeros((nv, 3)), np.zeros((nv, 3)), np.zeros((nv, 3))
    sc = [C.c_double() for _ in range(5)]
    lib().oracle_mesh_forces(nv, nf, _p(q), _p(X), faces.ctypes.data_as(_ip), _p(_f64(alpha)),
                             float(kv), int(bool(walls)), z_lo, z_hi, eps_lo, eps_hi, xi, r_cut,
                             _p(pS), _p(pV), _p(pW), *[C.byref(s) for s in sc])
    W, V, dV, V0, A = (s.value for s in sc)
    return {"phiS": pS, "phiV": pV, "phiW": pW, "W": W, "V": V, "dV": dV, "V0": V0, "A": A}


def spread(nx, ny, nz, walls, q, phi) -> np.ndarray:
    """F [3, nz_f, ny, nx] spread from vertex forces phi [N_v, 3] at positions q."""
    nzf = nz - 2 if walls else nz
    F = np.zeros((3, nzf, ny, nx))
    q = _f64(q)
    lib().oracle_spread(nx, ny, nz, int(bool(walls)), q.shape[0], _p(q), _p(_f64(phi)), _p(F))
    return F


def interp(nx, ny, nz, walls, q, u, u_lo=(0, 0, 0), u_hi=(0, 0, 0)) -> np.ndarray:
    """qdot [N_v, 3] interpolated from u [3, nz_f, ny, nx]."""
    q = _f64(q)
    out = np.zeros((q.shape[0], 3))
    lib().oracle_interp(nx, ny, nz, int(bool(walls)), q.shape[0], _p(q), _p(_f64(u)),
                        _p(_f64(u_lo)), _p(_f64(u_hi)), _p(out))
    return out


# ---------------------------------------------------------------- simulation

class OracleSim:
    """One lattice with at most one mesh, stepped in FP64 on the CPU."""

    def __init__(self, domain, mesh=None):
        L = lib()
        self.dom = domain
        self.h = L.oracle_create(domain.nx, domain.ny, domain.nz, 1 if domain.wall_mode == 0 else 0,
                                 domain.tau, domain.rho0, _p(_f64(domain.u_wall_lo)),
                                 _p(_f64(domain.u_wall_hi)), _p(_f64(domain.body_force)),
                                 int(domain.init_couette))
        self.n = L.oracle_n_fluid(self.h)
        self.shape = (domain.nz_fluid, domain.ny, domain.nx)
        self.nv = 0
        if mesh is not None:
            self.add_mesh(mesh)

    def add_mesh(self, m):
        self.mesh = m
        self.nv = m.n_vertices
        faces = np.ascontiguousarray(m.faces, dtype=np.int32)
        rc = lib().oracle_add_mesh(self.h, m.n_vertices, m.n_faces, _p(_f64(m.vertices)),
                                   _p(_f64(m.ref_vertices)), faces.ctypes.data_as(_ip),
                                   _p(_f64(m.alpha)), m.k_v, m.eps_wall_lo, m.eps_wall_hi,
                                   m.xi_wall, m.r_cut_wall)
        if rc != 0:
            raise RuntimeError("oracle supports one mesh")

    def set_force(self, F: np.ndarray):
        lib().oracle_set_force(self.h, _p(_f64(F).reshape(-1)))

    def step(self, n: int = 1) -> int:
        return lib().oracle_step(self.h, int(n))

    @property
    def t(self) -> int:
        return lib().oracle_step_count(self.h)

    def vertices(self) -> np.ndarray:
        out = np.zeros((self.nv, 3))
        lib().oracle_get_vertices(self.h, _p(out))
        return out

    def nodal_forces(self) -> np.ndarray:
        out = np.zeros((self.nv, 3))
        lib().oracle_get_nodal_forces(self.h, _p(out))
        return out

    def populations(self) -> np.ndarray:
        """Deviations f_i - w_i rho0, shape [19, nz_f, ny, nx]."""
        out = np.zeros((19,) + self.shape)
        lib().oracle_get_populations(self.h, _p(out))
        return out

    def set_populations(self, d: np.ndarray):
        lib().oracle_set_populations(self.h, _p(_f64(d).reshape(-1)))

    def force(self) -> np.ndarray:
        out = np.zeros((3,) + self.shape)
        lib().oracle_get_force(self.h, _p(out))
        return out

    def fields(self):
        rho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        lib().oracle_get_fields(self.h, _p(rho), _p(u))
        return rho, u

    def close(self):
        if self.h:
            lib().oracle_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- observables

def volume_area_centroid(q, faces):
    """V, A and the volume centroid of a closed, outward-oriented triangle mesh."""
    q = np.asarray(q, dtype=np.float64)
    f = np.asarray(faces)
    o = q.mean(axis=0)
    a, b, c = q[f[:, 0]] - o, q[f[:, 1]] - o, q[f[:, 2]] - o
    vt = np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0
    V = vt.sum()
    A = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1).sum()
    xc = (vt[:, None] * (a + b + c) / 4.0).sum(axis=0) / V + o
    return V, A, xc


def second_moment(q, faces):
    """Central second-moment tensor of the enclosed volume and the volume."""
    q = np.asarray(q, dtype=np.float64)
    f = np.asarray(faces)
    o = q.mean(axis=0)
    a, b, c = q[f[:, 0]] - o, q[f[:, 1]] - o, q[f[:, 2]] - o
    vt = np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0
    s = a + b + c
    M = np.zeros((3, 3))
    for p in (a, b, c, s):
        M += np.einsum("t,ti,tj->ij", vt / 20.0, p, p)
    V = vt.sum()
    xc = (vt[:, None] * s / 4.0).sum(axis=0) / V
    return M - V * np.outer(xc, xc), V


def shape_dtheta(q, faces):
    """(D, Theta) in the x-z shear plane; Theta is the angle of r1 from +x."""
    M, V = second_moment(q, faces)
    B = M[np.ix_([0, 2], [0, 2])]
    lam, vec = np.linalg.eigh(B)
    r = np.sqrt(5.0 * lam / V)
    r1, r3 = r[1], r[0]
    v = vec[:, 1]
    th = np.arctan2(v[1], v[0])
    if th > np.pi / 2:
        th -= np.pi
    elif th <= -np.pi / 2:
        th += np.pi
    return (r1 - r3) / (r1 + r3), th


def contact_angle_sphere(q, z_wall: float, exclude: float = 2.0, wall_hi: bool = False):
    """Algebraic least-squares sphere through the vertices at least `exclude`
    from the wall plane z = z_wall (the lower wall, or the upper one with
    wall_hi, the liquid then lying below it).

    Solves |p|^2 = 2 c.p + k for (c, k); R^2 = k + |c|^2; the centre's height
    hc above the wall into the liquid gives theta = arccos(-hc / R).  Returns
    (theta_deg, contact_radius, height, centre, R)."""
    q = np.asarray(q, dtype=np.float64)
    dist = (z_wall - q[:, 2]) if wall_hi else (q[:, 2] - z_wall)
    p = q[dist >= exclude]
    A = np.hstack([2.0 * p, np.ones((p.shape[0], 1))])
    rhs = (p * p).sum(axis=1)
    sol, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    cen, k = sol[:3], sol[3]
    R = np.sqrt(k + cen @ cen)
    hc = (z_wall - cen[2]) if wall_hi else (cen[2] - z_wall)
    theta = np.degrees(np.arccos(np.clip(-hc / R, -1.0, 1.0)))
    r = np.sqrt(max(0.0, R * R - hc * hc))
    return theta, r, hc + R, cen, R


def slice_count(n_faces: int) -> int:
    """Nodes in the paper's fitting slice, (4 / 3^(1/4)) sqrt(pi N_f), rounded
    (appendix on the resolution test).  For a sphere meshed by N_f nearly
    equilateral triangles this is the number of nodes within two edge lengths
    of a plane through the centre."""
    return int(np.floor(4.0 / 3.0 ** 0.25 * np.sqrt(np.pi * n_faces) + 0.5))


def contact_angle_slice(q, faces, z_wall: float, exclude: float = 2.0, wall_hi: bool = False, K=None):
    """The paper's contact angle (appendix on the resolution test): a circle cut
    by the wall chord fitted to a slice of the mesh.  The slice is the K nodes
    nearest the plane y = y of the volume centroid (ties to the lower vertex
    index), K = slice_count(N_f) unless given; they are projected on (x, z),
    those at least `exclude` from the wall plane kept, and the circle
    x^2 + z^2 = 2 c.p + k fitted by algebraic least squares.  Returns
    (theta_deg, contact_radius, height, centre_xz, R) as contact_angle_sphere."""
    q = np.asarray(q, dtype=np.float64)
    nv = q.shape[0]
    K = slice_count(len(faces)) if K is None else int(K)
    K = max(1, min(nv, K))
    _, _, xc = volume_area_centroid(q, faces)
    d = np.abs(q[:, 1] - xc[1])
    order = np.lexsort((np.arange(nv), d))[:K]
    p = q[order]
    dist = (z_wall - p[:, 2]) if wall_hi else (p[:, 2] - z_wall)
    p = p[dist >= exclude]
    xz = p[:, [0, 2]]
    A = np.hstack([2.0 * xz, np.ones((xz.shape[0], 1))])
    rhs = (xz * xz).sum(axis=1)
    sol, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    cen, k = sol[:2], sol[2]
    R = np.sqrt(k + cen @ cen)
    hc = (z_wall - cen[1]) if wall_hi else (cen[1] - z_wall)
    theta = np.degrees(np.arccos(np.clip(-hc / R, -1.0, 1.0)))
    r = np.sqrt(max(0.0, R * R - hc * hc))
    return theta, r, hc + R, cen, R


def shear_deformation_ode(a, t_end: float, n_steps: int, lam: float = 1.0, n_samples: int = 0):
    """Small-deformation dynamics of a particle in simple shear (Interface
    model section, Eqs. evJK and L_M), integrated by the classical fourth-order
    Runge-Kutta method from a sphere at rest (J = K = 0).

    Units: time in 1 / gammadot, lengths in the radius R; a = (a1, a2, a3) =
    alpha_k / (mu R gammadot), i.e. alpha_k / (alpha Ca) with Ca = mu R
    gammadot / alpha.  The shear flow is u = (z, 0, 0) (flow along x,
    gradient along z): velocity gradient G_ij = du_i/dx_j, E = (G + G^T) / 2,
    Omega = (G - G^T) / 2, and the Jaumann derivative D A / Dt = dA/dt -
    (Omega A - A Omega).  J here is the deformation itself (the paper's J
    times Ca), so Eq. deformation_J reads D = (J_xx^2 + J_xz^2)^(1/2); the
    inclination is that of the principal axis of J's x-z block, measured from
    x toward z.  Returns a dict with t, D and Theta at n_samples + 1 equally
    spaced times (start and end included; the end alone if n_samples = 0) and
    the final J and K."""
    a1, a2, a3 = (float(v) for v in a)
    G = np.zeros((3, 3))
    G[0, 2] = 1.0
    E = 0.5 * (G + G.T)
    W = 0.5 * (G - G.T)
    c_lam = 2.0 * lam + 3.0
    c_m = 19.0 * lam + 16.0

    def rates(J, K):
        L = 4.0 * (a2 + a3) * J - (6.0 * a2 + 10.0 * a3) * K
        M = -4.0 * (a1 + 2.0 * a2 + 2.0 * a3) * J + (12.0 * a2 + 16.0 * a3) * K
        DK = 5.0 * E / c_lam + L / c_lam + M * (6.0 * lam + 4.0) / (c_lam * c_m)
        DJ_K = 2.0 * M / c_m
        # dA/dt = D A / Dt + (Omega A - A Omega), for K and for J = (J - K) + K
        dK = DK + W @ K - K @ W
        dJ = DJ_K + DK + W @ J - J @ W
        return dJ, dK

    def observe(J):
        return np.hypot(J[0, 0], J[0, 2]), 0.5 * np.arctan2(2.0 * J[0, 2], J[0, 0] - J[2, 2])

    dt = t_end / n_steps
    every = n_steps // n_samples if n_samples else n_steps
    J = np.zeros((3, 3))
    K = np.zeros((3, 3))
    ts, Ds, Ths = [], [], []
    if n_samples:
        ts.append(0.0)
        Ds.append(0.0)
        Ths.append(0.0)
    for s in range(1, n_steps + 1):
        k1 = rates(J, K)
        k2 = rates(J + 0.5 * dt * k1[0], K + 0.5 * dt * k1[1])
        k3 = rates(J + 0.5 * dt * k2[0], K + 0.5 * dt * k2[1])
        k4 = rates(J + dt * k3[0], K + dt * k3[1])
        J = J + dt / 6.0 * (k1[0] + 2.0 * k2[0] + 2.0 * k3[0] + k4[0])
        K = K + dt / 6.0 * (k1[1] + 2.0 * k2[1] + 2.0 * k3[1] + k4[1])
        if s % every == 0 or s == n_steps:
            D, th = observe(J)
            if not ts or ts[-1] < s * dt:
                ts.append(s * dt)
                Ds.append(D)
                Ths.append(th)
    return {"t": np.array(ts), "D": np.array(Ds), "Theta": np.array(Ths), "J": J, "K": K}
