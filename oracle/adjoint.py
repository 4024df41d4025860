"""Reference gradients of the IB-LB step (test infrastructure only).

Like the rest of ``oracle/`` this module may be imported only by the tests,
the smoke check and the CPU-baseline leg of the benchmark.  It shares no code
with the GPU library.

The coupled step of the C oracle is restated with PyTorch tensor operations
in float64 on the CPU, step for step in the same order:
  1. nodal forces phi = phi^S + phi^V + phi^W (Eqs. generalised_energy1,
     nodal_force_S, nodal_force_V, LJ_interaction);
  2. spreading F(x) = sum_i phi_i delta(x - q_i) (Eq. ibm-governing_eq2);
  3. BGK collision with Guo forcing, propagation, half-way bounce-back with
     the moving-wall term (Eqs. LBeq, feq);
  4. u(t+1) = (sum c f(t+1) + F/2) / rho(t+1) with this step's F;
  5. interpolation and move q += sum_x u(x) delta(x - q) (Eq.
     ibm-governing_eq1), wall velocities at the stencil nodes outside the
     fluid.
The tests pin this restatement to the C oracle's trajectory.  Reverse-mode
differentiation of exactly these operations (torch.autograd) then gives the
gradient of an observable of the final vertex positions with respect to the
parameters abar (alpha = abar * model), k_V, eps (lower wall strength) and
tau, and with respect to the initial positions.  Those gradients are in turn
pinned by central finite differences of the C oracle.

Observables (the algebraic sphere fit of the contact-angle query: vertices at
least r_c above the lower wall plane z_lo):
  h  = z_c + R - z_lo                 height of the fitted cap,
  r2 = R^2 - (z_c - z_lo)^2           signed squared contact radius: the
                                      squared radius of the circle the fitted
                                      sphere cuts from the wall plane when
                                      positive (no contact when negative).
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64

# D3Q19, the canonical order of the library and the oracle
_C = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
      (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
      (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
C = torch.tensor(_C, dtype=F64)
W = torch.tensor([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12, dtype=F64)
OPP = [0] + [i + 1 if i % 2 else i - 1 for i in range(1, 19)]


def phi4(r: torch.Tensor) -> torch.Tensor:
    """4-point stencil (Eq. ibm-interpolation_stencil).  Both square-root
    arguments are >= 1 where their branch is used; clamping them there keeps
    the unused branch's derivative finite."""
    a = r.abs()
    inner = (3.0 - 2.0 * a + torch.sqrt(torch.clamp(1.0 + 4.0 * a - 4.0 * a * a, min=1.0))) / 8.0
    outer = (5.0 - 2.0 * a - torch.sqrt(torch.clamp(-7.0 + 12.0 * a - 4.0 * a * a, min=1.0))) / 8.0
    zero = torch.zeros_like(a)
    return torch.where(a <= 1.0, inner, torch.where(a <= 2.0, outer, zero))


def lj(eps, xi: float, rc: float, d: torch.Tensor) -> torch.Tensor:
    """Wall force along the wall normal, 48 eps [(xi/d)^12 - (xi/d)^6 / 2] / d
    (Eq. LJ_interaction), zero from r_c on, d clamped from below at xi/2."""
    dd = torch.clamp(d, min=0.5 * xi)
    s6 = (xi / dd) ** 6
    f = 48.0 * eps * (s6 * s6 - 0.5 * s6) / dd
    return torch.where(d < rc, f, torch.zeros_like(f))


def _triple(a, b, c):
    return (a * torch.cross(b, c, dim=1)).sum(1)


class Case:
    """A lattice with one mesh; index tables of the propagation and the
    reference geometry of the faces (all constant)."""

    def __init__(self, domain, mesh, model):
        self.nx, self.ny, self.nz = domain.nx, domain.ny, domain.nz
        self.walls = domain.wall_mode == 0
        self.zoff = 1 if self.walls else 0
        self.nzf = self.nz - 2 if self.walls else self.nz
        self.n = self.nx * self.ny * self.nzf
        self.rho0 = float(domain.rho0)
        self.ulo = torch.tensor(domain.u_wall_lo, dtype=F64)
        self.uhi = torch.tensor(domain.u_wall_hi, dtype=F64)
        self.g = torch.tensor(domain.body_force, dtype=F64)
        self.z_lo, self.z_hi = 0.5, self.nz - 1.5
        self.model = torch.tensor(model, dtype=F64)
        self.xi, self.rc = float(mesh.xi_wall), float(mesh.r_cut_wall)
        self.eps_hi = float(mesh.eps_wall_hi)
        self.faces = torch.tensor(np.asarray(mesh.faces), dtype=torch.long)
        self.X = torch.tensor(np.asarray(mesh.ref_vertices), dtype=F64)
        self.q0 = torch.tensor(np.asarray(mesh.vertices), dtype=F64)
        self.nv = self.q0.shape[0]
        f = self.faces
        Xa, Xb, Xc = self.X[f[:, 0]], self.X[f[:, 1]], self.X[f[:, 2]]
        E1, E2 = Xb - Xa, Xc - Xa
        G11, G12, G22 = (E1 * E1).sum(1), (E1 * E2).sum(1), (E2 * E2).sum(1)
        self.detG = G11 * G22 - G12 * G12
        self.Ginv = torch.stack([G22, -G12, G11], 1) / self.detG[:, None]
        self.A0 = 0.5 * torch.sqrt(self.detG)
        self.o = self.X.mean(0)
        self.V0 = (_triple(Xa - self.o, Xb - self.o, Xc - self.o) / 6.0).sum()
        # propagation: destination of each (direction, node), or a wall link
        zf, y, x = np.meshgrid(np.arange(self.nzf), np.arange(self.ny), np.arange(self.nx), indexing="ij")
        zf, y, x = zf.ravel(), y.ravel(), x.ravel()
        self.dest, self.interior, self.wall_lo = [], [], []
        for (cx, cy, cz) in _C:
            tx, ty, tz = (x + cx) % self.nx, (y + cy) % self.ny, zf + self.zoff + cz
            if self.walls:
                inside = (tz >= 1) & (tz <= self.nz - 2)
            else:
                inside = np.ones_like(tz, dtype=bool)
                tz = tz % self.nz
            tzf = np.where(inside, tz - self.zoff, 0)
            self.dest.append(torch.tensor((tzf * self.ny + ty) * self.nx + tx, dtype=torch.long))
            self.interior.append(torch.tensor(inside))
            self.wall_lo.append(torch.tensor(tz < 1))

    # -- step 1
    def forces(self, q, alpha, kv, eps_lo):
        f = self.faces
        a, b, c = q[f[:, 0]], q[f[:, 1]], q[f[:, 2]]
        e1, e2 = b - a, c - a
        g11, g12, g22 = (e1 * e1).sum(1), (e1 * e2).sum(1), (e2 * e2).sum(1)
        detg = g11 * g22 - g12 * g12
        J = detg / self.detG
        lnJ = torch.log(J)
        w1 = 0.5 * alpha[2]
        w2 = (0.5 * (alpha[0] - alpha[2]) + 0.25 * (alpha[0] + alpha[1]) * lnJ) / J
        S11 = self.A0 * (w1 * self.Ginv[:, 0] + w2 * g22 / self.detG)
        S12 = self.A0 * (w1 * self.Ginv[:, 1] - w2 * g12 / self.detG)
        S22 = self.A0 * (w1 * self.Ginv[:, 2] + w2 * g11 / self.detG)
        Fb = -2.0 * (S11[:, None] * e1 + S12[:, None] * e2)
        Fc = -2.0 * (S12[:, None] * e1 + S22[:, None] * e2)
        Fa = -Fb - Fc
        z = torch.zeros(self.nv, 3, dtype=F64)
        phiS = z.index_add(0, f[:, 0], Fa).index_add(0, f[:, 1], Fb).index_add(0, f[:, 2], Fc)
        # volume: V - V0 summed face by face from the displacements (trilinear
        # expansion of the triple product), and its gradient
        o = self.o
        A_, B_, C_ = self.X[f[:, 0]] - o, self.X[f[:, 1]] - o, self.X[f[:, 2]] - o
        da, db, dc = a - self.X[f[:, 0]], b - self.X[f[:, 1]], c - self.X[f[:, 2]]
        dV = (_triple(da, B_, C_) + _triple(A_, db, C_) + _triple(A_, B_, dc) + _triple(da, db, C_)
              + _triple(da, B_, dc) + _triple(A_, db, dc) + _triple(da, db, dc)).sum() / 6.0
        ao, bo, co = a - o, b - o, c - o
        gV = (z.index_add(0, f[:, 0], torch.cross(bo, co, dim=1) / 6.0)
              .index_add(0, f[:, 1], torch.cross(co, ao, dim=1) / 6.0)
              .index_add(0, f[:, 2], torch.cross(ao, bo, dim=1) / 6.0))
        phiV = -kv * dV / self.V0 * gV
        phiW = z
        if self.walls:
            cz = (a[:, 2] + b[:, 2] + c[:, 2]) / 3.0
            fz = lj(eps_lo, self.xi, self.rc, cz - self.z_lo) - lj(self.eps_hi, self.xi, self.rc, self.z_hi - cz)
            fw = torch.stack([torch.zeros_like(fz), torch.zeros_like(fz), fz / 3.0], 1)
            phiW = z.index_add(0, f[:, 0], fw).index_add(0, f[:, 1], fw).index_add(0, f[:, 2], fw)
        return phiS + phiV + phiW

    # stencil of every vertex: weights [nv, 64], node ids [nv, 64], fluid mask,
    # and the side of each non-fluid node (for the wall velocity)
    def stencil(self, q):
        base = torch.floor(q.detach()) - 1.0
        k = torch.arange(4, dtype=F64)
        r = base[:, :, None] + k[None, None, :] - q[:, :, None]
        w = phi4(r)
        Wt = (w[:, 2, :, None, None] * w[:, 1, None, :, None] * w[:, 0, None, None, :]).reshape(self.nv, 64)
        bi = base.long()
        kk = torch.arange(4)
        xs = (bi[:, 0, None] + kk) % self.nx
        ys = (bi[:, 1, None] + kk) % self.ny
        zs = bi[:, 2, None] + kk
        if self.walls:
            inside = (zs >= 1) & (zs <= self.nz - 2)
            zfs = torch.where(inside, zs - self.zoff, torch.zeros_like(zs))
        else:
            inside = torch.ones_like(zs, dtype=torch.bool)
            zfs = zs % self.nz
        ids = ((zfs[:, :, None, None] * self.ny + ys[:, None, :, None]) * self.nx + xs[:, None, None, :])
        fluid = inside[:, :, None, None].expand(-1, 4, 4, 4)
        below = (zs < 1)[:, :, None, None].expand(-1, 4, 4, 4)
        return Wt, ids.reshape(self.nv, 64), fluid.reshape(self.nv, 64), below.reshape(self.nv, 64)

    def step(self, d, q, alpha, kv, eps_lo, tau):
        phi = self.forces(q, alpha, kv, eps_lo)
        Wt, ids, fluid, below = self.stencil(q)
        contrib = (Wt[:, :, None] * phi[:, None, :])[fluid]
        F = torch.zeros(self.n, 3, dtype=F64).index_add(0, ids[fluid], contrib).T + self.g[:, None]
        # collision (deviations d = f - w rho0)
        rho = self.rho0 + d.sum(0)
        u = (C.T @ d + 0.5 * F) / rho
        cu = C @ u
        uu = (u * u).sum(0)
        deq = W[:, None] * (rho - self.rho0) + W[:, None] * rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu)
        cF = C @ F
        S = W[:, None] * (1.0 - 1.0 / (2.0 * tau)) * (3.0 * (cF - (u * F).sum(0)) + 9.0 * cF * cu)
        post = d - (d - deq) / tau + S
        # propagation and half-way bounce-back
        rows = [torch.zeros(self.n, dtype=F64) for _ in range(19)]
        for i in range(19):
            inn = self.interior[i]
            rows[i] = rows[i].index_add(0, self.dest[i][inn], post[i][inn])
            if not bool(inn.all()):
                wl = ~inn
                uw = torch.where(self.wall_lo[i][wl][:, None], self.ulo[None, :], self.uhi[None, :])
                cuw = (uw * C[i][None, :]).sum(1)
                node = torch.nonzero(wl).squeeze(1)
                rows[OPP[i]] = rows[OPP[i]].index_add(0, node, post[i][wl] - 6.0 * W[i] * rho[wl] * cuw)
        dn = torch.stack(rows)
        # u(t+1) with this step's force, interpolation and move
        rho1 = self.rho0 + dn.sum(0)
        u1 = (C.T @ dn + 0.5 * F) / rho1
        un = u1.T[ids]
        wallu = torch.where(below[:, :, None], self.ulo[None, None, :], self.uhi[None, None, :])
        un = torch.where(fluid[:, :, None], un, wallu)
        qn = q + (Wt[:, :, None] * un).sum(1)
        return dn, qn

    def initial(self):
        return torch.zeros(19, self.n, dtype=F64), self.q0.clone()

    def run(self, steps, abar, kv, eps_lo, tau, q0=None):
        d, q = self.initial()
        if q0 is not None:
            q = q0
        alpha = abar * self.model
        for _ in range(steps):
            d, q = self.step(d, q, alpha, kv, eps_lo, tau)
        return d, q


def sphere_fit(q: torch.Tensor, z_lo: float, rc: float) -> dict:
    """Algebraic least-squares sphere |p|^2 = 2 c.p + k through the vertices
    with z - z_lo >= rc (normal equations), R^2 = k + |c|^2."""
    sel = (q[:, 2].detach() - z_lo) >= rc
    p = q[sel]
    A = torch.cat([2.0 * p, torch.ones(p.shape[0], 1, dtype=F64)], 1)
    rhs = (p * p).sum(1)
    sol = torch.linalg.solve(A.T @ A, A.T @ rhs)
    cen, k = sol[:3], sol[3]
    R = torch.sqrt(k + cen @ cen)
    hc = cen[2] - z_lo
    return {"h": cen[2] + R - z_lo, "r2": R * R - hc * hc, "R": R, "zc": cen[2]}


def gradients(domain, mesh, model, abar, kv, eps_lo, tau, steps: int, observable: str = "h"):
    """Value of the observable after `steps` steps and its gradient with
    respect to (abar, k_V, eps_lo, tau) and the initial positions [nv, 3]."""
    case = Case(domain, mesh, model)
    p = [torch.tensor(float(v), dtype=F64, requires_grad=True) for v in (abar, kv, eps_lo, tau)]
    q0 = case.q0.clone().requires_grad_(True)
    _, q = case.run(steps, *p, q0=q0)
    J = sphere_fit(q, case.z_lo, case.rc)[observable]
    grads = torch.autograd.grad(J, p + [q0])
    return float(J.detach()), np.array([float(g) for g in grads[:4]]), grads[4].numpy()
