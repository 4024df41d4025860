"""Seeded synthetic inputs for the IB-LB step: meshes, perturbations, workloads.

This module only *prepares inputs*.  It holds none of the method's arithmetic
(no lattice Boltzmann, no interface mechanics, no delta kernel) and it imports
neither the HIP binding nor the oracle, so both sides can take their inputs
from here without sharing any of the computation.

Mesh: the paper resolves the particle interface with a closed triangular mesh
obtained by recursively refining an icosahedron (Sec. "Numerical
implementation", the paragraph introducing the immersed boundary method).  Here
refinement level k splits every triangle into four and projects the new edge
midpoints onto the sphere, giving 10*4^k + 2 vertices and 20*4^k faces.

Perturbation: vertices are displaced by seeded uniform noise drawn from
splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), so that the same numbers can be regenerated from the
published definition anywhere.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

WALLS_Z = 0
PERIODIC_ALL = 1

# LJ zero-force separation 2^(1/6) * xi for xi = 0.5 (wall interaction, Eq. LJ_interaction).
LJ_XI = 0.5
LJ_R0 = 2.0 ** (1.0 / 6.0) * LJ_XI

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """splitmix64 generator (Steele, Lea, Flood 2014), 64-bit state."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


def icosphere(level: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit icosphere: (vertices [N_v,3] float64, faces [N_f,3] int32), outward CCW.

    Vertex order: the 12 icosahedron corners first, then edge midpoints in the
    order they are first created while sweeping faces level by level.
    """
    if level < 0:
        raise ValueError("level must be >= 0")
    p = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0),
             (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
             (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    v = [np.array(x, dtype=np.float64) / np.linalg.norm(x) for x in verts]
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                m = v[a] + v[b]
                v.append(m / np.linalg.norm(m))
                idx = len(v) - 1
                cache[key] = idx
            return idx

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.array(v, dtype=np.float64)
    F = np.array(faces, dtype=np.int32)
    # orient every face outward: (b-a) x (c-a) must point away from the centre
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, a + b + c) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def perturb(vertices: np.ndarray, amplitude: float, seed: int) -> np.ndarray:
    """Add uniform noise in [-amplitude, amplitude) to every coordinate.

    For vertex v and axis a (x, y, z in turn) the draw is
    amplitude * (2u - 1), u = (splitmix64() >> 11) * 2^-53.
    """
    rng = SplitMix64(seed)
    out = np.array(vertices, dtype=np.float64, copy=True)
    flat = out.reshape(-1)
    for k in range(flat.size):
        flat[k] += amplitude * (2.0 * rng.uniform() - 1.0)
    return out


def random_force_field(shape_fluid: tuple[int, int, int], amplitude: float, seed: int) -> np.ndarray:
    """Smooth random body-force density [3, nz_f, ny, nx] for LB-only tests.

    A sum of a few random periodic Fourier modes plus white noise at 10 % of
    the amplitude, drawn from numpy's PCG64 with the given seed.
    """
    nzf, ny, nx = shape_fluid
    g = np.random.Generator(np.random.PCG64(seed))
    z, y, x = np.meshgrid(np.arange(nzf), np.arange(ny), np.arange(nx), indexing="ij")
    F = np.zeros((3, nzf, ny, nx))
    for c in range(3):
        for _ in range(4):
            kx, ky = g.integers(0, 3, size=2)
            kz = g.uniform(0.0, 2.0)
            ph = g.uniform(0, 2 * np.pi, size=3)
            F[c] += (np.cos(2 * np.pi * kx * x / nx + ph[0]) * np.cos(2 * np.pi * ky * y / ny + ph[1])
                     * np.cos(np.pi * kz * z / max(nzf, 1) + ph[2]))
        F[c] += 0.1 * g.standard_normal(F[c].shape)
    F *= amplitude / max(np.abs(F).max(), 1e-300)
    return F


@dataclass
class Domain:
    nx: int
    ny: int
    nz: int
    wall_mode: int = WALLS_Z
    tau: float = 1.0
    rho0: float = 1.0
    u_wall_lo: tuple = (0.0, 0.0, 0.0)
    u_wall_hi: tuple = (0.0, 0.0, 0.0)
    body_force: tuple = (0.0, 0.0, 0.0)
    init_couette: int = 0

    @property
    def nz_fluid(self) -> int:
        return self.nz - 2 if self.wall_mode == WALLS_Z else self.nz

    @property
    def n_fluid(self) -> int:
        return self.nx * self.ny * self.nz_fluid

    @property
    def z_lo(self) -> float:
        """Half-way wall plane between solid layer 0 and fluid layer 1."""
        return 0.5

    @property
    def z_hi(self) -> float:
        return self.nz - 1.5


@dataclass
class Mesh:
    vertices: np.ndarray          # [N_v,3] float64, initial (perturbed) positions
    faces: np.ndarray             # [N_f,3] int32, outward CCW
    ref_vertices: np.ndarray      # [N_v,3] float64, stress-free reference shape
    alpha: tuple = (1e-4, 0.0, 0.0)
    k_v: float = 1.0
    eps_wall_lo: float = 0.0
    eps_wall_hi: float = 0.0
    xi_wall: float = LJ_XI
    r_cut_wall: float = 2.0

    @property
    def n_vertices(self) -> int:
        return int(self.vertices.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.faces.shape[0])


@dataclass
class Workload:
    name: str
    domain: Domain
    mesh: Mesh | None
    steps: int
    precision: str                # "f64" or "f32"
    notes: dict = field(default_factory=dict)


def sphere_mesh(level: int, radius: float, centre, alpha, *, amplitude: float = 0.0,
                seed: int = 230518919, k_v: float = 1.0, eps_lo: float = 0.0,
                eps_hi: float = 0.0, r_cut: float = 2.0) -> Mesh:
    """Icosphere of the given level and radius; reference = the unperturbed sphere."""
    V, F = icosphere(level)
    ref = V * radius + np.asarray(centre, dtype=np.float64)
    q = perturb(ref, amplitude, seed) if amplitude > 0 else ref.copy()
    return Mesh(vertices=q, faces=F, ref_vertices=ref, alpha=tuple(float(a) for a in alpha),
                k_v=k_v, eps_wall_lo=eps_lo, eps_wall_hi=eps_hi, r_cut_wall=r_cut)


ABAR_WETTING = 1e-4           # alpha-bar of the wetting runs (Sec. "Results")
SEED = 230518919


def c1_droplet(eps_over_abar: float = 0.0) -> Workload:
    """32^3 walls, pure droplet abar(1,0,0), level 3 (642/1280), R = 8, FP64, 500 steps.

    With eps = 0 the centre sits one radius above the lower wall plane; with a
    wall interaction it is lifted by the LJ zero-force distance so that no face
    starts on the wall plane.
    """
    abar = ABAR_WETTING
    zc = 0.5 + 8.0 + (LJ_R0 if eps_over_abar > 0 else 0.0)
    mesh = sphere_mesh(3, 8.0, (15.5, 15.5, zc), (abar, 0.0, 0.0), amplitude=0.01,
                       eps_lo=eps_over_abar * abar)
    name = "droplet32_f64" if eps_over_abar == 0 else "droplet32_wall_f64"
    return Workload(name, Domain(32, 32, 32), mesh, 500, "f64")


def shear_capillary(ca: float) -> float:
    """abar for the 64^3 shear case at capillary number ca (Ca = mu R gammadot / alpha1)."""
    mu = 1.0 / 6.0
    gdot = 0.02 / 62.0
    return mu * 10.0 * gdot / ca


def c2_shear(ca: float = 0.05) -> Workload:
    """64^3, walls moving -+0.01 in x, coated capsule abar(1,1,1), level 4, R = 10, FP32 populations."""
    abar = shear_capillary(ca)
    dom = Domain(64, 64, 64, u_wall_lo=(-0.01, 0.0, 0.0), u_wall_hi=(0.01, 0.0, 0.0), init_couette=1)
    mesh = sphere_mesh(4, 10.0, (31.5, 31.5, 31.5), (abar, abar, abar))
    return Workload("shear64_capsule_f32", dom, mesh, 20000, "f32", {"Ca": ca, "abar": abar})


def c3_wetting(eps_over_abar: float = 1.0) -> Workload:
    """128x128x96 walls, softly coated droplet abar(1,0,1), level 5, R = 24, wetting lower wall."""
    abar = ABAR_WETTING
    mesh = sphere_mesh(5, 24.0, (63.5, 63.5, 0.5 + 24.0 + LJ_R0), (abar, 0.0, abar),
                       eps_lo=eps_over_abar * abar)
    return Workload("wetting128_f32", Domain(128, 128, 96), mesh, 1000, "f32",
                    {"eps_over_abar": eps_over_abar})


# Batched parameter sweep: cubic edges, and the three pre-stressed particle
# models of Table 1 (pure droplet, softly and rigidly coated droplet).
BATCH_EDGES = (32, 48, 64, 80)
BATCH_MODELS = ((1.0, 0.0, 0.0), (1.0, 0.0, 1.0), (1.0, 1.0, 1.0))


def batch_sweep(n: int = 48, seed: int = SEED + 5) -> list[Workload]:
    """n independent wetting domains of a parameter sweep, FP32 populations.

    Per domain, drawn from splitmix64 in this order: the cubic edge uniform
    over {32, 48, 64, 80} (walls at z = 0 and edge-1), the radius R uniform in
    [6, 14], the particle model uniform over the three pre-stressed models of
    Table 1, and abar log-uniform in [1e-3, 1e-1].  The droplet is an
    icosphere of level 3 below R = 10 and level 4 from there on, centred in x
    and y and lifted R + 2^(1/6) xi above the lower wall plane, with a wetting
    lower wall of eps = abar.
    """
    rng = SplitMix64(seed)
    out = []
    for k in range(n):
        edge = BATCH_EDGES[min(3, int(rng.uniform() * 4))]
        R = 6.0 + 8.0 * rng.uniform()
        model = BATCH_MODELS[min(2, int(rng.uniform() * 3))]
        abar = 10.0 ** (-3.0 + 2.0 * rng.uniform())
        level = 3 if R < 10.0 else 4
        centre = (edge / 2.0 - 0.5, edge / 2.0 - 0.5, 0.5 + R + LJ_R0)
        mesh = sphere_mesh(level, R, centre, tuple(abar * a for a in model), eps_lo=abar)
        out.append(Workload(f"sweep{k:02d}_e{edge}", Domain(edge, edge, edge), mesh, 5000, "f32",
                            {"edge": edge, "R": R, "model": model, "abar": abar, "level": level}))
    return out


def wetting_case(model=(1.0, 0.0, 0.0), eps_over_abar: float = 1.0, abar: float = 1e-3, kv: float = 1.0,
                 tau: float = 1.0) -> Workload:
    """64x64x48 walls, a droplet alpha = abar * model of radius R = 12 at
    level 4 (2562/5120), lifted R + 2^(1/6) xi above the wetting lower wall
    (eps = eps_over_abar * abar), FP32 populations."""
    mesh = sphere_mesh(4, 12.0, (31.5, 31.5, 0.5 + 12.0 + LJ_R0), tuple(abar * m for m in model), k_v=kv,
                       eps_lo=eps_over_abar * abar)
    return Workload("wetting64x48_f32", Domain(64, 64, 48, tau=tau), mesh, 2000, "f32",
                    {"model": tuple(model), "abar": abar, "kv": kv, "eps": eps_over_abar * abar, "tau": tau})


def differentiation_case(abar: float = 1e-3, kv: float = 1.0, eps_over_abar: float = 1.0,
                         tau: float = 1.0) -> Workload:
    """The run whose final contact radius and height are differentiated: the
    pure droplet abar(1,0,0) of wetting_case, 2000 steps."""
    return wetting_case((1.0, 0.0, 0.0), eps_over_abar, abar, kv, tau)
