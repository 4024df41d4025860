"""Oracle pins for the interface forces: elastic (Eqs. generalised_energy1 and
nodal_force_S), volume penalty (Eq. nodal_force_V) and wall interaction
(Eq. LJ_interaction).

The elastic energy is recomputed here by a different route: the in-plane
deformation gradient of each triangle and the eigenvalues of its right
Cauchy-Green tensor (principal stretches), which is how the strain invariants
are defined.  The oracle's closed-form nodal forces must be minus the finite
difference gradient of that energy.  Further pins are exact identities:
translation and rotation invariance, the isotropic pre-stress alpha1 at rest,
the Laplace virial of a sphere, exact polyhedron volumes and Euler's theorem
for the degree-3 homogeneous volume.
"""
import numpy as np
import pytest

from paper_2305_18919_amd.inputs import icosphere

ALPHAS = [(1.0, 0.0, 0.0), (1.0, 0.0, 1.0), (1.0, 1.0, 1.0), (0.0, 0.0, 1.0), (0.0, 1.0, 1.0),
          (0.3, 2.0, 0.7)]


def _invariants_by_stretches(q, X, faces):
    I1 = np.zeros(len(faces))
    I2 = np.zeros(len(faces))
    A0 = np.zeros(len(faces))
    for j, (a, b, c) in enumerate(faces):
        E1, E2 = X[b] - X[a], X[c] - X[a]
        e1, e2 = q[b] - q[a], q[c] - q[a]

        def local(v1, v2):
            t1 = v1 / np.linalg.norm(v1)
            t2 = v2 - (v2 @ t1) * t1
            t2 /= np.linalg.norm(t2)
            return np.array([[v1 @ t1, v2 @ t1], [v1 @ t2, v2 @ t2]])

        P, p = local(E1, E2), local(e1, e2)
        Fd = p @ np.linalg.inv(P)
        lam2 = np.linalg.eigvalsh(Fd.T @ Fd)
        I1[j] = lam2.sum() - 2.0
        I2[j] = lam2.prod() - 1.0
        A0[j] = 0.5 * np.linalg.norm(np.cross(E1, E2))
    return I1, I2, A0


def energy_by_stretches(q, X, faces, alpha):
    a1, a2, a3 = alpha
    I1, I2, A0 = _invariants_by_stretches(q, X, faces)
    L = np.log(I2 + 1.0)
    wS = 0.5 * (a1 - a3) * L + 0.125 * (a1 + a2) * L * L + a3 * (0.5 * (I1 + 2.0) - 1.0)
    return (A0 * wS).sum()


def _deformed(level=1, seed=0, amp=0.08):
    V, F = icosphere(level)
    X = 3.0 * V + np.array([1.0, -2.0, 0.5])
    g = np.random.default_rng(seed)
    A = np.eye(3) + 0.1 * g.standard_normal((3, 3))
    q = (X - X.mean(0)) @ A.T + X.mean(0) + amp * g.standard_normal(X.shape)
    return q, X, F


@pytest.mark.parametrize("alpha", ALPHAS)
def test_energy_matches_principal_stretches(O, alpha):
    q, X, F = _deformed()
    r = O.mesh_forces(q, X, F, alpha)
    assert r["W"] == pytest.approx(energy_by_stretches(q, X, F, alpha), rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("alpha", ALPHAS)
def test_elastic_force_is_minus_energy_gradient(O, alpha):
    q, X, F = _deformed(seed=1)
    phiS = O.mesh_forces(q, X, F, alpha)["phiS"]
    h = 1e-6
    grad = np.zeros_like(q)
    for i in range(q.shape[0]):
        for k in range(3):
            qp, qm = q.copy(), q.copy()
            qp[i, k] += h
            qm[i, k] -= h
            grad[i, k] = (energy_by_stretches(qp, X, F, alpha) - energy_by_stretches(qm, X, F, alpha)) / (2 * h)
    scale = np.abs(grad).max()
    assert np.abs(phiS + grad).max() < 1e-7 * scale


@pytest.mark.parametrize("alpha", ALPHAS)
def test_elastic_force_translation_rotation_invariance(O, alpha):
    q, X, F = _deformed(level=2, seed=2)
    phiS = O.mesh_forces(q, X, F, alpha)["phiS"]
    scale = np.abs(phiS).max()
    assert np.abs(phiS.sum(0)).max() < 1e-13 * scale * len(q)
    assert np.abs(np.cross(q, phiS).sum(0)).max() < 1e-12 * scale * len(q)


def _area_gradient(q, F):
    """dA/dq per vertex for A = sum of triangle areas: dA_j/da = n x (c - b) / 2, cyclic."""
    g = np.zeros_like(q)
    for a, b, c in F:
        n = np.cross(q[b] - q[a], q[c] - q[a])
        n /= np.linalg.norm(n)
        g[a] += 0.5 * np.cross(n, q[c] - q[b])
        g[b] += 0.5 * np.cross(n, q[a] - q[c])
        g[c] += 0.5 * np.cross(n, q[b] - q[a])
    return g


@pytest.mark.parametrize("alpha", ALPHAS)
def test_prestress_at_rest_is_alpha1(O, alpha):
    """In the reference shape every model carries the isotropic tension alpha1:
    phi^S = -alpha1 dA/dq (alpha1 = 0 gives no force)."""
    V, F = icosphere(2)
    X = 5.0 * V
    phiS = O.mesh_forces(X, X, F, alpha)["phiS"]
    assert np.allclose(phiS, -alpha[0] * _area_gradient(X, F), rtol=1e-12, atol=1e-14)


def test_pure_droplet_tension(O):
    """alpha = (s,0,0): W_j = A0 [s ln(A/A0) + s/2 ln^2(A/A0)], so
    phi^S = -sum_j s (A0/A)(1 + ln(A/A0)) dA_j/dq."""
    s = 0.7
    q, X, F = _deformed(seed=3)
    phiS = O.mesh_forces(q, X, F, (s, 0.0, 0.0))["phiS"]
    expect = np.zeros_like(q)
    for a, b, c in F:
        A0 = 0.5 * np.linalg.norm(np.cross(X[b] - X[a], X[c] - X[a]))
        n = np.cross(q[b] - q[a], q[c] - q[a])
        A = 0.5 * np.linalg.norm(n)
        n /= 2 * A
        k = -s * (A0 / A) * (1.0 + np.log(A / A0))
        expect[a] += k * 0.5 * np.cross(n, q[c] - q[b])
        expect[b] += k * 0.5 * np.cross(n, q[a] - q[c])
        expect[c] += k * 0.5 * np.cross(n, q[b] - q[a])
    assert np.allclose(phiS, expect, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("level", [2, 3])
def test_static_laplace_virial(O, level):
    """Unperturbed icosphere, any alpha1: sum_i n_i.phi^S_i / A = -2 alpha1 / R."""
    R, sig = 7.0, 2e-3
    V, F = icosphere(level)
    X = R * V + 10.0
    r = O.mesh_forces(X, X, F, (sig, 0.3, 0.1))
    n = (X - 10.0) / R
    assert (n * r["phiS"]).sum() / r["A"] == pytest.approx(-2 * sig / R, rel=1e-12)


CUBE_V = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], float)
CUBE_F = np.array([[0, 2, 1], [0, 3, 2], [4, 5, 6], [4, 6, 7], [0, 1, 5], [0, 5, 4],
                   [1, 2, 6], [1, 6, 5], [2, 3, 7], [2, 7, 6], [3, 0, 4], [3, 4, 7]], np.int32)
TET_V = np.array([[0, 0, 0], [2, 0, 0], [0, 3, 0], [0, 0, 4]], float)
TET_F = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], np.int32)


@pytest.mark.parametrize("s,shift", [(1.0, (0, 0, 0)), (2.5, (3.0, -1.0, 7.0)), (0.3, (2.0, 1.5, -1.0))])
def test_polyhedron_volumes_exact(O, s, shift):
    q = CUBE_V * s + np.array(shift)
    r = O.mesh_forces(q, CUBE_V, CUBE_F, (1.0, 0, 0))
    assert r["V"] == pytest.approx(s ** 3, rel=1e-12)
    assert r["V0"] == pytest.approx(1.0, rel=1e-14)
    assert r["dV"] == pytest.approx(s ** 3 - 1.0, rel=1e-13, abs=1e-14)
    assert r["A"] == pytest.approx(6 * s * s, rel=1e-14)
    t = O.mesh_forces(TET_V * s + np.array(shift), TET_V, TET_F, (1.0, 0, 0))
    assert t["V"] == pytest.approx(4.0 * s ** 3, rel=1e-14)


def test_volume_gradient(O):
    """phi^V = -kv (V-V0)/V0 dV/dq; dV/dq sums to zero, obeys Euler (degree 3)
    and equals the finite-difference gradient of the exact volume."""
    q, X, F = _deformed(level=2, seed=4)
    r = O.mesh_forces(q, X, F, (1.0, 0, 0), kv=1.0)
    gV = -r["phiV"] * r["V0"] / r["dV"]
    assert np.abs(gV.sum(0)).max() < 1e-12 * np.abs(gV).max() * len(q)
    assert (q * gV).sum() == pytest.approx(3 * r["V"], rel=1e-12)

    def vol(p):
        a, b, c = p[F[:, 0]], p[F[:, 1]], p[F[:, 2]]
        return np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0

    assert r["V"] == pytest.approx(vol(q), rel=1e-13)
    h = 1e-6
    fd = np.zeros_like(q)
    for i in range(len(q)):
        for k in range(3):
            qp, qm = q.copy(), q.copy()
            qp[i, k] += h
            qm[i, k] -= h
            fd[i, k] = (vol(qp) - vol(qm)) / (2 * h)
    assert np.abs(fd - gV).max() < 1e-7 * np.abs(gV).max()
    assert r["dV"] == pytest.approx(r["V"] - r["V0"], rel=1e-10)


def test_icosphere_volume_converges_to_ball(O):
    R = 4.0
    vols = []
    for k in range(1, 6):
        V, F = icosphere(k)
        vols.append(O.mesh_forces(R * V, R * V, F, (1.0, 0, 0))["V"])
    ball = 4.0 / 3.0 * np.pi * R ** 3
    assert all(v < ball for v in vols)
    assert all(b > a for a, b in zip(vols, vols[1:]))
    assert ball - vols[-1] < 2e-3 * ball


def test_lj_formula(O):
    xi, eps, rc = 0.5, 2e-4, 2.0
    for d in (0.3, 0.5, 0.6, 0.9, 1.5, 1.99):
        s = xi / d
        assert O.lj(eps, xi, rc, d) == pytest.approx(48 * eps * (s ** 12 - 0.5 * s ** 6) / d, rel=1e-15)
    r0 = 2 ** (1 / 6) * xi
    assert abs(O.lj(eps, xi, rc, r0)) < 1e-18
    assert O.lj(eps, xi, rc, r0 - 0.01) > 0 > O.lj(eps, xi, rc, r0 + 0.01)
    assert O.lj(eps, xi, rc, 2.0) == 0.0 and O.lj(eps, xi, rc, 2.5) == 0.0
    assert O.lj(0.0, xi, rc, 0.6) == 0.0
    assert O.lj(eps, xi, rc, 0.1) == O.lj(eps, xi, rc, 0.25)  # clamp at xi/2


def test_wall_force_one_third_per_vertex(O):
    """A flat triangle parallel to the lower wall: each vertex gets F/3 along +z,
    and the upper wall pushes down with the same law."""
    X = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    F = np.array([[0, 1, 2]], np.int32)
    z_lo, z_hi, eps, xi, rc = 0.5, 20.5, 1e-3, 0.5, 2.0
    d = 0.6
    q = X + np.array([0, 0, z_lo + d])
    r = O.mesh_forces(q, X, F, (0, 0, 0), kv=0.0, walls=True, z_lo=z_lo, z_hi=z_hi, eps_lo=eps, xi=xi, r_cut=rc)
    f = O.lj(eps, xi, rc, d)
    assert np.allclose(r["phiW"], [[0, 0, f / 3]] * 3, rtol=1e-15)
    q2 = X + np.array([0, 0, z_hi - d])
    r2 = O.mesh_forces(q2, X, F, (0, 0, 0), kv=0.0, walls=True, z_lo=z_lo, z_hi=z_hi, eps_hi=eps, xi=xi, r_cut=rc)
    assert np.allclose(r2["phiW"], [[0, 0, -f / 3]] * 3, rtol=1e-15)
