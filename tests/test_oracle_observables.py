"""Oracle pins for the query-time observables: contact angle from a sphere
fit (the paper fits a circle cut by the wall chord, appendix on the resolution
test), Taylor deformation and inclination (Eq. taylor_deform), volume
centroid.  Synthetic shapes with known answers fix each routine exactly."""
import numpy as np
import pytest

from paper_2305_18919_amd.inputs import icosphere


@pytest.mark.parametrize("theta", [95.0, 120.0, 157.0, 88.0, 60.0])
@pytest.mark.parametrize("wall_hi", [False, True])
def test_contact_angle_of_exact_cap(O, theta, wall_hi):
    """Vertices of a sphere cut by the wall at angle theta (on the upper wall
    the cap hangs below it): the fit returns theta, the contact radius
    R sin(theta) and the height R (1 - cos(theta)) exactly."""
    R, zw = 11.0, (0.5 if not wall_hi else 60.5)
    V, _ = icosphere(4)
    sgn = -1.0 if wall_hi else 1.0
    zc = zw - sgn * R * np.cos(np.radians(theta))
    p = R * V + np.array([30.0, 31.0, zc])
    p = p[sgn * (p[:, 2] - zw) >= 0.0]
    th, r, h, cen, Rs = O.contact_angle_sphere(p, zw, exclude=2.0, wall_hi=wall_hi)
    # the fit runs in absolute coordinates: near 180 degrees, 60 units from the
    # origin, the normal equations lose a few more digits
    assert th == pytest.approx(theta, abs=1e-9)
    assert Rs == pytest.approx(R, rel=1e-12)
    assert r == pytest.approx(R * np.sin(np.radians(theta)), rel=1e-10)
    assert h == pytest.approx(R * (1 - np.cos(np.radians(theta))), rel=1e-10)


@pytest.mark.parametrize("a,c,psi", [(1.1, 0.9, 0.3), (1.05, 1.0, -0.2), (1.3, 0.8, 0.7854)])
def test_deformation_and_inclination_of_linear_map(O, a, c, psi):
    """x' = A x with A = Rot_y(psi) diag(a,1,c) Rot_y(psi)^T: the icosphere's
    second moment is isotropic (icosahedral symmetry), so D = (a-c)/(a+c) and
    Theta = psi exactly."""
    V, F = icosphere(3)
    Rm = np.array([[np.cos(psi), 0, -np.sin(psi)], [0, 1, 0], [np.sin(psi), 0, np.cos(psi)]])
    A = Rm @ np.diag([a, 1.0, c]) @ Rm.T
    q = (8.0 * V) @ A.T + np.array([20.0, 20.0, 20.0])
    D, th = O.shape_dtheta(q, F)
    assert D == pytest.approx((a - c) / (a + c), rel=1e-12, abs=1e-15)
    assert th == pytest.approx(psi, abs=1e-12)


def test_volume_centroid_translates(O):
    V, F = icosphere(3)
    q = 6.0 * V * np.array([1.0, 0.9, 1.2]) + np.array([3.0, 4.0, 5.0])
    Vol, A, xc = O.volume_area_centroid(q, F)
    assert np.allclose(xc, [3.0, 4.0, 5.0], atol=1e-13)


# Closed meshes with known volume, area and centroid.  The unit cube's twelve
# outward triangles; a tetrahedron with vertices at the origin and on the axes.
CUBE_V = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                   [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], float)
CUBE_F = np.array([[0, 2, 1], [0, 3, 2], [4, 5, 6], [4, 6, 7], [0, 1, 5], [0, 5, 4],
                   [2, 3, 7], [2, 7, 6], [1, 2, 6], [1, 6, 5], [0, 4, 7], [0, 7, 3]], np.int32)
TET_F = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], np.int32)


@pytest.mark.parametrize("dims,shift", [((1.0, 1.0, 1.0), (0, 0, 0)), ((2.0, 0.5, 3.0), (4.0, -2.0, 7.0)),
                                        ((0.3, 1.7, 0.9), (-1.0, 12.5, 0.25))])
def test_volume_area_centroid_of_a_box(O, dims, shift):
    """A box a x b x c: V = abc, A = 2(ab + bc + ca), centroid at its centre.
    A scale error in the signed tetrahedra or in the triangle areas fails."""
    a, b, c = dims
    q = CUBE_V * np.array(dims) + np.array(shift)
    V, A, xc = O.volume_area_centroid(q, CUBE_F)
    assert V == pytest.approx(a * b * c, rel=1e-13)
    assert A == pytest.approx(2 * (a * b + b * c + c * a), rel=1e-13)
    assert np.allclose(xc, np.array(shift) + 0.5 * np.array(dims), rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_volume_area_centroid_of_a_tetrahedron(O, seed):
    """A random tetrahedron (outward faces): V = |det(b-a, c-a, d-a)| / 6, the
    area from Heron's formula on the edge lengths, the centroid the mean of
    the four corners."""
    rng = np.random.default_rng(seed)
    p = rng.normal(size=(4, 3)) * 3.0 + 5.0
    if np.linalg.det(np.array([p[1] - p[0], p[2] - p[0], p[3] - p[0]])) < 0:
        p[[1, 2]] = p[[2, 1]]
    # faces of TET_F point outward for a positively oriented (0, 1, 2, 3)
    vol = np.linalg.det(np.array([p[1] - p[0], p[2] - p[0], p[3] - p[0]])) / 6.0

    def heron(i, j, k):
        la, lb, lc = (np.linalg.norm(p[i] - p[j]), np.linalg.norm(p[j] - p[k]), np.linalg.norm(p[k] - p[i]))
        s = 0.5 * (la + lb + lc)
        return np.sqrt(s * (s - la) * (s - lb) * (s - lc))

    area = sum(heron(*f) for f in TET_F)
    V, A, xc = O.volume_area_centroid(p, TET_F)
    assert V == pytest.approx(vol, rel=1e-12)
    assert A == pytest.approx(area, rel=1e-10)
    assert np.allclose(xc, p.mean(axis=0), rtol=0, atol=1e-12)


def test_volume_area_match_the_force_routine_on_a_deformed_icosphere(O):
    """The query routine (numpy) and the C force routine compute V and A
    independently; they agree on a randomly deformed icosphere."""
    Vt, F = icosphere(3)
    rng = np.random.default_rng(7)
    X = 9.0 * Vt + 20.0
    q = X + rng.uniform(-0.4, 0.4, size=X.shape)
    V, A, _ = O.volume_area_centroid(q, F)
    r = O.mesh_forces(q, X, F, (1.0, 0.0, 0.0))
    assert V == pytest.approx(r["V"], rel=1e-12)
    assert A == pytest.approx(r["A"], rel=1e-12)
    # and both sit near the ball's values for this near-spherical shape
    assert V == pytest.approx(4.0 / 3.0 * np.pi * 9.0 ** 3, rel=0.05)
    assert A == pytest.approx(4.0 * np.pi * 81.0, rel=0.1)  # the perturbation roughens the surface


def _chord_cut_cylinder(R, theta, z_wall=0.5, ny=41, nphi=90, wall_hi=False):
    """Points exactly on a circular cylinder of radius R along y, cut by the
    wall plane z = z_wall at contact angle theta (measured inside the liquid):
    every slice across y projects onto the same circle in (x, z)."""
    zc = z_wall - R * np.cos(np.radians(theta))
    if wall_hi:
        zc = z_wall + R * np.cos(np.radians(theta))
    phi = np.linspace(0.0, 2.0 * np.pi, nphi, endpoint=False)
    pts = []
    for y in np.linspace(5.0, 25.0, ny):
        for f in phi:
            p = (30.0 + R * np.cos(f), y, zc + R * np.sin(f))
            if (p[2] >= z_wall) != wall_hi or p[2] == z_wall:
                pts.append(p)
    return np.array(pts)


@pytest.mark.parametrize("theta", [60.0, 95.0, 140.0])
@pytest.mark.parametrize("wall_hi", [False, True])
def test_slice_contact_angle_of_an_exact_chord_cut_circle(O, theta, wall_hi):
    """Every slice across a chord-cut cylinder lies on one circle, so the slice
    fit returns the angle, contact radius and height exactly.  The slice plane
    comes from the volume centroid of the faces; here the faces are a small
    tetrahedron with its centroid at y = 15, placed inside the excluded band
    next to the wall so that its corners never enter the fit."""
    R, zw = 9.0, (0.5 if not wall_hi else 40.5)
    p = _chord_cut_cylinder(R, theta, zw, wall_hi=wall_hi)
    tet = np.array([[0.0, 15.0, 0.0], [1.0, 15.0, 0.0], [0.0, 16.0, 0.0], [0.0, 15.0, 1.0]])
    tet[:, 1] -= 0.25
    tet[:, 2] += zw - 0.5
    q = np.vstack([tet, p])
    F = TET_F
    th, r, h, cen, Rs = O.contact_angle_slice(q, F, zw, exclude=2.0, wall_hi=wall_hi, K=400)
    assert th == pytest.approx(theta, abs=1e-9)
    assert Rs == pytest.approx(R, rel=1e-11)
    hc = R * np.cos(np.radians(180.0 - theta))
    assert r == pytest.approx(np.sqrt(R * R - hc * hc), rel=1e-9)
    assert h == pytest.approx(hc + R, rel=1e-10)


def test_slice_selects_the_nodes_nearest_the_centroid_plane(O):
    """The slice is the K nodes nearest the plane through the volume centroid,
    ties to the lower index: checked against brute force on a symmetric mesh
    (the unperturbed icosphere has many exact ties)."""
    V, F = icosphere(2)
    q = 7.0 * V + np.array([20.0, 21.0, 9.0])
    _, _, xc = O.volume_area_centroid(q, F)
    d = np.abs(q[:, 1] - xc[1])
    for K in (1, 12, 40, 41, 100, len(q)):
        want = sorted(range(len(q)), key=lambda v: (d[v], v))[:K]
        got = np.lexsort((np.arange(len(q)), d))[:K]
        assert list(got) == want


def test_slice_count_is_nodes_within_two_edges_of_the_midplane():
    """(4 / 3^(1/4)) sqrt(pi N_f) = N_v (2a) / R for N_v = N_f / 2 nodes on a
    sphere of radius R triangulated with equilateral faces of side a:
    the number of nodes within two edge lengths of a mid-plane."""
    from oracle import oracle as Ox
    for nf in (1280, 5120, 16820, 20480, 42320):
        R = 1.0
        a = np.sqrt(4.0 * np.pi * R * R / nf * 4.0 / np.sqrt(3.0))
        assert Ox.slice_count(nf) == round((nf / 2) * (2 * a) / R)
    assert Ox.slice_count(16820) == 699
