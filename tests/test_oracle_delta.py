"""Oracle pins for the 4-point stencil (Eq. ibm-interpolation_stencil) and for
spreading / interpolation (Eqs. ibm-governing_eq1, ibm-governing_eq2).

phi4 is fixed by Peskin's moment conditions, which hold for every shift; the
two delta-kernel operations are fixed by partition of unity, exact
interpolation of linear fields and by being transposes of each other.
"""
import numpy as np
import pytest


def test_phi4_values(O):
    # closed-form values of the two branches at 0, 1/2, 1, 3/2, 2
    assert O.phi4(0.0) == 0.5
    assert O.phi4(1.0) == 0.25
    assert O.phi4(2.0) == 0.0
    assert O.phi4(2.5) == 0.0
    assert O.phi4(0.5) == pytest.approx((2 + np.sqrt(2)) / 8, abs=1e-16)
    assert O.phi4(1.5) == pytest.approx((2 - np.sqrt(2)) / 8, abs=1e-16)
    assert O.phi4(-0.7) == O.phi4(0.7)


@pytest.mark.parametrize("q", [0.0, 0.125, 0.3, 0.5, 0.77, 0.999999])
def test_peskin_identities(O, q):
    k = np.arange(-4, 6)
    w = np.array([O.phi4(kk - q) for kk in k])
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert ((k - q) * w).sum() == pytest.approx(0.0, abs=1e-15)
    assert (w * w).sum() == pytest.approx(3.0 / 8.0, abs=1e-15)
    assert w[k % 2 == 0].sum() == pytest.approx(0.5, abs=1e-15)
    assert w[k % 2 == 1].sum() == pytest.approx(0.5, abs=1e-15)
    assert (w > 0).sum() <= 4


def test_phi4_continuous_and_c1(O):
    h = 1e-7
    for r in (1.0, 2.0):
        assert abs(O.phi4(r - 1e-12) - O.phi4(r + 1e-12)) < 1e-11
        left = (O.phi4(r - h) - O.phi4(r - 2 * h)) / h
        right = (O.phi4(r + 2 * h) - O.phi4(r + h)) / h
        assert abs(left - right) < 1e-5


def _rand_vertices(g, n, lo, hi):
    return g.uniform(lo, hi, size=(n, 3))


def test_spread_partition_of_unity_periodic(O):
    g = np.random.default_rng(1)
    nx, ny, nz = 11, 9, 10
    q = _rand_vertices(g, 40, -3.0, 13.0)
    phi = g.standard_normal((40, 3))
    F = O.spread(nx, ny, nz, False, q, phi)
    assert np.allclose(F.reshape(3, -1).sum(1), phi.sum(0), rtol=1e-13, atol=1e-13)


def test_spread_interp_are_transposes(O):
    """sum_x F(x).u(x) == sum_i phi_i . qdot_i for any phi and u (periodic)."""
    g = np.random.default_rng(2)
    nx, ny, nz = 12, 10, 9
    q = _rand_vertices(g, 60, 0.0, 12.0)
    phi = g.standard_normal((60, 3))
    u = g.standard_normal((3, nz, ny, nx))
    F = O.spread(nx, ny, nz, False, q, phi)
    qd = O.interp(nx, ny, nz, False, q, u)
    lhs = (F * u).sum()
    rhs = (phi * qd).sum()
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_spread_interp_transposes_with_walls(O):
    """With walls the dropped nodes carry zero force, and interpolation with
    zero wall velocity sees zero there: the identity still holds."""
    g = np.random.default_rng(3)
    nx, ny, nz = 10, 10, 12
    q = _rand_vertices(g, 50, 0.0, 10.0)
    q[:, 2] = g.uniform(-0.5, 12.0, size=50)
    phi = g.standard_normal((50, 3))
    u = g.standard_normal((3, nz - 2, ny, nx))
    F = O.spread(nx, ny, nz, True, q, phi)
    qd = O.interp(nx, ny, nz, True, q, u)
    assert (F * u).sum() == pytest.approx((phi * qd).sum(), rel=1e-13)


def test_interp_linear_field_exact(O):
    """u = a + B x is interpolated exactly away from the periodic seam."""
    g = np.random.default_rng(4)
    nx = ny = nz = 16
    a = g.standard_normal(3)
    B = g.standard_normal((3, 3))
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = np.stack([x, y, z])
    u = a[:, None, None, None] + np.einsum("kj,jzyx->kzyx", B, X)
    q = _rand_vertices(g, 30, 3.0, 12.0)
    qd = O.interp(nx, ny, nz, False, q, u)
    assert np.allclose(qd, a + q @ B.T, rtol=1e-13, atol=1e-13)


def test_interp_wall_velocity(O):
    """A field equal to the wall velocities everywhere comes back exactly, also
    for vertices whose stencil reaches into the walls."""
    nx, ny, nz = 10, 10, 12
    ulo = np.array([0.01, -0.02, 0.0])
    u = np.broadcast_to(ulo[:, None, None, None], (3, nz - 2, ny, nx)).copy()
    q = np.array([[3.3, 4.7, 0.6], [5.1, 2.2, 1.2], [7.0, 7.0, 5.5], [1.5, 8.5, 10.9]])
    qd = O.interp(nx, ny, nz, True, q, u, ulo, ulo)
    assert np.allclose(qd, ulo, atol=1e-16)


def test_spread_drops_nodes_outside_fluid(O):
    nx, ny, nz = 10, 10, 12
    q = np.array([[4.2, 5.5, 0.8]])
    phi = np.array([[1.0, 2.0, 3.0]])
    F = O.spread(nx, ny, nz, True, q, phi)
    # share of the nodes z = 1, 2 only (z = -1, 0 are not fluid)
    wz = sum(O.phi4(z - 0.8) for z in (1, 2))
    assert np.allclose(F.reshape(3, -1).sum(1), phi[0] * wz, rtol=1e-13)
