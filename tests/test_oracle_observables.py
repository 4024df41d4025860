"""Oracle pins for the query-time observables: contact angle from a sphere
fit (the paper fits a circle cut by the wall chord, appendix on the resolution
test), Taylor deformation and inclination (Eq. taylor_deform), volume
centroid.  Synthetic shapes with known answers fix each routine exactly."""
import numpy as np
import pytest

from paper_2305_18919_amd.inputs import icosphere


@pytest.mark.parametrize("theta", [95.0, 120.0, 157.0, 88.0, 60.0])
def test_contact_angle_of_exact_cap(O, theta):
    R, zw = 11.0, 0.5
    V, _ = icosphere(4)
    zc = zw - R * np.cos(np.radians(theta))
    p = R * V + np.array([30.0, 31.0, zc])
    p = p[p[:, 2] >= zw]
    th, r, h, cen, Rs = O.contact_angle_sphere(p, zw, exclude=2.0)
    assert th == pytest.approx(theta, abs=1e-10)
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
