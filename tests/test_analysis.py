"""Host-side observables of the wetting campaigns (paper_2305_18919_amd/analysis.py)."""
import math

import numpy as np
import pytest

from paper_2305_18919_amd.analysis import contact_patch_radius, power_law_fit
from paper_2305_18919_amd.inputs import icosphere


def fan(n: int, rho: float, z: float, apex_z: float):
    """A flat regular n-gon of circumradius rho at height z, fanned from its
    centre, closed by a cone to an apex at apex_z: the polygon's area is
    n rho^2 sin(2 pi / n) / 2."""
    ang = 2 * np.pi * np.arange(n) / n
    ring = np.stack([rho * np.cos(ang), rho * np.sin(ang), np.full(n, z)], axis=1)
    q = np.vstack([[0.0, 0.0, z], ring, [0.0, 0.0, apex_z]])
    faces = [(0, 1 + k, 1 + (k + 1) % n) for k in range(n)]
    faces += [(n + 1, 1 + (k + 1) % n, 1 + k) for k in range(n)]
    return q, np.array(faces)


def test_flat_patch_has_the_polygon_area():
    n, rho = 24, 5.0
    q, f = fan(n, rho, 0.5 + 0.3, 0.5 + 10.0)
    r = contact_patch_radius(q, f, z_wall=0.5, band=1.0)
    assert r == pytest.approx(math.sqrt(n * rho * rho * math.sin(2 * math.pi / n) / 2 / math.pi), rel=1e-14)


def test_patch_above_the_band_or_facing_the_other_wall_is_empty():
    q, f = fan(12, 3.0, 0.5 + 1.2, 0.5 + 8.0)
    assert contact_patch_radius(q, f, z_wall=0.5, band=1.0) == 0.0
    # the same fan mirrored under an upper wall at z = 20
    qm = q.copy()
    qm[:, 2] = 20.0 - (q[:, 2] - 0.5)
    assert contact_patch_radius(qm, f, z_wall=20.0, band=1.5, wall=1) == pytest.approx(
        contact_patch_radius(q, f, z_wall=0.5, band=1.5), rel=1e-14)


def test_sphere_tangent_to_the_wall_has_the_cap_radius():
    """A fine icosphere resting at height s on the plane: the patch within
    the band b is close to the spherical cap of depth b - s, radius
    sqrt(2 R (b - s)) (to the mesh's resolution)."""
    v, f = icosphere(6)
    R, s, b = 12.0, 0.1, 1.0
    q = v * R + [0.0, 0.0, 0.5 + s + R]
    r = contact_patch_radius(q, f, z_wall=0.5, band=b)
    cap = math.sqrt(2 * R * (b - s) - (b - s) ** 2)
    assert abs(r - cap) < 0.06 * cap


def test_power_law_recovered_on_the_spreading_window():
    t_star, R = 1314.0, 12.0
    t = np.unique(np.round(np.geomspace(16, 16000, 60)))
    C, delta = 0.9, 0.27
    r = R * C * (t / t_star) ** delta
    r = np.minimum(r, R * C * (4.0) ** delta)  # plateau from t = 4 t*
    fit = power_law_fit(t, r, R, t_star)
    assert fit["delta"] == pytest.approx(delta, rel=1e-12)
    assert fit["C"] == pytest.approx(C, rel=1e-12)
    # from the first sample at t >= 0.2 t* to the first that reaches 90 % of
    # the plateau, r/R = 0.9 C 4^delta at t/t* = 4 * 0.9^(1/delta)
    x = t / t_star
    assert fit["window_t_over_tstar"] == [x[x >= 0.2][0], x[x >= 4.0 * 0.9 ** (1 / delta) * (1 - 1e-12)][0]]


def test_power_law_needs_samples():
    with pytest.raises(ValueError):
        power_law_fit(np.array([1.0, 2.0]), np.array([1.0, 2.0]), 1.0, 1.0)
