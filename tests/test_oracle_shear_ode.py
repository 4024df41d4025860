"""Pins of the oracle's small-deformation shear dynamics (Eqs. evJK, L_M,
deformation_J) against closed forms the paper prints: the steady deformation
of Eq. deformation for the coated particles of Table 1, Eq.
deformation_droplet (35/32 Ca at viscosity ratio 1) and the Chaffey-Brenner
inclination of Eq. inclination_angle (pi/4 - 35/32 Ca) for the pure droplet,
and, for the pure droplet, the exponential approach to the steady state that
the equations reduce to when the rotation terms are negligible (small Ca):
D(t) = D_ss (1 - exp(-k t)), k = 40 (lam + 1) a1 / ((2 lam + 3)(19 lam + 16))
(16/35 a1 at lam = 1)."""
import math

import numpy as np
import pytest

CA = 1e-4


def eq_deformation(shape):
    """Eq. deformation, written in a_k = alpha_k / (mu R gammadot) with the
    moduli of `shape` in units of alpha and Ca = 1 (the alpha_1 of the
    printed form cancels)."""
    a1, a2, a3 = shape
    return 5.0 * (3 * a2 + 4 * a3) / (4.0 * (3 * a1 * a2 + 5 * a1 * a3 + 2 * a2 * a3 + 2 * a3 * a3))


def steady(O, shape, ca=CA):
    a = tuple(s / ca for s in shape)
    return O.shear_deformation_ode(a, 100.0 * ca, 8000)


def test_pure_droplet_steady_deformation_and_inclination(O):
    r = steady(O, (1.0, 0.0, 0.0))
    D, th = r["D"][-1], r["Theta"][-1]
    assert D / CA == pytest.approx(35.0 / 32.0, rel=1e-4)               # Eq. deformation_droplet
    assert (math.pi / 4 - th) / CA == pytest.approx(35.0 / 32.0, rel=1e-3)  # Eq. inclination_angle
    assert th < math.pi / 4  # the flow turns the shape toward its direction


@pytest.mark.parametrize("shape", [(1.0, 0.0, 1.0), (1.0, 1.0, 1.0), (0.0, 0.0, 1.0), (0.0, 1.0, 1.0)])
def test_coated_and_capsule_steady_deformation(O, shape):
    """Eq. deformation for the softly and rigidly coated droplets and both
    non-pre-stressed capsules of Table 1 (alpha_3 > 0 in all of them)."""
    r = steady(O, shape)
    assert r["D"][-1] / CA == pytest.approx(eq_deformation(shape), rel=2e-4)
    assert r["Theta"][-1] < math.pi / 4


def test_pure_droplet_transient_is_exponential(O):
    a1 = 1.0 / CA
    k = 16.0 / 35.0 * a1
    r = O.shear_deformation_ode((a1, 0.0, 0.0), 8.0 / k, 16000, n_samples=64)
    D_ss = 35.0 / 32.0 * CA
    t, D = r["t"], r["D"]
    sel = (t * k > 0.25)
    assert np.allclose(D[sel], D_ss * (1.0 - np.exp(-k * t[sel])), rtol=2e-3, atol=0)


def test_tensors_stay_symmetric_traceless_and_in_the_shear_plane(O):
    r = O.shear_deformation_ode((20.0, 10.0, 20.0), 3.0, 6000)
    for A in (r["J"], r["K"]):
        s = np.abs(A).max()
        assert np.allclose(A, A.T, atol=1e-14 * s)
        assert abs(np.trace(A)) <= 1e-13 * s
        assert abs(A[0, 1]) + abs(A[1, 2]) <= 1e-14 * s


def test_time_step_converges(O):
    a = (1.0 / 0.05, 1.0 / 0.05, 1.0 / 0.05)
    r1 = O.shear_deformation_ode(a, 2.0, 2000)
    r2 = O.shear_deformation_ode(a, 2.0, 4000)
    assert abs(r1["D"][-1] - r2["D"][-1]) <= 1e-8 * r2["D"][-1]
