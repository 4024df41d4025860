"""Oracle pins for the lattice, the equilibrium (Eq. feq) and the Guo source (Eq. LBeq).

These check the oracle against what the mathematics fixes: lattice isotropy,
the hydrodynamic moments of the equilibrium, and the moments of the Guo
forcing term.  A wrong weight, a wrong velocity, the printed 2 c_s^2
denominator of Eq. feq or a wrong sign in the Guo term each fails one of them.
"""
import json
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_weights_match_paper_footnote(O):
    c, w, opp = O.lattice()
    g = GOLD["d3q19_weights"]
    speed2 = (c * c).sum(1)
    assert w[speed2 == 0] == pytest.approx([g["rest"]], abs=1e-17)
    assert (speed2 == 1).sum() == g["axis_count"] and np.allclose(w[speed2 == 1], g["axis"], atol=1e-17)
    assert (speed2 == 2).sum() == g["diagonal_count"] and np.allclose(w[speed2 == 2], g["diagonal"], atol=1e-17)
    # index ranges of the footnote: 0 rest, 1..6 axis, 7..18 diagonal
    assert speed2[0] == 0 and (speed2[1:7] == 1).all() and (speed2[7:] == 2).all()


def test_lattice_isotropy(O):
    c, w, opp = O.lattice()
    cs2 = GOLD["cs2"]["value"]
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs((w[:, None] * c).sum(0)).max() < 1e-16
    assert np.allclose(np.einsum("i,ij,ik->jk", w, c, c), cs2 * np.eye(3), atol=1e-16)
    third = np.einsum("i,ij,ik,il->jkl", w, c, c, c)
    assert np.abs(third).max() < 1e-16
    four = np.einsum("i,ij,ik,il,im->jklm", w, c, c, c, c)
    d = np.eye(3)
    iso = cs2 ** 2 * (np.einsum("jk,lm->jklm", d, d) + np.einsum("jl,km->jklm", d, d)
                      + np.einsum("jm,kl->jklm", d, d))
    assert np.allclose(four, iso, atol=1e-16)
    for i in range(19):
        assert (c[opp[i]] == -c[i]).all()


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(O, seed):
    """sum f = rho, sum c f = rho u, sum cc f = rho c_s^2 I + rho u u (pins 2 c_s^4)."""
    g = np.random.default_rng(seed)
    rho = 1.0 + 0.1 * g.standard_normal()
    u = 0.05 * g.standard_normal(3)
    c, w, _ = O.lattice()
    f = O.feq(rho, u)
    assert f.sum() == pytest.approx(rho, rel=1e-15)
    assert np.allclose((c * f[:, None]).sum(0), rho * u, rtol=1e-14, atol=1e-17)
    P = np.einsum("i,ij,ik->jk", f, c, c)
    assert np.allclose(P, rho / 3 * np.eye(3) + rho * np.outer(u, u), rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_deviation_form_is_exact(O, seed):
    """f^eq - w rho0 as computed from small terms equals the printed form minus w rho0."""
    g = np.random.default_rng(100 + seed)
    rho0, drho = 1.0, 1e-3 * g.standard_normal()
    u = 0.03 * g.standard_normal(3)
    _, w, _ = O.lattice()
    full = O.feq(rho0 + drho, u)
    dev = O.feq_dev(rho0, drho, u)
    assert np.allclose(dev + w * rho0, full, rtol=0, atol=2e-16)
    # and the deviation itself has the right moments without cancellation
    c, _, _ = O.lattice()
    assert dev.sum() == pytest.approx(drho, rel=1e-13)
    assert np.allclose((c * dev[:, None]).sum(0), (rho0 + drho) * u, rtol=1e-13)


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_guo_moments(O, tau):
    """sum S = 0, sum c S = (1 - 1/2tau) F, sum cc S = (1 - 1/2tau)(uF + Fu)."""
    g = np.random.default_rng(7)
    u = 0.05 * g.standard_normal(3)
    F = 1e-3 * g.standard_normal(3)
    c, _, _ = O.lattice()
    S = O.guo(tau, u, F)
    k = 1 - 1 / (2 * tau)
    assert abs(S.sum()) < 1e-18
    assert np.allclose((c * S[:, None]).sum(0), k * F, rtol=1e-13, atol=1e-20)
    P = np.einsum("i,ij,il->jl", S, c, c)
    assert np.allclose(P, k * (np.outer(u, F) + np.outer(F, u)), rtol=1e-12, atol=1e-13 * np.abs(P).max())


def test_guo_vanishes_at_tau_half(O):
    assert np.abs(O.guo(0.5, [0.01, 0.0, 0.02], [1e-3, 2e-3, -1e-3])).max() == 0.0
