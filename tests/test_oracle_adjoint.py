"""Pins of the reference gradients (oracle/adjoint.py).

The PyTorch restatement of the step must follow the C oracle's trajectory,
and its reverse-mode gradients must agree with central finite differences of
the C oracle, which shares no code with it.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle.adjoint import Case, gradients, sphere_fit
from paper_2305_18919_amd.inputs import Domain, sphere_mesh

MODEL = (1.0, 0.5, 1.0)
BASE = dict(abar=2e-3, kv=1.0, eps=2e-3, tau=0.9)
STEPS = 20


def make(abar, kv, eps, tau):
    """An 18x16x16 lattice with moving walls; a perturbed level-2 mesh that
    straddles the x seam and feels the wetting lower wall; every alpha term on."""
    d = Domain(18, 16, 16, tau=tau, u_wall_lo=(0.002, 0, 0), u_wall_hi=(-0.003, 0.001, 0))
    m = sphere_mesh(2, 4.5, (1.3, 8.2, 0.5 + 4.5 + 0.6), tuple(abar * k for k in MODEL), amplitude=0.02, seed=5,
                    eps_lo=eps, k_v=kv)
    return d, m


def oracle_observable(p, which, dq0=None):
    d, m = make(**p)
    if dq0 is not None:
        m.vertices = m.vertices + dq0
    o = O.OracleSim(d, m)
    o.step(STEPS)
    _, _, h, cen, R = O.contact_angle_sphere(o.vertices(), 0.5, 2.0)
    return h if which == "h" else R * R - (cen[2] - 0.5) ** 2


def test_restatement_follows_the_oracle():
    d, m = make(**BASE)
    o = O.OracleSim(d, m)
    o.step(STEPS)
    case = Case(d, m, MODEL)
    t = lambda v: torch.tensor(v, dtype=torch.float64)
    with torch.no_grad():
        f, q = case.run(STEPS, t(BASE["abar"]), t(BASE["kv"]), t(BASE["eps"]), t(BASE["tau"]))
    assert np.abs(q.numpy() - o.vertices()).max() / 4.5 < 1e-13
    fo = o.populations().reshape(19, -1)
    assert np.abs(f.numpy() - fo).max() / np.abs(fo).max() < 1e-12
    fit = sphere_fit(q, 0.5, 2.0)
    _, _, h, cen, R = O.contact_angle_sphere(o.vertices(), 0.5, 2.0)
    assert float(fit["h"]) == pytest.approx(h, rel=1e-12)
    assert float(fit["r2"]) == pytest.approx(R * R - (cen[2] - 0.5) ** 2, rel=1e-10)


@pytest.mark.parametrize("which", ["h", "r2"])
def test_parameter_gradients_match_oracle_finite_differences(which):
    d, m = make(**BASE)
    _, g, _ = gradients(d, m, MODEL, BASE["abar"], BASE["kv"], BASE["eps"], BASE["tau"], STEPS, which)
    for k, name in enumerate(("abar", "kv", "eps", "tau")):
        h = BASE[name] * 1e-4
        pp, pm = dict(BASE), dict(BASE)
        pp[name] += h
        pm[name] -= h
        fd = (oracle_observable(pp, which) - oracle_observable(pm, which)) / (2 * h)
        assert abs(fd - g[k]) <= 2e-6 * abs(g[k]), (which, name, g[k], fd)


def test_initial_position_gradient_matches_directional_difference():
    d, m = make(**BASE)
    _, _, gq = gradients(d, m, MODEL, BASE["abar"], BASE["kv"], BASE["eps"], BASE["tau"], STEPS, "h")
    rng = np.random.default_rng(11)
    for _ in range(2):
        v = rng.standard_normal(gq.shape)
        eps = 1e-5
        fd = (oracle_observable(BASE, "h", eps * v) - oracle_observable(BASE, "h", -eps * v)) / (2 * eps)
        assert abs(fd - (gq * v).sum()) <= 1e-6 * np.abs(gq).sum() * np.abs(v).max()


def test_wall_gradient_vanishes_beyond_the_cutoff():
    """Lifted 3 lattice units: no face centroid comes within r_c = 2 of the
    wall in 20 steps, so the observable cannot depend on eps."""
    d, m = make(**BASE)
    m.vertices = m.vertices + [0.0, 0.0, 3.0]
    m.ref_vertices = m.ref_vertices + [0.0, 0.0, 3.0]
    _, g, _ = gradients(d, m, MODEL, BASE["abar"], BASE["kv"], BASE["eps"], BASE["tau"], STEPS, "h")
    assert g[2] == 0.0 and g[0] != 0.0 and g[3] != 0.0
