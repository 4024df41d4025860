"""Oracle pins for the coupled IB-LB step (the enumerated algorithm in the
Numerical implementation section).  No closed form exists for the coupled
trajectory; these are the invariants it must keep:

* internal interface forces (elastic + volume) sum to zero, and spreading
  preserves the sum, so in a fully periodic box the fluid momentum stays at
  its initial value;
* total fluid mass is conserved with walls;
* a mesh at rest in a fluid at rest, in its reference shape with alpha1 = 0
  and no wall force, feels no force and does not move;
* a uniform fluid velocity carries every vertex with it exactly (partition of
  unity of the interpolation).
"""
import numpy as np
import pytest

from paper_2305_18919_amd.inputs import PERIODIC_ALL, Domain, sphere_mesh


def test_fluid_momentum_conserved_periodic(O):
    d = Domain(20, 20, 20, wall_mode=PERIODIC_ALL)
    m = sphere_mesh(2, 5.0, (10.2, 9.7, 10.4), (1e-3, 0.0, 1e-3), amplitude=0.05, seed=11)
    s = O.OracleSim(d, m)
    c, _, _ = O.lattice()
    s.step(40)
    p = np.einsum("ia,izyx->a", c, s.populations())
    phi = s.nodal_forces()
    assert np.abs(phi.sum(0)).max() < 1e-14 * np.abs(phi).max() * len(phi)
    assert np.abs(p).max() < 1e-15 * d.n_fluid * np.abs(phi).max()


def test_mass_conserved_coupled_with_walls(O):
    d = Domain(16, 16, 18, u_wall_lo=(-0.005, 0, 0), u_wall_hi=(0.005, 0, 0))
    m = sphere_mesh(2, 4.5, (7.5, 8.0, 8.5), (1e-3, 1e-3, 1e-3), amplitude=0.02, seed=12)
    s = O.OracleSim(d, m)
    s.step(60)
    assert abs(s.populations().sum()) < 1e-13 * d.n_fluid


def test_reference_capsule_at_rest_stays(O):
    d = Domain(16, 16, 16)
    m = sphere_mesh(2, 4.0, (8.0, 8.0, 8.0), (0.0, 1e-3, 1e-3))
    s = O.OracleSim(d, m)
    s.step(20)
    assert np.abs(s.nodal_forces()).max() < 1e-17
    assert np.abs(s.vertices() - m.vertices).max() == 0.0
    assert np.abs(s.populations()).max() < 1e-18


def test_uniform_flow_advects_mesh(O):
    """Periodic box, uniform velocity U, capsule with no forces: q moves by U per step."""
    d = Domain(16, 16, 16, wall_mode=PERIODIC_ALL)
    U = np.array([0.01, -0.004, 0.002])
    m = sphere_mesh(2, 3.0, (8.0, 8.0, 8.0), (0.0, 0.0, 0.0))
    s = O.OracleSim(d, m)
    dev = O.feq_dev(1.0, 0.0, U)
    s.set_populations(np.broadcast_to(dev[:, None, None, None], (19, 16, 16, 16)).copy())
    s.step(5)
    assert np.allclose(s.vertices(), m.vertices + 5 * U, rtol=0, atol=1e-13)
