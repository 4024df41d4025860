"""iblb_get_fields_noalloc, the allocation-free form of iblb_get_fields,
called through the C ABI: the same fields bit for bit on two calls in a row,
the second on a smaller lattice (stale contents of the shared staging array
would show there), and a clear error above the array's size."""
import ctypes as C

import numpy as np
import pytest

from paper_2305_18919_amd import iblb
from paper_2305_18919_amd.inputs import PERIODIC_ALL, Domain, c3_wetting, sphere_mesh
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

MAX_NODES = 2097152  # IBLB_NOALLOC_MAX_NODES


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def noalloc_fields(sim):
    rho = np.full(sim.shape, np.nan)
    u = np.full((3,) + sim.shape, np.nan)
    rc = iblb.lib().iblb_get_fields_noalloc(sim.h, _p(rho), _p(u))
    return rc, rho, u


def check_same(sim, what):
    rho_a, u_a = sim.fields()  # iblb_get_fields
    rc, rho, u = noalloc_fields(sim)
    assert rc == iblb.IBLB_OK, iblb.lib().iblb_last_error(sim.h)
    announce(f"  {what}: max |u| {np.abs(u).max():.3e}, identical {np.array_equal(u, u_a)}")
    assert np.array_equal(rho, rho_a) and np.array_equal(u, u_a)
    assert np.abs(u).max() > 0.0


def test_noalloc_fields_equal_get_fields_on_two_calls():
    big = c3_wetting(1.0)
    announce("noalloc fields: 128x128x96 wetting, fp32, 5 steps")
    with iblb.Simulation(big.domain, big.mesh, precision=iblb.FP32_DEV) as g:
        g.step(5)
        check_same(g, "first call, 1540096 nodes")
    small = Domain(26, 21, 18, tau=0.9, u_wall_lo=(0.002, 0, 0), u_wall_hi=(-0.003, 0.001, 0))
    mesh = sphere_mesh(2, 4.5, (1.3, 10.2, 5.6), (2e-3, 1e-3, 1e-3), amplitude=0.02, seed=5, eps_lo=2e-3)
    announce("noalloc fields: 26x21x18 ragged, fp64, 3 steps")
    with iblb.Simulation(small, mesh, precision=iblb.FP64) as g:
        g.step(3)
        check_same(g, "second call, smaller lattice")


def test_noalloc_fields_reject_lattices_above_the_limit():
    over = Domain(130, 130, 126, wall_mode=PERIODIC_ALL)
    assert over.n_fluid > MAX_NODES
    announce(f"noalloc fields: {over.n_fluid} nodes, over the limit")
    with iblb.Simulation(over, precision=iblb.FP16_DEV) as g:
        rc, rho, _ = noalloc_fields(g)
        assert rc == iblb.IBLB_E_INVAL
        assert b"IBLB_NOALLOC_MAX_NODES" in iblb.lib().iblb_last_error(g.h)
        assert np.isnan(rho).all()  # nothing written
        g.step(1)  # the context is still usable
        g.sync()
