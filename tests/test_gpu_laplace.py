"""Dynamic Laplace balance on the GPU (the physics check of the oracle's
test_oracle_laplace, at a larger size): a pure droplet at rest, 48^3
periodic, R = 12, level-4 icosphere, after 1000 steps in FP64 and FP32
population storage.  Volume and centroid come from the library's own
queries."""
import numpy as np
import pytest

from paper_2305_18919_amd import iblb
from paper_2305_18919_amd.inputs import PERIODIC_ALL, Domain, sphere_mesh
from tests.gpu_util import announce
from tests.test_oracle_laplace import CS2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [iblb.FP64, iblb.FP32_DEV])
def test_dynamic_laplace_balance_on_gpu(prec):
    N, R, sigma = 48, 12.0, 1e-3
    d = Domain(N, N, N, wall_mode=PERIODIC_ALL)
    m = sphere_mesh(4, R, (N / 2 + 0.1, N / 2 + 0.2, N / 2 + 0.15), (sigma, 0.0, 0.0))
    announce(f"dynamic Laplace prec={prec}")
    with iblb.Simulation(d, m, precision=prec) as g:
        V0, _ = g.volume()
        g.step(1000)
        V, _ = g.volume()
        _, _, xc = g.shape_dtheta()
        rho, _ = g.fields()
    Reff = (3.0 * V / (4.0 * np.pi)) ** (1.0 / 3.0)
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    dd = [(c - xc[k] + N / 2) % N - N / 2 for k, c in enumerate((x, y, z))]
    r = np.sqrt(dd[0] ** 2 + dd[1] ** 2 + dd[2] ** 2)
    jump = CS2 * (rho[r < Reff - 3.0].mean() - rho[r > Reff + 3.0].mean())
    pen = m.k_v * (V0 - V) / V0
    load = 2.0 * sigma / Reff
    announce(f"  jump {jump:.4e} + penalty {pen:.4e} = {jump + pen:.4e} vs 2 sigma / R_eff {load:.4e}")
    assert jump > 0.1 * load and pen > 0.1 * load
    assert jump + pen == pytest.approx(load, rel=0.01)
