"""Dynamic Laplace balance of a pure droplet at rest (alpha = sigma (1, 0, 0),
the pre-stressed model of the Interface model section; no wall force):
the membrane load 2 sigma / R_eff is carried by the fluid's pressure jump
c_s^2 (rho_in - rho_out) and the volume penalty k_V (V0 - V) / V0 of Eq.
nodal_force_V together, with R_eff = (3 V / 4 pi)^(1/3).  A dropped term
(the penalty, which carries most of the load here, or the pressure jump) or
a wrong sign of the tension misses by far more than the tolerance."""
import numpy as np
import pytest

from paper_2305_18919_amd.inputs import PERIODIC_ALL, Domain, sphere_mesh

CS2 = 1.0 / 3.0


def laplace_terms(rho, q, faces, V0, k_v, sigma, vol):
    """(pressure-jump term, penalty term, 2 sigma / R_eff): densities averaged
    over the nodes more than three lattice units inside and outside the
    volume-equivalent sphere (clear of the 4-point stencil's smearing)."""
    V, _, xc = vol(q, faces)
    Reff = (3.0 * V / (4.0 * np.pi)) ** (1.0 / 3.0)
    nz, ny, nx = rho.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = [(c - xc[k] + n / 2) % n - n / 2 for k, (c, n) in enumerate(((x, nx), (y, ny), (z, nz)))]
    r = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
    jump = CS2 * (rho[r < Reff - 3.0].mean() - rho[r > Reff + 3.0].mean())
    return jump, k_v * (V0 - V) / V0, 2.0 * sigma / Reff


@pytest.mark.parametrize("R,sigma", [(8.0, 1e-3), (6.5, 2e-3)])
def test_dynamic_laplace_balance(O, R, sigma):
    N = 32
    d = Domain(N, N, N, wall_mode=PERIODIC_ALL)
    m = sphere_mesh(3, R, (N / 2 + 0.1, N / 2 + 0.2, N / 2 + 0.15), (sigma, 0.0, 0.0))
    V0, _, _ = O.volume_area_centroid(m.ref_vertices, m.faces)
    o = O.OracleSim(d, m)
    o.step(500)
    rho, _ = o.fields()
    jump, pen, load = laplace_terms(rho, o.vertices(), m.faces, V0, m.k_v, sigma, O.volume_area_centroid)
    assert jump > 0.1 * load and pen > 0.1 * load  # both carry a share
    assert jump + pen == pytest.approx(load, rel=0.01)
