"""The shear runs against the small-deformation theory (Interface model
section): D(t) of a particle on the 64^3 shear workload (walls at -+0.01,
R = 10, level-4 icosphere, Couette start, FP32 storage, captured graphs),
sampled every 0.1 shear times up to gammadot t = 3, against the oracle's
integration of Eqs. evJK and L_M from the same start.

This is a model check, not parity.  The theory is the Stokes limit of small
deformations: it has no time for the flow to adjust around the particle
(R^2 / nu = 600 steps, about 0.2 shear times here), and a 10-unit sphere of
5120 faces in a 62-unit channel departs from it by the finite Ca, the mesh
and the confinement.  Observed (one run): in the first 0.4 shear times the
GPU curve overshoots by up to 35 % of the steady value; from gammadot t = 0.6
on it stays 3-12 % above the theory (12 % for the non-pre-stressed capsule
at Ca = 0.05, D = 0.107, where small-deformation theory is least accurate).
The bound: from gammadot t = 0.6 on, every sample within 15 % of the
theory's steady deformation of the theory curve."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_18919_amd import iblb
from paper_2305_18919_amd.inputs import c2_shear, sphere_mesh
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

T_END = 3.0
SAMPLES = 30


def gpu_trace(shape, ca):
    w = c2_shear(ca)
    abar = w.mesh.alpha[0]
    mesh = sphere_mesh(4, 10.0, (31.5, 31.5, 31.5), tuple(abar * s for s in shape))
    gdot = 0.02 / (w.domain.z_hi - w.domain.z_lo)
    n = int(round(T_END / SAMPLES / gdot))
    t, D = [], []
    with iblb.Simulation(w.domain, mesh, precision=iblb.FP32_DEV, graph=True) as g:
        for k in range(SAMPLES):
            g.step(n)
            t.append(gdot * n * (k + 1))
            D.append(g.shape_dtheta()[0])
    return np.array(t), np.array(D)


@pytest.mark.parametrize("shape", [(1.0, 1.0, 1.0), (1.0, 0.0, 1.0), (0.0, 1.0, 1.0), (0.0, 0.0, 1.0)])
@pytest.mark.parametrize("ca", [0.01, 0.05])
def test_deformation_follows_small_deformation_theory(shape, ca):
    announce(f"shear D(t) shape={shape} Ca={ca}")
    t, D = gpu_trace(shape, ca)
    a = tuple(s / ca for s in shape)
    r = O.shear_deformation_ode(a, T_END, 12000, n_samples=300)
    D_ss = r["D"][-1]
    Dth = np.interp(t, r["t"], r["D"])
    gap = np.abs(D - Dth) / D_ss
    announce("  t     " + " ".join(f"{v:6.2f}" for v in t[::3]))
    announce("  D gpu " + " ".join(f"{v:6.4f}" for v in D[::3]))
    announce("  D ode " + " ".join(f"{v:6.4f}" for v in Dth[::3]))
    announce(f"  max gap from 0.6: {gap[t > 0.59].max():.3f} of D_ss = {D_ss:.5f}; last {D[-1] / D_ss - 1:+.3f}")
    assert gap[t > 0.59].max() <= 0.15
