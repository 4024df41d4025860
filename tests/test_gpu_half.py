"""16-bit population storage (FP16 and BF16 deviations relative to w_i, FP32
arithmetic) against the FP64 oracle.

Each stored population is rounded to nearest once per step, with relative
error at most 2^-11 (FP16: 11 significand bits) or 2^-8 (BF16: 8 bits); the
BGK collision with Guo forcing does not amplify a perturbation of the
populations, so after n LB steps the populations differ from the FP64 ones by
at most n times that bound relative to the largest deviation, plus the FP32
arithmetic (~1e-7)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_18919_amd import iblb
from paper_2305_18919_amd.inputs import PERIODIC_ALL, Domain, random_force_field
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

UNIT = {iblb.FP16_DEV: 2.0 ** -11, iblb.BF16_DEV: 2.0 ** -8}
CASES = {
    "walls_ragged": Domain(30, 22, 19, tau=0.8, u_wall_lo=(0.01, -0.005, 0), u_wall_hi=(-0.02, 0.01, 0)),
    "periodic_ragged": Domain(20, 13, 11, wall_mode=PERIODIC_ALL, tau=1.3, body_force=(1e-5, 0, -2e-5)),
    "wide_rows_ragged": Domain(140, 9, 10, tau=0.9, u_wall_lo=(0.004, 0.002, 0), u_wall_hi=(-0.003, 0, 0)),
    "rows128_walls": Domain(128, 11, 9, tau=0.85, u_wall_lo=(0.006, -0.002, 0), u_wall_hi=(-0.004, 0.003, 0)),
}


@pytest.mark.parametrize("prec", [iblb.FP16_DEV, iblb.BF16_DEV])
@pytest.mark.parametrize("name", sorted(CASES))
def test_lb_one_step_within_one_rounding(prec, name):
    """One step from rest: every population is the FP64 value rounded once."""
    d = CASES[name]
    announce(f"lb 16-bit prec={prec} {name} 1 step")
    F = random_force_field((d.nz_fluid, d.ny, d.nx), 2e-4, seed=7)
    o = O.OracleSim(d)
    o.set_force(F)
    o.step(1)
    fo = o.populations()
    with iblb.Simulation(d, precision=prec) as g:
        g.set_force(F)
        g.step(1)
        fg = g.populations()
    err = np.abs(fg - fo)
    bound = UNIT[prec] * np.abs(fo) + 1e-6 * np.abs(fo).max()
    assert np.all(err <= bound), float((err / np.maximum(bound, 1e-300)).max())


@pytest.mark.parametrize("prec", [iblb.FP16_DEV, iblb.BF16_DEV])
@pytest.mark.parametrize("nsteps", [2, 7])
@pytest.mark.parametrize("name", ["walls_ragged", "rows128_walls"])
def test_lb_error_grows_at_most_one_rounding_per_step(prec, nsteps, name):
    d = CASES[name]
    announce(f"lb 16-bit prec={prec} {name} {nsteps} steps")
    F = random_force_field((d.nz_fluid, d.ny, d.nx), 2e-4, seed=8)
    o = O.OracleSim(d)
    o.set_force(F)
    o.step(nsteps)
    fo = o.populations()
    with iblb.Simulation(d, precision=prec) as g:
        g.set_force(F)
        g.step(nsteps)
        fg = g.populations()
    e = np.abs(fg - fo).max() / np.abs(fo).max()
    announce(f"  max |df| / max |f - w rho0| = {e:.3e} (unit {UNIT[prec]:.3e})")
    assert e <= nsteps * UNIT[prec] * 1.05 + 1e-6


@pytest.mark.parametrize("prec", [iblb.FP16_DEV, iblb.BF16_DEV])
def test_set_populations_roundtrip_rounds_once(prec):
    d = CASES["walls_ragged"]
    w = O.lattice()[1]
    g0 = np.random.default_rng(1).standard_normal((19, d.nz_fluid, d.ny, d.nx)) * 1e-3 * w[:, None, None, None]
    with iblb.Simulation(d, precision=prec) as g:
        for _ in range(2):
            g.set_populations(g0)
            back = g.populations()
            assert np.all(np.abs(back - g0) <= UNIT[prec] * np.abs(g0) * 1.001 + 1e-12)
            g.step(1)
