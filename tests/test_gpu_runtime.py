"""Execution modes, determinism, checkpoints, queries and error paths of the
C ABI on the GPU."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_18919_amd import iblb
from paper_2305_18919_amd.inputs import Domain, c1_droplet, c3_wetting, sphere_mesh
from tests.gpu_util import announce, rel

pytestmark = pytest.mark.gpu


def _run(w, prec, n, graph=True, timing=False):
    with iblb.Simulation(w.domain, w.mesh, precision=prec, graph=graph) as g:
        g.set_timing(timing)
        g.step(n)
        return g.vertices(), g.populations()


@pytest.mark.parametrize("prec", [iblb.FP64, iblb.FP32_DEV])
def test_graph_eager_timed_bitwise_equal_and_deterministic(prec):
    w = c1_droplet(eps_over_abar=1.0)
    announce(f"modes prec={prec}")
    a = _run(w, prec, 37, graph=True)
    b = _run(w, prec, 37, graph=False)
    c = _run(w, prec, 37, graph=False, timing=True)
    d = _run(w, prec, 37, graph=True)
    for x in (b, c, d):
        assert np.array_equal(a[0], x[0]) and np.array_equal(a[1], x[1])


def test_checkpoint_resume_bitwise():
    w = c1_droplet(eps_over_abar=1.0)
    with iblb.Simulation(w.domain, w.mesh, precision=iblb.FP64) as g:
        g.step(25)
        st = g.save_state()
        g.step(26)
        q1, f1 = g.vertices(), g.populations()
    with iblb.Simulation(w.domain, w.mesh, precision=iblb.FP64) as h:
        h.load_state(st)
        assert h.t == 25
        h.step(26)
        assert np.array_equal(h.vertices(), q1) and np.array_equal(h.populations(), f1)


def test_queries_match_oracle():
    w = c3_wetting(1.0)
    with iblb.Simulation(w.domain, w.mesh, precision=iblb.FP32_DEV) as g:
        g.step(3)
        q = g.vertices()
        V, A = g.volume()
        D, th, cen = g.shape_dtheta()
        ang, r, h = g.contact_angle(0)
    Vo, Ao, xco = O.volume_area_centroid(q, w.mesh.faces)
    Do, tho = O.shape_dtheta(q, w.mesh.faces)
    ango, ro, ho, _, _ = O.contact_angle_sphere(q, 0.5, 2.0)
    assert V == pytest.approx(Vo, rel=1e-12) and A == pytest.approx(Ao, rel=1e-12)
    assert np.allclose(cen, xco, rtol=0, atol=1e-10)
    assert abs(D - Do) < 1e-10 and abs(th - tho) < 1e-8
    assert abs(ang - ango) < 1e-3 and r == pytest.approx(ro, rel=1e-8) and h == pytest.approx(ho, rel=1e-8)


def test_mesh_validation_errors():
    d = Domain(16, 16, 16)
    m = sphere_mesh(1, 3.0, (8.0, 8.0, 8.0), (1e-3, 0, 0))
    with iblb.Simulation(d, precision=iblb.FP64) as g:
        open_mesh = sphere_mesh(1, 3.0, (8.0, 8.0, 8.0), (1e-3, 0, 0))
        open_mesh.faces = open_mesh.faces[1:]
        with pytest.raises(iblb.IBLBError) as e:
            g.add_mesh(open_mesh)
        assert e.value.code == iblb.IBLB_E_MESH
        flipped = sphere_mesh(1, 3.0, (8.0, 8.0, 8.0), (1e-3, 0, 0))
        flipped.faces = flipped.faces[:, [0, 2, 1]].copy()
        with pytest.raises(iblb.IBLBError) as e:
            g.add_mesh(flipped)
        assert e.value.code == iblb.IBLB_E_MESH
        bad = sphere_mesh(1, 3.0, (8.0, 8.0, 8.0), (1e-3, 0, 0))
        bad.vertices = bad.vertices.copy()
        bad.vertices[3, 1] = np.nan
        with pytest.raises(iblb.IBLBError) as e:
            g.add_mesh(bad)
        assert e.value.code == iblb.IBLB_E_INVAL
        huge = sphere_mesh(1, 3.0, (8.0, 8.0, 8.0), (1e-3, 0, 0))
        huge.vertices = np.full((65537, 3), 8.0)  # one vertex beyond the limit of 65536
        huge.ref_vertices = huge.vertices.copy()
        with pytest.raises(iblb.IBLBError) as e:
            g.add_mesh(huge)
        assert e.value.code == iblb.IBLB_E_INVAL
        g.add_mesh(m)
        with pytest.raises(iblb.IBLBError) as e:
            g.add_mesh(m)
        assert e.value.code == iblb.IBLB_E_STATE
        with pytest.raises(iblb.IBLBError) as e:
            g.set_force(np.zeros((3, 14, 16, 16)))
        assert e.value.code == iblb.IBLB_E_STATE
        with pytest.raises(iblb.IBLBError):
            g.contact_angle(wall=2)


def test_unstable_state_reported():
    """A non-finite population planted from the host is reported, not hidden."""
    d = Domain(16, 16, 16)
    with iblb.Simulation(d, precision=iblb.FP64) as g:
        f = np.zeros((19, 14, 16, 16))
        f[0, 3, 4, 5] = np.nan
        g.set_populations(f)
        g.step(2)
        with pytest.raises(iblb.IBLBError) as e:
            g.sync()
        assert e.value.code == iblb.IBLB_E_UNSTABLE


def test_load_state_rejects_mismatch():
    w = c1_droplet()
    with iblb.Simulation(w.domain, w.mesh, precision=iblb.FP64) as g:
        st = g.save_state()
    with iblb.Simulation(w.domain, w.mesh, precision=iblb.FP32_DEV) as h:
        with pytest.raises(iblb.IBLBError):
            h.load_state(st)
        with pytest.raises(iblb.IBLBError):
            h.load_state(b"garbage" * 10)


@pytest.mark.parametrize("prec", [iblb.FP64, iblb.FP32_DEV])
def test_graph_with_odd_starts_and_counts(prec):
    """The two-step graph is only replayed from even times; odd starts and odd
    counts fall back to single launches.  Any split gives the same state."""
    w = c1_droplet(eps_over_abar=1.0)
    with iblb.Simulation(w.domain, w.mesh, precision=prec, graph=True) as g:
        for n in (1, 4, 3, 2, 1, 5):
            g.step(n)
        assert g.t == 16
        qa, fa = g.vertices(), g.populations()
    with iblb.Simulation(w.domain, w.mesh, precision=prec, graph=False) as h:
        h.step(16)
        assert np.array_equal(h.vertices(), qa) and np.array_equal(h.populations(), fa)


def _stencil_tile_nodes(q, dom):
    """Fluid nodes of the library's tiles reached by the 4^3 stencils of the
    vertices at q (x, y periodic; z periodic or clipped to the fluid layers)."""
    TX, TY, TZ = iblb.tile_shape()
    walls = dom.wall_mode == iblb.WALLS_Z
    zoff, nzf = (1, dom.nz - 2) if walls else (0, dom.nz)
    tiles = set()
    for p in q:
        b = np.floor(p).astype(np.int64) - 1
        for k in range(64):
            x = (b[0] + (k & 3)) % dom.nx
            y = (b[1] + ((k >> 2) & 3)) % dom.ny
            z = b[2] + (k >> 4)
            zf = z - zoff if walls else z % dom.nz
            if 0 <= zf < nzf:
                tiles.add((x // TX, y // TY, zf // TZ))
    return sum(min(TX, dom.nx - TX * tx) * min(TY, dom.ny - TY * ty) * min(TZ, nzf - TZ * tz)
               for tx, ty, tz in tiles)


@pytest.mark.parametrize("case", ["walls_ragged", "periodic_ragged"])
def test_active_nodes_are_the_stencil_tiles(case):
    """The tiles the step treats as active (their LB runs with the spreading)
    are exactly those reached by a vertex stencil at the step's positions."""
    if case == "walls_ragged":
        dom = Domain(26, 21, 18, tau=0.9, u_wall_lo=(0.002, 0, 0))
        mesh = sphere_mesh(2, 4.5, (1.3, 10.2, 0.5 + 4.5 + 0.6), (2e-3, 1e-3, 1e-3), amplitude=0.02, seed=5,
                           eps_lo=2e-3, r_cut=2.0)
    else:
        dom = Domain(21, 19, 17, wall_mode=iblb.PERIODIC_ALL)
        mesh = sphere_mesh(2, 4.0, (19.6, 0.7, 16.2), (1e-3, 0.0, 1e-3), amplitude=0.05, seed=3)
    announce(f"active nodes {case}")
    with iblb.Simulation(dom, mesh, precision=iblb.FP64) as g:
        assert g.active_nodes() == 0
        for before in (0, 5):
            g.step(before)
            q = g.vertices()
            g.step(1)
            n = g.active_nodes()
            assert 0 < n < dom.n_fluid and n == _stencil_tile_nodes(q, dom)


def test_tile_list_overflow_is_reported():
    """More than 512 vertices whose stencils reach one tile (a level-4
    icosphere of radius 1, 2562 vertices, inside one 4^3 neighbourhood): the
    spreading keeps the first 512 of the tile's list, raises the overflow bit
    and the step reports IBLB_E_UNSTABLE naming it; nothing is written out of
    bounds, so the fields stay finite."""
    d = Domain(32, 32, 32, wall_mode=iblb.PERIODIC_ALL)
    m = sphere_mesh(4, 1.0, (16.3, 16.2, 16.1), (1e-3, 0.0, 0.0))
    assert m.n_vertices > 512
    announce("tile list overflow")
    with iblb.Simulation(d, m, precision=iblb.FP32_DEV) as g:
        g.step(1)
        with pytest.raises(iblb.IBLBError) as e:
            g.sync()
        assert e.value.code == iblb.IBLB_E_UNSTABLE
        assert "tile list overflow" in str(e.value)
        # the error stays raised; the fields are still copied out
        rho, u = np.zeros(g.shape), np.zeros((3,) + g.shape)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = iblb.lib().iblb_get_fields(g.h, rho.ctypes.data_as(dp), u.ctypes.data_as(dp))
        assert rc == iblb.IBLB_E_UNSTABLE
        assert np.isfinite(rho).all() and np.isfinite(u).all()


def test_phase_sync_probe():
    """Both orderings run and pass every phase (the probe checks that the
    barrier's generation count reached the number of rounds); sizes it
    cannot hold at once are refused."""
    for blocks in (256, 1024):
        announce(f"phase sync probe blocks={blocks}")
        b, g = iblb.probe_phase_sync(blocks, 200)
        announce(f"  boundary {b:.3f} us, barrier {g:.3f} us")
        assert 0.0 < b < 1e3 and 0.0 < g < 1e3
    x, y = ctypes.c_double(), ctypes.c_double()
    assert iblb.lib().iblb_probe_phase_sync(1 << 24, 10, ctypes.byref(x), ctypes.byref(y)) == iblb.IBLB_E_INVAL
    assert iblb.lib().iblb_probe_phase_sync(256, 0, ctypes.byref(x), ctypes.byref(y)) == iblb.IBLB_E_INVAL
