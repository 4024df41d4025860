"""The seeded input generators: icosphere counts and orientation, splitmix64."""
import numpy as np
import pytest

from paper_2305_18919_amd.inputs import SplitMix64, c1_droplet, c2_shear, c3_wetting, icosphere, perturb


def test_splitmix64_published_sequence():
    # first outputs of splitmix64 seeded with 0 (Steele, Lea, Flood 2014 reference code)
    r = SplitMix64(0)
    assert [r.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


@pytest.mark.parametrize("k", range(6))
def test_icosphere_counts_and_orientation(k):
    V, F = icosphere(k)
    assert V.shape == (10 * 4 ** k + 2, 3) and F.shape == (20 * 4 ** k, 3)
    assert np.allclose(np.linalg.norm(V, axis=1), 1.0)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    assert (np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) > 0).all()
    # closed 2-manifold: every directed edge appears once and its reverse once
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    s = set(map(tuple, e))
    assert len(s) == len(e) and all((j, i) in s for i, j in s)


def test_perturbation_bounds_and_determinism():
    V, _ = icosphere(2)
    p1, p2 = perturb(V, 0.01, 7), perturb(V, 0.01, 7)
    assert np.array_equal(p1, p2)
    assert 0 < np.abs(p1 - V).max() <= 0.01


def test_workloads():
    w1, w2, w3 = c1_droplet(), c2_shear(0.05), c3_wetting()
    assert (w1.mesh.n_vertices, w1.mesh.n_faces, w1.domain.n_fluid) == (642, 1280, 32 * 32 * 30)
    assert (w2.mesh.n_vertices, w2.mesh.n_faces, w2.domain.n_fluid) == (2562, 5120, 64 * 64 * 62)
    assert (w3.mesh.n_vertices, w3.mesh.n_faces, w3.domain.n_fluid) == (10242, 20480, 128 * 128 * 94)
    assert w2.notes["abar"] == pytest.approx(1.0753e-2, rel=1e-3)


def test_batch_sweep_recipe():
    from paper_2305_18919_amd.inputs import BATCH_EDGES, BATCH_MODELS, LJ_R0, batch_sweep
    ws, again = batch_sweep(), batch_sweep()
    assert len(ws) == 48
    for w, v in zip(ws, again):
        assert np.array_equal(w.mesh.vertices, v.mesh.vertices) and w.notes == v.notes
        e, R, abar = w.notes["edge"], w.notes["R"], w.notes["abar"]
        assert e in BATCH_EDGES and (w.domain.nx, w.domain.ny, w.domain.nz) == (e, e, e)
        assert 6.0 <= R < 14.0 and 1e-3 <= abar < 1e-1
        assert w.notes["model"] in BATCH_MODELS
        assert w.mesh.alpha == tuple(abar * a for a in w.notes["model"])
        assert w.mesh.n_vertices == (642 if R < 10.0 else 2562)
        assert w.mesh.eps_wall_lo == abar
        # the droplet fits between the walls, its lowest point at the LJ zero-force distance
        z = w.mesh.vertices[:, 2]
        assert z.min() == pytest.approx(0.5 + LJ_R0) and z.max() < w.domain.z_hi
    # every edge and every model is drawn
    assert {w.notes["edge"] for w in ws} == set(BATCH_EDGES)
    assert {w.notes["model"] for w in ws} == set(BATCH_MODELS)
