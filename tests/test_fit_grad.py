"""The library's host-side sphere fit and its gradient (iblb_sphere_fit_grad)
against the oracle's fit differentiated by torch.autograd; no GPU needed."""
import numpy as np
import pytest
import torch

from oracle.adjoint import sphere_fit
from paper_2305_18919_amd import iblb
from paper_2305_18919_amd.inputs import sphere_mesh


def cap(shift_z):
    m = sphere_mesh(3, 8.0, (15.2, 15.9, 8.8), (1e-3, 0, 0), amplitude=0.3, seed=3)
    q = m.vertices.copy()
    q[:, 2] += shift_z
    return q


@pytest.mark.parametrize("shift_z", [-3.0, 0.0, 2.0])
def test_fit_and_gradient_match_oracle(shift_z):
    q = cap(shift_z)
    h, r2, dh, dr2 = iblb.sphere_fit_grad(q, 0, 0.5, 2.0)
    for name, val, grad in (("h", h, dh), ("r2", r2, dr2)):
        qt = torch.tensor(q, requires_grad=True)
        ref = sphere_fit(qt, 0.5, 2.0)[name]
        g, = torch.autograd.grad(ref, qt)
        assert val == pytest.approx(float(ref.detach()), rel=1e-11, abs=1e-11)
        assert np.abs(grad - g.numpy()).max() <= 1e-10 * np.abs(g.numpy()).max()


def test_upper_wall_is_the_mirror_image():
    q = cap(0.0)
    zw = 30.5
    mirrored = q.copy()
    mirrored[:, 2] = zw + 0.5 - q[:, 2]
    h0, r0, dh0, dr0 = iblb.sphere_fit_grad(q, 0, 0.5, 2.0)
    h1, r1, dh1, dr1 = iblb.sphere_fit_grad(mirrored, 1, zw, 2.0)
    assert h1 == pytest.approx(h0, rel=1e-12) and r1 == pytest.approx(r0, rel=1e-12)
    assert np.allclose(dh1[:, :2], dh0[:, :2], atol=1e-12) and np.allclose(dh1[:, 2], -dh0[:, 2], atol=1e-12)


def test_too_few_vertices_is_an_error():
    q = cap(0.0)
    with pytest.raises(iblb.IBLBError):
        iblb.sphere_fit_grad(q, 0, 0.5, 100.0)
