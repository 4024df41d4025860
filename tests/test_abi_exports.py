"""The C-ABI library loads without a GPU and exports every function that
include/iblb.h declares; argument validation that needs no device works."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iblb.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(iblb_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("iblb_create", "iblb_add_mesh", "iblb_step", "iblb_get_vertices", "iblb_contact_angle",
                 "iblb_volume", "iblb_destroy", "iblb_save_state", "iblb_load_state"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2305_18919_amd import iblb
    L = iblb.lib()
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_workspace_bytes_validates_domain_without_gpu():
    from paper_2305_18919_amd import iblb
    from paper_2305_18919_amd.inputs import Domain, c2_shear
    w = c2_shear()
    n = iblb.workspace_bytes(w.domain, iblb.FP32_DEV, w.mesh)
    # populations + force field at least
    assert n >= w.domain.n_fluid * (19 + 3) * 4
    assert iblb.workspace_bytes(w.domain, iblb.FP64) >= w.domain.n_fluid * 22 * 8
    for bad in (Domain(4, 32, 32), Domain(32, 32, 32, tau=0.5), Domain(32, 32, 32, wall_mode=7),
                Domain(32, 32, 32, u_wall_lo=(0, 0, 0.1))):
        with pytest.raises(iblb.IBLBError):
            iblb.workspace_bytes(bad, iblb.FP64)
    with pytest.raises(iblb.IBLBError):
        iblb.workspace_bytes(w.domain, 5)


def test_workspace_bytes_enforces_the_lattice_size_limits():
    """The populations must fit in 4 GiB (19 x nodes x bytes per population,
    32-bit byte offsets) and the lattice hold at most 2^31 nodes."""
    from paper_2305_18919_amd import iblb
    from paper_2305_18919_amd.inputs import Domain
    under = Domain(512, 512, 200)   # 52.4 M nodes: 3.98 GB of FP32 populations
    over = Domain(512, 512, 240)    # 62.9 M nodes: 4.78 GB in FP32, 2.39 GB in FP16
    assert iblb.workspace_bytes(under, iblb.FP32_DEV) >= under.n_fluid * 19 * 4
    with pytest.raises(iblb.IBLBError):
        iblb.workspace_bytes(over, iblb.FP32_DEV)
    with pytest.raises(iblb.IBLBError):
        iblb.workspace_bytes(under, iblb.FP64)
    assert iblb.workspace_bytes(over, iblb.FP16_DEV) >= over.n_fluid * 19 * 2
    with pytest.raises(iblb.IBLBError):
        iblb.workspace_bytes(Domain(2048, 2048, 600), iblb.BF16_DEV)  # beyond 2^31 nodes


def test_tile_shape_is_one_wavefront_of_power_of_two_extents():
    from paper_2305_18919_amd import iblb
    tx, ty, tz = iblb.tile_shape()
    assert tx * ty * tz == 64
    assert all(e >= 1 and (e & (e - 1)) == 0 for e in (tx, ty, tz))


def test_step_geometry_counts_the_stencil_tiles_by_brute_force():
    """bench.step_geometry's active nodes (the tiles reached by some vertex's
    4^3 stencil, in the library's tile shape) against a direct count over the
    stencil nodes, on a small droplet next to a wall and across the x seam."""
    import numpy as np
    import bench
    from paper_2305_18919_amd import iblb
    from paper_2305_18919_amd.inputs import Domain, sphere_mesh
    dom = Domain(37, 26, 20, tau=0.9)
    mesh = sphere_mesh(2, 5.0, (1.2, 12.3, 0.5 + 5.0 + 0.4), (1e-3, 1e-3, 1e-3), amplitude=0.03, seed=2)
    q = np.asarray(mesh.vertices)
    TX, TY, TZ = iblb.tile_shape()
    nzf = dom.nz - 2
    tiles = set()
    for p in q:
        b = np.floor(p).astype(int) - 1
        for k in range(64):
            x = (b[0] + (k & 3)) % dom.nx
            y = (b[1] + ((k >> 2) & 3)) % dom.ny
            zf = b[2] + (k >> 4) - 1
            if 0 <= zf < nzf:
                tiles.add((x // TX, y // TY, zf // TZ))
    want = sum(min(TX, dom.nx - TX * a) * min(TY, dom.ny - TY * c) * min(TZ, nzf - TZ * e) for a, c, e in tiles)
    geo = bench.step_geometry(dom, q, {"block_x": 32, "share_forces": 0.5})
    assert geo["active_nodes"] == want
    assert sum(geo["lb_nodes"].values()) == dom.n_fluid
