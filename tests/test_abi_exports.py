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
