"""Host-side checks of the Python binding that need no GPU."""
import pytest

from paper_2305_18919_amd import iblb

MAPS = """\
7f1a00000000-7f1a00400000 r-xp 00000000 08:01 1201 /opt/rocm-7.2.0/lib/libamdhip64.so.7.2.0
7f1b00000000-7f1b00400000 r-xp 00000000 08:01 1202 /usr/local/lib/python3.10/dist-packages/torch/lib/libamdhip64.so
7f1c00000000-7f1c00021000 rw-p 00000000 00:00 0
7f1d00000000-7f1d00200000 r-xp 00000000 08:01 1203 /usr/lib/x86_64-linux-gnu/libc.so.6
"""


def test_runtime_scan_finds_every_mapped_hip_runtime(tmp_path):
    maps = tmp_path / "maps"
    maps.write_text(MAPS)
    assert iblb._hip_runtimes(str(maps)) == {
        "/opt/rocm-7.2.0/lib/libamdhip64.so.7.2.0",
        "/usr/local/lib/python3.10/dist-packages/torch/lib/libamdhip64.so",
    }
    one = tmp_path / "one"
    one.write_text("".join(l + "\n" for l in MAPS.splitlines() if "torch" not in l))
    assert len(iblb._hip_runtimes(str(one))) == 1
    assert iblb._hip_runtimes(str(tmp_path / "absent")) == set()


def test_library_load_is_refused_with_two_runtimes(monkeypatch):
    """Two HIP runtimes in one process crashed when a stream of one was used
    by the other: the binding refuses to load the library then."""
    monkeypatch.setattr(iblb, "_hip_runtimes", lambda maps="/proc/self/maps": {"/a/libamdhip64.so", "/b/libamdhip64.so"})
    monkeypatch.setattr(iblb, "_lib", None)
    with pytest.raises(RuntimeError, match="two HIP runtimes"):
        iblb.lib()


def test_library_loads_with_one_runtime(monkeypatch):
    monkeypatch.setattr(iblb, "_hip_runtimes", lambda maps="/proc/self/maps": {"/a/libamdhip64.so"})
    monkeypatch.setattr(iblb, "_lib", None)
    assert iblb.lib() is not None
