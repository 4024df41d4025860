"""ctypes binding of libiblb (include/iblb.h): argument marshalling only.

Every step of the IB-LB path runs in the library's HIP kernels; this module
only converts numpy arrays and the workload descriptions of ``inputs`` into
the C structs, allocates the device workspace and stream through PyTorch when
it is available, and turns status codes into exceptions.  If the compiled
library is missing the import of :class:`Simulation` fails loudly: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libiblb.so")

IBLB_OK, IBLB_E_INVAL, IBLB_E_DEVICE, IBLB_E_MESH, IBLB_E_UNSTABLE, IBLB_E_STATE = 0, -1, -2, -3, -4, -5
FP64, FP32_DEV, FP16_DEV, BF16_DEV = 0, 1, 2, 3
WALLS_Z, PERIODIC_ALL = 0, 1

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_vp = C.c_void_p


class DomainDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("wall_mode", C.c_int32),
                ("precision", C.c_int32), ("init_couette", C.c_int32), ("tau", C.c_double),
                ("rho0", C.c_double), ("u_wall_lo", C.c_double * 3), ("u_wall_hi", C.c_double * 3),
                ("body_force", C.c_double * 3)]


class MeshDesc(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_faces", C.c_int32), ("vertices", _dp),
                ("ref_vertices", _dp), ("faces", _ip), ("alpha", C.c_double * 3), ("k_v", C.c_double),
                ("eps_wall_lo", C.c_double), ("eps_wall_hi", C.c_double), ("xi_wall", C.c_double),
                ("r_cut_wall", C.c_double)]


class BatchConfig(C.Structure):
    _fields_ = [("lb_block_x", C.c_int32), ("spread_blocks_per_cu", C.c_int32),
                ("vertices_per_wave", C.c_int32), ("reserved", C.c_int32), ("lb_share_forces", C.c_double)]


class IBLBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"iblb error {code}: {msg}")
        self.code = code


_lib = None


def _hip_runtimes(maps: str = "/proc/self/maps") -> set:
    """Paths of HIP runtime libraries mapped into this process (read from its
    memory map, /proc/self/maps unless another file in that format is given)."""
    found = set()
    try:
        with open(maps) as fh:
            for line in fh:
                path = line.split()[-1] if line.strip() else ""
                if "libamdhip64.so" in path:
                    found.add(path)
    except OSError:
        pass
    return found


def lib():
    """Load libiblb.so (raises if it has not been built).

    PyTorch ships its own HIP runtime and its libraries name it in a way that
    does not match an already loaded system runtime, so loading libiblb first
    would put two HIP runtimes in the process.  PyTorch is therefore imported
    first (when installed) and libiblb binds to the runtime it brought; the
    load is refused if two runtimes are mapped anyway.
    """
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2305_18919_amd.build`")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        runtimes = _hip_runtimes()
        if len(runtimes) > 1:
            raise RuntimeError(f"two HIP runtimes are loaded in this process: {sorted(runtimes)}; import torch "
                               f"before anything that loads /opt/rocm's libamdhip64")
        pp = C.POINTER(_vp)
        sig = {
            "iblb_workspace_bytes": [C.POINTER(DomainDesc), C.POINTER(MeshDesc), C.POINTER(C.c_size_t)],
            "iblb_create": [C.POINTER(DomainDesc), _vp, C.c_size_t, _vp, pp],
            "iblb_add_mesh": [_vp, C.POINTER(MeshDesc), _ip],
            "iblb_step": [_vp, C.c_int32],
            "iblb_sync": [_vp],
            "iblb_step_count": [_vp, C.POINTER(C.c_int64)],
            "iblb_get_vertices": [_vp, C.c_int32, _dp],
            "iblb_vertices_device": [_vp, C.c_int32, C.POINTER(_dp)],
            "iblb_volume": [_vp, C.c_int32, _dp, _dp],
            "iblb_shape": [_vp, C.c_int32, _dp, _dp, _dp],
            "iblb_contact_angle": [_vp, C.c_int32, C.c_int32, C.c_int32, _dp, _dp, _dp],
            "iblb_get_fields": [_vp, _dp, _dp],
            "iblb_get_fields_noalloc": [_vp, _dp, _dp],
            "iblb_probe_phase_sync": [C.c_int32, C.c_int32, _dp, _dp],
            "iblb_debug_set_force": [_vp, _dp],
            "iblb_debug_get_force": [_vp, _dp],
            "iblb_debug_get_populations": [_vp, _dp],
            "iblb_debug_set_populations": [_vp, _dp],
            "iblb_debug_get_nodal_forces": [_vp, C.c_int32, _dp],
            "iblb_save_state": [_vp, _vp, C.POINTER(C.c_size_t)],
            "iblb_load_state": [_vp, _vp, C.c_size_t],
            "iblb_set_graph": [_vp, C.c_int32],
            "iblb_set_timing": [_vp, C.c_int32],
            "iblb_get_lb_split": [_vp, _ip, _dp],
            "iblb_kernel_time": [_vp, C.c_char_p, _dp, C.POINTER(C.c_int64)],
            "iblb_reset_timing": [_vp],
            "iblb_active_nodes": [_vp, C.POINTER(C.c_int64)],
            "iblb_tile_shape": [_ip, _ip, _ip],
            "iblb_destroy": [_vp],
            "iblb_batch_create": [C.POINTER(_vp), C.c_int32, _vp, pp],
            "iblb_batch_step": [_vp, C.c_int32],
            "iblb_batch_sync": [_vp],
            "iblb_batch_check": [_vp, _ip, _ip],
            "iblb_batch_get_config": [_vp, C.POINTER(BatchConfig)],
            "iblb_batch_set_config": [_vp, C.POINTER(BatchConfig)],
            "iblb_batch_tune": [_vp, C.c_int32, _dp],
            "iblb_batch_destroy": [_vp],
            "iblb_adjoint_record": [_vp, C.c_int32, C.c_int32],
            "iblb_adjoint_backward": [_vp, _dp, _dp, _dp],
            "iblb_adjoint_release": [_vp],
            "iblb_sphere_fit_grad": [C.c_int32, _dp, C.c_int32, C.c_double, C.c_double, _dp, _dp, _dp, _dp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.iblb_tile_shape.restype = None
        L.iblb_last_error.argtypes = [_vp]
        L.iblb_last_error.restype = C.c_char_p
        L.iblb_batch_last_error.argtypes = [_vp]
        L.iblb_batch_last_error.restype = C.c_char_p
        L.iblb_batch_member_error.argtypes = [_vp, C.c_int32]
        L.iblb_batch_member_error.restype = C.c_char_p
        _lib = L
    return _lib


def tile_shape() -> tuple:
    """Extents (x, y, z) in fluid nodes of the tiles the spreading works on."""
    t = [C.c_int32() for _ in range(3)]
    lib().iblb_tile_shape(*[C.byref(v) for v in t])
    return tuple(v.value for v in t)


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def domain_desc(dom, precision: int) -> DomainDesc:
    d = DomainDesc()
    d.nx, d.ny, d.nz = int(dom.nx), int(dom.ny), int(dom.nz)
    d.wall_mode = int(dom.wall_mode)
    d.precision = int(precision)
    d.init_couette = int(dom.init_couette)
    d.tau, d.rho0 = float(dom.tau), float(dom.rho0)
    for k in range(3):
        d.u_wall_lo[k] = float(dom.u_wall_lo[k])
        d.u_wall_hi[k] = float(dom.u_wall_hi[k])
        d.body_force[k] = float(dom.body_force[k])
    return d


def mesh_desc(mesh, keep: list) -> MeshDesc:
    """MeshDesc over contiguous copies; `keep` holds them alive for the call."""
    q = _f64(mesh.vertices)
    X = _f64(mesh.ref_vertices)
    F = np.ascontiguousarray(mesh.faces, dtype=np.int32)
    keep += [q, X, F]
    m = MeshDesc()
    m.n_vertices, m.n_faces = q.shape[0], F.shape[0]
    m.vertices, m.ref_vertices = _p(q), _p(X)
    m.faces = F.ctypes.data_as(_ip)
    for k in range(3):
        m.alpha[k] = float(mesh.alpha[k])
    m.k_v = float(mesh.k_v)
    m.eps_wall_lo, m.eps_wall_hi = float(mesh.eps_wall_lo), float(mesh.eps_wall_hi)
    m.xi_wall, m.r_cut_wall = float(mesh.xi_wall), float(mesh.r_cut_wall)
    return m


def workspace_bytes(dom, precision: int, mesh=None) -> int:
    keep: list = []
    n = C.c_size_t()
    md = C.byref(mesh_desc(mesh, keep)) if mesh is not None else None
    rc = lib().iblb_workspace_bytes(C.byref(domain_desc(dom, precision)), md, C.byref(n))
    if rc != IBLB_OK:
        raise IBLBError(rc, "iblb_workspace_bytes rejected the domain")
    return n.value


def sphere_fit_grad(q, wall: int = 0, z_wall: float = 0.5, exclude: float = 2.0):
    """Height h and signed squared contact radius r2 of the contact-angle fit
    (iblb_sphere_fit_grad) and their gradients [nv, 3] with respect to q."""
    qa = _f64(q)
    h, r2 = C.c_double(), C.c_double()
    dh, dr2 = np.zeros_like(qa), np.zeros_like(qa)
    rc = lib().iblb_sphere_fit_grad(qa.shape[0], _p(qa), int(wall), float(z_wall), float(exclude), C.byref(h),
                                    C.byref(r2), _p(dh), _p(dr2))
    if rc != IBLB_OK:
        raise IBLBError(rc, "sphere fit failed (fewer than 4 vertices away from the wall, or singular)")
    return h.value, r2.value, dh, dr2


class Simulation:
    """One IB-LB context on the current GPU.

    use_torch: take the device workspace (a uint8 tensor) and the stream (a
    torch.cuda.Stream at default priority) from PyTorch; otherwise the library
    allocates both itself.
    """

    def __init__(self, domain, mesh=None, precision: int = FP64, graph: bool = True, use_torch: bool = True):
        L = lib()
        self.dom = domain
        self.precision = precision
        self.shape = (domain.nz_fluid, domain.ny, domain.nx)
        self.n = int(np.prod(self.shape))
        self._ws = None
        self._stream = None
        ws_ptr, ws_bytes, stream = None, 0, None
        if use_torch:
            import torch
            ws_bytes = workspace_bytes(domain, precision, mesh)
            self._ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
            self._stream = torch.cuda.Stream()
            torch.cuda.synchronize()
            ws_ptr, stream = self._ws.data_ptr(), self._stream.cuda_stream
        h = _vp()
        rc = L.iblb_create(C.byref(domain_desc(domain, precision)), ws_ptr, ws_bytes, stream, C.byref(h))
        if rc != IBLB_OK:
            raise IBLBError(rc, "iblb_create failed")
        self.h = h
        self.nv = 0
        if mesh is not None:
            self.add_mesh(mesh)
        self.set_graph(graph)

    @property
    def stream(self):
        """The torch.cuda.Stream all of this context's work runs on (None when
        the library owns its stream)."""
        return self._stream

    # -- plumbing
    def _check(self, rc: int):
        if rc != IBLB_OK:
            msg = lib().iblb_last_error(self.h)
            raise IBLBError(rc, msg.decode() if msg else "")

    def add_mesh(self, mesh):
        keep: list = []
        mid = C.c_int32()
        self._check(lib().iblb_add_mesh(self.h, C.byref(mesh_desc(mesh, keep)), C.byref(mid)))
        self.nv = mesh.n_vertices
        self.mesh = mesh
        return mid.value

    def set_graph(self, on: bool):
        self._check(lib().iblb_set_graph(self.h, int(bool(on))))

    def set_timing(self, on: bool):
        self._check(lib().iblb_set_timing(self.h, int(bool(on))))

    def lb_split(self) -> dict:
        """Launch shape of the LB outside the active tiles (iblb_get_lb_split)."""
        bx = C.c_int32()
        sh = C.c_double()
        self._check(lib().iblb_get_lb_split(self.h, C.byref(bx), C.byref(sh)))
        return {"block_x": bx.value, "share_forces": sh.value}

    def reset_timing(self):
        self._check(lib().iblb_reset_timing(self.h))

    def kernel_time(self, name: str):
        ms = C.c_double()
        n = C.c_int64()
        self._check(lib().iblb_kernel_time(self.h, name.encode(), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def active_nodes(self) -> int:
        """Fluid nodes in the active tiles of the last completed step."""
        n = C.c_int64()
        self._check(lib().iblb_active_nodes(self.h, C.byref(n)))
        return n.value

    # -- stepping
    def step(self, n: int = 1):
        self._check(lib().iblb_step(self.h, int(n)))

    def sync(self):
        self._check(lib().iblb_sync(self.h))

    @property
    def t(self) -> int:
        v = C.c_int64()
        self._check(lib().iblb_step_count(self.h, C.byref(v)))
        return v.value

    # -- state access
    def vertices(self) -> np.ndarray:
        out = np.zeros((self.nv, 3))
        self._check(lib().iblb_get_vertices(self.h, 0, _p(out)))
        return out

    def vertices_device_ptr(self) -> int:
        p = _dp()
        self._check(lib().iblb_vertices_device(self.h, 0, C.byref(p)))
        return C.cast(p, C.c_void_p).value

    def populations(self) -> np.ndarray:
        out = np.zeros((19,) + self.shape)
        self._check(lib().iblb_debug_get_populations(self.h, _p(out)))
        return out

    def set_populations(self, d: np.ndarray):
        self._check(lib().iblb_debug_set_populations(self.h, _p(_f64(d).reshape(-1))))

    def fields(self):
        rho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        self._check(lib().iblb_get_fields(self.h, _p(rho), _p(u)))
        return rho, u

    def force(self) -> np.ndarray:
        out = np.zeros((3,) + self.shape)
        self._check(lib().iblb_debug_get_force(self.h, _p(out)))
        return out

    def set_force(self, F: np.ndarray):
        self._check(lib().iblb_debug_set_force(self.h, _p(_f64(F).reshape(-1))))

    def nodal_forces(self) -> np.ndarray:
        out = np.zeros((self.nv, 3))
        self._check(lib().iblb_debug_get_nodal_forces(self.h, 0, _p(out)))
        return out

    # -- queries
    def volume(self):
        V, A = C.c_double(), C.c_double()
        self._check(lib().iblb_volume(self.h, 0, C.byref(V), C.byref(A)))
        return V.value, A.value

    def shape_dtheta(self):
        D, th = C.c_double(), C.c_double()
        cen = np.zeros(3)
        self._check(lib().iblb_shape(self.h, 0, C.byref(D), C.byref(th), _p(cen)))
        return D.value, th.value, cen

    def contact_angle(self, wall: int = 0, method: int = 0):
        """(theta_deg, contact_radius, height): method 0 sphere fit, 1 the
        slice circle fit."""
        th, r, h = C.c_double(), C.c_double(), C.c_double()
        self._check(lib().iblb_contact_angle(self.h, 0, wall, method, C.byref(th), C.byref(r), C.byref(h)))
        return th.value, r.value, h.value

    # -- adjoint
    def adjoint_record(self, n: int, every: int = 100):
        """Step n times recording the window for adjoint_backward: every time
        level and the step's own fields in device memory (every = 0), or a
        device checkpoint every `every` steps that the sweep recomputes from."""
        self._check(lib().iblb_adjoint_record(self.h, int(n), int(every)))

    def adjoint_backward(self, dJdq: np.ndarray):
        """Reverse sweep over the recorded steps for an observable J of the
        final positions with gradient dJdq [nv, 3].  Returns dJ/d(alpha_1,
        alpha_2, alpha_3, k_V, eps_lo, tau) and dJ/dq at the window's start."""
        src = _f64(dJdq).reshape(-1)
        g = np.zeros(6)
        dq0 = np.zeros((self.nv, 3))
        self._check(lib().iblb_adjoint_backward(self.h, _p(src), _p(g), _p(dq0)))
        return g, dq0

    def adjoint_release(self):
        self._check(lib().iblb_adjoint_release(self.h))

    # -- checkpoints
    def save_state(self) -> bytes:
        n = C.c_size_t()
        self._check(lib().iblb_save_state(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(lib().iblb_save_state(self.h, C.cast(buf, _vp), C.byref(n)))
        return buf.raw

    def load_state(self, state: bytes):
        buf = C.create_string_buffer(state, len(state))
        self._check(lib().iblb_load_state(self.h, C.cast(buf, _vp), len(state)))

    def close(self):
        if getattr(self, "h", None):
            lib().iblb_destroy(self.h)
            self.h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Several Simulations advanced together by one launch of each step
    kernel per step (iblb_batch_*).  The members keep answering their own
    queries; they must stay open while the batch exists.

    use_torch: the batch's launches go to a torch.cuda.Stream at default
    priority; otherwise the library creates the stream.
    """

    def __init__(self, sims, use_torch: bool = True):
        L = lib()
        self.sims = list(sims)
        n = len(self.sims)
        arr = (_vp * n)(*[s.h for s in self.sims])
        self._stream = None
        stream = None
        if use_torch:
            import torch
            self._stream = torch.cuda.Stream()
            stream = self._stream.cuda_stream
        h = _vp()
        rc = L.iblb_batch_create(arr, n, stream, C.byref(h))
        if rc != IBLB_OK:
            raise IBLBError(rc, "iblb_batch_create failed")
        self.h = h

    def _check(self, rc: int):
        if rc != IBLB_OK:
            msg = lib().iblb_batch_last_error(self.h)
            raise IBLBError(rc, msg.decode() if msg else "")

    @property
    def stream(self):
        return self._stream

    def step(self, n: int = 1):
        self._check(lib().iblb_batch_step(self.h, int(n)))

    def sync(self):
        self._check(lib().iblb_batch_sync(self.h))

    def check(self):
        """Per-member status after freezing the members whose device error
        bits are set: IBLB_OK or IBLB_E_UNSTABLE."""
        st = (C.c_int32 * len(self.sims))()
        nf = C.c_int32()
        self._check(lib().iblb_batch_check(self.h, st, C.byref(nf)))
        return list(st)

    def member_error(self, k: int) -> str:
        return lib().iblb_batch_member_error(self.h, int(k)).decode()

    @property
    def config(self) -> dict:
        c = BatchConfig()
        self._check(lib().iblb_batch_get_config(self.h, C.byref(c)))
        return {"lb_block_x": c.lb_block_x, "spread_blocks_per_cu": c.spread_blocks_per_cu,
                "vertices_per_wave": c.vertices_per_wave, "lb_share_forces": c.lb_share_forces}

    def set_config(self, **kw):
        cur = self.config
        cur.update(kw)
        c = BatchConfig()
        c.lb_block_x = int(cur["lb_block_x"])
        c.spread_blocks_per_cu = int(cur["spread_blocks_per_cu"])
        c.vertices_per_wave = int(cur["vertices_per_wave"])
        c.reserved = 0
        c.lb_share_forces = float(cur["lb_share_forces"])
        self._check(lib().iblb_batch_set_config(self.h, C.byref(c)))

    def tune(self, trial_steps: int = 64) -> float:
        """Autotune the launch shape; returns the best time per step (ms)."""
        ms = C.c_double()
        self._check(lib().iblb_batch_tune(self.h, int(trial_steps), C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "h", None):
            lib().iblb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def probe_phase_sync(blocks: int, rounds: int = 1000):
    """Microseconds per kernel boundary and per grid-wide barrier between two
    phases of `blocks` blocks (iblb_probe_phase_sync)."""
    b, g = C.c_double(), C.c_double()
    rc = lib().iblb_probe_phase_sync(int(blocks), int(rounds), C.byref(b), C.byref(g))
    if rc != IBLB_OK:
        raise IBLBError(rc, "iblb_probe_phase_sync failed")
    return b.value, g.value
