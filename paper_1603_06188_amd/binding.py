"""ctypes binding of libapic (C ABI in include/apic.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libapic.so``.  PyTorch provides device memory and the stream.  Importing
this module fails loudly when the library has not been built; there is no
CPU fallback.

The functions ``apic_*`` mirror the C entry points one to one and take a
ctypes ``ApicScene``.  ``DeviceScene`` owns the torch tensors behind one
scene and is a convenience for tests, the benchmark and users.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # first: the library must bind to the HIP runtime torch loaded

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapic.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")

_lib = ctypes.CDLL(LIB_PATH)

APIC_OK = 0
APIC_E_INVAL, APIC_E_UNSUPPORTED, APIC_E_HIP, APIC_E_WORKSPACE = -1, -2, -3, -4
APIC_MULTILINEAR, APIC_QUADRATIC, APIC_CUBIC = 1, 2, 3
APIC_F32, APIC_F64 = 0, 1
APIC_MODEL_NONE, APIC_MODEL_NEO_HOOKEAN = 0, 1
APIC_TRANSFER_APIC, APIC_TRANSFER_RPIC, APIC_TRANSFER_PIC = 0, 1, 2
APIC_OPT_COMPENSATED = 1
APIC_OPT_FUSED_TRANSFER = 2
APIC_OPT_ADAPTIVE_DT = 4
APIC_OPT_ABSOLUTE_POSITIONS = 8
APIC_OPT_BATCH_GRAPH = 16
APIC_FLAG_OUT_OF_DOMAIN, APIC_FLAG_NONFINITE, APIC_FLAG_INVERTED, APIC_FLAG_CFL = 1, 2, 4, 8
APIC_FLAG_UNSORTED = 16
APIC_GRID_MASS, APIC_GRID_MOMENTUM, APIC_GRID_VELOCITY = 0, 1, 2
APIC_DIAG_PARTICLES, APIC_DIAG_GRID, APIC_DIAG_GRID_NEW, APIC_DIAG_ENERGY = 0, 1, 2, 3

EXPORTED = [
    "apic_workspace_bytes", "apic_reset", "apic_sort", "apic_p2g", "apic_grid_update", "apic_g2p", "apic_step",
    "apic_batch_workspace_bytes", "apic_step_batch", "apic_grid_export", "apic_diagnostics", "apic_cfl_dt", "apic_step_time",
    "apic_get_flags", "apic_clear_flags",
    "apic_positions_from_absolute", "apic_positions_to_absolute", "apic_timing_enable", "apic_timing_read",
    "apic_last_error", "apic_version", "apic_midpoint_workspace_bytes", "apic_step_midpoint",
    "apic_noalloc_max_bytes", "apic_step_noalloc",
    "apic_batch_plan_count", "apic_batch_plan_info", "apic_batch_set_plan", "apic_batch_tuning",
]
APIC_PHASES = ["p2g", "grid_update", "bin", "g2p", "sort", "mid_force", "mid_apply"]


class ApicGridDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("degree", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("options", ctypes.c_int32), ("cells", ctypes.c_int32 * 3), ("dx", ctypes.c_double)]


class ApicParticles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("stride", ctypes.c_int64), ("cell", ctypes.c_void_p),
                ("off", ctypes.c_void_p), ("v", ctypes.c_void_p), ("B", ctypes.c_void_p), ("F", ctypes.c_void_p),
                ("mass", ctypes.c_void_p), ("id", ctypes.c_void_p)]


class ApicParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("gravity", ctypes.c_double * 3), ("model", ctypes.c_int32),
                ("band", ctypes.c_int32 * 6), ("transfer", ctypes.c_int32), ("mu", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("rho0", ctypes.c_double), ("cfl", ctypes.c_double)]


class ApicScene(ctypes.Structure):
    _fields_ = [("grid", ApicGridDesc), ("p", ApicParticles), ("prm", ApicParams),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


class ApicMidpointOpts(ctypes.Structure):
    _fields_ = [("newton_tol", ctypes.c_double), ("cg_tol", ctypes.c_double), ("max_newton", ctypes.c_int32),
                ("max_cg", ctypes.c_int32)]


class ApicMidpointStats(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int32), ("cg_iters", ctypes.c_int32), ("halvings", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32),
                ("res0", ctypes.c_double), ("res", ctypes.c_double)]


_S = ctypes.POINTER(ApicScene)
_V = ctypes.c_void_p
_sigs = {
    "apic_workspace_bytes": [ctypes.POINTER(ApicGridDesc), ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)],
    "apic_reset": [_S, _V],
    "apic_sort": [_S, _V],
    "apic_p2g": [_S, _V],
    "apic_grid_update": [_S, _V],
    "apic_g2p": [_S, _V],
    "apic_step": [_S, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _V],
    "apic_batch_workspace_bytes": [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "apic_step_batch": [_S, ctypes.c_int32, ctypes.c_int32, _V, ctypes.c_size_t, _V],
    "apic_grid_export": [_S, ctypes.c_int32, _V, _V],
    "apic_diagnostics": [_S, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), _V],
    "apic_cfl_dt": [_S, ctypes.c_double, ctypes.POINTER(ctypes.c_double), _V],
    "apic_step_time": [_S, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _V],
    "apic_get_flags": [_S, ctypes.POINTER(ctypes.c_uint32), _V],
    "apic_clear_flags": [_S, _V],
    "apic_positions_from_absolute": [_S, _V, _V],
    "apic_positions_to_absolute": [_S, _V, _V],
    "apic_midpoint_workspace_bytes": [ctypes.POINTER(ApicGridDesc), ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)],
    "apic_step_midpoint": [_S, ctypes.c_int32, ctypes.POINTER(ApicMidpointOpts), ctypes.POINTER(ApicMidpointStats), _V],
    "apic_noalloc_max_bytes": [ctypes.POINTER(ctypes.c_size_t)],
    "apic_step_noalloc": [_S, ctypes.c_int32, _V],
    "apic_batch_plan_count": [ctypes.POINTER(ctypes.c_int32)],
    "apic_batch_plan_info": [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
    "apic_batch_set_plan": [ctypes.c_int32],
    "apic_batch_tuning": [_S, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)],
}
for _name, _args in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int32
_lib.apic_timing_enable.argtypes = [ctypes.c_int32]
_lib.apic_timing_enable.restype = ctypes.c_int32
_lib.apic_timing_read.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
_lib.apic_timing_read.restype = ctypes.c_int32
_lib.apic_last_error.restype = ctypes.c_char_p
_lib.apic_last_error.argtypes = []
_lib.apic_version.restype = ctypes.c_char_p
_lib.apic_version.argtypes = []


class ApicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"apic error {code}: {msg}")
        self.code = code


def _check(rc: int) -> None:
    if rc != APIC_OK:
        raise ApicError(rc, _lib.apic_last_error().decode())


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# --- one-to-one wrappers of the C entry points -------------------------------

def apic_workspace_bytes(grid: ApicGridDesc, max_particles: int) -> int:
    out = ctypes.c_size_t()
    _check(_lib.apic_workspace_bytes(ctypes.byref(grid), int(max_particles), ctypes.byref(out)))
    return out.value


def apic_midpoint_workspace_bytes(grid: ApicGridDesc, max_particles: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.apic_midpoint_workspace_bytes(ctypes.byref(grid), int(max_particles), ctypes.byref(out)))
    return out.value


def apic_step_midpoint(scene: ApicScene, n_steps: int = 1, newton_tol: float = 0.0, cg_tol: float = 0.0,
                       max_newton: int = 0, max_cg: int = 0, stream=None) -> dict:
    """Implicit midpoint steps; returns the solver statistics."""
    o = ApicMidpointOpts(float(newton_tol), float(cg_tol), int(max_newton), int(max_cg))
    st = ApicMidpointStats()
    _check(_lib.apic_step_midpoint(ctypes.byref(scene), int(n_steps), ctypes.byref(o), ctypes.byref(st),
                                   _stream(stream)))
    return {k: getattr(st, k) for k, _ in ApicMidpointStats._fields_ if k != "reserved"}


def apic_noalloc_max_bytes() -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.apic_noalloc_max_bytes(ctypes.byref(out)))
    return out.value


def apic_step_noalloc(scene: ApicScene, n_steps: int = 1, stream=None) -> None:
    """Steps without a workspace (the library's own device array)."""
    _check(_lib.apic_step_noalloc(ctypes.byref(scene), int(n_steps), _stream(stream)))


def apic_reset(scene: ApicScene, stream=None) -> None:
    _check(_lib.apic_reset(ctypes.byref(scene), _stream(stream)))


def apic_sort(scene: ApicScene, stream=None) -> None:
    _check(_lib.apic_sort(ctypes.byref(scene), _stream(stream)))


def apic_p2g(scene: ApicScene, stream=None) -> None:
    _check(_lib.apic_p2g(ctypes.byref(scene), _stream(stream)))


def apic_grid_update(scene: ApicScene, stream=None) -> None:
    _check(_lib.apic_grid_update(ctypes.byref(scene), _stream(stream)))


def apic_g2p(scene: ApicScene, stream=None) -> None:
    _check(_lib.apic_g2p(ctypes.byref(scene), _stream(stream)))


def apic_step(scenes, n_steps: int, sort_every: int = 0, stream=None) -> None:
    arr = (ApicScene * len(scenes))(*scenes)
    _check(_lib.apic_step(arr, len(scenes), int(n_steps), int(sort_every), _stream(stream)))
    # the C side does not modify the structs; nothing to copy back


def apic_batch_workspace_bytes(n_scenes: int) -> int:
    out = ctypes.c_size_t()
    _check(_lib.apic_batch_workspace_bytes(int(n_scenes), ctypes.byref(out)))
    return out.value


def apic_step_batch(scenes, n_steps: int, batch_ws_ptr: int, batch_ws_bytes: int, stream=None) -> None:
    arr = (ApicScene * len(scenes))(*scenes)
    _check(_lib.apic_step_batch(arr, len(scenes), int(n_steps), ctypes.c_void_p(batch_ws_ptr),
                                int(batch_ws_bytes), _stream(stream)))


def apic_batch_plan_count() -> int:
    out = ctypes.c_int32()
    _check(_lib.apic_batch_plan_count(ctypes.byref(out)))
    return out.value


def apic_batch_plan_info(plan: int):
    """(particles per share block, blocks per CU; 0: one block per item)."""
    pb, bc = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.apic_batch_plan_info(int(plan), ctypes.byref(pb), ctypes.byref(bc)))
    return pb.value, bc.value


def apic_batch_set_plan(plan: int) -> None:
    """Force launch plan `plan` for later apic_step_batch calls (-1: tune)."""
    _check(_lib.apic_batch_set_plan(int(plan)))


def apic_batch_tuning(scenes):
    """(chosen plan or -1, measured ns per particle-step of each plan)."""
    arr = (ApicScene * len(scenes))(*scenes)
    plan = ctypes.c_int32()
    n = apic_batch_plan_count()
    ns = (ctypes.c_double * n)()
    _check(_lib.apic_batch_tuning(arr, len(scenes), ctypes.byref(plan), ns))
    return plan.value, [float(v) for v in ns]


def apic_grid_export(scene: ApicScene, field: int, out_ptr: int, stream=None) -> None:
    _check(_lib.apic_grid_export(ctypes.byref(scene), int(field), ctypes.c_void_p(out_ptr), _stream(stream)))


def apic_diagnostics(scene: ApicScene, which: int, stream=None) -> np.ndarray:
    out = (ctypes.c_double * 8)()
    _check(_lib.apic_diagnostics(ctypes.byref(scene), int(which), out, _stream(stream)))
    return np.array(out[:], dtype=np.float64)


def apic_cfl_dt(scene: ApicScene, nu: float = 1.0, stream=None) -> float:
    out = ctypes.c_double()
    _check(_lib.apic_cfl_dt(ctypes.byref(scene), float(nu), ctypes.byref(out), _stream(stream)))
    return out.value


def apic_step_time(scene: ApicScene, stream=None):
    """(dt of the last adaptive step, time advanced by adaptive steps)."""
    dt_last, t = ctypes.c_double(), ctypes.c_double()
    _check(_lib.apic_step_time(ctypes.byref(scene), ctypes.byref(dt_last), ctypes.byref(t), _stream(stream)))
    return dt_last.value, t.value


def apic_get_flags(scene: ApicScene, stream=None) -> int:
    out = ctypes.c_uint32()
    _check(_lib.apic_get_flags(ctypes.byref(scene), ctypes.byref(out), _stream(stream)))
    return out.value


def apic_clear_flags(scene: ApicScene, stream=None) -> None:
    _check(_lib.apic_clear_flags(ctypes.byref(scene), _stream(stream)))


def apic_positions_from_absolute(scene: ApicScene, x_ptr: int, stream=None) -> None:
    _check(_lib.apic_positions_from_absolute(ctypes.byref(scene), ctypes.c_void_p(x_ptr), _stream(stream)))


def apic_positions_to_absolute(scene: ApicScene, x_ptr: int, stream=None) -> None:
    _check(_lib.apic_positions_to_absolute(ctypes.byref(scene), ctypes.c_void_p(x_ptr), _stream(stream)))


def apic_timing_enable(enable: bool = True) -> None:
    _check(_lib.apic_timing_enable(1 if enable else 0))


def apic_timing_read() -> dict:
    """{phase: (launches, mean ms)} of the phases apic_step recorded."""
    n = len(APIC_PHASES)
    counts = (ctypes.c_int64 * n)()
    mean = (ctypes.c_double * n)()
    _check(_lib.apic_timing_read(counts, mean))
    return {APIC_PHASES[k]: (int(counts[k]), float(mean[k])) for k in range(n)}


def apic_last_error() -> str:
    return _lib.apic_last_error().decode()


def apic_version() -> str:
    return _lib.apic_version().decode()


# --- device-resident scene ----------------------------------------------------

def pack_cells(cell: np.ndarray) -> np.ndarray:
    """Per-axis int cell indices [n, dim] -> packed uint32 (layout of apic.h)."""
    c = cell.astype(np.uint64)
    if cell.shape[1] == 3:
        packed = c[:, 0] | (c[:, 1] << np.uint64(10)) | (c[:, 2] << np.uint64(20))
    else:
        packed = c[:, 0] | (c[:, 1] << np.uint64(16))
    return packed.astype(np.uint32)


def unpack_cells(packed: np.ndarray, dim: int) -> np.ndarray:
    p = packed.astype(np.uint64)
    if dim == 3:
        return np.stack([p & 1023, (p >> 10) & 1023, p >> 20], axis=1).astype(np.int64)
    return np.stack([p & 0xFFFF, p >> 16], axis=1).astype(np.int64)


def grid_desc(scene, precision=None, compensated=False, fused=False, adaptive=False,
              absolute=False, batch_graph=False) -> ApicGridDesc:
    """The apic_grid_desc of a host scene."""
    precision = precision or scene.precision
    g = ApicGridDesc()
    g.dim = scene.dim
    g.degree = scene.degree
    g.precision = APIC_F32 if precision == "fp32" else APIC_F64
    g.options = ((APIC_OPT_COMPENSATED if compensated else 0) | (APIC_OPT_FUSED_TRANSFER if fused else 0)
                 | (APIC_OPT_ADAPTIVE_DT if adaptive else 0) | (APIC_OPT_ABSOLUTE_POSITIONS if absolute else 0)
                 | (APIC_OPT_BATCH_GRAPH if batch_graph else 0))
    for a in range(3):
        g.cells[a] = scene.cells[a] if a < scene.dim else 0
    g.dx = scene.dx
    return g


def plane_capacity(n: int) -> int:
    """Plane stride, in particles, of a DeviceScene for n particles: n rounded
    up to a whole number of 64-particle blocks, so that every plane starts on
    a 256-byte boundary (the transfers move aligned runs of 64 particles per
    plane and cover whole cache lines only when all planes share the first
    plane's alignment)."""
    return (max(int(n), 1) + 63) // 64 * 64


def scene_footprint_bytes(scene, precision=None, compensated=False, with_id=True, capacity=None) -> int:
    """Device bytes a DeviceScene of `scene` holds: its particle planes, cell
    (and id) arrays and its workspace."""
    precision = precision or scene.precision
    cap = plane_capacity(capacity or scene.n)
    d = scene.dim
    elem = 4 if precision == "fp32" else 8
    planes = (2 * d + 2 * d * d + 1) * cap * elem
    ints = cap * 4 * (2 if with_id else 1)
    return planes + ints + apic_workspace_bytes(grid_desc(scene, precision, compensated), cap) + 256


class DeviceScene:
    """Device copy of a ``scenes.Scene`` plus its workspace.

    Particle planes live in one tensor ``f`` of shape [planes, stride]:
    off (dim), v (dim), B (dim*dim), F (dim*dim), mass (1)."""

    def __init__(self, scene, device="cuda", precision=None, compensated=False, capacity=None, with_id=True,
                 packed=None, fused=False, adaptive=False, midpoint=False, absolute=False, batch_graph=False):
        self.host = scene
        self.absolute = bool(absolute)   # positions as plain binary32 coordinates (APIC_OPT_ABSOLUTE_POSITIONS)
        self.dim = scene.dim
        self.precision = precision or scene.precision
        self.dtype = torch.float32 if self.precision == "fp32" else torch.float64
        self.n = scene.n
        self.capacity = plane_capacity(capacity or self.n)
        d = self.dim
        self.nplanes = 2 * d + 2 * d * d + 1
        cap = self.capacity
        self.f = torch.zeros((self.nplanes, cap), dtype=self.dtype, device=device)
        self.cell = torch.zeros(cap, dtype=torch.int32, device=device)
        self.id = torch.arange(cap, dtype=torch.int32, device=device) if with_id else None
        self.upload(scene, packed)
        g = grid_desc(scene, self.precision, compensated, fused, adaptive, self.absolute, batch_graph)
        self.wbytes = apic_workspace_bytes(g, cap)
        if midpoint:
            self.wbytes = max(self.wbytes, apic_midpoint_workspace_bytes(g, cap))
        self.ws = torch.empty(self.wbytes + 256, dtype=torch.uint8, device=device)
        s = ApicScene()
        s.grid = g
        s.workspace = (self.ws.data_ptr() + 255) // 256 * 256
        s.workspace_bytes = self.wbytes
        prm = s.prm
        prm.dt = scene.dt
        for a in range(3):
            prm.gravity[a] = scene.gravity[a] if a < len(scene.gravity) else 0.0
        prm.model = scene.model
        for k in range(6):
            prm.band[k] = scene.band[k]
        prm.transfer = scene.transfer
        prm.mu = scene.mu
        prm.lambda_ = scene.lam
        prm.rho0 = scene.rho0
        prm.cfl = scene.cfl
        self.s = s
        self._bind()
        apic_reset(self.s)

    def _plane(self, k):
        return self.f[k].data_ptr()

    def _bind(self):
        d = self.dim
        p = self.s.p
        p.n = self.n
        p.stride = self.capacity
        p.cell = self.cell.data_ptr()
        p.off = self._plane(0)
        p.v = self._plane(d)
        p.B = self._plane(2 * d)
        p.F = self._plane(2 * d + d * d)
        p.mass = self._plane(2 * d + 2 * d * d)
        p.id = self.id.data_ptr() if self.id is not None else None

    @staticmethod
    def pack(scene, dtype, absolute=False):
        """Host tensors in the device layout: planes [2d+2d^2+1, n] and packed cells [n].
        absolute: the position planes hold the coordinates x_p (rounded to the
        plane type) instead of the offsets in the cell."""
        d, n = scene.dim, scene.n
        pos = scene.off.T
        cell = scene.cell
        if absolute:
            x = scene.x.astype(np.float32 if dtype == torch.float32 else np.float64)
            pos = x.T.astype(np.float64)
            cell = np.floor(x.astype(np.float64) / scene.dx).astype(np.int64)
        planes = np.concatenate([pos, scene.v.T, scene.B.reshape(n, d * d).T, scene.F.reshape(n, d * d).T,
                                 scene.m[None, :]], axis=0)
        return (torch.from_numpy(np.ascontiguousarray(planes)).to(dtype),
                torch.from_numpy(pack_cells(cell).view(np.int32)))

    def upload(self, scene, packed=None):
        n = scene.n
        if n > self.capacity:
            raise ValueError("scene larger than capacity")
        self.n = n
        host, cells = packed if packed is not None else self.pack(scene, self.dtype, self.absolute)
        self.f[:, :n].copy_(host, non_blocking=True)
        self.cell[:n].copy_(cells, non_blocking=True)
        if self.id is not None:
            self.id[:n].copy_(torch.arange(n, dtype=torch.int32))
        if hasattr(self, "s"):
            self._bind()
            apic_sort(self.s)  # particle data changed outside the library: re-bin

    # --- the path -----------------------------------------------------------
    def sort(self):
        apic_sort(self.s)

    def p2g(self):
        apic_p2g(self.s)

    def grid_update(self):
        apic_grid_update(self.s)

    def g2p(self):
        apic_g2p(self.s)

    def step(self, n_steps=1, sort_every=0):
        apic_step([self.s], n_steps, sort_every)

    def step_midpoint(self, n_steps=1, **opts):
        """Implicit midpoint steps (needs ``midpoint=True``); solver stats."""
        return apic_step_midpoint(self.s, n_steps, **opts)

    # --- observation (copies to host) ---------------------------------------
    @property
    def node_shape(self):
        return tuple(c + 1 for c in self.host.cells)

    def export(self, field):
        """Grid field as a host array [nodes, comps] in the oracle's node order."""
        nodes = int(np.prod(self.node_shape))
        comps = 1 if field == APIC_GRID_MASS else self.dim
        out = torch.empty(comps * nodes, dtype=self.dtype, device=self.f.device)
        apic_grid_export(self.s, field, out.data_ptr())
        a = out.cpu().numpy().astype(np.float64).reshape(comps, nodes).T
        return a[:, 0] if comps == 1 else a

    def diagnostics(self, which=APIC_DIAG_PARTICLES):
        return apic_diagnostics(self.s, which)

    def cfl_dt(self, nu=1.0):
        """Largest dt the CFL rule of Sec. 4.3 admits for the current state."""
        return apic_cfl_dt(self.s, nu)

    def step_time(self):
        """(dt of the last adaptive step, time advanced by adaptive steps)."""
        return apic_step_time(self.s)

    def flags(self):
        return apic_get_flags(self.s)

    def clear_flags(self):
        apic_clear_flags(self.s)

    def state(self, raw=False):
        """Particle state on the host: cell [n,dim], off, x (float64 absolute),
        v, B [n,d,d], F [n,d,d], m, id.  The library keeps particles binned
        (it reorders them); unless `raw`, rows are returned in id order, i.e.
        in the order the scene was uploaded."""
        d, n = self.dim, self.n
        f = self.f[:, :n].cpu().numpy().astype(np.float64)
        cell = unpack_cells(self.cell[:n].cpu().numpy().view(np.uint32), d)
        if not raw and self.id is not None:
            ids = self.id[:n].cpu().numpy()
            order = np.empty(n, dtype=np.int64)
            order[ids] = np.arange(n)
            f = f[:, order]
            cell = cell[order]
        off = f[0:d].T.copy()
        if self.absolute:
            # the position planes hold the coordinates
            x = off
            off = x / self.host.dx - cell
        else:
            x = (cell.astype(np.float64) + off) * self.host.dx
        out = {
            "cell": cell,
            "off": off,
            "x": x,
            "v": f[d:2 * d].T.copy(),
            "B": f[2 * d:2 * d + d * d].T.reshape(n, d, d).copy(),
            "F": f[2 * d + d * d:2 * d + 2 * d * d].T.reshape(n, d, d).copy(),
            "m": f[2 * d + 2 * d * d].copy(),
        }
        if self.id is not None:
            ids = self.id[:n].cpu().numpy().copy()
            out["id"] = np.sort(ids) if not raw else ids
        return out


class SceneBatch:
    """Device scenes advanced together by apic_step_batch (one launch per
    phase for all of them).  Owns the batch workspace (the scene table)."""

    def __init__(self, device_scenes, device="cuda"):
        self.scenes = list(device_scenes)
        self.bbytes = apic_batch_workspace_bytes(len(self.scenes))
        self.bws = torch.empty(self.bbytes + 256, dtype=torch.uint8, device=device)
        self.bptr = (self.bws.data_ptr() + 255) // 256 * 256

    def step(self, n_steps=1, stream=None):
        apic_step_batch([d.s for d in self.scenes], n_steps, self.bptr, self.bbytes, stream)

    def tuning(self):
        """(chosen launch plan or -1, ns per particle-step of each plan)."""
        return apic_batch_tuning([d.s for d in self.scenes])

    def step_each(self, n_steps=1, stream=None):
        """The same steps as one apic_step call over the scenes (per-scene
        kernel launches, one scene after the other)."""
        apic_step([d.s for d in self.scenes], n_steps, 0, stream)
