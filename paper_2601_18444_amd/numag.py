"""Thin Python binding of the numag C ABI (include/numag.h).

Argument marshalling only: every numerical step runs in the HIP kernels of
``libnumag.so``.  Device arrays are torch tensors (float64, contiguous) on the
current HIP device; work is enqueued on torch's current stream.  There is no
CPU fallback: if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnumag.so")

OBSERVABLES = ("N", "M", "NM", "P", "CHI", "SF", "PP", "MM", "PM", "MP", "PLUS", "MINUS", "UNPOL")
GRID_CARTESIAN, GRID_POLAR = 0, 1
PATH_DIRECT, PATH_SEPARABLE_F64, PATH_SEPARABLE_BF16X3, PATH_DIRECT_HERMITIAN, PATH_SEPARABLE_BF16X6 = 0, 1, 2, 3, 4
PATH_SEPARABLE_F64_HERMITIAN = 5
MODE_COHERENT, MODE_DILUTE, MODE_SPLIT = 0, 1, 2
OK, E_INVALID, E_WORKSPACE, E_HIP, E_UNSUPPORTED = 0, -1, -2, -4, -5


class NumagError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


class Regular(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("reserved", ctypes.c_int32),
                ("origin", ctypes.c_double * 3), ("step", ctypes.c_double * 3)]


class CSample(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("pos", ctypes.c_void_p), ("nuc", ctypes.c_void_p),
                ("mag", ctypes.c_void_p), ("n_objects", ctypes.c_int64), ("obj_offsets", ctypes.c_void_p),
                ("obj_pos", ctypes.c_void_p), ("regular", ctypes.c_void_p)]


class QGrid(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n0", ctypes.c_int32), ("n1", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("qmax", ctypes.c_double)]

    @property
    def n_pixels(self) -> int:
        return int(self.n0) * int(self.n1)


class Consts(ctypes.Structure):
    _fields_ = [("V", ctypes.c_double), ("bH", ctypes.c_double), ("scale", ctypes.c_double),
                ("P", ctypes.c_double * 3)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2601_18444_amd.build` "
                          "(the HIP library is required; there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, d, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                               ctypes.c_double, ctypes.c_size_t)
    sig = {
        "numag_workspace_size": (sz, [P, i64, P, i32, i32]),
        "numag_amplitudes": (ctypes.c_int, [P, i64, P, P, i32, i32, i32, P, P, P, sz, P]),
        "numag_cross_section": (ctypes.c_int, [P, i64, P, P, P, u32, P, P]),
        "numag_azimuthal_average": (ctypes.c_int, [P, P, i32, i32, d, P, P, P]),
        "numag_correlation": (ctypes.c_int, [P, P, i32, i32, P, i32, d, P, P, P]),
        "numag_grad": (ctypes.c_int, [P, P, P, P, P, P, P, P, P, P, P, sz, P]),
        "numag_grad_path": (ctypes.c_int, [P, P, P, i32, P, P, P, P, P, P, P, P, sz, P]),
        "numag_amplitudes_noalloc": (ctypes.c_int, [P, i64, P, P, i32, P, P]),
        "numag_plan_create": (ctypes.c_int, [P, i64, P, P, i32, i32, i32, P]),
        "numag_plan_workspace_size": (sz, [P]),
        "numag_plan_upload": (ctypes.c_int, [P, P, sz, P]),
        "numag_amplitudes_plan": (ctypes.c_int, [P, P, P, P, P, sz, P]),
        "numag_plan_destroy": (None, [P]),
        "numag_correlation_2d_workspace_size": (sz, [P, P]),
        "numag_correlation_2d": (ctypes.c_int, [P, P, i32, P, P, P, sz, P]),
        "numag_angular_spectrum": (ctypes.c_int, [P, P, i32, i32, P, P, P, P, P]),
        "numag_spectral_matrix": (ctypes.c_int, [P, i64, P, P, P]),
        "numag_snapshots_workspace_size": (sz, [P, i64, P, i32]),
        "numag_amplitudes_snapshots": (ctypes.c_int, [P, i64, P, P, P, i32, P, P, sz, P]),
        "numag_tune_get": (ctypes.c_int, [i32, P, i32, i64, P, P]),
        "numag_tune_set": (ctypes.c_int, [i32, P, i32, i64, P]),
        "numag_tune_clear": (ctypes.c_int, []),
        "numag_autotune": (ctypes.c_int, [P, i64, P, P, i32, i32, i64, P, P]),
        "numag_kernel_timer": (ctypes.c_int, [i32]),
        "numag_kernel_timer_read": (ctypes.c_int, [i32, P, P]),
        "numag_last_error": (ctypes.c_char_p, []),
        "numag_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def last_error() -> str:
    return _lib.numag_last_error().decode()


def version() -> str:
    return _lib.numag_version().decode()


def _check(fn, rc):
    if rc != OK:
        raise NumagError(fn, rc, last_error())


KERNEL_DIRECT, KERNEL_ADJOINT, KERNEL_OBJECTS = 0, 1, 2


def kernel_timer(enable: bool) -> None:
    """Enable (and clear) or disable the library's per-launch kernel timer."""
    _check("numag_kernel_timer", _lib.numag_kernel_timer(1 if enable else 0))


def kernel_timer_read(kernel: int):
    """(summed milliseconds, launches) of the recorded launches of `kernel`; waits for them."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check("numag_kernel_timer_read", _lib.numag_kernel_timer_read(kernel, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(x, device, shape=None):
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=torch.float64)
    else:
        a = np.asarray(x, dtype=np.float64)
        if not a.flags.writeable:  # read-only views (broadcasts): torch wants a writable buffer
            a = a.copy()
        t = torch.as_tensor(a, device=device)
    t = t.contiguous()
    if shape is not None:
        t = t.reshape(shape)
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


_ws_cache: dict = {}


def workspace(nbytes: int, device) -> torch.Tensor:
    """A cached device workspace of at least nbytes, one per (device, stream): calls
    on one stream run in order and may share it, calls on different streams may
    overlap and must not."""
    dev = torch.device(device)
    key = (str(dev), torch.cuda.current_stream(dev).cuda_stream)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=dev)
        _ws_cache[key] = buf
    return buf


def clear_workspace_cache() -> None:
    """Drop the cached workspaces (the next call allocates exactly what it needs)."""
    _ws_cache.clear()


def qgrid(kind: int, n0: int, n1: int, qmax: float) -> QGrid:
    return QGrid(int(kind), int(n0), int(n1), 0, float(qmax))


def consts(V: float = 1.0, bH: float = 1.0, scale: float = 1.0, P: Sequence[float] = (0.0, 0.0, 1.0)) -> Consts:
    return Consts(float(V), float(bH), float(scale), (ctypes.c_double * 3)(*[float(x) for x in P]))


class Sample:
    """Real-space input (Sec. 3.2) resident on the device."""

    def __init__(self, pos=None, nuc=None, mag=None, obj_offsets=None, obj_pos=None, regular=None,
                 n_points=None, device="cuda"):
        self.device = torch.device(device)
        self.pos = _dev(pos, self.device, (-1, 3)) if pos is not None else None
        self.nuc = _dev(nuc, self.device, (-1,)) if nuc is not None else None
        self.mag = _dev(mag, self.device, (-1, 3)) if mag is not None else None
        self.obj_pos = _dev(obj_pos, self.device, (-1, 3)) if obj_pos is not None else None
        if n_points is None:
            for t in (self.pos, self.nuc, self.mag):
                if t is not None:
                    n_points = t.shape[0]
                    break
        self.n_points = int(n_points or 0)
        if obj_offsets is not None:
            self.offsets = np.ascontiguousarray(obj_offsets, dtype=np.int64)
            self.n_objects = int(self.offsets.size - 1)
        else:
            self.offsets = None
            self.n_objects = 1
        self.regular = None
        if regular is not None:
            self.regular = Regular((ctypes.c_int32 * 3)(*[int(v) for v in regular["n"]]), 0,
                                   (ctypes.c_double * 3)(*[float(v) for v in regular["origin"]]),
                                   (ctypes.c_double * 3)(*[float(v) for v in regular["step"]]))
        self._c = CSample(self.n_points, _ptr(self.pos), _ptr(self.nuc), _ptr(self.mag), self.n_objects,
                          self.offsets.ctypes.data_as(ctypes.c_void_p) if self.offsets is not None else None,
                          _ptr(self.obj_pos),
                          ctypes.cast(ctypes.pointer(self.regular), ctypes.c_void_p) if self.regular else None)

    @property
    def c(self):
        return ctypes.byref(self._c)

    def with_weights(self, nuc=None, mag=None) -> "Sample":
        """Same geometry with other weights (device tensors)."""
        s = Sample.__new__(Sample)
        s.__dict__.update(self.__dict__)
        s.nuc = _dev(nuc, self.device, (-1,)) if nuc is not None else None
        s.mag = _dev(mag, self.device, (-1, 3)) if mag is not None else None
        s._c = CSample(self._c.n_points, self._c.pos, _ptr(s.nuc), _ptr(s.mag), self._c.n_objects,
                       self._c.obj_offsets, self._c.obj_pos, self._c.regular)
        return s


def _rot_array(rot):
    if rot is None:
        return None, 1
    r = np.ascontiguousarray(np.asarray(rot, dtype=np.float64).reshape(-1, 9))
    return r, r.shape[0]


def workspace_size(sample: Sample, grid: QGrid, n_rot=1, path=PATH_DIRECT, mode=MODE_COHERENT) -> int:
    n = _lib.numag_workspace_size(sample.c, int(n_rot), ctypes.byref(grid), int(path), int(mode))
    if n == 0 and last_error():
        raise NumagError("numag_workspace_size", E_INVALID, last_error())
    return int(n)


def amplitudes(sample: Sample, grid: QGrid, rot=None, path=PATH_DIRECT, mode=MODE_COHERENT,
               spec_per_object=False, out=None, spec_out=None, ws: Optional[torch.Tensor] = None):
    """numag_amplitudes.  Returns (amp [n_rot, P, 4, 2] or None, spec [n_spec, P, 16] or None).
    In SPLIT mode amp has one rotation.  `ws` is an optional dedicated workspace."""
    r, n_rot = _rot_array(rot)
    dev = sample.device
    P = grid.n_pixels
    amp = spec = None
    if mode in (MODE_COHERENT, MODE_SPLIT):
        n_amp = n_rot if mode == MODE_COHERENT else 1
        amp = out if out is not None else torch.empty((n_amp, P, 4, 2), dtype=torch.float64, device=dev)
    if mode in (MODE_DILUTE, MODE_SPLIT):
        n_spec = sample.n_objects if spec_per_object else 1
        spec = spec_out if spec_out is not None else torch.empty((n_spec, P, 16), dtype=torch.float64, device=dev)
    if ws is None:
        ws = workspace(workspace_size(sample, grid, n_rot, path, mode), dev)
    rc = _lib.numag_amplitudes(sample.c, n_rot, r.ctypes.data_as(ctypes.c_void_p) if r is not None else None,
                               ctypes.byref(grid), int(path), int(mode), int(bool(spec_per_object)),
                               _ptr(amp), _ptr(spec), _ptr(ws), ws.numel(), _stream())
    _check("numag_amplitudes", rc)
    return amp, spec


def amplitudes_noalloc(sample: Sample, grid: QGrid, rot=None, path=PATH_DIRECT, out=None):
    """numag_amplitudes_noalloc: the coherent sums with the library's static scratch
    (no workspace, nothing allocated by the library).  Returns amp [n_rot, P, 4, 2]."""
    r, n_rot = _rot_array(rot)
    amp = out if out is not None else torch.empty((n_rot, grid.n_pixels, 4, 2), dtype=torch.float64,
                                                  device=sample.device)
    rc = _lib.numag_amplitudes_noalloc(sample.c, n_rot, r.ctypes.data_as(ctypes.c_void_p) if r is not None else None,
                                       ctypes.byref(grid), int(path), _ptr(amp), _stream())
    _check("numag_amplitudes_noalloc", rc)
    return amp


TUNE_DIRECT, TUNE_ADJOINT, TUNE_OBJECTS = 0, 1, 2


class TuneShape(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("target", ctypes.c_int32)]

    def as_tuple(self):
        return int(self.shape), int(self.target)


def tune_get(kernel: int, grid: QGrid, n_points: int, path=PATH_DIRECT):
    """(default (shape, target), shape in use (shape, target), tuned entry in use?)"""
    d, c = TuneShape(), TuneShape()
    rc = _lib.numag_tune_get(int(kernel), ctypes.byref(grid), int(path), int(n_points), ctypes.byref(d),
                             ctypes.byref(c))
    if rc < 0:
        raise NumagError("numag_tune_get", rc, last_error())
    return d.as_tuple(), c.as_tuple(), rc == 1


def tune_set(kernel: int, grid: QGrid, n_points: int, shape=None, path=PATH_DIRECT) -> None:
    """Store (shape, target) for the kernel, detector and point-count class; None removes it."""
    s = None if shape is None else ctypes.byref(TuneShape(int(shape[0]), int(shape[1])))
    _check("numag_tune_set", _lib.numag_tune_set(int(kernel), ctypes.byref(grid), int(path), int(n_points), s))


def tune_clear() -> None:
    _check("numag_tune_clear", _lib.numag_tune_clear())


def autotune(sample: Sample, grid: QGrid, kernel: int = TUNE_DIRECT, rot=None, path=PATH_DIRECT, max_points: int = 0):
    """numag_autotune: time the candidate shapes of `kernel` on this sample and keep the
    fastest.  Returns the chosen (shape, target)."""
    r, n_rot = _rot_array(rot)
    ch = TuneShape()
    rc = _lib.numag_autotune(sample.c, n_rot, r.ctypes.data_as(ctypes.c_void_p) if r is not None else None,
                             ctypes.byref(grid), int(path), int(kernel), int(max_points), ctypes.byref(ch), _stream())
    _check("numag_autotune", rc)
    return ch.as_tuple()


def regular_grid(n, origin, step) -> Regular:
    """A numag_regular descriptor (point j = (ix n1 + iy) n2 + iz at origin + i * step)."""
    return Regular((ctypes.c_int32 * 3)(*[int(v) for v in n]), 0, (ctypes.c_double * 3)(*[float(v) for v in origin]),
                   (ctypes.c_double * 3)(*[float(v) for v in step]))


def amplitudes_snapshots(points: Regular, grid: QGrid, nuc=None, mag=None, path=PATH_SEPARABLE_F64, out=None,
                         device="cuda"):
    """numag_amplitudes_snapshots (loop mode): nuc [B, W] and/or mag [B, W, 3] on the
    regular grid `points`; returns amp [B, P, 4, 2]."""
    dev = torch.device(device)
    W = int(points.n[0]) * int(points.n[1]) * int(points.n[2])

    def batch(x, per):
        # [B, W] / [B, W, 3] or flat; B = 0 passes through (the library refuses it)
        t = _dev(x, dev)
        n = W * per
        if n <= 0 or t.numel() % n != 0:
            raise ValueError("amplitudes_snapshots: weights do not match the grid size")
        return t.reshape((t.numel() // n, W) + ((3,) if per == 3 else ()))

    nt = batch(nuc, 1) if nuc is not None else None
    mt = batch(mag, 3) if mag is not None else None
    if nt is None and mt is None:
        raise ValueError("amplitudes_snapshots: nuc or mag is required")
    B = (nt if nt is not None else mt).shape[0]
    if nt is not None and mt is not None and nt.shape[0] != mt.shape[0]:
        raise ValueError("amplitudes_snapshots: nuc and mag hold different snapshot counts")
    amp = out if out is not None else torch.empty((B, grid.n_pixels, 4, 2), dtype=torch.float64, device=dev)
    nbytes = _lib.numag_snapshots_workspace_size(ctypes.byref(points), B, ctypes.byref(grid), int(path))
    if nbytes == 0:
        raise NumagError("numag_snapshots_workspace_size", E_INVALID, last_error())
    ws = workspace(nbytes, dev)
    rc = _lib.numag_amplitudes_snapshots(ctypes.byref(points), B, _ptr(nt), _ptr(mt), ctypes.byref(grid), int(path),
                                         _ptr(amp), _ptr(ws), ws.numel(), _stream())
    _check("numag_amplitudes_snapshots", rc)
    return amp


class Plan:
    """numag_plan_*: an object-mode (DILUTE / SPLIT) plan of a sample's object
    offsets and a set of rotations, uploaded once into its own workspace; calls
    then enqueue kernels only.  The sample's device arrays are read at call time.
    Calls that may overlap (on different streams) each need a workspace of their
    own: upload(ws) into it and pass ws= to the call."""

    def __init__(self, sample: Sample, grid: QGrid, rotations=None, mode: int = MODE_DILUTE,
                 spec_per_object: bool = True, path: int = PATH_DIRECT):
        r, n_rot = _rot_array(rotations)
        self.sample, self.grid, self.mode, self.n_rot = sample, grid, mode, n_rot
        self.spec_per_object = spec_per_object
        self._rot = r
        h = ctypes.c_void_p()
        rc = _lib.numag_plan_create(sample.c, n_rot, r.ctypes.data_as(ctypes.c_void_p) if r is not None else None,
                                    ctypes.byref(grid), int(path), int(mode), int(bool(spec_per_object)),
                                    ctypes.byref(h))
        _check("numag_plan_create", rc)
        self._h = h
        nws = _lib.numag_plan_workspace_size(self._h)
        self.ws = torch.empty(max(int(nws), 256), dtype=torch.uint8, device=sample.device)

    def upload(self, ws: Optional[torch.Tensor] = None) -> None:
        """Enqueue the copy of the plan's tables into `ws` (default: its own workspace)."""
        w = self.ws if ws is None else ws
        _check("numag_plan_upload", _lib.numag_plan_upload(self._h, _ptr(w), w.numel(), _stream()))

    def __call__(self, sample: Optional[Sample] = None, spec_out=None, amp_out=None,
                 ws: Optional[torch.Tensor] = None):
        """numag_amplitudes_plan: returns (amp [1, P, 4, 2] or None, spec [n_spec, P, 16])."""
        s = self.sample if sample is None else sample
        w = self.ws if ws is None else ws
        P = self.grid.n_pixels
        n_spec = s.n_objects if self.spec_per_object else 1
        spec = spec_out if spec_out is not None else torch.empty((n_spec, P, 16), dtype=torch.float64,
                                                                 device=s.device)
        amp = None
        if self.mode == MODE_SPLIT:
            amp = amp_out if amp_out is not None else torch.empty((1, P, 4, 2), dtype=torch.float64, device=s.device)
        rc = _lib.numag_amplitudes_plan(self._h, s.c, _ptr(amp), _ptr(spec), _ptr(w), w.numel(), _stream())
        _check("numag_amplitudes_plan", rc)
        return amp, spec

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            try:
                torch.cuda.synchronize()  # an upload may still read the plan's host tables
            except Exception:  # interpreter shutdown
                pass
            _lib.numag_plan_destroy(h)
            self._h = None


class BatchedOrientations:
    """Orientational average of a dilute sample (Sec. 3.3 dilute limit) over many
    sample rotations, recorded once into a HIP graph and replayed.  A plan holds
    the rotations and object offsets; its tables are uploaded once, and the graph
    records the plan's kernels (one persistent launch over (object, rotation range,
    pixel block) work items, on either detector kind).

    The graph reads the sample's device arrays at replay time, so weights may
    be updated in place between replays; rotations and object offsets are fixed
    at construction.  path=PATH_DIRECT_HERMITIAN sums half of a symmetric
    detector and completes the spectral matrices by G(-q) = conj G(q)."""

    def __init__(self, sample: Sample, grid: QGrid, rotations, spec_per_object: bool = True, path: int = PATH_DIRECT):
        self.sample, self.grid, self.path = sample, grid, path
        self.plan = Plan(sample, grid, rotations, mode=MODE_DILUTE, spec_per_object=spec_per_object, path=path)
        dev = sample.device
        n_spec = sample.n_objects if spec_per_object else 1
        self.spec = torch.empty((n_spec, grid.n_pixels, 16), dtype=torch.float64, device=dev)
        self.plan.upload()
        self._call()
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._call()

    def _call(self):
        self.plan(spec_out=self.spec)

    def eager(self) -> torch.Tensor:
        self._call()
        return self.spec

    def replay(self) -> torch.Tensor:
        self.graph.replay()
        return self.spec


def obs_mask(obs: Iterable[str]) -> int:
    m = 0
    for o in obs:
        m |= 1 << OBSERVABLES.index(o)
    return m


def cross_section(grid: QGrid, amp=None, spec=None, c: Optional[Consts] = None, obs=("UNPOL",), out=None):
    """numag_cross_section.  Returns [n_sets, n_obs, P] in the bit order of `obs`."""
    c = c if c is not None else consts()
    src = amp if amp is not None else spec
    P = grid.n_pixels
    n_sets = src.numel() // (P * (8 if amp is not None else 16))
    mask = obs_mask(obs)
    n_obs = bin(mask).count("1")
    res = out if out is not None else torch.empty((n_sets, n_obs, P), dtype=torch.float64, device=src.device)
    rc = _lib.numag_cross_section(ctypes.byref(grid), n_sets, _ptr(amp), _ptr(spec), ctypes.byref(c), mask,
                                  _ptr(res), _stream())
    _check("numag_cross_section", rc)
    return res


def spectral_matrix(grid: QGrid, amp: torch.Tensor, out=None):
    """numag_spectral_matrix: G = A A^H per amplitude set, [n_sets, P, 16] packed."""
    a = amp.reshape(-1, grid.n_pixels, 4, 2)
    if not a.is_contiguous():
        raise ValueError("spectral_matrix: amp must be contiguous")
    G = out if out is not None else torch.empty((a.shape[0], grid.n_pixels, 16), dtype=torch.float64,
                                                device=a.device)
    _check("numag_spectral_matrix", _lib.numag_spectral_matrix(ctypes.byref(grid), a.shape[0], _ptr(a), _ptr(G),
                                                                _stream()))
    return G


def ordered(obs: Iterable[str]):
    """Observable names in the row order numag_cross_section writes them."""
    s = set(obs)
    return [o for o in OBSERVABLES if o in s]


def azimuthal_average(grid: QGrid, f: torch.Tensor, n_bins: int, qmax_avg: Optional[float] = None,
                      out=None, count_out=None):
    """numag_azimuthal_average.  f is [n_f, P]; returns (I [n_f, n_bins], count [n_bins] int64)."""
    f2 = f.reshape(-1, grid.n_pixels)
    if not f2.is_contiguous():
        f2 = f2.contiguous()
    n_f = f2.shape[0]
    I = out if out is not None else torch.empty((n_f, n_bins), dtype=torch.float64, device=f.device)
    cnt = count_out if count_out is not None else torch.empty(n_bins, dtype=torch.int64, device=f.device)
    qa = float(grid.qmax if qmax_avg is None else qmax_avg)
    rc = _lib.numag_azimuthal_average(ctypes.byref(grid), _ptr(f2), n_f, int(n_bins), qa, _ptr(I), _ptr(cnt),
                                      _stream())
    _check("numag_azimuthal_average", rc)
    return I, cnt


def correlation(q: torch.Tensor, I: torch.Tensor, r: torch.Tensor, scale: float = 1.0, c_out=None, p_out=None):
    """numag_correlation.  I is [n_f, n_q]; returns (c, p) [n_f, n_r]."""
    I2 = I.reshape(-1, q.numel()).contiguous()
    n_f = I2.shape[0]
    c = c_out if c_out is not None else torch.empty((n_f, r.numel()), dtype=torch.float64, device=I.device)
    p = p_out if p_out is not None else torch.empty_like(c)
    rc = _lib.numag_correlation(_ptr(q), _ptr(I2), q.numel(), n_f, _ptr(r), r.numel(), float(scale), _ptr(c),
                                _ptr(p), _stream())
    _check("numag_correlation", rc)
    return c, p


def correlation_2d(grid: QGrid, f: torch.Tensor, rgrid: QGrid, out=None):
    """numag_correlation_2d (eq. crav2d).  f is [n_f, P] on `grid`; returns complex
    [n_f, R, 2] on the real-space grid `rgrid` (its qmax is r_max)."""
    f2 = f.reshape(-1, grid.n_pixels).contiguous()
    n_f = f2.shape[0]
    C = out if out is not None else torch.empty((n_f, rgrid.n_pixels, 2), dtype=torch.float64, device=f.device)
    nws = _lib.numag_correlation_2d_workspace_size(ctypes.byref(grid), ctypes.byref(rgrid))
    if nws == 0:
        raise NumagError("numag_correlation_2d_workspace_size", E_INVALID, last_error())
    ws = workspace(nws, f.device)
    rc = _lib.numag_correlation_2d(ctypes.byref(grid), _ptr(f2), n_f, ctypes.byref(rgrid), _ptr(C), _ptr(ws),
                                   ws.numel(), _stream())
    _check("numag_correlation_2d", rc)
    return C


def angular_spectrum(grid: QGrid, f: torch.Tensor, k_max: int, amplitudes: bool = True):
    """numag_angular_spectrum on a polar detector.  Returns (Is, Ic [n_f, n_q, k_max+1],
    As, Ac [n_f, k_max+1] or None)."""
    f2 = f.reshape(-1, grid.n_pixels).contiguous()
    n_f = f2.shape[0]
    dev = f.device
    Is = torch.empty((n_f, grid.n0, k_max + 1), dtype=torch.float64, device=dev)
    Ic = torch.empty_like(Is)
    As = torch.empty((n_f, k_max + 1), dtype=torch.float64, device=dev) if amplitudes else None
    Ac = torch.empty_like(As) if amplitudes else None
    rc = _lib.numag_angular_spectrum(ctypes.byref(grid), _ptr(f2), n_f, int(k_max), _ptr(Is), _ptr(Ic), _ptr(As),
                                     _ptr(Ac), _stream())
    _check("numag_angular_spectrum", rc)
    return Is, Ic, As, Ac


def grad(sample: Sample, grid: QGrid, c: Consts, weight: torch.Tensor, target: Optional[torch.Tensor] = None,
         rot=None, amp: Optional[torch.Tensor] = None, want_nuc=True, want_mag=True, path=PATH_DIRECT):
    """numag_grad_path.  Returns (loss [1] or None, dnuc [W] or None, dmag [W, 3] or None).
    path=PATH_DIRECT_HERMITIAN runs the sums and the adjoint on half of the detector."""
    r, n_rot = _rot_array(rot)
    if n_rot != 1:
        raise ValueError("grad takes one rotation")
    dev = sample.device
    W = sample.n_points
    loss = torch.empty(1, dtype=torch.float64, device=dev) if target is not None else None
    dn = torch.empty(W, dtype=torch.float64, device=dev) if want_nuc else None
    dm = torch.empty((W, 3), dtype=torch.float64, device=dev) if want_mag else None
    nws = workspace_size(sample, grid, 1, path, MODE_COHERENT)
    ws = workspace(nws, dev)
    rc = _lib.numag_grad_path(sample.c, r.ctypes.data_as(ctypes.c_void_p) if r is not None else None,
                              ctypes.byref(grid), int(path), ctypes.byref(c), _ptr(amp), _ptr(target), _ptr(weight),
                              _ptr(loss), _ptr(dn), _ptr(dm), _ptr(ws), ws.numel(), _stream())
    _check("numag_grad_path", rc)
    return loss, dn, dm


class UnpolarizedCrossSection(torch.autograd.Function):
    """Unpolarized 2D cross section (Sec. 2.4) as a differentiable function of
    the nuclear and magnetic weights; backward is the adjoint Fourier sum.
    path=PATH_DIRECT_HERMITIAN runs the sums and the adjoint on half of a
    symmetric detector."""

    @staticmethod
    def forward(ctx, nuc, mag, sample: Sample, grid: QGrid, c: Consts, rot=None, path=PATH_DIRECT):
        s = sample.with_weights(nuc.detach(), mag.detach())
        amp, _ = amplitudes(s, grid, rot=rot, path=path)
        I = cross_section(grid, amp=amp, c=c, obs=("UNPOL",))[0, 0]
        ctx.sample, ctx.grid, ctx.c, ctx.rot, ctx.path = s, grid, c, rot, path
        ctx.save_for_backward(amp)
        return I

    @staticmethod
    def backward(ctx, gI):
        (amp,) = ctx.saved_tensors
        _, dn, dm = grad(ctx.sample, ctx.grid, ctx.c, weight=gI.contiguous().to(torch.float64), target=None,
                         rot=ctx.rot, amp=amp[0], path=ctx.path)
        return dn, dm, None, None, None, None, None


def unpolarized(nuc, mag, sample: Sample, grid: QGrid, c: Consts, rot=None, path=PATH_DIRECT):
    return UnpolarizedCrossSection.apply(nuc, mag, sample, grid, c, rot, path)
