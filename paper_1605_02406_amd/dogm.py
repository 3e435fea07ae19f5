"""Python binding of libdogm (include/dogm.h): argument marshalling only.

Device memory comes from PyTorch (one uint8 arena tensor per grid) and work is enqueued on
PyTorch's current HIP stream; every step of the filter runs in the library's HIP kernels.
The binding refuses to work without the built library: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdogm.so")

DOGM_OK, DOGM_EINVAL, DOGM_ESIZE, DOGM_EHIP, DOGM_ESTATE, DOGM_ENOTIMPL = 0, -1, -2, -3, -4, -5
ST_CONFLICT, ST_NOCARRIER, ST_NONFINITE, ST_INTERNAL = 1, 2, 4, 8
MODEL_DS, MODEL_PHD_MIB = 0, 1  # Sec. VI (Dempster-Shafer), Sec. V (particle PHD/MIB)
PRECISION_FP32, PRECISION_FP64 = 0, 1  # real-valued arrays in FP32, or everything in FP64

# Names of the functions include/dogm.h declares.
ABI = ["dogm_arena_bytes", "dogm_init_grid", "dogm_destroy", "dogm_set_stream", "dogm_set_cycle",
       "dogm_get_cycle", "dogm_view", "dogm_predict", "dogm_assign", "dogm_update",
       "dogm_moments", "dogm_resample", "dogm_step", "dogm_step_noalloc", "dogm_step_batch",
       "dogm_status_string",
       "dogm_last_error", "dogm_trace_begin", "dogm_trace_end", "dogm_sensor_truth",
       "dogm_sensor_scan"]


class DogmError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_string(code)} ({code})")
        self.code = code


class CParams(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("cell_size", ct.c_float),
                ("dt", ct.c_float), ("p_s", ct.c_float), ("p_b", ct.c_float),
                ("sigma_pos", ct.c_float), ("sigma_vel", ct.c_float),
                ("sigma_birth_vel", ct.c_float), ("alpha_free", ct.c_float),
                ("n_pers", ct.c_int64), ("n_born", ct.c_int64), ("seed", ct.c_uint64),
                ("grid_id", ct.c_uint32), ("model", ct.c_uint32), ("precision", ct.c_uint32),
                ("sort_passes", ct.c_uint32), ("scan_parts", ct.c_uint32),
                ("resample", ct.c_uint32)]


class CMeas(ct.Structure):
    _fields_ = [(k, ct.c_void_p) for k in ("m_occ", "m_free", "p_assoc", "mu_vx", "mu_vy",
                                          "var_v", "p_tp", "p_fp", "det")]


_VIEW_ARRAYS = [  # (name, dtype, length kind)
    ("x", torch.float32, "nu"), ("y", torch.float32, "nu"), ("vx", torch.float32, "nu"),
    ("vy", torch.float32, "nu"), ("w", torch.float32, "nu"), ("key", torch.int32, "nu"),
    ("sx", torch.float32, "nu"), ("sy", torch.float32, "nu"), ("svx", torch.float32, "nu"),
    ("svy", torch.float32, "nu"), ("sw", torch.float32, "nu"), ("skey", torch.int32, "nu"),
    ("perm", torch.int32, "nu"), ("cell_start", torch.int32, "C"),
    ("cell_end", torch.int32, "C"), ("sum_w", torch.float64, "C"),
    ("m_pO", torch.float32, "C"), ("m_pF", torch.float32, "C"), ("m_O", torch.float32, "C"),
    ("m_F", torch.float32, "C"), ("rho_b", torch.float32, "C"), ("rho_p", torch.float32, "C"),
    ("pign", torch.float32, "C"), ("mu_A", torch.float64, "C"), ("mu_UA", torch.float64, "C"),
    ("born_off", torch.int32, "C1"), ("mean_x", torch.float32, "C"),
    ("mean_y", torch.float32, "C"), ("var_x", torch.float32, "C"),
    ("var_y", torch.float32, "C"), ("cov_xy", torch.float32, "C"),
    ("mom_flag", torch.uint8, "C"), ("bx", torch.float32, "nb"), ("by", torch.float32, "nb"),
    ("bvx", torch.float32, "nb"), ("bvy", torch.float32, "nb"), ("bw", torch.float32, "nb"),
    ("bkey", torch.int32, "nb"), ("bassoc", torch.uint8, "nb"), ("status", torch.int32, "1"),
    ("cycle", torch.int32, "1"), ("W_fixed", torch.int64, "1"), ("S_fixed", torch.int64, "1"),
]


class CViews(ct.Structure):
    _fields_ = [(name, ct.c_void_p) for name, _, _ in _VIEW_ARRAYS] + [
        ("n_pers", ct.c_int64), ("n_born", ct.c_int64), ("n_cells", ct.c_int64)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1605_02406_amd.build`")
        L = ct.CDLL(LIB_PATH)
        vp, i = ct.c_void_p, ct.c_int
        L.dogm_arena_bytes.argtypes = [ct.POINTER(CParams), ct.POINTER(ct.c_size_t)]
        L.dogm_init_grid.argtypes = [ct.POINTER(CParams), vp, ct.c_size_t, vp, ct.POINTER(vp)]
        for name in ("dogm_destroy", "dogm_predict", "dogm_assign", "dogm_moments",
                     "dogm_resample"):
            getattr(L, name).argtypes = [vp]
        L.dogm_set_stream.argtypes = [vp, vp]
        L.dogm_set_cycle.argtypes = [vp, ct.c_uint32]
        L.dogm_get_cycle.argtypes = [vp, ct.POINTER(ct.c_uint32)]
        L.dogm_view.argtypes = [vp, ct.POINTER(CViews)]
        L.dogm_update.argtypes = [vp, ct.POINTER(CMeas)]
        L.dogm_step.argtypes = [vp, ct.POINTER(CMeas)]
        L.dogm_step_noalloc.argtypes = [vp, ct.POINTER(CMeas)]
        L.dogm_step_batch.argtypes = [ct.POINTER(vp), ct.POINTER(CMeas), i, vp]
        L.dogm_status_string.argtypes = [i]
        L.dogm_status_string.restype = ct.c_char_p
        L.dogm_last_error.restype = ct.c_char_p
        L.dogm_trace_begin.argtypes = [ct.POINTER(vp), ct.POINTER(ct.c_char_p), i, ct.c_char_p]
        L.dogm_trace_end.argtypes = [ct.POINTER(i)]
        L.dogm_sensor_truth.argtypes = [vp, ct.c_int32, vp, ct.c_int32, ct.c_int32, ct.c_double,
                                        vp, vp]
        L.dogm_sensor_scan.argtypes = [vp, ct.c_int32, ct.c_int32, ct.c_double, ct.c_double,
                                       ct.c_uint64, ct.c_uint32, vp, vp, vp, vp]
        for name in ABI:
            if name not in ("dogm_status_string", "dogm_last_error"):
                getattr(L, name).restype = i
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().dogm_status_string(code).decode()


def _check(code: int, what: str):
    if code != DOGM_OK:
        raise DogmError(code, what)


def make_params(nx, ny, cell_size, n_pers, n_born, dt=0.1, p_s=0.99, p_b=0.02, sigma_pos=0.1,
                sigma_vel=0.5, sigma_birth_vel=4.0, alpha_free=0.9, seed=0, grid_id=0,
                model=MODEL_DS, precision=PRECISION_FP32, sort_passes=0,
                scan_parts=0, resample=0) -> CParams:
    return CParams(nx, ny, cell_size, dt, p_s, p_b, sigma_pos, sigma_vel, sigma_birth_vel,
                   alpha_free, n_pers, n_born, seed, grid_id, model, precision, sort_passes,
                   scan_parts, resample)


def arena_bytes(p: CParams) -> int:
    n = ct.c_size_t()
    _check(lib().dogm_arena_bytes(ct.byref(p), ct.byref(n)), "dogm_arena_bytes")
    return n.value


def _stream_ptr(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Meas:
    """A measurement grid of device tensors (float32, C each): m_occ, m_free (and the optional
    velocity evidence) for the Dempster-Shafer model; p_tp, p_fp, det for the particle PHD/MIB
    model (Sec. V)."""

    def __init__(self, m_occ=None, m_free=None, p_assoc=None, mu_vx=None, mu_vy=None,
                 var_v=None, p_tp=None, p_fp=None, det=None):
        self.t = dict(m_occ=m_occ, m_free=m_free, p_assoc=p_assoc, mu_vx=mu_vx, mu_vy=mu_vy,
                      var_v=var_v, p_tp=p_tp, p_fp=p_fp, det=det)
        for k, v in self.t.items():
            if v is not None:
                assert v.dtype == torch.float32 and v.is_cuda and v.is_contiguous(), k
        self.c = CMeas(*[None if v is None else v.data_ptr() for v in self.t.values()])


class Grid:
    """One filter grid whose whole state lives in a device arena tensor."""

    def __init__(self, params: CParams, device="cuda", stream=None):
        self.params = params
        self.nbytes = arena_bytes(params)
        self.arena = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.stream = stream
        h = ct.c_void_p()
        _check(lib().dogm_init_grid(ct.byref(params), ct.c_void_p(self.arena.data_ptr()),
                                    self.nbytes, ct.c_void_p(_stream_ptr(stream)), ct.byref(h)),
               "dogm_init_grid")
        self.handle = h
        cv = CViews()
        _check(lib().dogm_view(h, ct.byref(cv)), "dogm_view")
        self.nu, self.nb, self.C = cv.n_pers, cv.n_born, cv.n_cells
        base = self.arena.data_ptr()
        sizes = {"nu": self.nu, "nb": self.nb, "C": self.C, "C1": self.C + 1, "1": 1}
        self.v = {}
        real = torch.float64 if params.precision == PRECISION_FP64 else torch.float32
        self.real = real
        for name, dt, kind in _VIEW_ARRAYS:
            if dt == torch.float32:  # the real-valued arrays follow the precision mode
                dt = real
            off = getattr(cv, name) - base
            n = sizes[kind]
            item = torch.empty((), dtype=dt).element_size()
            self.v[name] = self.arena[off:off + n * item].view(dt)
        self._keep = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.dogm_destroy(h)
            self.handle = None

    def _sync_stream(self):
        lib().dogm_set_stream(self.handle, ct.c_void_p(_stream_ptr(self.stream)))

    def predict(self):
        self._sync_stream()
        _check(lib().dogm_predict(self.handle), "dogm_predict")

    def assign(self):
        self._sync_stream()
        _check(lib().dogm_assign(self.handle), "dogm_assign")

    def update(self, meas: Meas):
        self._sync_stream()
        self._keep = meas
        _check(lib().dogm_update(self.handle, ct.byref(meas.c)), "dogm_update")

    def moments(self):
        self._sync_stream()
        _check(lib().dogm_moments(self.handle), "dogm_moments")

    def resample(self):
        self._sync_stream()
        _check(lib().dogm_resample(self.handle), "dogm_resample")

    def step(self, meas: Meas):
        self._sync_stream()
        self._keep = meas
        _check(lib().dogm_step(self.handle, ct.byref(meas.c)), "dogm_step")

    def step_noalloc(self, meas: Meas):
        """The cycle of step() with its per-cycle scratch in the library's static array."""
        self._sync_stream()
        self._keep = meas
        _check(lib().dogm_step_noalloc(self.handle, ct.byref(meas.c)), "dogm_step_noalloc")

    def set_cycle(self, k: int):
        self._sync_stream()
        _check(lib().dogm_set_cycle(self.handle, k), "dogm_set_cycle")

    @property
    def cycle(self) -> int:
        c = ct.c_uint32()
        _check(lib().dogm_get_cycle(self.handle, ct.byref(c)), "dogm_get_cycle")
        return c.value

    def status(self) -> int:
        return int(self.v["status"].item())

    def state(self, sorted_: bool = False) -> dict:
        """Host copies of the particle state (x, y, vx, vy, w) as numpy arrays."""
        names = ("sx", "sy", "svx", "svy", "sw") if sorted_ else ("x", "y", "vx", "vy", "w")
        return {k: self.v[n].cpu().numpy() for k, n in zip(("x", "y", "vx", "vy", "w"), names)}

    def load_state(self, st: dict):
        """Writes a host particle state (x, y, vx, vy, w) into the grid (stream-ordered)."""
        for k in ("x", "y", "vx", "vy", "w"):
            self.v[k].copy_(torch.as_tensor(st[k], dtype=self.real), non_blocking=False)


class KernelTrace:
    """Times every launch of one kernel (or of all kernels) with HIP events on the launch's
    stream while the context is active:

        with dogm.KernelTrace("k_sort_scatter", capacity=256) as tr:
            ...calls...
        torch.cuda.synchronize(); tr.durations_ms()
    """

    def __init__(self, kernel: str | None = None, capacity: int = 1024):
        self.kernel = kernel
        self.cap = capacity
        self.events = [torch.cuda.Event(enable_timing=True) for _ in range(2 * capacity)]
        for e in self.events:  # the HIP event behind a torch event exists after its first record
            e.record()
        torch.cuda.synchronize()
        self._ev = (ct.c_void_p * (2 * capacity))(*[e.cuda_event for e in self.events])
        if not all(self._ev):
            raise RuntimeError("KernelTrace: a torch event has no HIP event behind it")
        self._names = (ct.c_char_p * capacity)()
        # the library keeps the pointer to the name until the trace ends
        self._kname = None if kernel is None else kernel.encode()
        self.count = 0

    def __enter__(self):
        _check(lib().dogm_trace_begin(self._ev, self._names, self.cap, self._kname),
               "dogm_trace_begin")
        return self

    def __exit__(self, *exc):
        n = ct.c_int()
        _check(lib().dogm_trace_end(ct.byref(n)), "dogm_trace_end")
        self.count = n.value
        return False

    def names(self) -> list:
        return [self._names[i].decode() for i in range(self.count)]

    def durations_ms(self) -> list:
        return [self.events[2 * i].elapsed_time(self.events[2 * i + 1]) for i in range(self.count)]


def step_batch(grids: list, meas: list, stream=None):
    """One cycle of several grids with one launch per kernel."""
    n = len(grids)
    hs = (ct.c_void_p * n)(*[g.handle.value for g in grids])
    ms = (CMeas * n)(*[m.c for m in meas])
    for g, m in zip(grids, meas):
        g._keep = m
    _check(lib().dogm_step_batch(hs, ms, n, ct.c_void_p(_stream_ptr(stream))),
           "dogm_step_batch")


def _ptr(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


def sensor_truth(rects, static_occ, nx: int, ny: int, cell: float, occ, stream=None):
    """Truth grid on the device: rects float64 [n, 4] (x0, y0, x1, y1), static_occ uint8 [C] or
    None, occ uint8 [C] (written)."""
    n = 0 if rects is None else int(rects.shape[0])
    _check(lib().dogm_sensor_truth(_ptr(rects), n, _ptr(static_occ), nx, ny, float(cell),
                                   _ptr(occ), ct.c_void_p(_stream_ptr(stream))),
           "dogm_sensor_truth")


def sensor_scan(occ, nx: int, ny: int, p_d: float, p_cl: float, seed: int, cycle: int, seen,
                m_occ=None, m_free=None, stream=None):
    """Ray cast and evidence masses of one cycle on the device (seen uint8 [C], m_occ and
    m_free float32 [C], all written)."""
    _check(lib().dogm_sensor_scan(_ptr(occ), nx, ny, float(p_d), float(p_cl), seed, cycle,
                                  _ptr(seen), _ptr(m_occ), _ptr(m_free),
                                  ct.c_void_p(_stream_ptr(stream))), "dogm_sensor_scan")
