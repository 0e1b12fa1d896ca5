"""Python binding of libcddt (ctypes).  Argument marshalling only.

Every computation runs in the library's HIP kernels; torch supplies device
buffers (``tensor.data_ptr()``) and the stream (``cuda_stream``).  The binding
refuses to run without the compiled library: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcddt.so")

OK, EINVAL, ENOMEM, EDEVICE, EBUSY, EINTERNAL = 0, -1, -2, -3, -4, -5
FLAG_FULL_MAP = 1
FLAG_STATIC = 2
FLAG_BUCKETS = 4
FLAG_ZP16 = 8
FLAG_PRUNE = 16


def bucket_flags(log2_width: int | None) -> int:
    """Flag bits for a bucket index of 2^log2_width cells (None: no index, 0: the default width)."""
    if log2_width is None:
        return 0
    return FLAG_BUCKETS | (int(log2_width) << 8)


class CddtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libcddt error {code}: {msg}")
        self.code = code


class Stats(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("theta_bins", C.c_int32),
                ("slices", C.c_int32), ("flags", C.c_uint32), ("reserved", C.c_uint32),
                ("rows", C.c_int64), ("edge_cells", C.c_int64), ("zero_points", C.c_int64),
                ("capacity", C.c_int64), ("max_row_len", C.c_int64), ("device_bytes", C.c_int64),
                ("rebuilds", C.c_int64), ("bucket_lines", C.c_int64), ("bucket_overflow", C.c_int64),
                ("bucket_log2", C.c_int32), ("reserved2", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("reserved")}


class Filter(C.Structure):
    _fields_ = [("map", C.c_void_p), ("px", C.c_void_p), ("py", C.c_void_p), ("ptheta", C.c_void_p),
                ("n_particles", C.c_int64), ("ray_offsets", C.c_void_p), ("n_rays", C.c_int32),
                ("pair_offset", C.c_int32), ("obs_ranges", C.c_void_p), ("log_table", C.c_void_p),
                ("max_range", C.c_int32), ("reserved", C.c_int32), ("logw_out", C.c_void_p),
                ("ranges_out", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("particles_per_tile", C.c_int32), ("waves_per_block", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("search_mode", C.c_int32)]

    def as_tuple(self):
        return (self.particles_per_tile, self.waves_per_block, self.blocks_per_cu, self.search_mode)


class ServerConfig(C.Structure):
    _fields_ = [("budget_bytes", C.c_int64), ("n_lanes", C.c_int32), ("max_batch", C.c_int32),
                ("max_rays", C.c_int32), ("resident", C.c_int32), ("tuning", Tuning)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("batches", C.c_int64), ("rays", C.c_int64), ("peak_bytes", C.c_int64),
                ("busy_seconds", C.c_double), ("device_seconds", C.c_double),
                ("max_batch_seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


_lib = None

# name -> (restype, argtypes)
_vp, _i32, _i64, _u32, _f32p = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_void_p
SIGNATURES = {
    "cddt_create": (_i32, [_vp, _i32, _i32, _i32, _u32, _vp, _vp, C.POINTER(_vp)]),
    "cddt_destroy": (_i32, [_vp]),
    "cddt_update": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp]),
    "cddt_cast": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _vp, _vp]),
    "cddt_weight": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp, _i32, _i32, _vp, _vp, _i32, _vp, _vp, _vp]),
    "cddt_pair_offset": (_i32, [_vp, _i32]),
    "cddt_info": (_i32, [_vp, C.POINTER(Stats)]),
    "cddt_slice_table": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "cddt_export": (_i32, [_vp, _vp, _vp, _vp]),
    "cddt_export_grid": (_i32, [_vp, _vp]),
    "cddt_export_buckets": (_i32, [_vp, _vp, _i64]),
    "cddt_plan_create": (_i32, [_vp, _i32, _vp, _vp, C.POINTER(_vp)]),
    "cddt_plan_set_tuning": (_i32, [_vp, C.POINTER(Tuning)]),
    "cddt_plan_get_tuning": (_i32, [_vp, C.POINTER(Tuning)]),
    "cddt_plan_run": (_i32, [_vp, _vp]),
    "cddt_plan_capture": (_i32, [_vp, _vp]),
    "cddt_plan_replay": (_i32, [_vp, _vp]),
    "cddt_plan_time": (_i32, [_vp, C.POINTER(Tuning), _i32, _vp, C.POINTER(C.c_float)]),
    "cddt_plan_run_plain": (_i32, [_vp, _vp]),
    "cddt_plan_destroy": (_i32, [_vp]),
    "cddt_tuning_cache_put": (_i32, [_vp, _i32, C.POINTER(Tuning)]),
    "cddt_tuning_cache_get": (_i32, [_vp, _i32, C.POINTER(Tuning), C.POINTER(_i32)]),
    "cddt_batch_weight": (_i32, [_vp, _i32, _vp, _vp]),
    "cddt_batch_weight_noalloc": (_i32, [_vp, _i32, _vp, _vp]),
    "cddt_device_clock_khz": (_i32, []),
    "cddt_cast_timed": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _vp, _vp, _vp]),
    "cddt_lut_build": (_i32, [_vp, _i32, _vp, _vp]),
    "cddt_lut_cast": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "cddt_march_cast": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _vp, _vp, _vp]),
    "cddt_device_cus": (_i32, []),
    "cddt_probe_gather": (_i32, [_vp, _i64, _i32, _i32, _i32, _u32, _vp, _vp]),
    "cddt_server_create": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, C.POINTER(ServerConfig), C.POINTER(_vp)]),
    "cddt_server_submit": (_i32, [_vp, _i32, _vp, _vp, _vp, _i32, _vp, C.POINTER(_i64)]),
    "cddt_server_replay": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cddt_server_replay_threads": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cddt_motion": (_i32, [_vp, _vp, _vp, _i64, C.c_float, C.c_float, C.c_float, _vp, _vp]),
    "cddt_resample": (_i32, [_vp, _i64, C.c_uint32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cddt_plan_set_mcl": (_i32, [_vp, _vp, _vp, _vp]),
    "cddt_plan_run_mcl": (_i32, [_vp, _vp]),
    "cddt_plan_capture_mcl": (_i32, [_vp, _vp]),
    "cddt_server_poll": (_i32, [_vp, _i64, _vp, C.POINTER(_i32)]),
    "cddt_server_wait": (_i32, [_vp, _i64, _vp]),
    "cddt_server_times": (_i32, [_vp, _i64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "cddt_server_stats_get": (_i32, [_vp, C.POINTER(ServerStats)]),
    "cddt_server_now": (C.c_double, [_vp]),
    "cddt_server_destroy": (_i32, [_vp]),
    "cddt_last_error": (C.c_char_p, []),
}


def lib():
    """Load libcddt.so; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1705_01167_amd/build_lib.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code: int):
    if code != OK:
        raise CddtError(code, lib().cddt_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _need(t, dtype, what, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous {dtype} tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what} must have {numel} elements, has {t.numel()}")


def pair_offset(offsets) -> int:
    a = np.ascontiguousarray(np.asarray(offsets, np.float32))
    return int(lib().cddt_pair_offset(a.ctypes.data_as(C.c_void_p), a.size))


def torch_allocator():
    """A cddt_allocator backed by torch's caching allocator (current device and stream)."""
    import torch

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    a = Allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
    return a


class Map:
    """A CDDT resident on the GPU (cddt_create / cddt_destroy)."""

    def __init__(self, occ, theta_bins: int, full_map: bool = False, static: bool = False,
                 allocator: Allocator | None = None, stream=None, buckets: int | None = None,
                 zp16: bool = False, prune: bool = False):
        """buckets: None for no bucket index, else log2 of the bucket width in cells (0: default 7);
        zp16: 16-bit zero points in the bucket index (the 16-bit reading; needs buckets);
        prune: PCDDT, only the zero points some grid state's cast returns (implies static)."""
        import torch
        _need(occ, torch.uint8, "occ")
        if occ.dim() != 2:
            raise ValueError("occ must be 2-D [height, width]")
        self.height, self.width = int(occ.shape[0]), int(occ.shape[1])
        self.theta_bins = int(theta_bins)
        self._alloc = allocator       # keep callbacks alive
        flags = (FLAG_FULL_MAP if full_map else 0) | (FLAG_STATIC if static else 0) | bucket_flags(buckets)
        flags |= FLAG_ZP16 if zp16 else 0
        flags |= (FLAG_PRUNE | FLAG_STATIC) if prune else 0
        h = C.c_void_p()
        _check(lib().cddt_create(_ptr(occ), self.width, self.height, self.theta_bins, flags,
                                 C.byref(allocator) if allocator is not None else None,
                                 _stream(stream), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().cddt_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- queries -----------------------------------------------------------
    def cast(self, x, y, theta, max_range: int, out=None, stream=None):
        import torch
        n = x.numel()
        for t, w in ((x, "x"), (y, "y"), (theta, "theta")):
            _need(t, torch.float32, w, n)
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=x.device)
        _need(out, torch.int32, "out", n)
        _check(lib().cddt_cast(self.handle, _ptr(x), _ptr(y), _ptr(theta), n, int(max_range), _ptr(out),
                               _stream(stream)))
        return out

    def weight(self, px, py, pth, offsets, obs, log_table, max_range: int, pair: int | None = None,
               logw=None, ranges=False, stream=None):
        import torch
        n = px.numel()
        for t, w in ((px, "px"), (py, "py"), (pth, "ptheta")):
            _need(t, torch.float32, w, n)
        nr = offsets.numel()
        _need(offsets, torch.float32, "ray_offsets")
        _need(obs, torch.int32, "obs_ranges", nr)
        _need(log_table, torch.float32, "log_table", (max_range + 1) ** 2)
        if pair is None:
            pair = pair_offset(offsets.cpu().numpy())
        if logw is None:
            logw = torch.empty(n, dtype=torch.float32, device=px.device)
        rng = torch.empty((n, nr), dtype=torch.int32, device=px.device) if ranges else None
        _check(lib().cddt_weight(self.handle, _ptr(px), _ptr(py), _ptr(pth), n, _ptr(offsets), nr, int(pair),
                                 _ptr(obs), _ptr(log_table), int(max_range), _ptr(logw), _ptr(rng),
                                 _stream(stream)))
        return (logw, rng) if ranges else logw

    def cast_timed(self, x, y, theta, max_range: int, stream=None):
        """(ranges, ticks): cddt_cast_timed; ticks in device wall-clock ticks (device_clock_khz per ms)."""
        import torch
        n = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (theta, "theta")):
            _need(t, torch.float32, nm, n)
        out = torch.empty(n, dtype=torch.int32, device=x.device)
        ticks = torch.empty(n, dtype=torch.int32, device=x.device)
        _check(lib().cddt_cast_timed(self.handle, _ptr(x), _ptr(y), _ptr(theta), n, int(max_range), _ptr(out),
                                     _ptr(ticks), _stream(stream)))
        return out, ticks

    def march(self, x, y, theta, max_range: int, timed: bool = False, stream=None):
        """The cell-walk comparator (cddt_march_cast) on this map's grid: ranges (and ticks when timed)."""
        import torch
        n = x.numel()
        out = torch.empty(n, dtype=torch.int32, device=x.device)
        ticks = torch.empty(n, dtype=torch.int32, device=x.device) if timed else None
        _check(lib().cddt_march_cast(self.handle, _ptr(x), _ptr(y), _ptr(theta), n, int(max_range), _ptr(out),
                                     _ptr(ticks), _stream(stream)))
        return (out, ticks) if timed else out

    def lut(self, max_range: int, stream=None):
        """Dense table [theta_bins, height, width] (uint16 stored in an int16 tensor) of casts from cell centres."""
        import torch
        t = torch.empty((self.theta_bins, self.height, self.width), dtype=torch.int16, device="cuda")
        _check(lib().cddt_lut_build(self.handle, int(max_range), _ptr(t), _stream(stream)))
        return t

    def update(self, xs, ys, values, stream=None):
        xs = np.ascontiguousarray(np.asarray(xs), np.int32)
        ys = np.ascontiguousarray(np.asarray(ys), np.int32)
        vs = np.ascontiguousarray(np.asarray(values), np.uint8)
        if not (xs.size == ys.size == vs.size):
            raise ValueError("xs, ys, values must have the same length")
        _check(lib().cddt_update(self.handle, xs.ctypes.data_as(C.c_void_p), ys.ctypes.data_as(C.c_void_p),
                                 vs.ctypes.data_as(C.c_void_p), xs.size, _stream(stream)))

    # -- inspection ----------------------------------------------------------
    def info(self) -> dict:
        s = Stats()
        _check(lib().cddt_info(self.handle, C.byref(s)))
        return s.as_dict()

    def slice_table(self):
        half = self.theta_bins // 2
        c = np.zeros(half, np.int32)
        s = np.zeros(half, np.int32)
        rmin = np.zeros(half, np.int32)
        nrows = np.zeros(half, np.int32)
        k = np.zeros(1, np.float32)
        _check(lib().cddt_slice_table(self.handle, *(a.ctypes.data_as(C.c_void_p) for a in (c, s, rmin, nrows, k))))
        return c, s, rmin, nrows, k[0]

    def export(self, with_starts: bool = False):
        """(nrows per slice, band lengths, zero points) in canonical order (host numpy); with_starts
        adds the compressed-row offsets (int64[rows + 1]) as a fourth element."""
        st = self.info()
        rl = np.zeros(st["rows"], np.int32)
        zz = np.zeros(max(st["zero_points"], 1), np.int32)
        rs = np.zeros(st["rows"] + 1, np.int64)
        _check(lib().cddt_export(self.handle, rs.ctypes.data_as(C.c_void_p), rl.ctypes.data_as(C.c_void_p),
                                 zz.ctypes.data_as(C.c_void_p)))
        out = (self.slice_table()[3], rl, zz[:st["zero_points"]])
        return out + (rs,) if with_starts else out

    def bucket_lines(self) -> np.ndarray:
        """The bucket index lines, int32[bucket_lines, 32] (the map must have a bucket index)."""
        n = int(self.info()["bucket_lines"])
        out = np.empty((n, 32), np.int32)
        _check(lib().cddt_export_buckets(self.handle, out.ctypes.data_as(C.c_void_p), n * 32))
        return out

    def grid(self) -> np.ndarray:
        g = np.zeros((self.height, self.width), np.uint8)
        _check(lib().cddt_export_grid(self.handle, g.ctypes.data_as(C.c_void_p)))
        return g


def make_filter(m: Map, px, py, pth, offsets, obs, log_table, max_range: int, logw, ranges=None,
                pair: int | None = None) -> Filter:
    if pair is None:
        pair = pair_offset(offsets.cpu().numpy())
    f = Filter()
    f.map = m.handle.value
    f.px, f.py, f.ptheta = px.data_ptr(), py.data_ptr(), pth.data_ptr()
    f.n_particles = px.numel()
    f.ray_offsets = offsets.data_ptr()
    f.n_rays = offsets.numel()
    f.pair_offset = int(pair)
    f.obs_ranges = obs.data_ptr()
    f.log_table = log_table.data_ptr()
    f.max_range = int(max_range)
    f.logw_out = logw.data_ptr()
    f.ranges_out = ranges.data_ptr() if ranges is not None else None
    return f


def motion(px, py, pth, odom, noise, stream=None):
    """Move particles in place (cddt_motion): odom = (dx, dy, dtheta), noise device float32[3n]."""
    n = px.numel()
    _check(lib().cddt_motion(_ptr(px), _ptr(py), _ptr(pth), n, float(odom[0]), float(odom[1]), float(odom[2]),
                             _ptr(noise), _stream(stream)))


def resample(logw, u: int, px, py, pth, stream=None):
    """Systematic resampling (cddt_resample): returns (idx, px', py', pth') as new device tensors."""
    import torch
    n = logw.numel()
    outs = [torch.empty_like(px), torch.empty_like(py), torch.empty_like(pth)]
    idx = torch.empty(n, dtype=torch.int32, device=logw.device)
    _check(lib().cddt_resample(_ptr(logw), n, int(u) & 0xffffffff, _ptr(px), _ptr(py), _ptr(pth),
                               _ptr(outs[0]), _ptr(outs[1]), _ptr(outs[2]), _ptr(idx), _stream(stream)))
    return (idx, *outs)


class Plan:
    """Many filters in one persistent launch (cddt_plan_*)."""

    def __init__(self, filters, tuning: tuple | None = None, stream=None, keepalive=None):
        arr = (Filter * len(filters))(*filters)
        t = Tuning(*tuning) if tuning is not None else None
        h = C.c_void_p()
        _check(lib().cddt_plan_create(C.cast(arr, C.c_void_p), len(filters),
                                      C.byref(t) if t is not None else None, _stream(stream), C.byref(h)))
        self.handle = h
        self.n_filters = len(filters)
        self._arr = arr
        self._keep = keepalive

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().cddt_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def tuning(self):
        t = Tuning()
        _check(lib().cddt_plan_get_tuning(self.handle, C.byref(t)))
        return t.as_tuple()

    @tuning.setter
    def tuning(self, v):
        t = Tuning(*v)
        _check(lib().cddt_plan_set_tuning(self.handle, C.byref(t)))

    def run(self, stream=None):
        _check(lib().cddt_plan_run(self.handle, _stream(stream)))

    def run_plain(self, stream=None):
        _check(lib().cddt_plan_run_plain(self.handle, _stream(stream)))

    def capture(self, stream):
        _check(lib().cddt_plan_capture(self.handle, _stream(stream)))

    def replay(self, stream=None):
        _check(lib().cddt_plan_replay(self.handle, _stream(stream)))

    # -- the whole particle-filter step (motion, weights, resampling) --------
    def set_mcl(self, odom, u, noise):
        """odom: device float32[3F]; u: device int32/uint32[F]; noise: device float32[3P] (kept alive here)."""
        self._mcl = (odom, u, noise)
        _check(lib().cddt_plan_set_mcl(self.handle, _ptr(odom), _ptr(u), _ptr(noise)))

    def run_mcl(self, stream=None):
        _check(lib().cddt_plan_run_mcl(self.handle, _stream(stream)))

    def capture_mcl(self, stream):
        _check(lib().cddt_plan_capture_mcl(self.handle, _stream(stream)))

    def time(self, tuning, reps: int = 5, stream=None) -> float:
        t = Tuning(*tuning)
        ms = C.c_float()
        _check(lib().cddt_plan_time(self.handle, C.byref(t), int(reps), _stream(stream), C.byref(ms)))
        return float(ms.value)


def tuning_cache_put(filters, tuning) -> None:
    """Record `tuning` in the library for this filter set (used when no tuning is given)."""
    arr = (Filter * len(filters))(*filters)
    t = Tuning(*tuning)
    _check(lib().cddt_tuning_cache_put(C.cast(arr, C.c_void_p), len(filters), C.byref(t)))


def tuning_cache_get(filters):
    """(tuning the library uses for this filter set when none is given, whether one was recorded)."""
    arr = (Filter * len(filters))(*filters)
    t = Tuning()
    found = C.c_int32()
    _check(lib().cddt_tuning_cache_get(C.cast(arr, C.c_void_p), len(filters), C.byref(t), C.byref(found)))
    return t.as_tuple(), bool(found.value)


def batch_weight(filters, tuning: tuple | None = None, stream=None) -> None:
    """All filters' log-weights in one persistent launch (cddt_batch_weight).

    tuning None: the tuning recorded for this filter set (tuning_cache_put), else
    the library default."""
    arr = (Filter * len(filters))(*filters)
    t = Tuning(*tuning) if tuning is not None else None
    _check(lib().cddt_batch_weight(C.cast(arr, C.c_void_p), len(filters), C.byref(t) if t is not None else None,
                                   _stream(stream)))


def batch_weight_noalloc(filters, tuning: tuple | None = None, stream=None) -> None:
    """batch_weight with the library's fixed device workspace (cddt_batch_weight_noalloc):
    allocates nothing; at most 1024 filters; calls that overlap on one GPU race."""
    arr = (Filter * len(filters))(*filters)
    t = Tuning(*tuning) if tuning is not None else None
    _check(lib().cddt_batch_weight_noalloc(C.cast(arr, C.c_void_p), len(filters),
                                           C.byref(t) if t is not None else None, _stream(stream)))


def lut_cast(lut, x, y, theta, timed: bool = False, stream=None):
    """Lookups in a table from Map.lut: ranges (and ticks when timed)."""
    import torch
    n = x.numel()
    th, h, w = (int(v) for v in lut.shape)
    out = torch.empty(n, dtype=torch.int32, device=x.device)
    ticks = torch.empty(n, dtype=torch.int32, device=x.device) if timed else None
    _check(lib().cddt_lut_cast(_ptr(lut), w, h, th, _ptr(x), _ptr(y), _ptr(theta), n, _ptr(out), _ptr(ticks),
                               _stream(stream)))
    return (out, ticks) if timed else out


def device_clock_khz() -> int:
    return int(lib().cddt_device_clock_khz())


def device_cus() -> int:
    return int(lib().cddt_device_cus())


def probe_gather(gib: float = 4.0, depth: int = 4, steps: int = 64, blocks: int | None = None, reps: int = 3,
                 stream=None) -> dict:
    """Achievable random 128-byte-line gather rate (cddt_probe_gather) over a `gib` GiB buffer."""
    import torch
    nbytes = int(gib * (1 << 30)) // 128 * 128
    buf = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    if blocks is None:
        blocks = device_cus() * 32
    sink = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    s = stream if stream is not None else torch.cuda.current_stream()
    args = (C.c_void_p(buf.data_ptr()), nbytes, int(blocks), int(steps), int(depth))
    _check(lib().cddt_probe_gather(*args, 1, C.c_void_p(sink.data_ptr()), C.c_void_p(s.cuda_stream)))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for r in range(reps):
        _check(lib().cddt_probe_gather(*args, 2 + r, C.c_void_p(sink.data_ptr()), C.c_void_p(s.cuda_stream)))
    e1.record(s)
    s.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    lines = blocks * 256 // 8 * steps * depth
    del buf
    return {"lines_per_s": lines / sec, "GBps": lines * 128 / sec / 1e9, "buffer_GiB": gib, "depth": depth,
            "blocks": blocks, "steps": steps}


class Server:
    """Continuous-batching server over resident maps (cddt_server_*)."""

    def __init__(self, maps, offsets, tables, max_ranges, budget_bytes: int = 1 << 30, n_lanes: int = 1,
                 max_batch: int = 256, tuning=(8, 4, 2, 7), resident: bool = False):
        """resident: one persistent kernel fed through a ring of max_batch slots (n_lanes must be 1)."""
        n = len(maps)
        self._offsets = [np.ascontiguousarray(np.asarray(o, np.float32)) for o in offsets]
        self._tables = list(tables)              # keep device tables alive
        self._maps = list(maps)
        self._n_rays = [o.size for o in self._offsets]
        cfg = ServerConfig(int(budget_bytes), int(n_lanes), int(max_batch), int(max(self._n_rays)),
                           1 if resident else 0, Tuning(*tuning))
        handles = (C.c_void_p * n)(*[m.handle.value for m in maps])
        offp = (C.c_void_p * n)(*[o.ctypes.data for o in self._offsets])
        nr = (C.c_int32 * n)(*self._n_rays)
        tabs = (C.c_void_p * n)(*[t.data_ptr() for t in tables])
        mr = (C.c_int32 * n)(*[int(v) for v in max_ranges])
        h = C.c_void_p()
        _check(lib().cddt_server_create(C.cast(handles, C.c_void_p), n, C.cast(offp, C.c_void_p),
                                        C.cast(nr, C.c_void_p), C.cast(tabs, C.c_void_p), C.cast(mr, C.c_void_p),
                                        C.byref(cfg), C.byref(h)))
        self.handle = h
        self._sizes = {}

    def submit(self, map_index: int, px, py, pth, obs) -> int:
        px = np.ascontiguousarray(px, np.float32)
        py = np.ascontiguousarray(py, np.float32)
        pth = np.ascontiguousarray(pth, np.float32)
        obs = np.ascontiguousarray(obs, np.int32)
        if obs.size != self._n_rays[map_index]:
            raise ValueError("obs must hold one range per ray of the map")
        rid = C.c_int64()
        _check(lib().cddt_server_submit(self.handle, int(map_index), px.ctypes.data_as(C.c_void_p),
                                        py.ctypes.data_as(C.c_void_p), pth.ctypes.data_as(C.c_void_p), px.size,
                                        obs.ctypes.data_as(C.c_void_p), C.byref(rid)))
        self._sizes[rid.value] = px.size
        return rid.value

    def replay(self, reqs, at, threads: int = 1):
        """Open-loop replay: request i = (map, px, py, pth, obs) submitted at[i] s after the call starts,
        from `threads` submitting threads (request i by thread i mod threads).

        Returns the request ids (-1 where refused); srv.times(id)[0] is the scheduled arrival."""
        n = len(reqs)
        keep = []
        arr = {k: (C.c_void_p * n)() for k in ("px", "py", "pth", "obs")}
        maps = np.zeros(n, np.int32)
        counts = np.zeros(n, np.int32)
        for i, (m, px, py, pth, obs) in enumerate(reqs):
            a = [np.ascontiguousarray(px, np.float32), np.ascontiguousarray(py, np.float32),
                 np.ascontiguousarray(pth, np.float32), np.ascontiguousarray(obs, np.int32)]
            if a[3].size != self._n_rays[m]:
                raise ValueError("obs must hold one range per ray of the map")
            keep.append(a)
            maps[i], counts[i] = m, a[0].size
            for k, v in zip(("px", "py", "pth", "obs"), a):
                arr[k][i] = v.ctypes.data
        at = np.ascontiguousarray(at, np.float64)
        ids = np.full(n, -1, np.int64)
        t0 = time.perf_counter()
        _check(lib().cddt_server_replay_threads(self.handle, int(threads), n, maps.ctypes.data_as(C.c_void_p),
                                                counts.ctypes.data_as(C.c_void_p), C.cast(arr["px"], C.c_void_p),
                                                C.cast(arr["py"], C.c_void_p), C.cast(arr["pth"], C.c_void_p),
                                                C.cast(arr["obs"], C.c_void_p), at.ctypes.data_as(C.c_void_p),
                                                ids.ctypes.data_as(C.c_void_p)))
        self.last_replay_seconds = time.perf_counter() - t0  # the native submission loop alone
        for i, rid in enumerate(ids.tolist()):
            if rid >= 0:
                self._sizes[rid] = int(counts[i])
        return ids

    def poll(self, rid: int):
        out = np.empty(self._sizes[rid], np.float32)
        done = C.c_int32()
        _check(lib().cddt_server_poll(self.handle, int(rid), out.ctypes.data_as(C.c_void_p), C.byref(done)))
        if done.value:
            del self._sizes[rid]
            return out
        return None

    def wait(self, rid: int):
        out = np.empty(self._sizes[rid], np.float32)
        _check(lib().cddt_server_wait(self.handle, int(rid), out.ctypes.data_as(C.c_void_p)))
        del self._sizes[rid]
        return out

    def times(self, rid: int):
        a, b = C.c_double(), C.c_double()
        _check(lib().cddt_server_times(self.handle, int(rid), C.byref(a), C.byref(b)))
        return a.value, b.value

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().cddt_server_stats_get(self.handle, C.byref(s)))
        return s.as_dict()

    def now(self) -> float:
        return float(lib().cddt_server_now(self.handle))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().cddt_server_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
