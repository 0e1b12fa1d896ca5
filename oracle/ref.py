"""ctypes front end of the plain C++ CDDT oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cddt_ref.cpp")
LIB = os.path.join(HERE, "libcddt_ref.so")


SRC_MCL = os.path.join(HERE, "mcl_ref.c")


def _compile(out: str, extra: list[str]) -> str:
    tmp = out + ".tmp"
    obj = out + ".mcl.o"
    subprocess.run(["gcc", "-std=c11", "-O2", *extra, "-ffp-contract=off", "-fPIC", "-c", SRC_MCL, "-o", obj],
                   check=True)
    cmd = ["g++", "-std=c++17", "-O2", *extra, "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
           SRC, obj, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.remove(obj)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with the host compilers (no GPU code involved)."""
    if force or not os.path.exists(LIB):
        _compile(LIB, [])
    return LIB


def select_native() -> str:
    """Load an oracle library compiled for this host's CPU (-O2 -march=native),
    built in a temporary directory, for timing the CPU baseline on the machine
    that runs it; the portable build in this directory stays the one the tests
    load.  Must come before the first call into the oracle.  Returns the flags
    in use."""
    global LIB
    if _lib is not None:
        return "-O2 -march=native" if LIB.endswith("_native.so") else "-O2"
    try:
        d = tempfile.mkdtemp(prefix="cddt_ref_")
        LIB = _compile(os.path.join(d, "libcddt_ref_native.so"), ["-march=native"])
        return "-O2 -march=native"
    except (OSError, subprocess.CalledProcessError):
        return "-O2"


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.ref_create.restype = vp
        L.ref_create.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32]
        L.ref_destroy.argtypes = [vp]
        L.ref_edge_count.restype = i64
        L.ref_edge_count.argtypes = [vp]
        L.ref_tables.argtypes = [vp, vp, vp, vp, vp, vp]
        L.ref_sizes.argtypes = [vp, vp, vp, vp]
        L.ref_export.argtypes = [vp, vp, vp]
        L.ref_cast.argtypes = [vp, vp, vp, vp, i64, i32, vp, i32]
        L.ref_cast_bruteforce.argtypes = [vp, vp, vp, vp, i64, i32, vp, i32]
        L.ref_weight.argtypes = [vp, vp, vp, vp, i64, vp, vp, i32, vp, i32, vp, vp, i32]
        L.ref_update.restype = i32
        L.ref_update.argtypes = [vp, vp, vp, vp, i64]
        L.ref_det_exp_neg.restype = C.c_double
        L.ref_det_exp_neg.argtypes = [C.c_double]
        L.ref_det_sincos.argtypes = [C.c_double, vp, vp]
        L.ref_motion.argtypes = [vp, vp, vp, i64, C.c_float, C.c_float, C.c_float, vp, vp, vp, vp, vp, vp]
        L.ref_resample.restype = i32
        L.ref_resample.argtypes = [vp, i64, C.c_uint32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.ref_resample_weights.restype = C.c_uint64
        L.ref_resample_weights.argtypes = [vp, i64, vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


class RefCDDT:
    """Plain CDDT built on the host: sorted std::vector rows, std::upper/lower_bound."""

    def __init__(self, occ: np.ndarray, theta_bins: int, full_map: bool = False, threads: int = 1,
                 zp16: bool = False, prune: bool = False):
        """zp16: the 16-bit reading (zero points rounded to 1/8-cell bin centres); prune: the PCDDT
        reading (only the zero points some discrete state's cast returns).  See cddt_ref.cpp."""
        self.occ = np.ascontiguousarray(occ, dtype=np.uint8)
        self.h, self.w = self.occ.shape
        self.n = int(theta_bins)
        self.h_ = lib().ref_create(_p(self.occ), self.w, self.h, self.n, int(full_map), int(threads), int(zp16),
                                   int(prune))
        if not self.h_:
            raise ValueError("invalid oracle arguments")

    def close(self):
        if self.h_:
            lib().ref_destroy(self.h_)
            self.h_ = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def edge_count(self) -> int:
        return int(lib().ref_edge_count(self.h_))

    def tables(self):
        half = self.n // 2
        c = np.zeros(half, np.int64)
        s = np.zeros(half, np.int64)
        rmin = np.zeros(half, np.int64)
        nrows = np.zeros(half, np.int64)
        k = np.zeros(1, np.float32)
        lib().ref_tables(self.h_, _p(c), _p(s), _p(rmin), _p(nrows), _p(k))
        return c, s, rmin, nrows, k[0]

    def sizes(self):
        v = np.zeros(3, np.int64)
        lib().ref_sizes(self.h_, _p(v[0:]), _p(v[1:]), _p(v[2:]))
        return int(v[0]), int(v[1]), int(v[2])

    def export(self):
        """(nrows per slice, row lengths, zero points) in canonical (slice, band) order."""
        rows, zeros, _ = self.sizes()
        rl = np.zeros(rows, np.int32)
        zz = np.zeros(max(zeros, 1), np.int32)
        lib().ref_export(self.h_, _p(rl), _p(zz))
        return self.tables()[3], rl, zz[:zeros]

    def cast(self, x, y, th, max_range: int, threads: int = 1, brute: bool = False) -> np.ndarray:
        x = np.ascontiguousarray(x, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        th = np.ascontiguousarray(th, np.float32)
        out = np.zeros(x.size, np.int32)
        f = lib().ref_cast_bruteforce if brute else lib().ref_cast
        f(self.h_, _p(x), _p(y), _p(th), x.size, int(max_range), _p(out), int(threads))
        return out

    def weight(self, px, py, pth, offsets, obs, log_table, max_range: int, threads: int = 1,
               want_ranges: bool = False):
        px = np.ascontiguousarray(px, np.float32)
        py = np.ascontiguousarray(py, np.float32)
        pth = np.ascontiguousarray(pth, np.float32)
        offsets = np.ascontiguousarray(offsets, np.float32)
        obs = np.ascontiguousarray(obs, np.int32)
        table = np.ascontiguousarray(log_table, np.float32).ravel()
        assert table.size == (max_range + 1) ** 2
        logw = np.zeros(px.size, np.float64)
        ranges = np.zeros(px.size * offsets.size, np.int32) if want_ranges else None
        lib().ref_weight(self.h_, _p(px), _p(py), _p(pth), px.size, _p(offsets), _p(obs),
                         offsets.size, _p(table), int(max_range), _p(logw),
                         _p(ranges) if want_ranges else None, int(threads))
        if want_ranges:
            return logw, ranges.reshape(px.size, offsets.size)
        return logw

    def update(self, xs, ys, vals) -> int:
        xs = np.ascontiguousarray(xs, np.int32)
        ys = np.ascontiguousarray(ys, np.int32)
        vals = np.ascontiguousarray(vals, np.uint8)
        r = lib().ref_update(self.h_, _p(xs), _p(ys), _p(vals), xs.size)
        if r < 0:
            raise ValueError("op off the map")
        for x, y, v in zip(xs.tolist(), ys.tolist(), vals.tolist()):
            self.occ[y, x] = 1 if v else 0
        return r


# ---------------------------------------------------------------------------
# Particle-filter steps around the sensor model (mcl_ref.c)
# ---------------------------------------------------------------------------
def det_exp_neg(x: float) -> float:
    return float(lib().ref_det_exp_neg(float(x)))


def det_sincos(a: float):
    s, c = C.c_double(), C.c_double()
    lib().ref_det_sincos(float(a), C.byref(s), C.byref(c))
    return s.value, c.value


def motion(px, py, pth, odom, ex, ey, eth):
    """Move every particle by the robot-frame odometry (dx, dy, dth) plus the given noise."""
    a = [np.ascontiguousarray(v, np.float32) for v in (px, py, pth, ex, ey, eth)]
    n = a[0].size
    out = [np.empty(n, np.float32) for _ in range(3)]
    dx, dy, dth = (float(v) for v in odom)
    lib().ref_motion(_p(a[0]), _p(a[1]), _p(a[2]), n, dx, dy, dth, _p(a[3]), _p(a[4]), _p(a[5]),
                     _p(out[0]), _p(out[1]), _p(out[2]))
    return tuple(out)


def resample_weights(logw):
    """Integer weights q_k and their total T."""
    lw = np.ascontiguousarray(logw, np.float32)
    q = np.zeros(max(lw.size, 1), np.uint64)
    total = int(lib().ref_resample_weights(_p(lw), lw.size, _p(q)))
    return q[:lw.size], total


def resample(logw, u: int, px, py, pth):
    """Systematic resampling: (source index per output, gathered px, py, pth)."""
    lw = np.ascontiguousarray(logw, np.float32)
    n = lw.size
    a = [np.ascontiguousarray(v, np.float32) for v in (px, py, pth)]
    idx = np.full(n, -1, np.int32)
    out = [np.empty(n, np.float32) for _ in range(3)]
    q = np.zeros(max(n, 1), np.uint64)
    r = lib().ref_resample(_p(lw), n, int(u) & 0xffffffff, _p(a[0]), _p(a[1]), _p(a[2]), _p(idx),
                           _p(out[0]), _p(out[1]), _p(out[2]), _p(q))
    if r != 0:
        raise ValueError("resample: n must be in 0..2^20")
    return idx, out[0], out[1], out[2]


# ---------------------------------------------------------------------------
# The cell-walk comparator (Sec. II: Bresenham's line family; here the exact
# traversal of Amanatides and Woo), a comparison system, not CDDT
# ---------------------------------------------------------------------------
def march_cast(occ, x, y, theta, max_range: int) -> int:
    """Range of a ray walked cell by cell along (cos theta, sin theta), theta not binned: the entry distance into
    the first occupied cell the exact ray enters (exact.grid_traversal, ties step in y), rounded half up and capped
    at max_range; max_range if the ray leaves the map first; 0 for a non-finite or |theta| >= 1e6 angle, a position
    off the map, or a position in an occupied cell.  sin and cos from det_sincos (fixed operation order)."""
    import math
    from oracle import exact
    occ = np.asarray(occ)
    h, w = occ.shape
    xf, yf, th = np.float32(x), np.float32(y), np.float32(theta)
    if not (abs(float(th)) < 1e6) or not (0.0 <= xf < w and 0.0 <= yf < h):
        return 0
    px, py = float(xf), float(yf)
    if occ[int(math.floor(py)), int(math.floor(px))]:
        return 0
    s, c = det_sincos(float(th))
    hit = exact.grid_traversal(occ, px, py, c, s)
    if hit is None:
        return int(max_range)
    return min(int(max_range), int(math.floor(hit[0] + 0.5)))
