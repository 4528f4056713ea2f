"""CPU oracle for the RTA low-level reconstruction — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It is a plain FP64 / int64 reference of
what the real-time reconstruction computes for every camera event (the paper's
Section 4.1 lists calibration, gamma/hadron separation, energy and direction
reconstruction of the DL0 data; Section 4.2 asks for a reduced, fast variant):

* ``oracle.c`` — calibration / signal extraction, two-level tailcut cleaning,
  islands, Hillas moments, time gradient, leakage and stereo direction, in
  straightforward loops (see the header of that file for each definition).
* ``mlp.py`` — the small gamma/hadron + energy network: forward with bfloat16
  rounding at the storage points, FP64 backward, loss and Adam.

It shares no code with the HIP library (``paper_1307_6489_amd``) and never
imports it.  Inputs come from ``dl0sim`` (the seeded generator) or from test
code.  Parity status of every function is recorded in the design notes: all
are pinned by the ``-m "not gpu"`` tests.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

HILLAS_INVALID = 1
TIME_INVALID = 2
LOW_GAIN = 4
STEREO_INVALID = 1

# signal extractors (window placement)
EX_SLIDING = 0
EX_FIXED = 1
EX_GLOBAL_PEAK = 2
EX_NEIGHBOUR_PEAK = 3


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (plain -O2, no vector intrinsics)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OracleCam(ctypes.Structure):
    _fields_ = [
        ("n_pix", ctypes.c_int32), ("n_pix_pad", ctypes.c_int32), ("n_samp", ctypes.c_int32),
        ("n_gain", ctypes.c_int32), ("window", ctypes.c_int32), ("hg_switch", ctypes.c_int32),
        ("max_nbr", ctypes.c_int32), ("extractor", ctypes.c_int32),
        ("fixed_start", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("ped", ctypes.c_void_p), ("a", ctypes.c_void_p),
        ("nbr", ctypes.c_void_p), ("t_pic", ctypes.c_double), ("t_bnd", ctypes.c_double),
        ("focal", ctypes.c_double),
    ]


PIX_DTYPE = np.dtype([("S", "<i8"), ("D", "<i8"), ("Nt", "<i8"), ("sstar", "<i4"), ("peak", "<i4"),
                      ("gain", "<i4"), ("pad_", "<i4"), ("q", "<f8"), ("t", "<f8")])

HILLAS_FIELDS = ("size", "cog_x", "cog_y", "length", "width", "psi", "skewness", "kurtosis",
                 "time_gradient", "time_intercept", "leakage", "cog_dist")
HILLAS_DTYPE = np.dtype([(f, "<f8") for f in HILLAS_FIELDS]
                        + [("n_pix", "<i8"), ("n_islands", "<i8"), ("n_lowgain", "<i8"), ("flags", "<i8")])


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.oracle_neighbours.argtypes = [i32, vp, vp, dbl, i32, vp]
        L.oracle_neighbours.restype = ctypes.c_int
        L.oracle_calibrate_event.argtypes = [vp, vp, vp]
        L.oracle_clean_event.argtypes = [vp, vp, vp, vp]
        L.oracle_islands.argtypes = [vp, vp]
        L.oracle_islands.restype = i64
        L.oracle_hillas_event.argtypes = [vp, vp, vp, vp, vp, vp]
        L.oracle_reconstruct_event.argtypes = [vp, vp, vp, vp, vp]
        L.oracle_stereo.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.oracle_reconstruct_batch.argtypes = [vp, i64, vp, vp, vp, vp, i32]
        L.oracle_crc16.argtypes = [vp, i64]
        L.oracle_crc16.restype = ctypes.c_uint16
        for f in ("oracle_sizeof_cam", "oracle_sizeof_pix", "oracle_sizeof_hillas"):
            getattr(L, f).restype = ctypes.c_int
        assert L.oracle_sizeof_cam() == ctypes.sizeof(OracleCam)
        assert L.oracle_sizeof_pix() == PIX_DTYPE.itemsize
        assert L.oracle_sizeof_hillas() == HILLAS_DTYPE.itemsize
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def neighbours(x, y, tol, max_nbr=6):
    """Brute-force neighbour lists: j is a neighbour of i iff 0 < |r_i - r_j| <= tol."""
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    nbr = np.empty((len(x), max_nbr), np.int32)
    most = lib().oracle_neighbours(len(x), _p(x), _p(y), float(tol), max_nbr, _p(nbr))
    if most < 0:
        raise ValueError("more than max_nbr neighbours within tol")
    return nbr


class Camera:
    """Oracle view of one camera type.  Takes positions and calibration tables
    (from any source, normally ``dl0sim.CameraType``) and derives its own
    neighbour lists by the O(N^2) distance test with tolerance 1.4 x pitch."""

    def __init__(self, n_pix, n_samp, n_gain, x, y, ped, adc_per_pe, pitch, window=4, hg_switch=4000,
                 t_pic=10.0, t_bnd=5.0, focal=1.0, extractor=EX_SLIDING, fixed_start=None):
        self.n_pix, self.n_samp, self.n_gain = int(n_pix), int(n_samp), int(n_gain)
        self.n_pix_pad = (self.n_pix + 7) // 8 * 8
        self.window, self.hg_switch = int(window), int(hg_switch)
        self.x = np.ascontiguousarray(x, np.float32)
        self.y = np.ascontiguousarray(y, np.float32)
        self.ped = np.ascontiguousarray(np.asarray(ped, np.float32).reshape(self.n_gain, self.n_pix))
        self.a = np.ascontiguousarray(np.asarray(adc_per_pe, np.float32).reshape(self.n_gain, self.n_pix))
        self.nbr = neighbours(self.x, self.y, 1.4 * pitch)
        self.t_pic, self.t_bnd, self.focal = float(t_pic), float(t_bnd), float(focal)
        self.extractor = int(extractor)
        self.fixed_start = (self.n_samp - self.window) // 2 if fixed_start is None else int(fixed_start)
        if self.extractor not in (EX_SLIDING, EX_FIXED, EX_GLOBAL_PEAK, EX_NEIGHBOUR_PEAK):
            raise ValueError("unknown extractor")
        if not 0 <= self.fixed_start <= self.n_samp - self.window:
            raise ValueError("fixed window outside the trace")
        self.c = OracleCam(self.n_pix, self.n_pix_pad, self.n_samp, self.n_gain, self.window, self.hg_switch,
                           self.nbr.shape[1], self.extractor, self.fixed_start, 0, _p(self.x), _p(self.y),
                           _p(self.ped), _p(self.a), _p(self.nbr), self.t_pic, self.t_bnd, self.focal)

    @classmethod
    def from_type(cls, cam, t_pic=10.0, t_bnd=5.0, extractor=EX_SLIDING):
        return cls(cam.n_pix, cam.n_samp, cam.n_gain, cam.geom.x, cam.geom.y, cam.ped, cam.adc_per_pe,
                   cam.pitch, cam.window, cam.hg_switch_adc, t_pic, t_bnd, cam.focal_m, extractor,
                   cam.fixed_start)

    @property
    def event_elems(self):
        return self.n_gain * self.n_samp * self.n_pix_pad

    # -- single-event steps ------------------------------------------------
    def calibrate(self, ev):
        ev = np.ascontiguousarray(ev, np.uint16).reshape(-1)
        assert ev.size == self.event_elems
        out = np.zeros(self.n_pix, PIX_DTYPE)
        lib().oracle_calibrate_event(ctypes.byref(self.c), _p(ev), _p(out))
        return out

    def clean(self, D, gain):
        D = np.ascontiguousarray(D, np.int64)
        g = np.ascontiguousarray(gain, np.int32)
        m = np.zeros(self.n_pix, np.uint8)
        lib().oracle_clean_event(ctypes.byref(self.c), _p(D), _p(g), _p(m))
        return m

    def islands(self, mask):
        m = np.ascontiguousarray(mask, np.uint8)
        return int(lib().oracle_islands(ctypes.byref(self.c), _p(m)))

    def hillas(self, q, t, mask, gain=None):
        q = np.ascontiguousarray(q, np.float64)
        t = np.ascontiguousarray(t, np.float64)
        m = np.ascontiguousarray(mask, np.uint8)
        g = None if gain is None else np.ascontiguousarray(gain, np.int32)
        h = np.zeros(1, HILLAS_DTYPE)
        lib().oracle_hillas_event(ctypes.byref(self.c), _p(q), _p(t), _p(m), _p(g), _p(h))
        return h[0]

    def reconstruct(self, ev):
        ev = np.ascontiguousarray(ev, np.uint16).reshape(-1)
        assert ev.size == self.event_elems
        pix = np.zeros(self.n_pix, PIX_DTYPE)
        mask = np.zeros(self.n_pix, np.uint8)
        h = np.zeros(1, HILLAS_DTYPE)
        lib().oracle_reconstruct_event(ctypes.byref(self.c), _p(ev), _p(pix), _p(mask), _p(h))
        return pix, mask, h[0]


def calibrate_events(cam: Camera, traces):
    """Per-pixel calibration of every event of ``traces`` [E][G][T][Npad]."""
    tr = np.ascontiguousarray(traces, np.uint16).reshape(-1, cam.event_elems)
    return np.stack([cam.calibrate(tr[e]) for e in range(tr.shape[0])]) if tr.shape[0] else \
        np.zeros((0, cam.n_pix), PIX_DTYPE)


def reconstruct_batch(cams, types, blob, offsets, n_threads=1):
    """Hillas records of many camera events: ``types[e]`` indexes ``cams``;
    event ``e``'s trace block starts at element ``offsets[e]`` of ``blob``."""
    types = np.ascontiguousarray(types, np.int32)
    offsets = np.ascontiguousarray(offsets, np.int64)
    blob = np.ascontiguousarray(blob).view(np.uint16).reshape(-1)
    arr = (OracleCam * len(cams))(*[c.c for c in cams])
    out = np.zeros(len(types), HILLAS_DTYPE)
    lib().oracle_reconstruct_batch(arr, len(types), _p(types), _p(blob), _p(offsets), _p(out), int(n_threads))
    return out


def stereo(size, cog_x, cog_y, length, width, psi, valid, focal):
    """Weighted least-squares intersection of the major axes of one array
    event.  Returns (dir_x, dir_y, cond, n_used, flags)."""
    arrs = [np.ascontiguousarray(v, np.float64) for v in (size, cog_x, cog_y, length, width, psi)]
    va = np.ascontiguousarray(valid, np.int32)
    f = np.ascontiguousarray(focal, np.float64)
    out = np.zeros(5, np.float64)
    lib().oracle_stereo(len(va), *[_p(a) for a in arrs], _p(va), _p(f), _p(out))
    return out[0], out[1], out[2], int(out[3]), int(out[4])
