"""dl0sim — seeded synthetic DL0 inputs for the RTA low-level reconstruction.

This package generates *inputs only*: hexagonal camera geometries, per-pixel
pedestal / gain tables, dual-gain uint16 waveform traces of Cherenkov ellipse
images, ragged array events and charge-domain gamma / hadron images.  It plays
the role of the Central Event Builder simulator of the paper (Section 5: the
DL0 stream built from simulated data), which is not available; it contains
none of the reconstruction arithmetic and is shared, as a plain input source,
by the HIP library's tests / benchmark and by the CPU oracle.

Trace layout of one camera event: ``uint16[G][T][Npad]`` (gain, sample,
pixel), ``Npad = round_up(N, 8)``; pad pixels hold 0.

The workload recipes (``C0`` … ``C4``) follow the statement of the problem:
a pitch-0.05 m hexagonal camera, pedestal 300 ADC, electronic noise sigma
5 ADC, night-sky background 0.1 p.e. per 1-ns sample at 10 ADC/p.e. (high
gain), Gaussian pulses of sigma 2 samples with a linear time gradient along
the major axis, 4-sample extraction window, tailcut 10/5 p.e.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dl0sim.c")
_LIB_PATH = os.path.join(_HERE, "libdl0sim.so")
_lib = None

PITCH_M = 0.05
MAX_BLOB = 4


def build(force: bool = True) -> str:
    """Compile the generator with gcc into ``dl0sim/libdl0sim.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _declare(_lib)
        if _lib.dl0sim_shower_size() != SHOWER_DTYPE.itemsize:
            raise RuntimeError("dl0sim shower struct size mismatch")
    return _lib


SHOWER_DTYPE = np.dtype([
    ("n_blob", "<i4"), ("kind", "<i4"), ("energy_tev", "<f4"), ("src_x", "<f4"), ("src_y", "<f4"),
    ("pad_", "<f4", 3),
    ("size", "<f4", MAX_BLOB), ("cog_x", "<f4", MAX_BLOB), ("cog_y", "<f4", MAX_BLOB),
    ("width", "<f4", MAX_BLOB), ("length", "<f4", MAX_BLOB), ("psi", "<f4", MAX_BLOB),
    ("t0", "<f4", MAX_BLOB), ("tgrad", "<f4", MAX_BLOB),
])


class DrawCfg(ctypes.Structure):
    _fields_ = [
        ("size_min", ctypes.c_double), ("size_max", ctypes.c_double),
        ("cog_rmax", ctypes.c_double),
        ("width_min", ctypes.c_double), ("width_max", ctypes.c_double),
        ("lw_min", ctypes.c_double), ("lw_max", ctypes.c_double),
        ("tgrad_max", ctypes.c_double),
        ("t0_center", ctypes.c_double), ("t0_halfwidth", ctypes.c_double),
        ("e_min", ctypes.c_double), ("e_max", ctypes.c_double),
        ("size_per_tev", ctypes.c_double), ("hadron_fraction", ctypes.c_double),
        ("had_width_min", ctypes.c_double), ("had_width_max", ctypes.c_double),
        ("had_lw_min", ctypes.c_double), ("had_lw_max", ctypes.c_double),
        ("had_blobs_max", ctypes.c_int32), ("pad_", ctypes.c_int32),
    ]


class RenderCfg(ctypes.Structure):
    _fields_ = [
        ("n_pix", ctypes.c_int32), ("n_pix_pad", ctypes.c_int32), ("n_samp", ctypes.c_int32),
        ("n_gain", ctypes.c_int32), ("hg_clip", ctypes.c_int32), ("lg_clip", ctypes.c_int32),
        ("n_threads", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("noise_sigma", ctypes.c_double), ("nsb_rate", ctypes.c_double),
        ("pulse_sigma", ctypes.c_double), ("pix_area", ctypes.c_double),
        ("image_window", ctypes.c_double),
    ]


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _declare(L):
    vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    L.dl0sim_camera_geometry.argtypes = [ctypes.c_int, dbl, vp, vp, vp, vp]
    L.dl0sim_camera_geometry.restype = ctypes.c_int
    L.dl0sim_draw_ellipses.argtypes = [ctypes.POINTER(DrawCfg), u64, i64, i64, vp]
    L.dl0sim_draw_ellipses.restype = None
    L.dl0sim_draw_gamma_hadron.argtypes = [ctypes.POINTER(DrawCfg), u64, i64, i64, vp]
    L.dl0sim_draw_gamma_hadron.restype = None
    L.dl0sim_draw_array.argtypes = [ctypes.POINTER(DrawCfg), u64, i64, i64, i32, i32, i32, vp, vp, dbl, i64,
                                    vp, vp, vp, vp]
    L.dl0sim_draw_array.restype = i64
    L.dl0sim_render_traces.argtypes = [ctypes.POINTER(RenderCfg), vp, vp, vp, vp, vp, vp, u64, i64, vp, vp]
    L.dl0sim_render_traces.restype = None
    L.dl0sim_render_images.argtypes = [ctypes.POINTER(RenderCfg), vp, vp, vp, vp, vp, u64, i64, vp, vp, vp]
    L.dl0sim_render_images.restype = None
    L.dl0sim_philox4x32_10.argtypes = [vp, vp, vp]
    L.dl0sim_philox4x32_10.restype = None
    L.dl0sim_shower_size.argtypes = []
    L.dl0sim_shower_size.restype = ctypes.c_int
    L.dl0sim_crc16.argtypes = [vp, i64]
    L.dl0sim_crc16.restype = ctypes.c_uint16
    L.dl0sim_serialize_packets.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp]
    L.dl0sim_serialize_packets.restype = None


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().dl0sim_philox4x32_10(_p(c), _p(k), _p(o))
    return o


# --------------------------------------------------------------------------
# Cameras
# --------------------------------------------------------------------------
def pad_pixels(n_pix: int) -> int:
    return (n_pix + 7) // 8 * 8


def full_hex_count(rings: int) -> int:
    return 1 + 3 * rings * (rings + 1)


@dataclass
class Geometry:
    n_pix: int
    pitch: float
    x: np.ndarray      # float32 [N] metres
    y: np.ndarray      # float32 [N]
    nbr: np.ndarray    # int32 [N][6], -1 padded
    ab: np.ndarray     # int32 [N][2] lattice coordinates


def hex_geometry(n_pix: int, pitch: float = PITCH_M) -> Geometry:
    x = np.zeros(n_pix, np.float32)
    y = np.zeros(n_pix, np.float32)
    nbr = np.zeros((n_pix, 6), np.int32)
    ab = np.zeros((n_pix, 2), np.int32)
    rc = lib().dl0sim_camera_geometry(n_pix, pitch, _p(x), _p(y), _p(nbr), _p(ab))
    if rc != 0:
        raise ValueError("dl0sim_camera_geometry failed (%d)" % rc)
    return Geometry(n_pix, pitch, x, y, nbr, ab)


@dataclass
class CameraType:
    """One camera type: geometry, sampling, and the calibration tables a
    reconstruction receives (pedestal per sample including the NSB mean, ADC
    counts per p.e.), plus the generator's electronic pedestal."""
    name: str
    n_pix: int
    n_samp: int
    n_gain: int
    focal_m: float
    window: int = 4
    hg_switch_adc: int = 4000
    pitch: float = PITCH_M
    adc_per_pe_hg: float = 10.0
    gain_ratio: float = 16.0
    base_pedestal: float = 300.0
    noise_sigma: float = 5.0
    nsb_rate: float = 0.1
    pulse_sigma: float = 2.0
    ped_jitter: float = 0.0        # optional per-pixel pedestal spread (ADC, uniform +-)
    gain_jitter: float = 0.0       # optional per-pixel relative gain spread (uniform +-)
    table_seed: int = 0
    fixed_start: int = -1          # fixed-window readout start; -1: (n_samp - window) // 2
    geom: Geometry = field(default=None, repr=False)
    adc_per_pe: np.ndarray = field(default=None, repr=False)   # float32 [G][N]
    base_ped: np.ndarray = field(default=None, repr=False)     # float32 [G][N]
    ped: np.ndarray = field(default=None, repr=False)          # float32 [G][N] per-sample pedestal table

    def __post_init__(self):
        if self.fixed_start < 0:
            self.fixed_start = (self.n_samp - self.window) // 2
        if self.geom is None:
            self.geom = hex_geometry(self.n_pix, self.pitch)
        G, N = self.n_gain, self.n_pix
        rng = np.random.default_rng(self.table_seed)
        a = np.empty((G, N), np.float64)
        a[0] = self.adc_per_pe_hg
        if G == 2:
            a[1] = self.adc_per_pe_hg / self.gain_ratio
        if self.gain_jitter:
            a *= 1.0 + self.gain_jitter * (2.0 * rng.random((1, N)) - 1.0)
        p = np.full((G, N), self.base_pedestal, np.float64)
        if self.ped_jitter:
            p += self.ped_jitter * (2.0 * rng.random((G, N)) - 1.0)
        self.adc_per_pe = a.astype(np.float32)
        self.base_ped = p.astype(np.float32)
        # the pedestal table a reconstruction subtracts: electronic pedestal plus
        # the mean night-sky background contribution per sample
        self.ped = (self.base_ped.astype(np.float64)
                    + self.adc_per_pe.astype(np.float64) * self.nsb_rate).astype(np.float32)

    @property
    def n_pix_pad(self) -> int:
        return pad_pixels(self.n_pix)

    @property
    def event_elems(self) -> int:
        """uint16 elements of one camera event's trace block (with pixel pad)."""
        return self.n_gain * self.n_samp * self.n_pix_pad

    @property
    def dl0_bytes(self) -> int:
        """Logical DL0 bytes of one camera event: N * T * G * 2."""
        return self.n_pix * self.n_samp * self.n_gain * 2

    @property
    def pix_area(self) -> float:
        return math.sqrt(3.0) / 2.0 * self.pitch ** 2

    @property
    def hg_clip(self) -> int:
        return 4095 if self.n_gain == 2 else 65535


def camera_c0() -> CameraType:
    """1855-pixel camera, 30 samples, single gain (the plain-method parity set)."""
    return CameraType("C0-1855x30", 1855, 30, 1, focal_m=28.0)


def camera_types_c1():
    """The three dual-gain camera types of the throughput mix, weights 1:3:6."""
    return [CameraType("1855x40", 1855, 40, 2, focal_m=28.0),
            CameraType("1764x25", 1764, 25, 2, focal_m=16.0),
            CameraType("2048x128", 2048, 128, 2, focal_m=5.6)]


C1_WEIGHTS = (1.0, 3.0, 6.0)


def draw_cfg_plain(n_samp: int) -> DrawCfg:
    """Ellipse draws of the plain-method configuration: cog uniform in the
    0.8 m disk, psi uniform, width U[0.02, 0.06] m, length U[1.5, 4] x width,
    size log-uniform 50..5000 p.e., t0 within +-2 samples of mid-trace, time
    gradient U[-5, 5] samples/m."""
    c = DrawCfg()
    c.size_min, c.size_max = 50.0, 5000.0
    c.cog_rmax = 0.8
    c.width_min, c.width_max = 0.02, 0.06
    c.lw_min, c.lw_max = 1.5, 4.0
    c.tgrad_max = 5.0
    c.t0_center, c.t0_halfwidth = n_samp / 2.0, 2.0
    c.e_min, c.e_max = 0.03, 100.0
    c.size_per_tev = 1000.0
    c.hadron_fraction = 0.75
    c.had_width_min, c.had_width_max = 0.06, 0.15
    c.had_lw_min, c.had_lw_max = 1.0, 2.0
    c.had_blobs_max = 4
    return c


def draw_ellipses(cfg: DrawCfg, seed: int, first_event: int, n: int) -> np.ndarray:
    out = np.zeros(n, SHOWER_DTYPE)
    lib().dl0sim_draw_ellipses(ctypes.byref(cfg), seed, first_event, n, _p(out))
    return out


def draw_gamma_hadron(cfg: DrawCfg, seed: int, first_event: int, n: int) -> np.ndarray:
    out = np.zeros(n, SHOWER_DTYPE)
    lib().dl0sim_draw_gamma_hadron(ctypes.byref(cfg), seed, first_event, n, _p(out))
    return out


@dataclass
class ArrayDraw:
    evt_tel_off: np.ndarray   # int64 [E+1]
    tel_type: np.ndarray      # int32 [n_tel]
    showers: np.ndarray       # SHOWER_DTYPE [n_tel]
    src_nominal: np.ndarray   # float64 [E][2] radians


def draw_array(cfg: DrawCfg, seed: int, first_event: int, n_evt: int, cams, weights=C1_WEIGHTS,
               mult=(2, 40), src_rmax=0.02) -> ArrayDraw:
    n_types = len(cams)
    w = np.asarray(weights, np.float64)
    f = np.asarray([c.focal_m for c in cams], np.float64)
    cap = n_evt * mult[1]
    off = np.zeros(n_evt + 1, np.int64)
    ty = np.zeros(cap, np.int32)
    sh = np.zeros(cap, SHOWER_DTYPE)
    src = np.zeros((n_evt, 2), np.float64)
    nt = lib().dl0sim_draw_array(ctypes.byref(cfg), seed, first_event, n_evt, mult[0], mult[1], n_types,
                                 _p(w), _p(f), src_rmax, cap, _p(off), _p(ty), _p(sh), _p(src))
    if nt < 0:
        raise RuntimeError("dl0sim_draw_array: capacity exceeded")
    return ArrayDraw(off, ty[:nt].copy(), sh[:nt].copy(), src)


def _render_cfg(cam: CameraType, n_threads: int) -> RenderCfg:
    r = RenderCfg()
    r.n_pix, r.n_pix_pad, r.n_samp, r.n_gain = cam.n_pix, cam.n_pix_pad, cam.n_samp, cam.n_gain
    r.hg_clip, r.lg_clip = cam.hg_clip, 65535
    r.n_threads = n_threads
    r.noise_sigma, r.nsb_rate, r.pulse_sigma = cam.noise_sigma, cam.nsb_rate, cam.pulse_sigma
    r.pix_area = cam.pix_area
    r.image_window = float(cam.window)
    return r


def default_threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def render_traces(cam: CameraType, showers: np.ndarray, seed: int, event_ids=None, out=None,
                  n_threads=None, want_npe=False):
    """Render camera events into ``uint16[n][G][T][Npad]`` (or into ``out``,
    any C-contiguous uint16 buffer of that many elements)."""
    n = len(showers)
    showers = np.ascontiguousarray(showers, SHOWER_DTYPE)
    if out is None:
        out = np.empty((n, cam.n_gain, cam.n_samp, cam.n_pix_pad), np.uint16)
    assert out.dtype == np.uint16 and out.flags.c_contiguous and out.size == n * cam.event_elems
    ids = None if event_ids is None else np.ascontiguousarray(event_ids, np.uint64)
    npe = np.zeros((n, cam.n_pix), np.float32) if want_npe else None
    cfg = _render_cfg(cam, n_threads or default_threads())
    g = cam.geom
    lib().dl0sim_render_traces(ctypes.byref(cfg), _p(g.x), _p(g.y), _p(cam.base_ped), _p(cam.adc_per_pe),
                               _p(showers), _p(ids), seed, n, _p(out), _p(npe))
    return (out, npe) if want_npe else out


def render_images(cam: CameraType, showers: np.ndarray, seed: int, event_ids=None, n_threads=None,
                  want_npe=False):
    """Charge-domain images: ``D int32[n][N]`` in Q8 units (256 x ADC) and
    arrival times ``t float32[n][N]`` (high gain only)."""
    n = len(showers)
    showers = np.ascontiguousarray(showers, SHOWER_DTYPE)
    d = np.empty((n, cam.n_pix), np.int32)
    t = np.empty((n, cam.n_pix), np.float32)
    npe = np.zeros((n, cam.n_pix), np.float32) if want_npe else None
    ids = None if event_ids is None else np.ascontiguousarray(event_ids, np.uint64)
    cfg = _render_cfg(cam, n_threads or default_threads())
    g = cam.geom
    a0 = np.ascontiguousarray(cam.adc_per_pe[0])
    lib().dl0sim_render_images(ctypes.byref(cfg), _p(g.x), _p(g.y), _p(a0), _p(showers), _p(ids), seed, n,
                               _p(d), _p(t), _p(npe))
    return (d, t, npe) if want_npe else (d, t)


# --------------------------------------------------------------------------
# Workload helpers
# --------------------------------------------------------------------------
def plain_events(cam: CameraType, seed: int, n: int, first_event: int = 0, n_threads=None):
    """Showers + traces for ``n`` plain single-ellipse camera events."""
    sh = draw_ellipses(draw_cfg_plain(cam.n_samp), seed, first_event, n)
    ids = np.arange(first_event, first_event + n, dtype=np.uint64)
    tr = render_traces(cam, sh, seed, event_ids=ids, n_threads=n_threads)
    return sh, tr


def mix_types(n: int, seed: int, weights=C1_WEIGHTS) -> np.ndarray:
    """Camera-type sequence of a mixed stream with exact type proportions
    (largest-remainder rounding), in a seeded random order."""
    w = np.asarray(weights, np.float64)
    w = w / w.sum()
    counts = np.floor(w * n).astype(np.int64)
    rem = w * n - counts
    for i in np.argsort(-rem)[: n - counts.sum()]:
        counts[i] += 1
    types = np.repeat(np.arange(len(w), dtype=np.int32), counts)
    rng = np.random.default_rng(seed)
    rng.shuffle(types)
    return types
