"""MI355X-native low-level reconstruction of the CTA real-time analysis.

Thin Python binding over ``librta.so`` (C ABI declared in ``include/rta.h``).
It only marshals arguments: every step of the reconstruction runs in the HIP
kernels of the library.  PyTorch supplies device memory and streams.  If the
library is missing or fails to load, every entry point raises; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librta.so")

RTA_OK = 0
STATUS_NAMES = {0: "ok", 1: "invalid argument", 2: "unsupported shape", 3: "HIP runtime error",
                4: "out of memory", 5: "unsupported option", 6: "no tuned schedule"}
RTA_E_UNTUNED = 6
EXTRACT_SLIDING = 0       # per pixel: earliest maximiser of the window sum
EXTRACT_FIXED = 1         # every pixel: the camera's fixed window start
EXTRACT_GLOBAL_PEAK = 2   # every pixel: earliest maximiser of the camera-summed window
EXTRACT_NEIGHBOUR_PEAK = 3  # per pixel: earliest maximiser of its neighbours' summed window
FLAG_HILLAS_INVALID = 0x1
FLAG_TIME_INVALID = 0x2
FLAG_LOW_GAIN = 0x4
FLAG_BAD_DESCRIPTOR = 0x8
FLAG_MLP_FALLBACK = 0x10
EVT_STEREO_INVALID = 0x1
EVT_NO_MLP = 0x2
STATUS_BAD_TYPE = 0x1
STATUS_BAD_OFFSET = 0x2
STATUS_BAD_EVENT = 0x4
STATUS_BAD_PACKET = 0x8
PKT_HEADER_BAD = 0x1
PKT_TYPE_BAD = 0x2
PKT_CRC_BAD = 0x4
MAX_PIX = 2048
MAX_SAMP = 255
MAX_TYPES = 8


class RTAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, msg))
        self.status = status


class CameraDesc(ctypes.Structure):
    _fields_ = [("n_pix", ctypes.c_int32), ("n_samp", ctypes.c_int32), ("n_gain", ctypes.c_int32),
                ("window", ctypes.c_int32), ("hg_switch_adc", ctypes.c_int32), ("max_nbr", ctypes.c_int32),
                ("pix_x", ctypes.c_void_p), ("pix_y", ctypes.c_void_p), ("nbr", ctypes.c_void_p),
                ("ped", ctypes.c_void_p), ("adc_per_pe", ctypes.c_void_p), ("focal_m", ctypes.c_float),
                ("t_pic", ctypes.c_float), ("t_bnd", ctypes.c_float), ("fixed_start", ctypes.c_int32)]


class CameraInfo(ctypes.Structure):
    _fields_ = [("n_pix", ctypes.c_int32), ("n_pix_pad", ctypes.c_int32), ("n_samp", ctypes.c_int32),
                ("n_gain", ctypes.c_int32), ("window", ctypes.c_int32), ("fixed_start", ctypes.c_int32),
                ("event_elems", ctypes.c_int64)]


class Batch(ctypes.Structure):
    _fields_ = [("traces", ctypes.c_void_p), ("traces_len", ctypes.c_int64), ("evt_tel_off", ctypes.c_void_p),
                ("tel_type", ctypes.c_void_p), ("tel_trace_off", ctypes.c_void_p), ("n_evt", ctypes.c_int64),
                ("n_tel", ctypes.c_int64), ("evt_done_clock", ctypes.c_void_p), ("tel_class", ctypes.c_void_p)]


class PipelineParams(ctypes.Structure):
    _fields_ = [("do_stereo", ctypes.c_int32), ("extractor", ctypes.c_int32), ("max_width_ratio", ctypes.c_float),
                ("max_cond", ctypes.c_float), ("tune_cache", ctypes.c_char_p), ("mlp", ctypes.c_void_p),
                ("boxcut", ctypes.c_void_p)]


class Schedule(ctypes.Structure):
    _fields_ = [("pix_per_lane", ctypes.c_int32), ("waves_per_wg", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("chunk", ctypes.c_int32)]

    def as_tuple(self):
        return (self.pix_per_lane, self.waves_per_wg, self.wg_per_cu, self.chunk)


HILLAS_FIELDS = ("size", "cog_x", "cog_y", "length", "width", "psi", "skewness", "kurtosis",
                 "time_gradient", "time_intercept", "leakage", "cog_dist")
HILLAS_DTYPE = np.dtype([(f, "<f4") for f in HILLAS_FIELDS]
                        + [("n_pix", "<i4"), ("n_islands", "<i4"), ("n_lowgain", "<i4"), ("flags", "<u4")])
EVENT_DTYPE = np.dtype([("dir_x", "<f4"), ("dir_y", "<f4"), ("cond", "<f4"), ("gammaness", "<f4"),
                        ("log10_energy", "<f4"), ("n_tel", "<i4"), ("n_used", "<i4"), ("flags", "<u4")])

PACKET_DTYPE = np.dtype([("event_number", "<u8"), ("coarse_time", "<u4"), ("fine_time", "<u2"), ("apid", "<u2"),
                         ("seq_count", "<u2"), ("cam_type", "<u2"), ("flags", "<u4"), ("crc_stored", "<u2"),
                         ("crc_computed", "<u2"), ("pad_", "<u4")])

PIXEL_HEALTH_DTYPE = np.dtype([("n", "<u8"), ("s1", "<u8"), ("s2", "<u8"), ("n_sat", "<u8"), ("mean", "<f8"),
                               ("rms", "<f8"), ("flags", "<u4"), ("pad_", "<u4"), ("reserved_", "<u8")])
CAMERA_HEALTH_DTYPE = np.dtype([("median_rms", "<f8", (2,)), ("n_bad", "<i4"), ("verdict", "<i4")])
HEALTH_DEAD, HEALTH_NOISY, HEALTH_PED_SHIFT, HEALTH_SATURATING = 0x1, 0x2, 0x4, 0x8


class HealthParams(ctypes.Structure):
    _fields_ = [("rms_dead", ctypes.c_float), ("noisy_factor", ctypes.c_float), ("ped_tol", ctypes.c_float),
                ("sat_frac", ctypes.c_float), ("bad_frac_max", ctypes.c_float), ("pad_", ctypes.c_int32)]


SAM_ALERT_DTYPE = np.dtype([("scale", "<i4"), ("ix", "<i4"), ("iy", "<i4"), ("n_on", "<i4"),
                            ("significance", "<f8"), ("n_off", "<i4"), ("pad_", "<i4")])


class SamParams(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("n_bins", ctypes.c_int32), ("t0", ctypes.c_double),
                ("bin_s", ctypes.c_double), ("cell", ctypes.c_float), ("r_on", ctypes.c_float),
                ("r_in", ctypes.c_float), ("r_out", ctypes.c_float), ("gamma_cut", ctypes.c_float),
                ("sigma_alert", ctypes.c_float), ("n_scales", ctypes.c_int32), ("scales", ctypes.c_int32 * 8)]


# C symbols declared in include/rta.h: name -> (argtypes, restype)
_vp, _i32, _i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
SYMBOLS = {
    "rta_status_str": ([ctypes.c_int], ctypes.c_char_p),
    "rta_last_error": ([], ctypes.c_char_p),
    "rta_version": ([], _i32),
    "rta_device_cus": ([_vp], ctypes.c_int),
    "rta_device_clock_hz": ([_vp], ctypes.c_int),
    "rta_device_stamp": ([_vp, _vp], ctypes.c_int),
    "rta_camera_create": ([_vp, _vp], ctypes.c_int),
    "rta_camera_destroy": ([_vp], ctypes.c_int),
    "rta_camera_get_info": ([_vp, _vp], ctypes.c_int),
    "rta_calibrate": ([_vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "rta_calibrate_ex": ([_vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "rta_clean": ([_vp, _vp, _vp, _vp, _i64, _vp, _vp], ctypes.c_int),
    "rta_hillas": ([_vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp], ctypes.c_int),
    "rta_hillas_q8": ([_vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp], ctypes.c_int),
    "rta_pipeline_create": ([_vp, _i32, _vp, _vp], ctypes.c_int),
    "rta_pipeline_destroy": ([_vp], ctypes.c_int),
    "rta_set_schedule": ([_vp, _vp], ctypes.c_int),
    "rta_get_schedule": ([_vp, _vp], ctypes.c_int),
    "rta_list_schedules": ([_vp, _i32, _vp], ctypes.c_int),
    "rta_pipeline_tune_key": ([_vp, ctypes.c_char_p, _i32], ctypes.c_int),
    "rta_pipeline_tune": ([_vp, _vp, _vp, _vp, _vp, _i32, _i32, _vp, _vp, _vp], ctypes.c_int),
    "rta_tune_cache_lookup": ([ctypes.c_char_p, ctypes.c_char_p, _vp, _vp], ctypes.c_int),
    "rta_tune_cache_store": ([ctypes.c_char_p, ctypes.c_char_p, _vp, ctypes.c_float], ctypes.c_int),
    "rta_process_batch": ([_vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "rta_process_batch_noalloc": ([_vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "rta_stereo": ([_vp, _vp, _vp, _i64, _i64, _vp, _vp, _vp], ctypes.c_int),
    "rta_batch_status": ([_vp, _vp], ctypes.c_int),
    "rta_graph_capture": ([_vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "rta_graph_launch": ([_vp, _vp], ctypes.c_int),
    "rta_graph_destroy": ([_vp], ctypes.c_int),
    "rta_health": ([_vp, _vp, _i64, _vp, _vp, _vp, _vp], ctypes.c_int),
    "rta_sam_create": ([_vp, _vp], ctypes.c_int),
    "rta_sam_destroy": ([_vp], ctypes.c_int),
    "rta_sam_clear": ([_vp, _vp], ctypes.c_int),
    "rta_sam_fill": ([_vp, _vp, _vp, _i64, _vp], ctypes.c_int),
    "rta_sam_search": ([_vp, _i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp], ctypes.c_int),
    "rta_sam_counts": ([_vp, _vp, _vp], ctypes.c_int),
    "rta_frame_packets": ([_vp, _i32, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "rta_decode_packets": ([_vp, _vp, _i64, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp], ctypes.c_int),
    "rta_mlp_create": ([_vp, _vp], ctypes.c_int),
    "rta_mlp_destroy": ([_vp], ctypes.c_int),
    "rta_mlp_set_params": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "rta_mlp_get_params": ([_vp, _vp], ctypes.c_int),
    "rta_mlp_forward": ([_vp, _vp, _i64, _vp, _vp], ctypes.c_int),
    "rta_mlp_loss_grad": ([_vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp], ctypes.c_int),
    "rta_mlp_train_step": ([_vp, _vp, _vp, _vp, _i64, _vp, _vp], ctypes.c_int),
    "rta_mlp_train_step_rows": ([_vp, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp], ctypes.c_int),
    "rta_mlp_stored": ([_vp, _i32, _i64, _vp, _vp], ctypes.c_int),
    "rta_features": ([_vp, _i64, _vp, _vp], ctypes.c_int),
    "rta_classify": ([_vp, _vp, _vp, _i64, _vp, _vp], ctypes.c_int),
    "rta_pipeline_attach_mlp": ([_vp, _vp, _vp], ctypes.c_int),
}
BOXCUT_MAX_BINS = 32
MLP_N_PARAMS = 9154
MLP_N_FEATURES = 10
MLP_N_STORED = 8


class BoxCutDesc(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("lgs_lo", ctypes.c_float), ("lgs_hi", ctypes.c_float),
                ("w_mean", ctypes.c_float * 32), ("w_std", ctypes.c_float * 32),
                ("l_mean", ctypes.c_float * 32), ("l_std", ctypes.c_float * 32),
                ("cut_w", ctypes.c_float), ("cut_l", ctypes.c_float), ("e_a", ctypes.c_float), ("e_b", ctypes.c_float),
                ("feat_lo", ctypes.c_float * 10), ("feat_hi", ctypes.c_float * 10), ("mlp_cut", ctypes.c_float)]


class MlpDesc(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]

_lib = None


def lib():
    """Load librta.so; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librta.so is not built (run __graft_entry__.build() or "
                               "python paper_1307_6489_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SYMBOLS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status):
    if status != RTA_OK:
        raise RTAError(status, lib().rta_last_error().decode())


def _ptr(t):
    """Device (or host) address of a tensor / array, None for None."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return ctypes.c_void_p(t.data_ptr())
    return t.ctypes.data_as(ctypes.c_void_p)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _require(t, dtype, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))


def device_cus():
    n = ctypes.c_int32()
    _check(lib().rta_device_cus(ctypes.byref(n)))
    return n.value


def device_clock_hz():
    """Rate of the device clock of device_stamp / evt_done_clock, Hz."""
    v = ctypes.c_int64()
    _check(lib().rta_device_clock_hz(ctypes.byref(v)))
    return v.value


def device_stamp(slot, stream=None):
    """Write the device clock into ``slot`` (int64 device tensor, one element)
    when ``stream`` reaches this point."""
    import torch
    _require(slot, torch.int64, name="slot")
    if slot.numel() < 1:
        raise ValueError("slot must hold one element")
    _check(lib().rta_device_stamp(_ptr(slot), _stream(stream)))


def list_schedules():
    n = ctypes.c_int32()
    _check(lib().rta_list_schedules(None, 0, ctypes.byref(n)))
    arr = (Schedule * n.value)()
    _check(lib().rta_list_schedules(arr, n.value, ctypes.byref(n)))
    return [s.as_tuple() for s in arr]


TUNE_KEY_MAX = 512


def tune_cache_lookup(path, key):
    """(schedule tuple, ms) the tune cache file holds for key, or None
    (no file, no entry, or a schedule this library does not compile)."""
    s, ms = Schedule(), ctypes.c_float()
    st = lib().rta_tune_cache_lookup(os.fsencode(path), key.encode(), ctypes.byref(s), ctypes.byref(ms))
    if st == RTA_E_UNTUNED:
        return None
    _check(st)
    return s.as_tuple(), ms.value


def tune_cache_store(path, key, sched, ms):
    """Record sched (4-tuple) with its time for key in the tune cache file."""
    s = Schedule(*sched)
    _check(lib().rta_tune_cache_store(os.fsencode(path), key.encode(), ctypes.byref(s), float(ms)))


class Camera:
    """A camera type on the current device (pedestals in Q8, integer cleaning
    thresholds, neighbour table)."""

    def __init__(self, n_pix, n_samp, n_gain, x, y, nbr, ped, adc_per_pe, focal_m, window=4, hg_switch_adc=4000,
                 t_pic=10.0, t_bnd=5.0, fixed_start=None):
        self._keep = dict(x=np.ascontiguousarray(x, np.float32), y=np.ascontiguousarray(y, np.float32),
                          nbr=np.ascontiguousarray(nbr, np.int32),
                          ped=np.ascontiguousarray(ped, np.float32).reshape(n_gain, n_pix),
                          a=np.ascontiguousarray(adc_per_pe, np.float32).reshape(n_gain, n_pix))
        k = self._keep
        d = CameraDesc(n_pix, n_samp, n_gain, window, hg_switch_adc, k["nbr"].shape[1] if k["nbr"].ndim == 2 else 0,
                       _ptr(k["x"]), _ptr(k["y"]), _ptr(k["nbr"]), _ptr(k["ped"]), _ptr(k["a"]), focal_m, t_pic,
                       t_bnd, (n_samp - window) // 2 if fixed_start is None else fixed_start)
        h = ctypes.c_void_p()
        _check(lib().rta_camera_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        info = CameraInfo()
        _check(lib().rta_camera_get_info(h, ctypes.byref(info)))
        self.n_pix, self.n_pix_pad, self.n_samp = info.n_pix, info.n_pix_pad, info.n_samp
        self.n_gain, self.window, self.event_elems = info.n_gain, info.window, info.event_elems
        self.fixed_start = info.fixed_start
        self.n_pix_pad = info.n_pix_pad
        self.focal_m = focal_m

    @classmethod
    def from_type(cls, ct, t_pic=10.0, t_bnd=5.0):
        """From any camera-type object with n_pix, n_samp, n_gain, geom.{x,y,nbr},
        ped, adc_per_pe, focal_m, window, hg_switch_adc and (optionally)
        fixed_start attributes."""
        return cls(ct.n_pix, ct.n_samp, ct.n_gain, ct.geom.x, ct.geom.y, ct.geom.nbr, ct.ped, ct.adc_per_pe,
                   ct.focal_m, ct.window, ct.hg_switch_adc, t_pic, t_bnd, getattr(ct, "fixed_start", None))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.rta_camera_destroy(h)
            self.handle = None

    def _n_evt(self, traces):
        import torch
        _require(traces, torch.uint16, name="traces")
        if traces.numel() % self.event_elems:
            raise ValueError("traces must hold whole events of %d elements" % self.event_elems)
        return traces.numel() // self.event_elems


def calibrate(cam: Camera, traces, stream=None, outputs=("S", "D", "sstar", "peak", "gain", "q", "t"),
              extractor=None):
    """Per-pixel calibration of every event of ``traces`` (uint16 [E][G][T][Npad]);
    ``extractor`` one of EXTRACT_* (default: the sliding window)."""
    import torch
    E = cam._n_evt(traces)
    dev = traces.device
    dt = {"S": torch.int32, "D": torch.int32, "sstar": torch.uint8, "peak": torch.uint8, "gain": torch.uint8,
          "q": torch.float32, "t": torch.float32}
    out = {k: torch.empty((E, cam.n_pix), dtype=dt[k], device=dev) for k in outputs}
    g = lambda k: _ptr(out.get(k))  # noqa: E731
    if extractor is None:
        _check(lib().rta_calibrate(cam.handle, _ptr(traces), E, g("S"), g("D"), g("sstar"), g("peak"), g("gain"),
                                   g("q"), g("t"), _stream(stream)))
    else:
        _check(lib().rta_calibrate_ex(cam.handle, int(extractor), _ptr(traces), E, g("S"), g("D"), g("sstar"),
                                      g("peak"), g("gain"), g("q"), g("t"), _stream(stream)))
    return out


class CleanParams(ctypes.Structure):
    _fields_ = [("t_pic", ctypes.c_float), ("t_bnd", ctypes.c_float)]


def clean(cam: Camera, D, gain=None, stream=None, levels=None):
    """rta_clean; levels: optional (t_pic, t_bnd) in p.e. (default: the
    camera's levels)."""
    import torch
    _require(D, torch.int32, name="D")
    E = D.numel() // cam.n_pix
    _require(D, torch.int32, (E, cam.n_pix), "D")
    if gain is not None:
        _require(gain, torch.uint8, (E, cam.n_pix), "gain")
    lv = None if levels is None else ctypes.byref(CleanParams(float(levels[0]), float(levels[1])))
    mask = torch.empty((E, cam.n_pix), dtype=torch.uint8, device=D.device)
    _check(lib().rta_clean(cam.handle, lv, _ptr(D), _ptr(gain), E, _ptr(mask), _stream(stream)))
    return mask


def hillas(cam: Camera, q, t, mask, gain=None, stream=None):
    """rta_hillas: records from charges q (p.e.), times t and the mask; gain
    (optional) for the low-gain pixel count."""
    import torch
    E = q.numel() // cam.n_pix
    _require(q, torch.float32, (E, cam.n_pix), "q")
    _require(t, torch.float32, (E, cam.n_pix), "t")
    _require(mask, torch.uint8, (E, cam.n_pix), "mask")
    if gain is not None:
        _require(gain, torch.uint8, (E, cam.n_pix), "gain")
    out = torch.empty((E, 16), dtype=torch.float32, device=q.device)
    _check(lib().rta_hillas(cam.handle, _ptr(q), _ptr(t), _ptr(mask), _ptr(gain), E, _ptr(out), _stream(stream)))
    return out


def hillas_q8(cam: Camera, D, t, mask, gain=None, stream=None):
    """rta_hillas_q8: records from the integer charges D (Q8) and their gain."""
    import torch
    E = D.numel() // cam.n_pix
    _require(D, torch.int32, (E, cam.n_pix), "D")
    _require(t, torch.float32, (E, cam.n_pix), "t")
    _require(mask, torch.uint8, (E, cam.n_pix), "mask")
    if gain is not None:
        _require(gain, torch.uint8, (E, cam.n_pix), "gain")
    out = torch.empty((E, 16), dtype=torch.float32, device=D.device)
    _check(lib().rta_hillas_q8(cam.handle, _ptr(D), _ptr(t), _ptr(mask), _ptr(gain), E, _ptr(out), _stream(stream)))
    return out


def records(t, dtype=HILLAS_DTYPE):
    """Device record tensor ([n][16] or [n][8] float32) -> numpy structured array."""
    a = t.detach().cpu().contiguous().numpy()
    return a.view(dtype).reshape(-1)


class Pipeline:
    """Fused batched path over several camera types."""

    def __init__(self, cams, do_stereo=True, max_width_ratio=0.9, max_cond=1e4, extractor=0, tune_cache=None,
                 mlp=None, boxcut=None):
        """tune_cache: optional path of a schedule tune cache.  With one, the
        pipeline takes the cached schedule for its key, or refuses to process
        (RTAError status RTA_E_UNTUNED) until tune() or set_schedule().
        mlp, boxcut: optional network and box-cut tables attached at creation
        (as attach_mlp does)."""
        self.cams = list(cams)
        arr = (ctypes.c_void_p * len(self.cams))(*[c.handle.value for c in self.cams])
        p = PipelineParams(1 if do_stereo else 0, int(extractor), max_width_ratio, max_cond,
                           None if tune_cache is None else os.fsencode(tune_cache),
                           None if mlp is None else mlp.handle.value,
                           None if boxcut is None else ctypes.cast(ctypes.pointer(boxcut), ctypes.c_void_p).value)
        self._mlp = mlp
        self.extractor = int(extractor)
        h = ctypes.c_void_p()
        _check(lib().rta_pipeline_create(arr, len(self.cams), ctypes.byref(p), ctypes.byref(h)))
        self.handle = h
        self.do_stereo = do_stereo

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.rta_pipeline_destroy(h)
            self.handle = None

    def set_schedule(self, pix_per_lane, waves_per_wg, wg_per_cu, chunk=8):
        s = Schedule(pix_per_lane, waves_per_wg, wg_per_cu, chunk)
        _check(lib().rta_set_schedule(self.handle, ctypes.byref(s)))

    def schedule(self):
        s = Schedule()
        _check(lib().rta_get_schedule(self.handle, ctypes.byref(s)))
        return s.as_tuple()

    def tune_key(self):
        buf = ctypes.create_string_buffer(TUNE_KEY_MAX)
        _check(lib().rta_pipeline_tune_key(self.handle, buf, TUNE_KEY_MAX))
        return buf.value.decode()

    def tune(self, batch, tel_out, evt_out=None, candidates=None, reps=3, stream=None):
        """rta_pipeline_tune: time candidate schedules (all compiled ones by
        default) on batch, apply the fastest, store it in the pipeline's tune
        cache if it has one.  Returns (best tuple, {schedule: median ms})."""
        cands = list(candidates) if candidates is not None else list_schedules()
        arr = (Schedule * len(cands))(*[Schedule(*c) for c in cands])
        ms = (ctypes.c_float * len(cands))()
        best = Schedule()
        _check(lib().rta_pipeline_tune(self.handle, ctypes.byref(batch), _ptr(tel_out), _ptr(evt_out), arr,
                                       len(cands), int(reps), ms, ctypes.byref(best), _stream(stream)))
        return best.as_tuple(), {tuple(c): ms[i] for i, c in enumerate(cands)}

    @staticmethod
    def make_batch(traces, tel_type, tel_trace_off, evt_tel_off=None, evt_done_clock=None, tel_class=None):
        """evt_done_clock: optional int64 device tensor [n_evt] that receives the
        device clock at each event record's write; tel_class: optional float32
        device tensor [n_tel][2] that receives each telescope's gamma score and
        log10 E, classified in the reconstruction kernel (needs attach_mlp)."""
        import torch
        _require(traces, torch.uint16, name="traces")
        _require(tel_type, torch.int32, name="tel_type")
        _require(tel_trace_off, torch.int64, name="tel_trace_off")
        n_tel = tel_type.numel()
        if tel_trace_off.numel() != n_tel:
            raise ValueError("tel_type and tel_trace_off differ in length")
        n_evt = 0
        if evt_tel_off is not None:
            _require(evt_tel_off, torch.int64, name="evt_tel_off")
            n_evt = evt_tel_off.numel() - 1
        if evt_done_clock is not None:
            _require(evt_done_clock, torch.int64, (n_evt,), "evt_done_clock")
        if tel_class is not None:
            _require(tel_class, torch.float32, (n_tel, 2), "tel_class")
        b = Batch(_ptr(traces), traces.numel(), _ptr(evt_tel_off), _ptr(tel_type), _ptr(tel_trace_off), n_evt, n_tel,
                  _ptr(evt_done_clock), _ptr(tel_class))
        b._keep = (traces, tel_type, tel_trace_off, evt_tel_off, evt_done_clock, tel_class)
        return b

    def alloc_outputs(self, batch, device):
        import torch
        tel = torch.empty((batch.n_tel, 16), dtype=torch.float32, device=device)
        evt = torch.empty((max(batch.n_evt, 0), 8), dtype=torch.float32, device=device) if self.do_stereo else None
        return tel, evt

    def process(self, batch, tel_out, evt_out=None, stream=None):
        _check(lib().rta_process_batch(self.handle, ctypes.byref(batch), _ptr(tel_out), _ptr(evt_out),
                                       _stream(stream)))

    def process_noalloc(self, batch, tel_out, evt_out=None, status_out=None, stream=None):
        """rta_process_batch_noalloc: the same batch through the library's
        static scratch (status_out: optional device uint32 tensor [1])."""
        _check(lib().rta_process_batch_noalloc(self.handle, ctypes.byref(batch), _ptr(tel_out), _ptr(evt_out),
                                               _ptr(status_out), _stream(stream)))

    def stereo(self, evt_tel_off, tel_type, tel_rec, stream=None):
        import torch
        n_evt = evt_tel_off.numel() - 1
        out = torch.empty((n_evt, 8), dtype=torch.float32, device=tel_rec.device)
        _check(lib().rta_stereo(self.handle, _ptr(evt_tel_off), _ptr(tel_type), n_evt, tel_type.numel(),
                                _ptr(tel_rec), _ptr(out), _stream(stream)))
        return out

    def attach_mlp(self, mlp, boxcut):
        """Classify telescopes in the per-event pass (mlp None: detach)."""
        if mlp is None:
            _check(lib().rta_pipeline_attach_mlp(self.handle, None, None))
            self._mlp = None
            return
        _check(lib().rta_pipeline_attach_mlp(self.handle, mlp.handle, ctypes.byref(boxcut)))
        self._mlp = mlp

    def status(self):
        s = ctypes.c_uint32()
        _check(lib().rta_batch_status(self.handle, ctypes.byref(s)))
        return s.value

    def capture(self, batch, tel_out, evt_out=None):
        return Graph(self, batch, tel_out, evt_out)


def frame_packets(cams, data, cap=None):
    """Host framing of a DL0 packet stream (``data``: host uint8 array) for
    the camera types ``cams`` (list of Camera, index = camera type).
    Returns (pkt_off int64, tel_type int32, tel_trace_off int64, pool_elems,
    consumed bytes) as numpy arrays / ints."""
    data = np.ascontiguousarray(data, np.uint8).reshape(-1)
    infos = (CameraInfo * max(len(cams), 1))()
    for i, c in enumerate(cams):
        infos[i] = CameraInfo(c.n_pix, c.n_pix_pad, c.n_samp, c.n_gain, c.window, c.fixed_start, c.event_elems)
    cap = data.size // 34 + 1 if cap is None else int(cap)
    off = np.empty(cap, np.int64)
    ty = np.empty(cap, np.int32)
    toff = np.empty(cap, np.int64)
    n, pool, used = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().rta_frame_packets(infos, len(cams), data.ctypes.data_as(ctypes.c_void_p), data.size, cap,
                                   off.ctypes.data_as(ctypes.c_void_p), ty.ctypes.data_as(ctypes.c_void_p),
                                   toff.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n), ctypes.byref(pool),
                                   ctypes.byref(used)))
    k = n.value
    return off[:k].copy(), ty[:k].copy(), toff[:k].copy(), pool.value, used.value


PACKET_PAD = 32


def packet_buffer(host_bytes, device):
    """A device copy of a host packet stream with the RTA_PACKET_PAD readable
    bytes the decode needs after it.  Returns (tensor, n_bytes)."""
    import torch
    h = np.ascontiguousarray(host_bytes, np.uint8).reshape(-1)
    t = torch.zeros(h.size + PACKET_PAD, dtype=torch.uint8, device=device)
    t[:h.size].copy_(torch.from_numpy(h))
    return t, h.size


def decode_packets(pipe, data, pkt_off, tel_type, tel_trace_off, pool_elems, pool=None, stream=None, want_rec=True,
                   n_bytes=None):
    """Device decode of framed packets: ``data`` uint8 device tensor (16-byte
    aligned) holding the stream in its first ``n_bytes`` bytes (default
    data.numel() - PACKET_PAD) and at least PACKET_PAD more; ``pkt_off`` /
    ``tel_trace_off`` int64 and ``tel_type`` int32 device tensors (tel_type is
    rewritten in place: -1 for rejected packets).  Returns (pool uint16
    tensor, packet records [n][8] float32-viewed tensor or None)."""
    import torch
    _require(data, torch.uint8, name="data")
    n_bytes = data.numel() - PACKET_PAD if n_bytes is None else int(n_bytes)
    if n_bytes < 0 or data.numel() < n_bytes + PACKET_PAD:
        raise ValueError("data must hold the stream and %d readable bytes after it" % PACKET_PAD)
    _require(pkt_off, torch.int64, name="pkt_off")
    _require(tel_type, torch.int32, name="tel_type")
    _require(tel_trace_off, torch.int64, name="tel_trace_off")
    n = pkt_off.numel()
    if tel_type.numel() != n or tel_trace_off.numel() != n:
        raise ValueError("packet arrays differ in length")
    if pool is None:
        pool = torch.empty(max(int(pool_elems), 8), dtype=torch.uint16, device=data.device)
    rec = torch.empty((n, 8), dtype=torch.float32, device=data.device) if want_rec else None
    _check(lib().rta_decode_packets(pipe.handle, _ptr(data), n_bytes, _ptr(pkt_off), _ptr(tel_type),
                                    _ptr(tel_trace_off), n, _ptr(pool), int(pool_elems), _ptr(rec),
                                    _stream(stream)))
    return pool, rec


def health(cam: Camera, traces, rms_dead=0.5, noisy_factor=3.0, ped_tol=20.0, sat_frac=0.01, bad_frac_max=0.05,
           stream=None, to_host=True):
    """Health statistics of the events of ``traces`` (uint16 [E][G][T][Npad],
    one camera type).  Returns (per-pixel records [G][N], camera summary) as
    numpy records, or the device tensors with to_host=False."""
    import torch
    E = cam._n_evt(traces)
    p = HealthParams(rms_dead, noisy_factor, ped_tol, sat_frac, bad_frac_max, 0)
    pix = torch.empty((cam.n_gain * cam.n_pix, 8), dtype=torch.float64, device=traces.device)
    out = torch.empty(3, dtype=torch.float64, device=traces.device)
    _check(lib().rta_health(cam.handle, _ptr(traces), E, ctypes.byref(p), _ptr(pix), _ptr(out), _stream(stream)))
    if not to_host:
        return pix, out
    pr = pix.cpu().numpy().view(PIXEL_HEALTH_DTYPE).reshape(cam.n_gain, cam.n_pix)
    cr = out.cpu().numpy().view(CAMERA_HEALTH_DTYPE)[0]
    return pr, cr


class Sam:
    """Science alert monitor: time-binned sky counts of selected events and
    the Li & Ma search on several timescales (definitions in rta.h)."""

    def __init__(self, grid, n_bins, t0, bin_s, cell, r_on, r_in, r_out, gamma_cut, sigma_alert, scales):
        sc = (ctypes.c_int32 * 8)(*(list(scales) + [1] * (8 - len(scales))))
        self.params = SamParams(grid, n_bins, t0, bin_s, cell, r_on, r_in, r_out, gamma_cut, sigma_alert,
                                len(scales), sc)
        h = ctypes.c_void_p()
        _check(lib().rta_sam_create(ctypes.byref(self.params), ctypes.byref(h)))
        self.handle = h
        self.grid, self.n_bins, self.scales = grid, n_bins, list(scales)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.rta_sam_destroy(h)
            self.handle = None

    def clear(self, stream=None):
        _check(lib().rta_sam_clear(self.handle, _stream(stream)))

    def fill(self, evt, t, stream=None):
        """evt: event records [n][8] float32 tensor; t: float64 times [n]."""
        import torch
        _require(t, torch.float64, name="t")
        n = t.numel()
        _require(evt, torch.float32, (n, 8), "evt")
        _check(lib().rta_sam_fill(self.handle, _ptr(evt), _ptr(t), n, _stream(stream)))

    def counts(self, stream=None):
        """Copy of the counts cube [n_bins][grid][grid] (int32 numpy)."""
        import torch
        out = torch.empty((self.n_bins, self.grid, self.grid), dtype=torch.int32, device="cuda")
        _check(lib().rta_sam_counts(self.handle, _ptr(out), _stream(stream)))
        torch.cuda.synchronize()
        return out.cpu().numpy()

    def search(self, end_bin, max_alerts=4096, stream=None, maps=True):
        """Significance / N_on / N_off maps [n_scales][grid][grid] (tensors, or
        None) and the alerts (numpy, sorted by scale, iy, ix)."""
        import torch
        dev = torch.device("cuda")
        shape = (len(self.scales), self.grid, self.grid)
        sig = torch.empty(shape, dtype=torch.float64, device=dev) if maps else None
        non = torch.empty(shape, dtype=torch.int32, device=dev) if maps else None
        noff = torch.empty(shape, dtype=torch.int32, device=dev) if maps else None
        al = torch.empty((max(max_alerts, 1), 4), dtype=torch.float64, device=dev)
        cnt = torch.zeros(1, dtype=torch.int32, device=dev)
        _check(lib().rta_sam_search(self.handle, int(end_bin), _ptr(sig), _ptr(non), _ptr(noff), _ptr(al),
                                    int(max_alerts), _ptr(cnt), _stream(stream)))
        k = min(int(cnt.cpu()[0]), max_alerts)
        a = al.cpu().numpy().view(SAM_ALERT_DTYPE).reshape(-1)[:k]
        a = a[np.lexsort((a["ix"], a["iy"], a["scale"]))]
        return sig, non, noff, a, int(cnt.cpu()[0])


class Graph:
    """A captured rta_process_batch (fixed pointers and sizes)."""

    def __init__(self, pipe, batch, tel_out, evt_out):
        h = ctypes.c_void_p()
        _check(lib().rta_graph_capture(pipe.handle, ctypes.byref(batch), _ptr(tel_out), _ptr(evt_out),
                                       ctypes.byref(h)))
        self.handle = h
        self._keep = (pipe, batch, tel_out, evt_out)

    def launch(self, stream=None):
        _check(lib().rta_graph_launch(self.handle, _stream(stream)))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.rta_graph_destroy(h)
            self.handle = None


class Mlp:
    """The gamma/hadron + energy network on the device (bf16 MFMA kernels)."""

    def __init__(self, max_batch=4096, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        d = MlpDesc(max_batch, lr, beta1, beta2, eps)
        h = ctypes.c_void_p()
        _check(lib().rta_mlp_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        self.max_batch = max_batch

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.rta_mlp_destroy(h)
            self.handle = None

    def set_params(self, params, feat_mean, feat_std):
        p = np.ascontiguousarray(params, np.float32)
        m = np.ascontiguousarray(feat_mean, np.float32)
        s = np.ascontiguousarray(feat_std, np.float32)
        if p.size != MLP_N_PARAMS or m.size != MLP_N_FEATURES or s.size != MLP_N_FEATURES:
            raise ValueError("parameter / normaliser sizes")
        _check(lib().rta_mlp_set_params(self.handle, _ptr(p), _ptr(m), _ptr(s)))

    def get_params(self):
        p = np.empty(MLP_N_PARAMS, np.float32)
        _check(lib().rta_mlp_get_params(self.handle, _ptr(p)))
        return p

    def forward(self, x, stream=None):
        import torch
        _require(x, torch.float32, name="x")
        B = x.shape[0]
        _require(x, torch.float32, (B, MLP_N_FEATURES), "x")
        out = torch.empty((B, 2), dtype=torch.float32, device=x.device)
        _check(lib().rta_mlp_forward(self.handle, _ptr(x), B, _ptr(out), _stream(stream)))
        return out

    def _batch(self, x, label, log10e):
        import torch
        B = x.shape[0]
        _require(x, torch.float32, (B, MLP_N_FEATURES), "x")
        _require(label, torch.float32, (B,), "label")
        _require(log10e, torch.float32, (B,), "log10e")
        return B

    def loss_grad(self, x, label, log10e, stream=None):
        import torch
        B = self._batch(x, label, log10e)
        grad = torch.empty(MLP_N_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(lib().rta_mlp_loss_grad(self.handle, _ptr(x), _ptr(label), _ptr(log10e), B, _ptr(grad), _ptr(loss),
                                       _stream(stream)))
        return loss, grad

    def stored(self, which, B, stream=None):
        """rta_mlp_stored: the bfloat16 values (as float32, feature-major
        [rows][B]) the last loss_grad / train_step pass stored; which 0..3:
        input and hidden activations, 4..6: gradients at the pre-activations
        of layers 1..3, 7: gradient at the outputs."""
        import torch
        rows = 16 if which in (0, 7) else 64
        out = torch.empty((rows, B), dtype=torch.int16, device="cuda")
        _check(lib().rta_mlp_stored(self.handle, which, B, _ptr(out), _stream(stream)))
        bits = out.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        return bits.view(np.float32)

    def train_step(self, x, label, log10e, loss_out=None, stream=None, rows=None):
        """One Adam step on the batch (x, label, log10e); with ``rows`` (int64
        device tensor) the batch is rows of those data arrays, gathered in the
        kernel."""
        if rows is None:
            B = self._batch(x, label, log10e)
            _check(lib().rta_mlp_train_step(self.handle, _ptr(x), _ptr(label), _ptr(log10e), B, _ptr(loss_out),
                                            _stream(stream)))
            return
        import torch
        n = self._batch(x, label, log10e)
        _require(rows, torch.int64, name="rows")
        _check(lib().rta_mlp_train_step_rows(self.handle, _ptr(x), _ptr(label), _ptr(log10e), n, _ptr(rows),
                                             rows.numel(), _ptr(loss_out), _stream(stream)))


def features(rec, stream=None):
    """Network inputs [n][10] of device records ([n][16] float32)."""
    import torch
    n = rec.shape[0]
    _require(rec, torch.float32, (n, 16), "rec")
    x = torch.empty((n, MLP_N_FEATURES), dtype=torch.float32, device=rec.device)
    _check(lib().rta_features(_ptr(rec), n, _ptr(x), _stream(stream)))
    return x


def classify(mlp, boxcut, rec, stream=None):
    """Per-record [score, log10 E, gamma (0/1), fallback (0/1)]; mlp may be None."""
    import torch
    n = rec.shape[0]
    _require(rec, torch.float32, (n, 16), "rec")
    out = torch.empty((n, 4), dtype=torch.float32, device=rec.device)
    _check(lib().rta_classify(None if mlp is None else mlp.handle, ctypes.byref(boxcut), _ptr(rec), n, _ptr(out),
                              _stream(stream)))
    return out
