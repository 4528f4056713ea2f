"""Parity comparison of GPU records against the oracle — TEST INFRASTRUCTURE.

Integer results (window sums, D, s*, peak, gain, masks, pixel / island /
low-gain counts, flags) must be bit-exact.  Floating-point Hillas fields are
compared as |gpu - oracle| <= tol * scale with tol = 1e-5 and per-field scales
chosen so that the bound reflects FP32 rounding of the field rather than its
size when the value itself is near zero:

  size, length            own value
  width                   length
  cog_x, cog_y, cog_dist  max(|cog|, length)
  psi                     compared modulo pi, only if (l+ - l-) >= 1e-2 l+,
                          with scale l+ / (l+ - l-)
  skewness, kurtosis      sum q |l|^3 / (S len^3), sum q l^4 / (S len^4)
  time_gradient           sqrt(sum (t - tbar)^2 / sum (l - lbar)^2)
  time_intercept          max |t| + time-gradient scale * max |l|
  leakage                 1

When the two psi values straddle +-pi/2 (they differ by about pi), the axis
orientation differs, so the GPU's skewness and time gradient are compared with
their sign flipped.
"""
from __future__ import annotations

import math

import numpy as np

TOL = 1e-5
INT_FIELDS = ("n_pix", "n_islands", "n_lowgain")


def _axis_diff(a, b):
    d = math.fmod(a - b, math.pi)
    return min(abs(d), math.pi - abs(d))


def hillas_mismatches(g, o, x, y, q, t, mask, tol=TOL, check_flags=True, t_input_f32=False):
    """Compare one GPU record ``g`` with one oracle record ``o``.  ``q``, ``t``
    and ``mask`` are the oracle's per-pixel charges, times and mask; ``x``,
    ``y`` the pixel positions.  Returns a list of human-readable mismatches.

    t_input_f32: the kernel received the peak times rounded to float32 (the
    unfused Hillas call takes them from the calibration call's float32
    output), so the time regression may further differ by the effect of that
    input rounding: at most sum |l - lbar| e_i / sum (l - lbar)^2 on the slope,
    with e_i = 2^-24 |t_i| the half-ulp of each time, and max e_i plus that
    times max |l| on the intercept."""
    bad = []
    for k in INT_FIELDS:
        if int(g[k]) != int(o[k]):
            bad.append("%s: gpu %d oracle %d" % (k, int(g[k]), int(o[k])))
    if check_flags and (int(g["flags"]) & 0x7) != (int(o["flags"]) & 0x7):
        bad.append("flags: gpu %#x oracle %#x" % (int(g["flags"]), int(o["flags"])))
    if not math.isclose(float(g["size"]), float(o["size"]), rel_tol=tol, abs_tol=1e-30):
        bad.append("size: gpu %r oracle %r" % (float(g["size"]), float(o["size"])))
    if int(o["flags"]) & 1:
        return bad
    m = mask.astype(bool)
    qm, xm, ym, tm = q[m], x[m].astype(np.float64), y[m].astype(np.float64), t[m]
    S = float(o["size"])
    length, width = float(o["length"]), float(o["width"])
    psi = float(o["psi"])
    l = (xm - o["cog_x"]) * math.cos(psi) + (ym - o["cog_y"]) * math.sin(psi)
    cog_scale = max(abs(float(o["cog_x"])), abs(float(o["cog_y"])), length)
    flip = _axis_diff(float(g["psi"]), psi) < 0.5 * math.pi and abs(float(g["psi"]) - psi) > 0.5 * math.pi
    sgn = -1.0 if flip else 1.0
    sc = {
        "length": length, "width": length, "cog_x": cog_scale, "cog_y": cog_scale, "cog_dist": cog_scale,
        "skewness": float(np.sum(qm * np.abs(l) ** 3) / (S * length ** 3)),
        "kurtosis": float(np.sum(qm * l ** 4) / (S * length ** 4)),
        "leakage": 1.0,
    }
    for k, s in sc.items():
        gv = float(g[k]) * (sgn if k == "skewness" else 1.0)
        if not (abs(gv - float(o[k])) <= tol * s):
            bad.append("%s: gpu %r oracle %r (scale %g)" % (k, gv, float(o[k]), s))
    lp, lm = length ** 2, width ** 2
    if lp - lm >= 1e-2 * lp:
        d = _axis_diff(float(g["psi"]), psi)
        if not d <= tol * lp / (lp - lm):
            bad.append("psi: gpu %r oracle %r (axis diff %g)" % (float(g["psi"]), psi, d))
    if not (int(o["flags"]) & 2):
        lb = l - l.mean()
        tb = tm - tm.mean()
        tg_scale = math.sqrt(float(np.sum(tb * tb)) / float(np.sum(lb * lb))) if np.sum(lb * lb) > 0 else 0.0
        gv = float(g["time_gradient"]) * sgn
        ds = di = 0.0
        if t_input_f32 and np.sum(lb * lb) > 0:
            e = 2.0 ** -24 * np.abs(tm)
            ds = float(np.sum(np.abs(lb) * e) / np.sum(lb * lb))
            di = float(np.max(e)) + ds * float(np.max(np.abs(l)))
        if not abs(gv - float(o["time_gradient"])) <= tol * max(tg_scale, 1e-30) + ds:
            bad.append("time_gradient: gpu %r oracle %r (scale %g)" % (gv, float(o["time_gradient"]), tg_scale))
        is_ = float(np.max(np.abs(tm))) + tg_scale * float(np.max(np.abs(l)))
        if not abs(float(g["time_intercept"]) - float(o["time_intercept"])) <= tol * is_ + di:
            bad.append("time_intercept: gpu %r oracle %r (scale %g)" % (float(g["time_intercept"]),
                                                                        float(o["time_intercept"]), is_))
    return bad


def stereo_mismatch(g_dir, o_dir, cond, c_max, tol=TOL):
    """Stereo point tolerance: FP32 accumulation of the 2x2 normal equations
    amplifies relative rounding by the condition number, so the bound is
    tol * max(1, cond / 100) * (|p| + c_max) with c_max the largest nominal
    cog offset of the event."""
    scale = (math.hypot(*o_dir) + c_max) * max(1.0, cond / 100.0)
    d = math.hypot(g_dir[0] - o_dir[0], g_dir[1] - o_dir[1])
    return d > tol * scale, d, tol * scale


# ---------------------------------------------------------------------------
# Network: float32 accumulation followed by bfloat16 rounding.
#
# A sum of n terms (products of bfloat16 values are exact in float32, and a
# bias is one more term) evaluated in float32 in any order, with each
# addition in error by at most one float32 ulp of its result (2^-23
# relative: round-to-nearest or truncation), differs from its exact value by
# at most n * 2^-23 * (sum of the absolute values of the terms), to first
# order.  Whatever the kernels' order, their float32 result lies inside that
# bracket, and after a monotone map (ReLU, or none) and rounding to bfloat16
# inside the rounded bracket.  An element whose bracket holds one bfloat16
# value must equal it exactly; one whose bracket straddles a rounding
# boundary may take either side.
ULP32 = 2.0 ** -23


def bf16_bracket(exact, mag, n_terms, relu=False):
    """(lo, hi) bfloat16 values (float64) that a float32 evaluation of the
    sums ``exact`` (FP64) with term magnitudes ``mag`` can round to."""
    from oracle.mlp import bf16
    d = n_terms * ULP32 * np.asarray(mag, np.float64)
    lo, hi = np.asarray(exact, np.float64) - d, np.asarray(exact, np.float64) + d
    if relu:
        lo, hi = np.maximum(lo, 0.0), np.maximum(hi, 0.0)
    return bf16(lo), bf16(hi)


def sum_bound(mag, n_terms):
    """Largest |float32 evaluation - exact| of a sum of n_terms terms whose
    absolute values add to ``mag``."""
    return n_terms * ULP32 * np.asarray(mag, np.float64)
