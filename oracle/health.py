"""Oracle of the real-time health monitor — TEST INFRASTRUCTURE ONLY.

In the paper's design a real-time monitor checks the quality of the incoming
data and its verdict lets the alert monitor hold back on bad data (Section
4.2).  It names no quantities; the reading implemented here (plain
numpy, integers exact, derived values FP64):

  accumulate   over n_evt camera events of one type, per gain g and pixel i:
               n = n_evt * T samples, S1 = sum x, S2 = sum x^2, n_sat =
               number of samples >= the saturation level (the high-gain
               switch level for the high gain of dual-gain cameras, 65535
               otherwise)
  derive       mean = S1 / n, rms = sqrt(max(S2 / n - mean^2, 0))
  median       per gain, the lower median of the rms over the pixels
               (element (N - 1) // 2 of the sorted values)
  flags        DEAD rms < rms_dead; NOISY rms > noisy_factor * median;
               PED_SHIFT |mean - P / 256| > ped_tol (P = nearest-even
               (256 ped), the Q8 pedestal the calibration uses, ADC);
               SATURATING n_sat > sat_frac * n
  verdict      bad pixels (any flag, any gain) > bad_frac_max * N  ->  1

Parity status: pinned by a direct loop, hand-made bad pixels, the lower
median and the generator's noise (tests/test_oracle_health.py).
"""
from __future__ import annotations

import numpy as np

DEAD, NOISY, PED_SHIFT, SATURATING = 1, 2, 4, 8


def f32(v):
    return float(np.float32(v))


def health(traces, n_pix, n_gain, ped, hg_switch, p):
    """traces uint16 [E][G][T][Npad].  Returns per-pixel dict of arrays
    [G][N] and the camera summary."""
    tr = np.asarray(traces)
    E, G, T, Np = tr.shape
    N = n_pix
    x = tr[:, :, :, :N].astype(np.int64)
    S1 = x.sum(axis=(0, 2))
    S2 = (x * x).sum(axis=(0, 2))
    lvl = np.array([hg_switch if (n_gain == 2 and g == 0) else 65535 for g in range(G)], np.int64)
    n_sat = (x >= lvl[None, :, None, None]).sum(axis=(0, 2))
    n = E * T
    mean = S1 / n
    var = S2 / n - mean * mean
    rms = np.sqrt(np.maximum(var, 0.0))
    med = np.array([np.sort(rms[g])[(N - 1) // 2] for g in range(G)])
    flags = np.zeros((G, N), np.int64)
    flags |= np.where(rms < f32(p["rms_dead"]), DEAD, 0)
    flags |= np.where(rms > f32(p["noisy_factor"]) * med[:, None], NOISY, 0)
    pedd = np.round(256.0 * np.asarray(ped, np.float32).reshape(G, N).astype(np.float64)) / 256.0
    flags |= np.where(np.abs(mean - pedd) > f32(p["ped_tol"]), PED_SHIFT, 0)
    flags |= np.where(n_sat > f32(p["sat_frac"]) * n, SATURATING, 0)
    bad = int(np.any(flags != 0, axis=0).sum())
    return ({"n": np.full((G, N), n, np.int64), "S1": S1, "S2": S2, "n_sat": n_sat, "mean": mean, "rms": rms,
             "flags": flags},
            {"median_rms": med, "n_bad": bad, "verdict": int(bad > f32(p["bad_frac_max"]) * N)})
