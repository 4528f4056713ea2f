"""Oracle of the science alert monitor (SAM) — TEST INFRASTRUCTURE ONLY.

The paper's real-time analysis must search for transients on several
integration timescales, from seconds to hours, inside a source region and
elsewhere in the field of view, and raise science alerts (Section 2,
requirement (ii); Section 4.2, the SAM sub-function).  It gives no method;
the reading implemented here (plain loops and numpy, FP64):

  selection    array events with a valid stereo direction and gammaness >=
               gamma_cut
  binning      time bin b = floor((t - t0) / bin_s), 0 <= b < n_bins; sky
               cell ix = floor(dir_x / cell + grid/2), iy likewise,
               0 <= ix, iy < grid (nominal frame, radians)
  counts       C[b][iy][ix] = number of selected events
  window       for a timescale of w bins ending at bin e:
               W[iy][ix] = sum of C[b][iy][ix] over e-w < b <= e (b >= 0)
  on / off     for the cell (x, y): N_on = sum of W over the grid cells at
               squared cell distance d2 <= r_on^2, N_off = sum over
               r_in^2 < d2 <= r_out^2; alpha = (number of on cells) /
               (number of off cells), both counted inside the grid (flat
               acceptance)
  significance Li & Ma (1983) eq. 17: S = sign(N_on - alpha N_off) *
               sqrt(2 (N_on ln[(1+alpha)/alpha * N_on/(N_on+N_off)]
                         + N_off ln[(1+alpha) N_off/(N_on+N_off)])),
               a term with a zero count contributes 0; S = 0 when
               N_on + N_off = 0, when there are no off cells, and when the
               excess is exactly zero (N_on * off cells == on cells * N_off,
               decided in integers)
  alert        S >= sigma_alert

Parity status: pinned by the Poisson likelihood ratio, closed special cases,
numpy.histogramdd, a flat sky, mirror symmetry and a planted flare
(tests/test_oracle_sam.py).
"""
from __future__ import annotations

import math

import numpy as np


def li_ma(n_on, n_off, alpha):
    """Li & Ma eq. 17 with the sign of the excess (scalar, FP64)."""
    n_on, n_off, alpha = float(n_on), float(n_off), float(alpha)
    if n_on + n_off <= 0 or alpha <= 0:
        return 0.0
    tot = n_on + n_off
    t1 = n_on * math.log((1.0 + alpha) / alpha * n_on / tot) if n_on > 0 else 0.0
    t2 = n_off * math.log((1.0 + alpha) * n_off / tot) if n_off > 0 else 0.0
    v = max(2.0 * (t1 + t2), 0.0)
    return math.copysign(math.sqrt(v), n_on - alpha * n_off) if n_on != alpha * n_off else 0.0


def li_ma_cells(n_on, n_off, c_on, c_off):
    """Li & Ma with alpha = c_on / c_off, the zero excess decided exactly."""
    if c_off <= 0 or n_on * c_off == c_on * n_off:
        return 0.0
    return li_ma(n_on, n_off, c_on / c_off)


def f32(v):
    """The float parameters (cell, radii, cuts) are 32-bit in the interface."""
    return float(np.float32(v))


def histogram(evt_dir, evt_time, gammaness, valid, p):
    """Counts cube [n_bins][grid][grid] (int64) and the number of selected
    events that fell inside it."""
    G, nb = p["grid"], p["n_bins"]
    cell, cut = f32(p["cell"]), np.float32(p["gamma_cut"])
    C = np.zeros((nb, G, G), np.int64)
    used = 0
    for k in range(len(evt_time)):
        if not valid[k] or not (np.float32(gammaness[k]) >= cut):
            continue
        b = math.floor((float(evt_time[k]) - p["t0"]) / p["bin_s"])
        ix = math.floor(float(evt_dir[k, 0]) / cell + G / 2)
        iy = math.floor(float(evt_dir[k, 1]) / cell + G / 2)
        if 0 <= b < nb and 0 <= ix < G and 0 <= iy < G:
            C[b, iy, ix] += 1
            used += 1
    return C, used


def window(C, end_bin, w):
    lo = max(end_bin - w + 1, 0)
    return C[lo:end_bin + 1].sum(axis=0)


def search(C, end_bin, p):
    """Per timescale: significance map [G][G], N_on, N_off, alpha maps, and
    the alerts [(scale index, ix, iy, S)]."""
    G = p["grid"]
    r_on2, r_in2, r_out2 = f32(p["r_on"]) ** 2, f32(p["r_in"]) ** 2, f32(p["r_out"]) ** 2
    reach = int(math.ceil(f32(p["r_out"])))
    thr = f32(p["sigma_alert"])
    out = []
    alerts = []
    for si, w in enumerate(p["scales"]):
        Wm = window(C, end_bin, w)
        S = np.zeros((G, G))
        Non = np.zeros((G, G), np.int64)
        Noff = np.zeros((G, G), np.int64)
        A = np.zeros((G, G))
        for y in range(G):
            for x in range(G):
                non = noff = con = coff = 0
                for dy in range(-reach, reach + 1):
                    for dx in range(-reach, reach + 1):
                        yy, xx = y + dy, x + dx
                        if not (0 <= yy < G and 0 <= xx < G):
                            continue
                        d2 = dx * dx + dy * dy
                        if d2 <= r_on2:
                            non += Wm[yy, xx]
                            con += 1
                        elif r_in2 < d2 <= r_out2:
                            noff += Wm[yy, xx]
                            coff += 1
                alpha = con / coff if coff else 0.0
                s = li_ma_cells(non, noff, con, coff)
                S[y, x], Non[y, x], Noff[y, x], A[y, x] = s, non, noff, alpha
                if s >= thr:
                    alerts.append((si, x, y, s))
        out.append({"S": S, "N_on": Non, "N_off": Noff, "alpha": A})
    return out, alerts
