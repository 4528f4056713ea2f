"""Scaled-width / scaled-length box cuts: table preparation from training data.

Prepares the rta_boxcut_desc tables the classification kernels apply:
per log10(size) bin, the mean and standard deviation of width and length of
training gammas; the pair of cuts (SW < cut_w and SL < cut_l) that reaches a
target gamma efficiency with the fewest hadrons; a linear log10 E fit on
log10 size; the feature range the network was trained on; and the network
score threshold that gives the same gamma efficiency.  This is offline table
preparation on the host (the per-telescope decisions run in the kernels).
"""
from __future__ import annotations

import numpy as np

import paper_1307_6489_amd as rta

# a tiny relative margin keeps training-set extremes off the range edges
RANGE_MARGIN = 1e-6


def _bin_index(lgs, lo, hi, n):
    b = np.floor((lgs - lo) / (hi - lo) * n).astype(np.int64)
    return np.clip(b, 0, n - 1)


def fit(feat_g, feat_h, log10e_g, target_eff=0.7, n_bins=20, grid=np.linspace(-3.0, 6.0, 181),
        feat_all=None) -> rta.BoxCutDesc:
    """feat_g / feat_h: [n][10] features of training gammas / hadrons (columns as
    in the network input: log10 size first, length second, width third)."""
    feat_g = np.asarray(feat_g, np.float64)
    feat_h = np.asarray(feat_h, np.float64)
    ok_g = np.all(np.isfinite(feat_g), 1)
    ok_h = np.all(np.isfinite(feat_h), 1)
    g, h = feat_g[ok_g], feat_h[ok_h]
    lgs = g[:, 0]
    lo, hi = float(np.min(lgs)), float(np.max(lgs)) + 1e-6
    bc = rta.BoxCutDesc()
    bc.n_bins, bc.lgs_lo, bc.lgs_hi = n_bins, lo, hi
    b = _bin_index(lgs, lo, hi, n_bins)
    gl_w = (float(np.mean(g[:, 2])), float(np.std(g[:, 2])) + 1e-6)
    gl_l = (float(np.mean(g[:, 1])), float(np.std(g[:, 1])) + 1e-6)
    for k in range(n_bins):
        sel = b == k
        if sel.sum() >= 10:
            bc.w_mean[k], bc.w_std[k] = float(np.mean(g[sel, 2])), float(np.std(g[sel, 2])) + 1e-6
            bc.l_mean[k], bc.l_std[k] = float(np.mean(g[sel, 1])), float(np.std(g[sel, 1])) + 1e-6
        else:
            (bc.w_mean[k], bc.w_std[k]), (bc.l_mean[k], bc.l_std[k]) = gl_w, gl_l
    sw_g, sl_g = scaled(bc, g)
    sw_h, sl_h = scaled(bc, h)
    best = None
    for cw in grid:
        pass_w_g = sw_g < cw
        pass_w_h = sw_h < cw
        for cl in grid:
            eff = np.mean(pass_w_g & (sl_g < cl))
            if eff < target_eff:
                continue
            acc = np.mean(pass_w_h & (sl_h < cl))
            key = (acc, eff)
            if best is None or key < best[0]:
                best = (key, cw, cl)
    bc.cut_w, bc.cut_l = float(best[1]), float(best[2])
    A = np.stack([np.ones_like(lgs), lgs], 1)
    coef = np.linalg.lstsq(A, np.asarray(log10e_g, np.float64)[ok_g], rcond=None)[0]
    bc.e_a, bc.e_b = float(coef[0]), float(coef[1])
    fa = np.concatenate([g, h]) if feat_all is None else np.asarray(feat_all, np.float64)
    fa = fa[np.all(np.isfinite(fa), 1)]
    for f in range(10):
        lo_f, hi_f = float(np.min(fa[:, f])), float(np.max(fa[:, f]))
        bc.feat_lo[f] = lo_f - RANGE_MARGIN * (abs(lo_f) + 1e-30)
        bc.feat_hi[f] = hi_f + RANGE_MARGIN * (abs(hi_f) + 1e-30)
    bc.mlp_cut = 0.5
    return bc


def scaled(bc, feat):
    """Scaled width and length of feature rows under the tables (float32,
    as the kernels compute them)."""
    f = np.asarray(feat, np.float32)
    b = _bin_index(f[:, 0].astype(np.float64), bc.lgs_lo, bc.lgs_hi, bc.n_bins)
    wm = np.array(bc.w_mean, np.float32)[b]
    ws = np.array(bc.w_std, np.float32)[b]
    lm = np.array(bc.l_mean, np.float32)[b]
    ls = np.array(bc.l_std, np.float32)[b]
    return (f[:, 2] - wm) / ws, (f[:, 1] - lm) / ls


def set_score_cut(bc, gamma_scores, target_eff=0.7):
    """Network threshold giving the target efficiency on training gammas."""
    s = np.sort(np.asarray(gamma_scores, np.float64))
    bc.mlp_cut = float(s[int(np.floor((1.0 - target_eff) * len(s)))])
    return bc
