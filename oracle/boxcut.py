"""Oracle of the classification decisions — TEST INFRASTRUCTURE ONLY.

Applies box-cut tables (any object with the rta_boxcut_desc fields) and the
network outputs to feature rows, following the stated rule: the network
decides when all ten features are finite and inside the trained range,
otherwise the scaled-width / scaled-length box cut decides and the energy is
the linear fit in log10 size.  Decisions that are integers are taken in
float32, the precision of the kernels.

Parity status: pinned by hand-derived decisions, bin clamping and fallback
cases (tests/test_oracle_boxcut.py).
"""
from __future__ import annotations

import math

import numpy as np


def classify(table, feat, logit=None, log10e_net=None):
    """feat [n][10] (float32 values).  Returns score, log10e, gamma, fallback."""
    f = np.asarray(feat, np.float32)
    n = f.shape[0]
    lo = np.array(table.feat_lo, np.float32)
    hi = np.array(table.feat_hi, np.float32)
    have = logit is not None
    in_range = np.all(np.isfinite(f) & (f >= lo) & (f <= hi), axis=1) & have
    lgs = f[:, 0]
    nb = int(table.n_bins)
    span = np.float32(table.lgs_hi) - np.float32(table.lgs_lo)
    b = np.floor((lgs - np.float32(table.lgs_lo)) / span * np.float32(nb))
    b = np.where(np.isfinite(b), b, 0).astype(np.int64)
    b = np.clip(b, 0, nb - 1)
    sw = (f[:, 2] - np.array(table.w_mean, np.float32)[b]) / np.array(table.w_std, np.float32)[b]
    sl = (f[:, 1] - np.array(table.l_mean, np.float32)[b]) / np.array(table.l_std, np.float32)[b]
    box = (sw < np.float32(table.cut_w)) & (sl < np.float32(table.cut_l))
    score = np.where(box, 1.0, 0.0)
    e = np.float64(table.e_a) + np.float64(table.e_b) * lgs.astype(np.float64)
    gamma = box.copy()
    if have:
        z = np.asarray(logit, np.float64)
        s = 1.0 / (1.0 + np.exp(-z))
        score = np.where(in_range, s, score)
        e = np.where(in_range, np.asarray(log10e_net, np.float64), e)
        gamma = np.where(in_range, s > table.mlp_cut, box)
    return score, e, gamma.astype(np.int64), (~in_range).astype(np.int64)


def bin_edge_distance(table, lgs):
    """Distance of log10 size to the nearest internal bin edge (to skip
    knife-edge comparisons in parity tests)."""
    edges = np.linspace(table.lgs_lo, table.lgs_hi, int(table.n_bins) + 1)
    return np.min(np.abs(np.asarray(lgs, np.float64)[:, None] - edges[None, :]), axis=1)
