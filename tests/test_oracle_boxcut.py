"""Pins of the classification-decision oracle against hand-derived cases: the
scaled width / length of a row in its log10-size bin (bins clamped at both
ends), the box decision and the linear energy, and the rule that hands a
row to the network only when every feature is finite and inside the trained
range.  CPU only."""
import math
from types import SimpleNamespace

import numpy as np

from oracle import boxcut


def table():
    """Two log10-size bins [1, 2) and [2, 3]; width mean / std 0.1 / 0.01
    and 0.2 / 0.02, length 0.3 / 0.05 and 0.5 / 0.1; cuts SW < 1.5,
    SL < 2.0; log10 E = -3 + log10 size; trained range [-10, 10] for every
    feature; network threshold 0.5."""
    return SimpleNamespace(n_bins=2, lgs_lo=1.0, lgs_hi=3.0, w_mean=[0.1, 0.2], w_std=[0.01, 0.02],
                           l_mean=[0.3, 0.5], l_std=[0.05, 0.1], cut_w=1.5, cut_l=2.0, e_a=-3.0, e_b=1.0,
                           feat_lo=[-10.0] * 10, feat_hi=[10.0] * 10, mlp_cut=0.5)


def row(lgs, length, width):
    f = np.zeros(10, np.float32)
    f[0], f[1], f[2] = lgs, length, width
    return f


def test_box_decisions_by_hand():
    """Row 0: bin 0, SW = (0.11 - 0.1) / 0.01 = 1, SL = (0.35 - 0.3) / 0.05 = 1:
    gamma, log10 E = -1.5.  Row 1: bin 1, SW = (0.25 - 0.2) / 0.02 = 2.5:
    hadron, log10 E = -0.5.  Row 2: bin 1, SW = 0, SL = (0.72 - 0.5) / 0.1
    = 2.2: hadron (length cut).  Row 3: log10 size 0.2 below the first bin
    (clamped to bin 0), SW = SL = 0: gamma, log10 E = -2.8.  Row 4: log10
    size 3.7 above the last bin (clamped to bin 1), width 0.23 -> SW = 1.5,
    not below the cut: hadron.  Without a network every row falls back."""
    f = np.stack([row(1.5, 0.35, 0.11), row(2.5, 0.5, 0.25), row(2.2, 0.72, 0.2), row(0.2, 0.3, 0.1),
                  row(3.7, 0.5, 0.2 + 1.5 * 0.02 + 1e-4)])
    score, e, gamma, fb = boxcut.classify(table(), f)
    assert list(gamma) == [1, 0, 0, 1, 0]
    assert list(score) == [1.0, 0.0, 0.0, 1.0, 0.0]
    assert np.allclose(e, [-1.5, -0.5, -0.8, -2.8, 0.7], atol=1e-6)
    assert list(fb) == [1, 1, 1, 1, 1]


def test_width_and_length_are_not_swapped():
    """A row narrow in width but long: the length cut rejects it; swapping
    the two features would accept it."""
    f = np.stack([row(1.5, 0.45, 0.1)])        # SL = 3 > 2, SW = 0
    _, _, gamma, _ = boxcut.classify(table(), f)
    assert list(gamma) == [0]
    _, _, gamma, _ = boxcut.classify(table(), np.stack([row(1.5, 0.3, 0.1)]))
    assert list(gamma) == [1]


def test_network_decides_only_inside_the_trained_range():
    """With network outputs: an in-range row takes sigmoid(logit) as score,
    the network energy and score > 0.5 as decision (logit 2 -> 0.8808,
    gamma even though the box says hadron; logit -1 -> 0.2689, hadron even
    though the box says gamma).  A NaN feature, an infinite one, and a
    feature above the trained range fall back to the box decision and the
    linear energy."""
    f = np.stack([row(2.5, 0.5, 0.25), row(1.5, 0.35, 0.11), row(1.5, 0.35, 0.11), row(1.5, 0.35, 0.11),
                  row(1.5, 0.35, 0.11)])
    f[2, 5] = np.nan
    f[3, 7] = np.inf
    f[4, 8] = 10.5
    logit = np.array([2.0, -1.0, 3.0, 3.0, 3.0])
    e_net = np.array([0.25, 0.5, 9.0, 9.0, 9.0])
    score, e, gamma, fb = boxcut.classify(table(), f, logit, e_net)
    s = 1.0 / (1.0 + math.exp(-2.0)), 1.0 / (1.0 + math.exp(1.0))
    assert abs(score[0] - s[0]) < 1e-12 and abs(score[1] - s[1]) < 1e-12
    assert list(gamma) == [1, 0, 1, 1, 1]
    assert list(fb) == [0, 0, 1, 1, 1]
    assert np.allclose(e, [0.25, 0.5, -1.5, -1.5, -1.5], atol=1e-6)
    assert list(score[2:]) == [1.0, 1.0, 1.0]


def test_range_edges_are_inside():
    """A feature exactly at the trained minimum or maximum is in range."""
    t = table()
    f = np.stack([row(1.5, 0.35, 0.11), row(1.5, 0.35, 0.11)])
    f[0, 4] = -10.0
    f[1, 4] = 10.0
    _, _, _, fb = boxcut.classify(t, f, np.zeros(2), np.zeros(2))
    assert list(fb) == [0, 0]
