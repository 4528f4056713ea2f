"""Pins of the alert-monitor oracle: the Li & Ma significance against the
on/off Poisson likelihood-ratio statistic evaluated with scipy, its closed
special cases, the counts cube against numpy's histogramdd, exact zero
significance for a flat sky (edge cells included), mirror symmetry, and a
planted flare found at its place and timescale.  CPU only."""
import math

import numpy as np
import pytest
from scipy.stats import poisson

import dl0sim.workloads as W
from oracle import sam

P = {"grid": 32, "cell": 0.002, "t0": 0.0, "bin_s": 1.0, "n_bins": 600, "r_on": 1.5, "r_in": 3.0, "r_out": 6.0,
     "gamma_cut": 0.7, "scales": [1, 10, 100, 600], "sigma_alert": 5.0}


def lr_statistic(n_on, n_off, alpha):
    """-2 ln(lambda) of the on/off problem (N_on ~ Pois(s + alpha b),
    N_off ~ Pois(b)) from Poisson log-likelihoods at the maximum-likelihood
    points: free fit s = N_on - alpha N_off, b = N_off; null fit s = 0,
    b = (N_on + N_off) / (1 + alpha)."""
    b0 = (n_on + n_off) / (1.0 + alpha)
    l1 = poisson.logpmf(n_on, max(n_on, 1e-300)) + poisson.logpmf(n_off, max(n_off, 1e-300))
    l0 = poisson.logpmf(n_on, alpha * b0) + poisson.logpmf(n_off, b0)
    return 2.0 * (l1 - l0)


def test_li_ma_equals_the_likelihood_ratio():
    rng = np.random.default_rng(0)
    for _ in range(300):
        alpha = float(rng.uniform(0.02, 3.0))
        n_off = int(rng.integers(0, 400))
        n_on = int(rng.integers(0, 400))
        if n_on + n_off == 0:
            continue
        s = sam.li_ma(n_on, n_off, alpha)
        assert s * s == pytest.approx(lr_statistic(n_on, n_off, alpha), rel=1e-9, abs=1e-9)
        assert (s > 0) == (n_on > alpha * n_off) or s == 0


def test_li_ma_special_cases():
    assert sam.li_ma(30, 60, 0.5) == 0.0
    assert sam.li_ma_cells(27, 312, 9, 104) == 0.0          # alpha * N_off = 27 only up to rounding
    assert sam.li_ma_cells(28, 312, 9, 104) > 0 > sam.li_ma_cells(26, 312, 9, 104)
    assert sam.li_ma(0, 0, 0.3) == 0.0
    a = 0.25
    assert sam.li_ma(17, 0, a) == pytest.approx(math.sqrt(2 * 17 * math.log((1 + a) / a)), rel=1e-14)
    assert sam.li_ma(0, 40, a) == pytest.approx(-math.sqrt(2 * 40 * math.log(1 + a)), rel=1e-14)
    # large counts: the Gaussian limit (N_on - alpha N_off) / sqrt(alpha (N_on + N_off))
    n_on, n_off, a = 1_000_000, 4_000_000, 0.249
    assert sam.li_ma(n_on, n_off, a) == pytest.approx((n_on - a * n_off) / math.sqrt(a * (n_on + n_off)), rel=2e-3)


def test_histogram_matches_histogramdd():
    t, d, g, v = W.sam_events(1, 600.0, 40.0, 0.03, [(0.01, -0.005, 100.0, 160.0, 2.0, 0.001)])
    C, used = sam.histogram(d, t, g, v, P)
    sel = v & (g >= P["gamma_cut"])
    edges_t = np.arange(P["n_bins"] + 1) * P["bin_s"] + P["t0"]
    edges_xy = (np.arange(P["grid"] + 1) - P["grid"] / 2) * P["cell"]
    H, _ = np.histogramdd(np.stack([t[sel], d[sel, 1], d[sel, 0]], 1).astype(np.float64),
                          bins=[edges_t, edges_xy, edges_xy])
    # histogramdd closes the last bin on the right; no event sits on an edge here
    assert np.array_equal(C, H.astype(np.int64)) and used == int(H.sum())


def test_flat_sky_has_zero_significance_everywhere():
    C = np.full((10, P["grid"], P["grid"]), 3, np.int64)
    out, alerts = sam.search(C, 9, dict(P, scales=[1, 4]))
    for o in out:
        assert np.all(o["S"] == 0.0)
        assert np.allclose(o["alpha"] * o["N_off"], o["N_on"])
    assert not alerts


def test_mirror_symmetry():
    t, d, g, v = W.sam_events(2, 200.0, 80.0, 0.03, [(0.012, 0.004, 50.0, 90.0, 3.0, 0.001)])
    p = dict(P, scales=[10, 200])
    C, _ = sam.histogram(d, t, g, v, p)
    dm = d.copy()
    dm[:, 0] = -dm[:, 0]
    Cm, _ = sam.histogram(dm, t, g, v, p)
    assert np.array_equal(Cm, C[:, :, ::-1])
    a, _ = sam.search(C, 199, p)
    b, _ = sam.search(Cm, 199, p)
    for x, y in zip(a, b):
        assert np.array_equal(y["N_on"], x["N_on"][:, ::-1]) and np.allclose(y["S"], x["S"][:, ::-1])


def test_planted_flare_is_found_at_its_place_and_timescale():
    """A 60 s flare 8 mrad off axis: the 10 s and 100 s windows ending in it
    alert at its cell; the background-only sky stays below 5 sigma."""
    src = (0.008, -0.006)
    t, d, g, v = W.sam_events(3, 600.0, 30.0, 0.03, [(src[0], src[1], 300.0, 360.0, 4.0, 0.0008)])
    C, _ = sam.histogram(d, t, g, v, P)
    out, alerts = sam.search(C, 359, P)
    ix = math.floor(src[0] / P["cell"] + P["grid"] / 2)
    iy = math.floor(src[1] / P["cell"] + P["grid"] / 2)
    by_scale = {}
    for si, x, y, s in alerts:
        by_scale.setdefault(si, []).append((x, y, s))
    for si in (1, 2):
        best = max(by_scale[si], key=lambda a: a[2])
        assert abs(best[0] - ix) <= 1 and abs(best[1] - iy) <= 1
    t0, d0, g0, v0 = W.sam_events(3, 600.0, 30.0, 0.03, [])
    C0, _ = sam.histogram(d0, t0, g0, v0, P)
    out0, alerts0 = sam.search(C0, 359, P)
    assert not alerts0 and max(o["S"].max() for o in out0) < 5.0
