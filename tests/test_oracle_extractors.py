"""Pins of the oracle's alternative signal extractors (fixed window, global
peak window, neighbour peak window) against hand-derived values, reductions
to the pinned sliding window, locality and translation invariances.  CPU
only."""
import numpy as np
import pytest

import dl0sim
import oracle

P = 0.05
EX = (oracle.EX_SLIDING, oracle.EX_FIXED, oracle.EX_GLOBAL_PEAK, oracle.EX_NEIGHBOUR_PEAK)


def cam_of(n_pix, T, G, ped, a, extractor, fixed_start=None, w=4, switch=4000, x=None, y=None):
    x = np.arange(n_pix, dtype=np.float32) * P if x is None else x
    y = np.zeros(n_pix, np.float32) if y is None else y
    return oracle.Camera(n_pix, T, G, x, y, np.full((G, n_pix), ped, np.float32),
                         np.full((G, n_pix), a, np.float32), P, window=w, hg_switch=switch,
                         extractor=extractor, fixed_start=fixed_start)


def event_of(traces):
    """traces [G][N][T] -> uint16 [G][T][Npad]."""
    tr = np.asarray(traces, np.int64)
    G, N, T = tr.shape
    ev = np.zeros((G, T, (N + 7) // 8 * 8), np.uint16)
    ev[:, :, :N] = np.transpose(tr, (0, 2, 1))
    return ev


def test_fixed_window_hand_case():
    """T = 8, w = 4, s0 = 2, pedestal 3 ADC (P = 768), 2 ADC/p.e.; trace
    0 0 9 1 1 1 50 50: the sliding window would take s = 4 (sum 102), the
    fixed window takes samples 2..5: S = 12, D = 256*12 - 4*768 = 0,
    Nt = 0*(2304-768) + 1*(256-768) + 2*(256-768) + 3*(256-768) = -3072,
    peak = 2 (the 9), t = s0 + (w-1)/2 = 3.5 because D <= 0."""
    trace = [0, 0, 9, 1, 1, 1, 50, 50]
    fx = cam_of(1, 8, 1, 3.0, 2.0, oracle.EX_FIXED, fixed_start=2).calibrate(event_of([[trace]]))[0]
    assert (int(fx["S"]), int(fx["D"]), int(fx["Nt"]), int(fx["sstar"]), int(fx["peak"])) == (12, 0, -3072, 2, 2)
    assert fx["t"] == 3.5 and fx["q"] == 0.0
    sl = cam_of(1, 8, 1, 3.0, 2.0, oracle.EX_SLIDING).calibrate(event_of([[trace]]))[0]
    assert (int(sl["S"]), int(sl["sstar"])) == (102, 4)
    # a positive charge: pedestal 0 -> D = 256*12 = 3072, q = 3072/(256*2) = 6,
    # Nt = 256*(0*9 + 1*1 + 2*1 + 3*1) = 1536, t = 2 + 1536/3072 = 2.5
    fx = cam_of(1, 8, 1, 0.0, 2.0, oracle.EX_FIXED, fixed_start=2).calibrate(event_of([[trace]]))[0]
    assert (int(fx["D"]), int(fx["Nt"])) == (3072, 1536)
    assert fx["q"] == 6.0 and fx["t"] == 2.5


def test_fixed_window_gain_looks_inside_the_window_only():
    """Dual gain: a saturated high-gain sample outside the window does not
    switch the pixel (the sliding window's rule would); one inside does, and
    then the charge comes from the low-gain samples of the same window."""
    T, s0 = 12, 4
    hg = np.full((3, T), 300)
    lg = np.full((3, T), 300)
    hg[0, 0] = 4095                       # pixel 0: saturated before the window
    hg[1, s0 + 1] = 4000                  # pixel 1: at the switch inside the window
    lg[1, s0:s0 + 4] = [310, 400, 320, 305]
    hg[2, s0 - 1] = hg[2, s0 + 4] = 4095  # pixel 2: saturated just outside both ends
    ev = event_of([hg, lg])
    fx = cam_of(3, T, 2, 300.0, 1.0, oracle.EX_FIXED, fixed_start=s0).calibrate(ev)
    sl = cam_of(3, T, 2, 300.0, 1.0, oracle.EX_SLIDING).calibrate(ev)
    assert list(fx["gain"]) == [0, 1, 0] and list(sl["gain"]) == [1, 1, 1]
    assert int(fx["S"][0]) == 4 * 300 and int(fx["S"][1]) == 310 + 400 + 320 + 305
    assert int(fx["sstar"][1]) == s0 and int(fx["peak"][1]) == s0 + 1


def test_fixed_window_reads_nothing_outside_the_window():
    """Random dual-gain traces: rewriting every sample outside s0..s0+w-1 (both
    gains) leaves every output unchanged; changing one sample inside moves S."""
    rng = np.random.default_rng(1)
    N, T, s0 = 19, 30, 11
    for trial in range(20):
        tr = rng.integers(250, 4200, size=(2, N, T))
        cam = cam_of(N, T, 2, 300.0, 10.0, oracle.EX_FIXED, fixed_start=s0)
        a = cam.calibrate(event_of(tr))
        tr2 = tr.copy()
        outside = np.ones(T, bool)
        outside[s0:s0 + 4] = False
        tr2[:, :, outside] = rng.integers(0, 65536, size=tr2[:, :, outside].shape)
        b = cam.calibrate(event_of(tr2))
        assert a.tobytes() == b.tobytes()
        tr3 = tr.copy()
        tr3[:, :, s0 + 2] += 1
        c = cam.calibrate(event_of(tr3))
        assert np.array_equal(c["S"], a["S"] + 1)


def test_fixed_window_equals_sliding_when_the_pulse_fills_the_window():
    """Zero outside the fixed window and positive inside: the sliding window's
    unique maximiser is s0, so every output equals the pinned sliding one."""
    rng = np.random.default_rng(2)
    N, T, s0 = 7, 25, 9
    tr = np.zeros((1, N, T), np.int64)
    tr[0, :, s0:s0 + 4] = rng.integers(1, 3000, size=(N, 4))
    a = cam_of(N, T, 1, 0.0, 7.0, oracle.EX_FIXED, fixed_start=s0).calibrate(event_of(tr))
    b = cam_of(N, T, 1, 0.0, 7.0, oracle.EX_SLIDING).calibrate(event_of(tr))
    assert a.tobytes() == b.tobytes()


def test_global_peak_planted_pulse():
    """Flat pedestals everywhere and one pulse in one pixel at samples p..p+3:
    every pixel's window starts at p, and the pulse pixel's charge is the
    pulse."""
    N, T = 7, 40
    for p in (0, 5, 17, T - 4):
        tr = np.full((1, N, T), 300, np.int64)
        tr[0, 3, p:p + 4] += [50, 200, 120, 30]
        r = cam_of(N, T, 1, 300.0, 10.0, oracle.EX_GLOBAL_PEAK).calibrate(event_of(tr))
        assert np.all(r["sstar"] == p)
        assert int(r["D"][3]) == 256 * 400 and int(r["peak"][3]) == p + 1
        assert np.all(r["D"][np.arange(N) != 3] == 0)


def test_global_peak_earliest_of_equal_pulses():
    """Two equal pulses in different pixels at p1 < p2: the first wins."""
    N, T = 5, 30
    tr = np.full((1, N, T), 300, np.int64)
    tr[0, 1, 20:24] += 100
    tr[0, 4, 6:10] += 100
    r = cam_of(N, T, 1, 300.0, 10.0, oracle.EX_GLOBAL_PEAK).calibrate(event_of(tr))
    assert np.all(r["sstar"] == 6)


def test_global_peak_reduces_to_sliding():
    """One pixel: the camera sum is the pixel's own window sum, so global peak
    and sliding window agree on random traces (ties included: both take the
    first maximiser).  Identical traces in every pixel: the same."""
    rng = np.random.default_rng(3)
    for trial in range(200):
        T = int(rng.integers(4, 20))
        tr = rng.integers(0, 4, size=(1, 1, T))
        a = cam_of(1, T, 1, 0.0, 1.0, oracle.EX_GLOBAL_PEAK).calibrate(event_of(tr))
        b = cam_of(1, T, 1, 0.0, 1.0, oracle.EX_SLIDING).calibrate(event_of(tr))
        assert a.tobytes() == b.tobytes()
    tr = np.repeat(rng.integers(250, 900, size=(1, 1, 33)), 9, axis=1)
    a = cam_of(9, 33, 1, 300.0, 10.0, oracle.EX_GLOBAL_PEAK).calibrate(event_of(tr))
    b = cam_of(9, 33, 1, 300.0, 10.0, oracle.EX_SLIDING).calibrate(event_of(tr))
    assert a.tobytes() == b.tobytes()


def test_global_peak_places_on_high_gain_and_integrates_the_selected_gain():
    """Dual gain: the window is placed by the raw high-gain camera sum even
    where the low gain peaks elsewhere; a switched pixel integrates its low
    gain at that start."""
    N, T = 3, 24
    hg = np.full((N, T), 300, np.int64)
    lg = np.full((N, T), 300, np.int64)
    hg[0, 8:12] = [1000, 4095, 4095, 2000]   # pixel 0 switches
    lg[0, 8:12] = [350, 800, 700, 420]
    lg[0, 16:20] = 2000                      # a larger low-gain bump elsewhere
    hg[2, 9:13] += 40
    r = cam_of(N, T, 2, 300.0, 10.0, oracle.EX_GLOBAL_PEAK).calibrate(event_of([hg, lg]))
    assert np.all(r["sstar"] == 8) and list(r["gain"]) == [1, 0, 0]
    assert int(r["S"][0]) == 350 + 800 + 700 + 420


def test_window_placement_is_translation_covariant():
    """Delaying every trace by d samples (the first d samples repeat the
    pedestal) delays the window start by d for every extractor (the fixed
    start moves with it), with identical charges."""
    rng = np.random.default_rng(4)
    N, T, d = 19, 40, 5
    tr = np.full((2, N, T), 300, np.int64)
    tr += rng.integers(-4, 5, size=tr.shape)
    tr[0, :, 10:14] += rng.integers(0, 3000, size=(N, 4))
    tr[1] = 300 + (tr[0] - 300) // 16
    late = np.full_like(tr, 300)
    late[:, :, d:] = tr[:, :, :T - d]
    for ex in EX:
        a = cam_of(N, T, 2, 300.0, 10.0, ex, fixed_start=10).calibrate(event_of(tr))
        b = cam_of(N, T, 2, 300.0, 10.0, ex, fixed_start=10 + d).calibrate(event_of(late))
        ok = a["sstar"] + d <= T - 4        # windows that do not run off the end
        assert np.array_equal(b["sstar"][ok], a["sstar"][ok] + d)
        for k in ("S", "D", "Nt", "gain"):
            assert np.array_equal(b[k][ok], a[k][ok]), (ex, k)


def test_generated_events_through_every_extractor():
    """Every extractor on generated C0 events: window starts inside the trace,
    S is the window sum at s*, and the global peak start is common to all
    pixels."""
    cam = dl0sim.camera_c0()
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(cam.n_samp), 0, 0, 4)
    tr = dl0sim.render_traces(cam, sh, 0, event_ids=np.arange(4, dtype=np.uint64))
    for ex in EX:
        oc = oracle.Camera.from_type(cam, extractor=ex)
        for e in range(4):
            r = oc.calibrate(tr[e])
            assert np.all((r["sstar"] >= 0) & (r["sstar"] <= cam.n_samp - cam.window))
            x = tr[e, 0, :, :cam.n_pix].astype(np.int64)
            s = r["sstar"]
            S = sum(x[s + k, np.arange(cam.n_pix)] for k in range(cam.window))
            assert np.array_equal(r["S"], S)
            if ex == oracle.EX_GLOBAL_PEAK:
                assert len(set(s.tolist())) == 1
            if ex == oracle.EX_FIXED:
                assert np.all(s == cam.fixed_start)


def test_unknown_extractor_and_bad_fixed_start_are_rejected():
    with pytest.raises(ValueError):
        cam_of(1, 8, 1, 0.0, 1.0, 7)
    with pytest.raises(ValueError):
        cam_of(1, 8, 1, 0.0, 1.0, oracle.EX_FIXED, fixed_start=5)


def test_neighbour_peak_hand_case():
    """Three pixels in a row (0-1-2 neighbours), T = 10, w = 4, pedestal 0:
    pixel 0 carries 100 at samples 1..4, pixel 1 500 at 5..8, pixel 2 60 at
    2..5.  Pixel 0's window follows its one neighbour (pixel 1): s* = 5, where
    its own samples are 0.  Pixel 1 sums pixels 0 and 2: C(0) = 300 + 120,
    C(1) = 400 + 180, C(2) = 300 + 240, C(3) = 200 + 180: s* = 1, S = 0.
    Pixel 2 follows pixel 1: s* = 5, S = 60 (its sample 5)."""
    T = 10
    tr = np.zeros((1, 3, T), np.int64)
    tr[0, 0, 1:5] = 100
    tr[0, 1, 5:9] = 500
    tr[0, 2, 2:6] = 60
    r = cam_of(3, T, 1, 0.0, 1.0, oracle.EX_NEIGHBOUR_PEAK).calibrate(event_of(tr))
    assert list(r["sstar"]) == [5, 1, 5] and list(r["S"]) == [0, 0, 60]
    assert list(r["peak"]) == [5, 1, 5]


def test_neighbour_peak_without_neighbours_starts_at_zero():
    """A lone pixel has C(s) = 0 for every s: the first start, 0."""
    tr = np.array([[[5, 1, 1, 1, 90, 90, 90, 90]]])
    r = cam_of(1, 8, 1, 0.0, 1.0, oracle.EX_NEIGHBOUR_PEAK).calibrate(event_of(tr))[0]
    assert int(r["sstar"]) == 0 and int(r["S"]) == 8


def test_neighbour_peak_reduces_to_sliding_for_identical_traces():
    """The same trace in every pixel of a row: C_i(s) = (number of
    neighbours) x W(s), whose first maximiser is the sliding window's (ties
    included), so every output is the pinned sliding one."""
    rng = np.random.default_rng(5)
    for trial in range(200):
        T = int(rng.integers(4, 20))
        N = int(rng.integers(2, 6))
        tr = np.repeat(rng.integers(0, 4, size=(1, 1, T)), N, axis=1)
        a = cam_of(N, T, 1, 0.0, 1.0, oracle.EX_NEIGHBOUR_PEAK).calibrate(event_of(tr))
        b = cam_of(N, T, 1, 0.0, 1.0, oracle.EX_SLIDING).calibrate(event_of(tr))
        assert a.tobytes() == b.tobytes()


def test_neighbour_peak_is_local():
    """On the 37-pixel hexagon: rewriting every sample of pixel j changes the
    outputs of j and of its neighbours at most; every other pixel is
    unchanged."""
    rng = np.random.default_rng(6)
    a_ = np.arange(-3, 4)
    pts = [(a, b) for a in a_ for b in a_ if abs(a) <= 3 and abs(b) <= 3 and abs(a + b) <= 3]
    x = np.array([P * (a + b / 2) for a, b in pts], np.float32)
    y = np.array([P * b * np.sqrt(3) / 2 for a, b in pts], np.float32)
    N, T = len(pts), 24
    d = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
    near = (d < 1.4 * P) & (d > 0)
    cam = cam_of(N, T, 2, 300.0, 10.0, oracle.EX_NEIGHBOUR_PEAK, x=x, y=y)
    for trial in range(10):
        tr = rng.integers(250, 4200, size=(2, N, T))
        base = cam.calibrate(event_of(tr))
        j = int(rng.integers(0, N))
        tr2 = tr.copy()
        tr2[:, j, :] = rng.integers(0, 65536, size=(2, T))
        got = cam.calibrate(event_of(tr2))
        same = ~near[j]
        same[j] = False
        assert got[same].tobytes() == base[same].tobytes()


def test_neighbour_peak_gain_uses_the_whole_trace():
    """Dual gain: a saturated high-gain sample anywhere in the pixel's trace
    switches it (as for the sliding window), and the low gain is integrated
    at the start the neighbours chose."""
    T = 16
    hg = np.zeros((2, T), np.int64)
    lg = np.zeros((2, T), np.int64)
    hg[0, 0] = 4095                      # pixel 0 saturates at sample 0
    lg[0, 9:13] = [7, 8, 9, 10]
    hg[1, 9:13] = 200                    # pixel 1 (pixel 0's neighbour) peaks at 9
    r = cam_of(2, T, 2, 0.0, 1.0, oracle.EX_NEIGHBOUR_PEAK).calibrate(event_of([hg, lg]))
    assert int(r["gain"][0]) == 1 and int(r["sstar"][0]) == 9 and int(r["S"][0]) == 34
