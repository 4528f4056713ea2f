"""Pins of the CPU oracle against facts fixed outside it: hand-derived cases,
closed forms, lattice symmetries, brute force on tiny inputs, exact integer
identities and textbook / library routines.  CPU only."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import dl0sim
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
P = 0.05


def one_pixel_cam(T, w, G, ped, a, switch=4000):
    return oracle.Camera(1, T, G, [0.0], [0.0], np.asarray(ped, np.float32).reshape(G, 1),
                         np.asarray(a, np.float32).reshape(G, 1), P, window=w, hg_switch=switch)


def one_pixel_event(trace_g_t):
    tr = np.asarray(trace_g_t, np.uint16)
    G, T = tr.shape
    ev = np.zeros((G, T, 8), np.uint16)
    ev[:, :, 0] = tr
    return ev


def geometry_cam(geom, T=8, G=1, a=10.0, ped=300.0, t_pic=10.0, t_bnd=5.0):
    N = geom.n_pix
    return oracle.Camera(N, T, G, geom.x, geom.y, np.full((G, N), ped, np.float32),
                         np.full((G, N), a, np.float32), geom.pitch, t_pic=t_pic, t_bnd=t_bnd)


# ---------------------------------------------------------------- extraction
def test_hand_derived_extraction_cases():
    cases = json.load(open(os.path.join(GOLDEN, "extraction_hand.json")))["cases"]
    for c in cases:
        cam = one_pixel_cam(c["T"], c["w"], c["G"], c["ped"], c["a"], c["switch"])
        r = cam.calibrate(one_pixel_event(c["trace"]))[0]
        for k in ("S", "D", "Nt", "sstar", "peak", "gain"):
            assert int(r[k]) == c[k], (c["name"], k, int(r[k]), c[k])
        assert r["q"] == pytest.approx(c["q"], rel=1e-12), c["name"]
        assert r["t"] == pytest.approx(c["t"], rel=1e-12), c["name"]


def all_windows(x, w):
    return np.array([int(np.sum(x[s:s + w], dtype=np.int64)) for s in range(len(x) - w + 1)])


@pytest.mark.parametrize("T,w", [(3, 1), (5, 2), (6, 3), (7, 4), (7, 7)])
def test_argmax_brute_force_all_ternary_traces(T, w):
    """Every trace of length T over {0, 1, 2}: s* is the first maximiser of the
    enumerated window sums and the peak the first maximum inside it."""
    cam = one_pixel_cam(T, w, 1, [0.0], [1.0])
    for code in range(3 ** T):
        x = np.array([(code // 3 ** k) % 3 for k in range(T)], np.int64)
        W = all_windows(x, w)
        best = max(W)
        s_ref = min(s for s in range(len(W)) if W[s] == best)
        win = list(x[s_ref:s_ref + w])
        p_ref = s_ref + win.index(max(win))
        r = cam.calibrate(one_pixel_event([x]))[0]
        assert (int(r["sstar"]), int(r["S"]), int(r["peak"])) == (s_ref, best, p_ref), x


@pytest.fixture(scope="module")
def c0_cam_and_events():
    cam = dl0sim.camera_c0()
    sh, tr = dl0sim.plain_events(cam, seed=11, n=6)
    return cam, oracle.Camera.from_type(cam), tr


def test_window_identities_on_generated_events(c0_cam_and_events):
    """W(s*) >= W(s) for all s with strict > for s < s*, by enumeration;
    sum_s W(s) = sum_k m_k x_k with m_k the number of windows covering k."""
    cam, oc, tr = c0_cam_and_events
    w, T = cam.window, cam.n_samp
    m = np.array([min(k, T - w) - max(0, k - w + 1) + 1 for k in range(T)])
    for e in range(tr.shape[0]):
        r = oc.calibrate(tr[e])
        for i in range(0, cam.n_pix, 37):
            x = tr[e, 0, :, i].astype(np.int64)
            W = all_windows(x, w)
            s = int(r["sstar"][i])
            assert W[s] == r["S"][i]
            assert np.all(W <= W[s]) and np.all(W[:s] < W[s])
            assert W.sum() == int(np.dot(m, x))


def test_constant_offset_invariance(c0_cam_and_events):
    """Adding a constant c to a pixel's samples keeps s* and the peak and moves
    S by w*c and D by 256*w*c; the time numerator moves by 256*c*w(w-1)/2."""
    cam, oc, tr = c0_cam_and_events
    w = cam.window
    base = oc.calibrate(tr[0])
    rng = np.random.default_rng(5)
    c = rng.integers(0, 2000, size=cam.n_pix)
    ev = tr[0].astype(np.int64)
    ev[:, :, :cam.n_pix] += c[None, None, :]
    shifted = oc.calibrate(ev.astype(np.uint16))
    assert np.array_equal(base["sstar"], shifted["sstar"])
    assert np.array_equal(base["peak"], shifted["peak"])
    assert np.array_equal(shifted["S"] - base["S"], w * c)
    assert np.array_equal(shifted["D"] - base["D"], 256 * w * c)
    assert np.array_equal(shifted["Nt"] - base["Nt"], 256 * c * (w * (w - 1) // 2))


def test_dual_gain_reduces_to_single_gain():
    """Below the switch everywhere, a dual-gain event gives the single-gain
    result of its high-gain block; a pixel forced over the switch gives the
    single-gain result of its low-gain block."""
    types = dl0sim.camera_types_c1()
    cam = types[1]
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(cam.n_samp), 3, 0, 3)
    sh["size"][:, 0] = 300.0  # far below the switch
    tr = dl0sim.render_traces(cam, sh, 3)
    assert tr[:, 0].max() < cam.hg_switch_adc
    od = oracle.Camera.from_type(cam)
    hg = oracle.Camera(cam.n_pix, cam.n_samp, 1, cam.geom.x, cam.geom.y, cam.ped[:1], cam.adc_per_pe[:1], P)
    lg = oracle.Camera(cam.n_pix, cam.n_samp, 1, cam.geom.x, cam.geom.y, cam.ped[1:], cam.adc_per_pe[1:], P)
    for e in range(3):
        a = od.calibrate(tr[e])
        b = hg.calibrate(tr[e, :1])
        for k in ("S", "D", "Nt", "sstar", "peak"):
            assert np.array_equal(a[k], b[k])
        assert np.all(a["gain"] == 0)
        ev = tr[e].copy()
        forced = np.arange(0, cam.n_pix, 7)
        ev[0, 3, forced] = cam.hg_switch_adc
        a = od.calibrate(ev)
        c = lg.calibrate(ev[1:])
        assert np.all(a["gain"][forced] == 1)
        for k in ("S", "D", "Nt", "sstar", "peak", "q", "t"):
            assert np.array_equal(a[k][forced], c[k][forced])


def test_extremes_do_not_overflow():
    T, w = 128, 4
    cam = one_pixel_cam(T, w, 1, [65535.0], [10.0])
    r = cam.calibrate(one_pixel_event([np.full(T, 65535)]))[0]
    assert int(r["S"]) == w * 65535 and int(r["D"]) == 0 and int(r["sstar"]) == 0
    cam = one_pixel_cam(T, w, 1, [0.0], [10.0])
    x = np.zeros(T, np.int64)
    x[-1] = 65535
    r = cam.calibrate(one_pixel_event([x]))[0]
    assert int(r["S"]) == 65535 and int(r["D"]) == 256 * 65535 and int(r["sstar"]) == T - w
    assert int(r["peak"]) == T - 1 and r["t"] == pytest.approx(T - 1, abs=0)


# ---------------------------------------------------------------- cleaning
def exact_threshold(a32, level):
    return math.ceil(Fraction(float(np.float32(a32))) * 256 * Fraction(level))


def ref_mask(xy, D, thr_p, thr_b, tol):
    n = len(D)
    nb = [{j for j in range(n) if j != i and math.dist(xy[i], xy[j]) <= tol} for i in range(n)]
    pic = {i for i in range(n) if D[i] >= thr_p[i]}
    bnd = {i for i in range(n) if D[i] >= thr_b[i]}
    keep = {i for i in bnd if nb[i] & pic} | {i for i in pic if nb[i] & bnd}
    return np.array([1 if i in keep else 0 for i in range(n)], np.uint8)


def test_tailcut_exhaustive_seven_pixels():
    """All 4^7 patterns of levels {0, Tb-1, Tb, Tp} on the 7-pixel hexagon,
    with per-pixel gains and two gain tables; reference = set definition over
    pairwise distances, thresholds in exact rational arithmetic."""
    g = dl0sim.hex_geometry(7)
    a = np.array([[9.7] * 7, [0.61] * 7], np.float32)
    cam = oracle.Camera(7, 8, 2, g.x, g.y, np.full((2, 7), 300, np.float32), a, P)
    gain = np.array([0, 1, 0, 1, 1, 0, 0], np.int32)
    tp = [exact_threshold(a[gain[i], i], 10.0) for i in range(7)]
    tb = [exact_threshold(a[gain[i], i], 5.0) for i in range(7)]
    xy = list(zip(g.x.astype(float), g.y.astype(float)))
    for code in range(4 ** 7):
        lv = [(code >> (2 * i)) & 3 for i in range(7)]
        D = np.array([[0, tb[i] - 1, tb[i], tp[i]][lv[i]] for i in range(7)], np.int64)
        m = cam.clean(D, gain)
        assert np.array_equal(m, ref_mask(xy, D, tp, tb, 1.4 * P)), D


def test_tailcut_random_nineteen_pixels():
    g = dl0sim.hex_geometry(19)
    cam = geometry_cam(g)
    tp, tb = exact_threshold(10.0, 10.0), exact_threshold(10.0, 5.0)
    assert (tp, tb) == (25600, 12800)
    xy = list(zip(g.x.astype(float), g.y.astype(float)))
    rng = np.random.default_rng(19)
    gain = np.zeros(19, np.int32)
    for _ in range(3000):
        D = rng.choice([0, tb - 1, tb, tb + 1, tp - 1, tp, tp + 5000], size=19).astype(np.int64)
        assert np.array_equal(cam.clean(D, gain), ref_mask(xy, D, [tp] * 19, [tb] * 19, 1.4 * P))


def test_neighbours_match_lattice_tables():
    """The oracle's distance-derived neighbour lists equal the generator's
    lattice-derived tables as sets, for every camera size in use."""
    for n in (7, 19, 37, 1764, 1801, 1855, 2048):
        g = dl0sim.hex_geometry(n)
        ob = oracle.neighbours(g.x, g.y, 1.4 * P)
        for i in range(n):
            assert set(ob[i][ob[i] >= 0]) == set(g.nbr[i][g.nbr[i] >= 0])
    g = dl0sim.hex_geometry(1801)   # closed under the 60 degree lattice rotation
    border = set(np.flatnonzero((g.nbr >= 0).sum(1) < 6))
    index = {(int(a), int(b)): i for i, (a, b) in enumerate(g.ab)}
    assert {index[(-int(g.ab[i, 1]), int(g.ab[i, 0] + g.ab[i, 1]))] for i in border} == border


# ---------------------------------------------------------------- islands
def test_islands_against_scipy_components():
    for n in (19, 37):
        g = dl0sim.hex_geometry(n)
        cam = geometry_cam(g)
        d = np.hypot(g.x[:, None] - g.x[None, :], g.y[:, None] - g.y[None, :])
        adj = (d <= 1.4 * P) & (d > 0)
        rng = np.random.default_rng(n)
        for _ in range(500):
            m = (rng.random(n) < rng.random()).astype(np.uint8)
            idx = np.flatnonzero(m)
            if len(idx) == 0:
                ref = 0
            else:
                ref = connected_components(csr_matrix(adj[np.ix_(idx, idx)]), directed=False)[0]
            assert cam.islands(m) == ref


def test_islands_hand_patterns():
    g = dl0sim.hex_geometry(37)
    cam = geometry_cam(g)
    ring1 = [i for i in range(37) if 0.9 * P < math.hypot(g.x[i], g.y[i]) < 1.1 * P]
    assert len(ring1) == 6
    m = np.zeros(37, np.uint8)
    assert cam.islands(m) == 0
    m[0] = 1
    assert cam.islands(m) == 1
    m[:] = 0
    m[ring1] = 1                        # the first ring without its centre is one loop
    assert cam.islands(m) == 1
    outer = [i for i in range(37) if math.hypot(g.x[i], g.y[i]) > 2.9 * P]
    m[:] = 0
    m[0] = 1
    m[outer[0]] = 1                     # centre and one outer-ring pixel: two islands
    assert cam.islands(m) == 2


# ---------------------------------------------------------------- Hillas
def point_cam(xs, ys):
    n = len(xs)
    return oracle.Camera(n, 8, 1, xs, ys, np.full((1, n), 300, np.float32), np.full((1, n), 10, np.float32), P)


def wrap_half_pi(a):
    """Map an axis angle into (-pi/2, pi/2]."""
    a = math.fmod(a, math.pi)
    if a > math.pi / 2:
        a -= math.pi
    if a <= -math.pi / 2:
        a += math.pi
    return a


def axis_diff(a, b):
    d = math.fmod(a - b, math.pi)
    return min(abs(d), math.pi - abs(d))


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.2, math.pi / 2, -0.7, 2.5])
def test_hillas_two_points(theta):
    d = 0.173
    x0, y0 = 0.11, -0.23
    xs = np.array([x0, x0 + d * math.cos(theta)], np.float32)
    ys = np.array([y0, y0 + d * math.sin(theta)], np.float32)
    cam = point_cam(xs, ys)
    h = cam.hillas([1.0, 1.0], [0.0, 0.0], [1, 1])
    dd = math.hypot(float(xs[1]) - float(xs[0]), float(ys[1]) - float(ys[0]))
    ang = math.atan2(float(ys[1]) - float(ys[0]), float(xs[1]) - float(xs[0]))
    assert h["length"] == pytest.approx(dd / 2, rel=1e-12)
    assert h["width"] <= 1e-7 * dd
    assert axis_diff(h["psi"], ang) < 1e-9
    assert -math.pi / 2 < h["psi"] <= math.pi / 2
    assert h["size"] == 2.0 and h["n_pix"] == 2


@pytest.mark.parametrize("p", [0.1, 0.25, 0.5, 0.8])
def test_hillas_two_point_skewness_kurtosis(p):
    """Two charges (1-p, p): along the axis the standardised third and fourth
    moments are those of a Bernoulli(p) variable."""
    xs = np.array([0.0, 0.3], np.float32)
    ys = np.array([0.1, 0.1], np.float32)
    cam = point_cam(xs, ys)
    h = cam.hillas([1 - p, p], [0, 0], [1, 1])
    skew = (1 - 2 * p) / math.sqrt(p * (1 - p))
    kurt = (1 - 3 * p * (1 - p)) / (p * (1 - p))
    assert abs(h["skewness"]) == pytest.approx(abs(skew), rel=1e-9, abs=1e-12)
    assert h["kurtosis"] == pytest.approx(kurt, rel=1e-9)


def test_hillas_seven_pixel_hexagon():
    g = dl0sim.hex_geometry(7)
    cam = geometry_cam(g)
    h = cam.hillas(np.ones(7), np.zeros(7), np.ones(7, np.uint8))
    r = P * math.sqrt(3.0 / 7.0)
    assert h["length"] == pytest.approx(r, rel=1e-6)
    assert h["width"] == pytest.approx(r, rel=1e-6)
    assert abs(h["cog_x"]) < 1e-9 and abs(h["cog_y"]) < 1e-9
    assert abs(h["skewness"]) < 1e-6
    assert h["leakage"] == pytest.approx(6.0 / 7.0, rel=1e-12)   # six ring pixels lack neighbours
    assert h["n_islands"] == 1


def gaussian_image(g, cx, cy, sl, sw, psi, size=1000.0):
    x = g.x.astype(np.float64)
    y = g.y.astype(np.float64)
    c, s = math.cos(psi), math.sin(psi)
    l = (x - cx) * c + (y - cy) * s
    w = -(x - cx) * s + (y - cy) * c
    area = math.sqrt(3) / 2 * g.pitch ** 2
    return size * area * np.exp(-0.5 * (l * l / sl ** 2 + w * w / sw ** 2)) / (2 * math.pi * sl * sw)


@pytest.fixture(scope="module")
def big_lattice():
    g = dl0sim.hex_geometry(dl0sim.full_hex_count(40))
    return g, geometry_cam(g)


def test_hillas_sampled_gaussian_matches_continuous_moments(big_lattice):
    """A Gaussian ellipse sampled on a fine lattice (sigma >= 1.2 pitch, far
    from the edge) has discrete moments equal to the continuous ones."""
    g, cam = big_lattice
    for (cx, cy, sl, sw, psi) in [(0.13, -0.07, 2.5 * P, 1.2 * P, 0.4), (-0.3, 0.2, 4 * P, 1.5 * P, -1.1),
                                  (0.05, 0.31, 3 * P, 1.3 * P, 1.5)]:
        q = gaussian_image(g, cx, cy, sl, sw, psi)
        h = cam.hillas(q, np.zeros_like(q), np.ones(g.n_pix, np.uint8))
        assert h["cog_x"] == pytest.approx(cx, abs=1e-7 * sl)
        assert h["cog_y"] == pytest.approx(cy, abs=1e-7 * sl)
        assert h["length"] == pytest.approx(sl, rel=1e-6)
        assert h["width"] == pytest.approx(sw, rel=1e-6)
        assert axis_diff(h["psi"], psi) < 1e-6
        assert abs(h["skewness"]) < 1e-6
        assert h["kurtosis"] == pytest.approx(3.0, rel=1e-5)   # Gaussian: non-excess kurtosis 3


def lattice_map(g, f):
    index = {(int(a), int(b)): i for i, (a, b) in enumerate(g.ab)}
    return np.array([index.get(f(int(a), int(b)), -1) for a, b in g.ab])


def test_hillas_lattice_rotation_reflection_translation():
    """Exact lattice symmetries of the full 24-ring camera: a 60 degree rotation
    adds pi/3 to psi and rotates the cog; a reflection negates psi; a lattice
    translation moves the cog by one pitch.  Size, length, width, kurtosis and
    |skewness| are unchanged."""
    g = dl0sim.hex_geometry(1801)
    cam = geometry_cam(g)
    rng = np.random.default_rng(7)
    q = gaussian_image(g, 0.21, -0.13, 3 * P, 1.4 * P, 0.7) * (1 + 0.3 * rng.random(g.n_pix))
    mask = (q > 0.5).astype(np.uint8)
    t = rng.random(g.n_pix)
    h0 = cam.hillas(q, t, mask)
    rot = lattice_map(g, lambda a, b: (-b, a + b))
    ref = lattice_map(g, lambda a, b: (a + b, -b))
    assert (rot >= 0).all() and (ref >= 0).all()
    for perm, kind in ((rot, "rot"), (ref, "ref")):
        q2 = np.zeros_like(q); q2[perm] = q
        m2 = np.zeros_like(mask); m2[perm] = mask
        t2 = np.zeros_like(t); t2[perm] = t
        h = cam.hillas(q2, t2, m2)
        for k in ("size", "length", "width", "kurtosis", "leakage"):
            assert h[k] == pytest.approx(h0[k], rel=1e-6), (kind, k)
        # float32 pixel positions are rotated only up to their rounding (~1e-7 m)
        assert abs(h["skewness"]) == pytest.approx(abs(h0["skewness"]), abs=1e-6)
        assert abs(h["time_gradient"]) == pytest.approx(abs(h0["time_gradient"]), rel=1e-6)
        assert h["n_islands"] == h0["n_islands"] and h["n_pix"] == h0["n_pix"]
        if kind == "rot":
            c, s = 0.5, math.sqrt(3) / 2
            ex, ey = c * h0["cog_x"] - s * h0["cog_y"], s * h0["cog_x"] + c * h0["cog_y"]
            assert axis_diff(h["psi"], h0["psi"] + math.pi / 3) < 1e-6
        else:
            ex, ey = h0["cog_x"], -h0["cog_y"]
            assert axis_diff(h["psi"], -h0["psi"]) < 1e-6
        assert h["cog_x"] == pytest.approx(ex, abs=1e-7) and h["cog_y"] == pytest.approx(ey, abs=1e-7)
    # translation by the lattice vector (1, 0) on an image well inside the camera
    tr = lattice_map(g, lambda a, b: (a + 1, b))
    inside = mask.astype(bool)
    assert (tr[inside] >= 0).all()
    q2 = np.zeros_like(q); q2[tr[inside]] = q[inside]
    m2 = np.zeros_like(mask); m2[tr[inside]] = 1
    h = cam.hillas(q2, t, m2)
    assert h["cog_x"] == pytest.approx(h0["cog_x"] + P, abs=1e-7)
    assert h["cog_y"] == pytest.approx(h0["cog_y"], abs=1e-7)
    assert h["length"] == pytest.approx(h0["length"], rel=1e-6)


def test_hillas_scaling_and_time_gradient(big_lattice):
    g, cam = big_lattice
    cx, cy, psi = 0.11, 0.05, -0.6
    q = gaussian_image(g, cx, cy, 3 * P, 1.3 * P, psi)
    l = (g.x - cx) * math.cos(psi) + (g.y - cy) * math.sin(psi)
    t = 17.0 + 6.5 * l
    mask = np.ones(g.n_pix, np.uint8)
    h = cam.hillas(q, t, mask)
    assert h["time_gradient"] == pytest.approx(6.5, rel=1e-7)
    assert h["time_intercept"] == pytest.approx(17.0, rel=1e-7)
    h3 = cam.hillas(3.5 * q, t, mask)
    assert h3["size"] == pytest.approx(3.5 * h["size"], rel=1e-12)
    for k in ("cog_x", "cog_y", "length", "width", "psi", "skewness", "kurtosis", "time_gradient"):
        assert h3[k] == pytest.approx(h[k], rel=1e-10, abs=1e-13)


def test_hillas_invalid_below_two_pixels():
    g = dl0sim.hex_geometry(19)
    cam = geometry_cam(g)
    h = cam.hillas(np.ones(19), np.zeros(19), np.zeros(19, np.uint8))
    assert h["n_pix"] == 0 and h["flags"] & oracle.HILLAS_INVALID and math.isnan(h["length"])
    m = np.zeros(19, np.uint8); m[3] = 1
    h = cam.hillas(np.ones(19), np.zeros(19), m)
    assert h["flags"] & oracle.HILLAS_INVALID


# ---------------------------------------------------------------- stereo
def test_stereo_common_point_and_two_line_intersection():
    rng = np.random.default_rng(3)
    p0 = np.array([0.0123, -0.0071])
    n = 9
    f = rng.choice([28.0, 16.0, 5.6], size=n)
    c = rng.uniform(-0.03, 0.03, size=(n, 2))
    psi = np.array([wrap_half_pi(math.atan2(c[i, 1] - p0[1], c[i, 0] - p0[0])) for i in range(n)])
    width = rng.uniform(0.02, 0.05, n)
    length = width * rng.uniform(1.5, 4, n)
    size = rng.uniform(100, 1000, n)
    dx, dy, cond, used, flags = oracle.stereo(size, c[:, 0] * f, c[:, 1] * f, length, width, psi,
                                              np.ones(n, np.int32), f)
    assert flags == 0 and used == n
    assert dx == pytest.approx(p0[0], abs=1e-12) and dy == pytest.approx(p0[1], abs=1e-12)
    # two lines: the closed-form intersection c1 + s d1 = c2 + u d2 (Cramer's rule)
    c1, c2 = np.array([0.01, 0.002]), np.array([-0.004, 0.011])
    a1, a2 = 0.3, 1.9
    d1, d2 = np.array([math.cos(a1), math.sin(a1)]), np.array([math.cos(a2), math.sin(a2)])
    det = d1[0] * (-d2[1]) - d1[1] * (-d2[0])
    s_ = ((c2 - c1)[0] * (-d2[1]) - (c2 - c1)[1] * (-d2[0])) / det
    x_ref = c1 + s_ * d1
    dx, dy, cond, used, flags = oracle.stereo([1, 1], [c1[0], c2[0]], [c1[1], c2[1]], [0.1, 0.1], [0.02, 0.05],
                                              [a1, wrap_half_pi(a2)], [1, 1], [1.0, 1.0])
    assert dx == pytest.approx(x_ref[0], abs=1e-13) and dy == pytest.approx(x_ref[1], abs=1e-13)


def test_stereo_weighted_least_squares_matches_lstsq():
    rng = np.random.default_rng(8)
    n = 12
    c = rng.uniform(-0.03, 0.03, (n, 2))
    psi = rng.uniform(-math.pi / 2, math.pi / 2, n)
    width = rng.uniform(0.01, 0.04, n)
    length = width * rng.uniform(1.2, 4, n)
    size = rng.uniform(50, 5000, n)
    valid = (rng.random(n) < 0.85).astype(np.int32)
    keep = valid.astype(bool) & (width / length <= 0.9)
    wgt = size * (1 - width / length)
    nv = np.stack([-np.sin(psi), np.cos(psi)], 1)
    A = np.sqrt(wgt[keep])[:, None] * nv[keep]
    b = np.sqrt(wgt[keep]) * np.sum(nv[keep] * c[keep], 1)
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    dx, dy, cond, used, flags = oracle.stereo(size, c[:, 0], c[:, 1], length, width, psi, valid, np.ones(n))
    assert used == keep.sum() and flags == 0
    assert dx == pytest.approx(ref[0], rel=1e-9) and dy == pytest.approx(ref[1], rel=1e-9)
    ev = np.linalg.eigvalsh(A.T @ A)
    assert cond == pytest.approx(ev[-1] / ev[0], rel=1e-9)


def test_stereo_degenerate_cases():
    # one telescope, parallel axes, and a near-round image dropped by the ratio cut
    r = oracle.stereo([100], [0.1], [0.0], [0.1], [0.02], [0.3], [1], [1.0])
    assert r[4] == oracle.STEREO_INVALID and math.isnan(r[0])
    r = oracle.stereo([100, 100], [0.1, 0.2], [0.0, 0.05], [0.1, 0.1], [0.02, 0.02], [0.3, 0.3], [1, 1], [1.0, 1.0])
    assert r[4] == oracle.STEREO_INVALID
    r = oracle.stereo([100, 100, 100], [0.1, 0.2, 0.0], [0.0, 0.05, 0.1], [0.1, 0.1, 0.1], [0.02, 0.02, 0.095],
                      [0.3, -0.8, 1.0], [1, 1, 1], [1.0, 1.0, 1.0])
    assert r[3] == 2 and r[4] == 0


# ---------------------------------------------------------------- generator
def test_generator_noise_statistics():
    """Pure background: mean = 300 + 10 * 0.1 = 301 ADC, variance = 25 (noise)
    + 100 * 0.1 (NSB at 10 ADC/p.e.) + 1/12 (rounding) ADC^2."""
    cam = dl0sim.camera_c0()
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(cam.n_samp), 2, 0, 40)
    sh["size"][:, 0] = 0.0
    tr = dl0sim.render_traces(cam, sh, 2)[:, 0, :, :cam.n_pix].astype(np.float64)
    n = tr.size
    assert abs(tr.mean() - 301.0) < 5 * math.sqrt(35 / n)
    assert abs(tr.var() - (35 + 1 / 12)) < 5 * 35 * math.sqrt(2 / n) + 0.05
    assert np.all(dl0sim.render_traces(cam, sh, 2)[:, :, :, cam.n_pix:] == 0)   # pixel pad


def test_generator_photon_count_matches_size():
    cam = dl0sim.CameraType("big", dl0sim.full_hex_count(40), 30, 1, 28.0)
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(30), 4, 0, 200)
    sh["cog_x"][:, 0] *= 0.5
    sh["cog_y"][:, 0] *= 0.5
    sh["size"][:, 0] = 2000.0
    _, npe = dl0sim.render_traces(cam, sh, 4, want_npe=True)
    tot = npe.sum(1)
    assert abs(tot.mean() - 2000.0) < 5 * math.sqrt(2000.0 / len(tot)) + 2.0


def test_generator_is_order_independent():
    cam = dl0sim.camera_c0()
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(30), 9, 0, 8)
    full = dl0sim.render_traces(cam, sh, 9, event_ids=np.arange(8))
    part = dl0sim.render_traces(cam, sh[5:7], 9, event_ids=np.arange(5, 7), n_threads=1)
    assert np.array_equal(full[5:7], part)
    assert dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(30), 9, 5, 2).tobytes() == sh[5:7].tobytes()


def test_philox_known_answers():
    """Known-answer vectors of Philox4x32-10 published with the generator."""
    assert [hex(v) for v in dl0sim.philox4x32_10([0, 0, 0, 0], [0, 0])] == \
        ["0x6627e8d5", "0xe169c58d", "0xbc57ac4c", "0x9b00dbd8"]
    assert [hex(v) for v in dl0sim.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2)] == \
        ["0x408f276d", "0x41c83b0e", "0xa20bc7c6", "0x6d5451fd"]


# ---------------------------------------------------------------- cog distance, low-gain count
def test_cog_distance_hand_cases():
    """cog distance is the distance of the charge-weighted centre from the
    camera centre.  Charges 2 and 1 at (0, 0) and (0.09, 0.12) m put the
    centre at (0.03, 0.04): distance 0.05, not the rms radius of the pixels
    (0.05 sqrt(3) = 0.0866) nor the mean pixel distance (0.05).  A third,
    bright pixel outside the mask does not move it; two charges placed
    symmetrically about (0.03, 0.04) give 0.05 as well."""
    xs = np.array([0.0, 0.09, -0.4], np.float32)
    ys = np.array([0.0, 0.12, 0.3], np.float32)
    cam = point_cam(xs, ys)
    h = cam.hillas([2.0, 1.0, 50.0], [0.0, 0.0, 0.0], [1, 1, 0])
    cx = (2 * float(xs[0]) + float(xs[1])) / 3
    cy = (2 * float(ys[0]) + float(ys[1])) / 3
    assert h["cog_x"] == pytest.approx(0.03, rel=1e-7) and h["cog_y"] == pytest.approx(0.04, rel=1e-7)
    assert h["cog_dist"] == pytest.approx(math.hypot(cx, cy), rel=1e-12)
    assert h["cog_dist"] == pytest.approx(0.05, rel=1e-7)
    xs = np.array([0.03 - 0.2, 0.03 + 0.2], np.float32)
    ys = np.array([0.04 + 0.1, 0.04 - 0.1], np.float32)
    h = point_cam(xs, ys).hillas([1.0, 1.0], [0.0, 0.0], [1, 1])
    assert h["cog_dist"] == pytest.approx(0.05, rel=1e-6)


def test_low_gain_count_over_all_pixels():
    """n_lowgain counts the pixels that used their low gain over the whole
    camera, inside and outside the cleaning mask, and the low-gain flag is
    set exactly when that count is non-zero."""
    g = dl0sim.hex_geometry(19)
    cam = geometry_cam(g, G=2)
    q = np.linspace(1.0, 3.0, 19)
    t = np.zeros(19)
    mask = np.zeros(19, np.uint8)
    mask[[0, 1, 2, 3]] = 1
    gain = np.zeros(19, np.int32)
    h = cam.hillas(q, t, mask, gain)
    assert h["n_lowgain"] == 0 and not h["flags"] & oracle.LOW_GAIN
    gain[[2, 7, 11, 18]] = 1          # one inside the mask, three outside
    h = cam.hillas(q, t, mask, gain)
    assert h["n_lowgain"] == 4 and h["flags"] & oracle.LOW_GAIN
    mask[:] = 0                       # empty mask: still counted, still flagged
    h = cam.hillas(q, t, mask, gain)
    assert h["n_lowgain"] == 4 and h["flags"] & oracle.LOW_GAIN and h["flags"] & oracle.HILLAS_INVALID


def test_low_gain_count_through_the_chain():
    """Whole-event reconstruction of a dual-gain event: with k pixels forced
    over the switch (most of them far from the image, so outside the mask)
    the record counts k and is flagged; with none forced, 0 and no flag."""
    types = dl0sim.camera_types_c1()
    ct = types[1]
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(ct.n_samp), 1, 0, 5)
    sh["size"][:, 0] = 400.0
    tr = dl0sim.render_traces(ct, sh, 5)
    ev = tr[0].copy()
    assert ev[0].max() < ct.hg_switch_adc
    od = oracle.Camera.from_type(ct)
    _, m0, h0 = od.reconstruct(ev)
    assert h0["n_lowgain"] == 0 and not h0["flags"] & oracle.LOW_GAIN
    forced = np.array([5, 77, 400, 901, 1500, 1763])
    ev[0, 2, forced] = ct.hg_switch_adc
    pix, m1, h1 = od.reconstruct(ev)
    assert np.all(pix["gain"][forced] == 1) and int(np.sum(pix["gain"])) == len(forced)
    assert int(np.sum(m1[forced])) < len(forced)
    assert h1["n_lowgain"] == len(forced) and h1["flags"] & oracle.LOW_GAIN
