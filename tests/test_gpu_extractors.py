"""GPU parity of the alternative signal extractors (fixed window, global peak
window, neighbour peak window) against the oracle, through the C ABI: per-pixel integers bit-exact
(S, D, s*, peak, gain), q / t within FP32 rounding, Hillas records of the
fused batch within the per-field tolerances of oracle/parity.py."""
import numpy as np
import pytest

import dl0sim
import dl0sim.workloads as W
import oracle
import oracle.parity as par
import paper_1307_6489_amd as rta

pytestmark = pytest.mark.gpu
EXS = [rta.EXTRACT_FIXED, rta.EXTRACT_GLOBAL_PEAK, rta.EXTRACT_NEIGHBOUR_PEAK]
NAME = {rta.EXTRACT_SLIDING: "sliding", rta.EXTRACT_FIXED: "fixed", rta.EXTRACT_GLOBAL_PEAK: "global peak",
        rta.EXTRACT_NEIGHBOUR_PEAK: "neighbour peak"}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rta.lib()
    return torch.device("cuda:0")


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def calib_parity(ct, traces, dev, ex):
    cam = rta.Camera.from_type(ct)
    oc = oracle.Camera.from_type(ct, extractor=ex)
    assert cam.fixed_start == oc.fixed_start
    out = rta.calibrate(cam, to_dev(traces, dev), extractor=ex)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    ref = oracle.calibrate_events(oc, traces)
    for k in ("S", "D", "sstar", "peak", "gain"):
        assert np.array_equal(g[k].astype(np.int64), ref[k].astype(np.int64)), (NAME[ex], k)
    assert np.allclose(g["q"], ref["q"], rtol=1e-6, atol=1e-6)
    assert np.allclose(g["t"], ref["t"], rtol=1e-6, atol=1e-5)
    return ref


@pytest.mark.parametrize("ex", EXS)
def test_calibrate_c0(torch_dev, ex):
    ct = dl0sim.camera_c0()
    say("C0 calibrate, %s: 1855 px x 30 samples, 64 events, seed 0" % NAME[ex])
    _, tr = dl0sim.plain_events(ct, 0, 64)
    ref = calib_parity(ct, tr, torch_dev, ex)
    if ex == rta.EXTRACT_GLOBAL_PEAK:
        assert all(len(set(ref["sstar"][e].tolist())) == 1 for e in range(len(tr)))


@pytest.mark.parametrize("ex", EXS)
@pytest.mark.parametrize("ti", [0, 1, 2])
def test_calibrate_dual_gain_with_switching(torch_dev, ex, ti):
    ct = dl0sim.camera_types_c1()[ti]
    say("dual-gain calibrate, %s: %s, seed 21" % (NAME[ex], ct.name))
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(ct.n_samp), 21, 0, 24)
    sh["size"][::2, 0] = 1.0e5
    tr = dl0sim.render_traces(ct, sh, 21)
    ref = calib_parity(ct, tr, torch_dev, ex)
    assert ref["gain"].sum() > 20


@pytest.mark.parametrize("ex", EXS)
def test_calibrate_per_pixel_tables_and_pad_garbage(torch_dev, ex):
    """Per-pixel pedestal / gain spreads, a non-default fixed start, and
    random values in the pad columns (pixels N..Npad-1, which every extractor
    must ignore: the global peak sums only real pixels)."""
    ct = dl0sim.CameraType("jitter", 1764, 25, 2, 16.0, ped_jitter=40.0, gain_jitter=0.3, table_seed=4,
                           fixed_start=7)
    say("per-pixel tables + pad garbage, %s: 1764 x 25 dual gain, seed 22" % NAME[ex])
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(25), 22, 0, 16)
    sh["size"][::2, 0] = 30000.0
    tr = dl0sim.render_traces(ct, sh, 22)
    rng = np.random.default_rng(5)
    tr[:, :, :, ct.n_pix:] = rng.integers(0, 65536, size=tr[:, :, :, ct.n_pix:].shape, dtype=np.uint16)
    calib_parity(ct, tr, torch_dev, ex)


@pytest.mark.parametrize("ex", EXS)
def test_calibrate_extremes(torch_dev, ex):
    """All-zero, all-65535 and random single-gain traces at 2048 x 255 (the
    global camera sum reaches 2048 * 4 * 65535), saturated dual gain."""
    say("extremes, %s: 2048 x 255" % NAME[ex])
    ct = dl0sim.CameraType("max", 2048, 255, 1, 5.6)
    tr = np.zeros((3, 1, 255, 2048), np.uint16)
    tr[1] = 65535
    rng = np.random.default_rng(1)
    tr[2] = rng.integers(0, 65536, size=(1, 255, 2048), dtype=np.uint16)
    calib_parity(ct, tr, torch_dev, ex)
    ct2 = dl0sim.CameraType("sat", 1855, 40, 2, 28.0)
    tr2 = np.full((2, 2, 40, 1856), 4095, np.uint16)
    tr2[:, 1] = rng.integers(0, 65536, size=(2, 40, 1856), dtype=np.uint16)
    ref = calib_parity(ct2, tr2, torch_dev, ex)
    assert ref["gain"].all()


@pytest.fixture(scope="module")
def c1_pool():
    cams = dl0sim.camera_types_c1()
    counts = [6, 18, 36]
    per = []
    for ty, ct in enumerate(cams):
        sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(ct.n_samp), 1, 1000 * ty, counts[ty])
        sh["size"][::3, 0] *= 10.0
        per.append(sh)
    return W.render_pool(cams, counts, 1, showers_per_type=per)


def fused_records(pool, dev, ex, schedule):
    import torch
    cams = [rta.Camera.from_type(c) for c in pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=False, extractor=ex)
    pipe.set_schedule(*schedule)
    b = pipe.make_batch(to_dev(pool.blob, dev), to_dev(pool.pool_type.astype(np.int32), dev),
                        to_dev(pool.pool_off.astype(np.int64), dev))
    tel, _ = pipe.alloc_outputs(b, dev)
    pipe.process(b, tel)
    torch.cuda.synchronize()
    assert pipe.status() == 0
    return rta.records(tel)


@pytest.mark.parametrize("ex", EXS)
def test_fused_c1_mix_parity_every_schedule(torch_dev, c1_pool, ex):
    """The fused batch with each extractor against the oracle's whole chain,
    in every pixels-per-lane / waves / chunk shape; a persistent schedule
    request runs the grid form and gives identical records."""
    pool = c1_pool
    ocs = [oracle.Camera.from_type(c, extractor=ex) for c in pool.cams]
    ref = []
    for k in range(pool.n):
        ty, off = pool.pool_type[k], pool.pool_off[k]
        ref.append(ocs[ty].reconstruct(pool.blob[off:off + pool.cams[ty].event_elems]))
    base = None
    for s in rta.list_schedules():
        if s[2] not in (0, 3):
            continue
        say("fused %s, schedule %s" % (NAME[ex], s))
        g = fused_records(pool, torch_dev, ex, s)
        bad = []
        for k in range(pool.n):
            ct = pool.cams[pool.pool_type[k]]
            p, m, h = ref[k]
            mm = par.hillas_mismatches(g[k], h, ct.geom.x, ct.geom.y, p["q"], p["t"], m)
            if mm:
                bad.append((k, mm))
        assert not bad, (NAME[ex], s, bad[:3])
        if s[:2] == (8, 4) and s[3] == 8:
            if base is None:
                base = g.tobytes()
            else:
                assert g.tobytes() == base      # (8,4,0,8) and (8,4,3,8): same grid-form kernel


@pytest.mark.parametrize("ex", EXS)
def test_full_size_stream_sampled(torch_dev, ex):
    """1e6 camera events of the 1:3:6 mix through a 600-event pool with each
    extractor in the benchmark's launch shape; 100 sampled telescopes against
    the oracle and record identity of repeated pool entries."""
    import torch
    pool = W.c1_pool(600, seed=1)
    n = 1_000_000
    idx, ty, off = W.stream_order(pool, n, seed=3)
    say("full-size stream, %s: %d telescopes" % (NAME[ex], n))
    cams = [rta.Camera.from_type(c) for c in pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=False, extractor=ex)
    pipe.set_schedule(8, 4, 0, 8)
    b = pipe.make_batch(to_dev(pool.blob, torch_dev), to_dev(ty, torch_dev), to_dev(off, torch_dev))
    tel, _ = pipe.alloc_outputs(b, torch_dev)
    pipe.process(b, tel)
    torch.cuda.synchronize()
    assert pipe.status() == 0
    g = rta.records(tel)
    ocs = [oracle.Camera.from_type(c, extractor=ex) for c in pool.cams]
    rng = np.random.default_rng(13)
    bad = []
    for k in np.concatenate([rng.choice(n, 96, replace=False), [0, n - 1, n // 2, n // 3]]):
        t_, o_ = ty[k], off[k]
        p, m, h = ocs[t_].reconstruct(pool.blob[o_:o_ + pool.cams[t_].event_elems])
        mm = par.hillas_mismatches(g[k], h, pool.cams[t_].geom.x, pool.cams[t_].geom.y, p["q"], p["t"], m)
        if mm:
            bad.append((k, mm))
    assert not bad, bad[:3]
    first = {}
    for k in range(0, 100_000):
        e = idx[k]
        if e in first:
            assert g[k].tobytes() == g[first[e]].tobytes()
        else:
            first[e] = k


def test_bad_extractor_is_rejected(torch_dev):
    ct = dl0sim.camera_c0()
    cam = rta.Camera.from_type(ct)
    _, tr = dl0sim.plain_events(ct, 0, 1)
    with pytest.raises(rta.RTAError):
        rta.calibrate(cam, to_dev(tr, torch_dev), extractor=4)
    with pytest.raises(rta.RTAError):
        rta.Pipeline([cam], do_stereo=False, extractor=-1)
    with pytest.raises(rta.RTAError):
        rta.Camera.from_type(dl0sim.CameraType("bad", 1855, 30, 1, 28.0, fixed_start=27))


@pytest.mark.parametrize("ex", [rta.EXTRACT_SLIDING] + EXS)
def test_calibrate_small_cameras(torch_dev, ex):
    """Cameras far below one workgroup's pixels (1, 7 and 61 pixels, padded
    to 8 / 8 / 64 columns with garbage in the padding), the shortest traces
    (T = w) and odd lengths, single and dual gain: every extractor against
    the oracle (the lone pixel has no neighbours)."""
    rng = np.random.default_rng(17)
    for n, T, G in ((1, 4, 1), (7, 9, 2), (61, 33, 2), (61, 4, 1)):
        ct = dl0sim.CameraType("tiny%d" % n, n, T, G, 5.0)
        npad = (n + 7) // 8 * 8
        tr = rng.integers(250, 4300, size=(5, G, T, npad), dtype=np.uint16)
        say("small camera %d px x %d samples x %d gains, %s" % (n, T, G, NAME[ex]))
        calib_parity(ct, tr, torch_dev, ex)


def layout_cameras():
    """Pixel layouts other than the generator's hexagon in distance order:
    the 61-pixel hexagon numbered at random, a 15 x 15 square grid (four
    neighbours), one row of 50 pixels, and a 331-pixel hexagon with every
    pixel moved by up to 0.1 pitch in x and y (its rows no longer share one
    y).  Neighbours: the oracle's distance rule (<= 1.4 pitch)."""
    p = dl0sim.PITCH_M
    rng = np.random.default_rng(31)
    h = dl0sim.hex_geometry(61)
    perm = rng.permutation(61)
    g = np.arange(15) * p
    gx, gy = np.meshgrid(g, g)
    j = dl0sim.hex_geometry(331)
    shapes = [("relabelled hexagon", h.x[perm], h.y[perm]), ("square grid", gx.ravel(), gy.ravel()),
              ("single row", np.arange(50) * p, np.zeros(50)),
              ("jittered hexagon", j.x + rng.uniform(-0.1, 0.1, 331) * p, j.y + rng.uniform(-0.1, 0.1, 331) * p)]
    out = []
    for name, x, y in shapes:
        x = np.ascontiguousarray(x, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        n = len(x)
        geom = dl0sim.Geometry(n, p, x, y, oracle.neighbours(x, y, 1.4 * p), np.zeros((n, 2), np.int32))
        out.append((name, dl0sim.CameraType(name, n, 40, 2, 5.0, geom=geom)))
    return out


@pytest.mark.parametrize("ex", EXS)
def test_calibrate_pixel_layouts(torch_dev, ex):
    """Every extractor against the oracle on the layouts above (random dual-
    gain traces, switching included): the lattice-row order in which the
    neighbour peak stages its words must not change any result."""
    rng = np.random.default_rng(37)
    for name, ct in layout_cameras():
        tr = rng.integers(250, 4300, size=(6, 2, 40, ct.n_pix_pad), dtype=np.uint16)
        say("pixel layout %s (%d px), %s" % (name, ct.n_pix, NAME[ex]))
        calib_parity(ct, tr, torch_dev, ex)


@pytest.mark.parametrize("ex", [rta.EXTRACT_SLIDING] + EXS)
def test_fused_small_cameras(torch_dev, ex):
    """The fused batch on a mix of 1-, 7- and 61-pixel cameras (random dual-
    and single-gain traces, switching included) in every extractor: records
    against the oracle's whole chain."""
    import torch
    cams = [dl0sim.CameraType("tiny1", 1, 4, 1, 5.0), dl0sim.CameraType("tiny7", 7, 9, 2, 5.0),
            dl0sim.CameraType("tiny61", 61, 33, 2, 5.0)]
    rng = np.random.default_rng(23)
    parts, ty, off, pos = [], [], [], 0
    for k in range(24):
        t = k % 3
        c = cams[t]
        ev = rng.integers(250, 4300, size=c.event_elems, dtype=np.uint16)
        parts.append(ev)
        ty.append(t)
        off.append(pos)
        pos += c.event_elems
    blob = np.concatenate(parts)
    say("fused small cameras, %s: 24 events" % NAME[ex])
    pipe = rta.Pipeline([rta.Camera.from_type(c) for c in cams], do_stereo=False, extractor=ex)
    b = pipe.make_batch(to_dev(blob, torch_dev), to_dev(np.array(ty, np.int32), torch_dev),
                        to_dev(np.array(off, np.int64), torch_dev))
    tel, _ = pipe.alloc_outputs(b, torch_dev)
    pipe.process(b, tel)
    torch.cuda.synchronize()
    assert pipe.status() == 0
    g = rta.records(tel)
    ocs = [oracle.Camera.from_type(c, extractor=ex) for c in cams]
    bad = []
    for k in range(len(ty)):
        c = cams[ty[k]]
        p, m, h = ocs[ty[k]].reconstruct(blob[off[k]:off[k] + c.event_elems])
        mm = par.hillas_mismatches(g[k], h, c.geom.x, c.geom.y, p["q"], p["t"], m)
        if mm:
            bad.append((k, mm))
    assert not bad, bad[:3]
