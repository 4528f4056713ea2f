"""GPU parity of the science alert monitor against the oracle: the counts
cube exactly (order-independent, accumulating over fills), N_on / N_off
exactly, the FP64 significance to rounding, the alert set exactly (away
from the threshold), zero significance on a flat sky."""
import numpy as np
import pytest

import dl0sim.workloads as W
import paper_1307_6489_amd as rta
from oracle import sam as osam

pytestmark = pytest.mark.gpu

P = {"grid": 48, "cell": 0.0015, "t0": 10.0, "bin_s": 0.5, "n_bins": 1200, "r_on": 1.5, "r_in": 3.5, "r_out": 7.0,
     "gamma_cut": 0.7, "scales": [2, 20, 120, 1200], "sigma_alert": 4.0}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rta.lib()
    return torch.device("cuda:0")


def records(d, g, valid):
    rec = np.zeros(len(g), rta.EVENT_DTYPE)
    rec["dir_x"], rec["dir_y"], rec["gammaness"] = d[:, 0], d[:, 1], g
    rec["flags"] = np.where(valid, 0, rta.EVT_STEREO_INVALID)
    return rec


def make_sam(p):
    return rta.Sam(p["grid"], p["n_bins"], p["t0"], p["bin_s"], p["cell"], p["r_on"], p["r_in"], p["r_out"],
                   p["gamma_cut"], p["sigma_alert"], p["scales"])


def to_dev(rec, t, dev):
    import torch
    e = torch.from_numpy(np.ascontiguousarray(rec).view(np.float32).reshape(-1, 8).copy()).to(dev)
    return e, torch.from_numpy(np.ascontiguousarray(t, np.float64)).to(dev)


@pytest.fixture(scope="module")
def events():
    t, d, g, v = W.sam_events(5, 620.0, 60.0, 0.04, [(0.01, 0.006, 400.0, 460.0, 6.0, 0.0008),
                                                    (-0.02, -0.012, 100.0, 105.0, 40.0, 0.0006)])
    t = t + P["t0"] - 5.0          # some events before bin 0, some after the last bin
    # events exactly on cell boundaries and at the grid edges
    k = np.arange(12)
    edge = ((k - P["grid"] // 2) * np.float32(P["cell"])).astype(np.float32)
    d[:12, 0] = edge
    d[12:24, 1] = edge
    g[:24] = 0.9
    v[:24] = True
    return t, d, g, v


def test_counts_exact_and_order_independent(torch_dev, events):
    t, d, g, v = events
    say("alert monitor fill: %d events" % len(t))
    C_ref, used = osam.histogram(d, t, g, v, P)
    sam = make_sam(P)
    e, td = to_dev(records(d, g, v), t, torch_dev)
    sam.fill(e, td)
    C = sam.counts()
    assert np.array_equal(C.astype(np.int64), C_ref) and int(C.sum()) == used
    # shuffled and split over three fills: the same cube
    sam.clear()
    perm = np.random.default_rng(1).permutation(len(t))
    for part in np.array_split(perm, 3):
        e, td = to_dev(records(d[part], g[part], v[part]), t[part], torch_dev)
        sam.fill(e, td)
    assert np.array_equal(sam.counts().astype(np.int64), C_ref)


def test_search_parity(torch_dev, events):
    t, d, g, v = events
    C_ref, _ = osam.histogram(d, t, g, v, P)
    sam = make_sam(P)
    e, td = to_dev(records(d, g, v), t, torch_dev)
    sam.fill(e, td)
    for end_bin in (0, 190, 919, P["n_bins"] - 1):
        say("alert monitor search, end bin", end_bin)
        ref, ref_alerts = osam.search(C_ref, end_bin, P)
        sig, non, noff, alerts, n_found = sam.search(end_bin)
        sig, non, noff = sig.cpu().numpy(), non.cpu().numpy(), noff.cpu().numpy()
        for si, r in enumerate(ref):
            assert np.array_equal(non[si].astype(np.int64), r["N_on"])
            assert np.array_equal(noff[si].astype(np.int64), r["N_off"])
            assert np.allclose(sig[si], r["S"], rtol=1e-12, atol=1e-12)
        near = {(si, x, y) for si, x, y, s in ref_alerts if abs(s - P["sigma_alert"]) < 1e-9}
        got = {(int(a["scale"]), int(a["ix"]), int(a["iy"])) for a in alerts} - near
        want = {(si, x, y) for si, x, y, s in ref_alerts} - near
        assert got == want and n_found == len(alerts)
    # the flares: the window ending inside the 400-460 s flare alerts
    sig, non, noff, alerts, n_found = sam.search(int((450.0 - P["t0"]) / P["bin_s"]))
    assert len(alerts) > 0


def test_flat_sky_and_alert_capacity(torch_dev):
    """A flat sky gives exactly zero everywhere; with more alerts than room,
    the count is still complete and only max_alerts are written."""
    p = dict(P, n_bins=4, scales=[1, 4], sigma_alert=-1.0)
    sam = make_sam(p)
    G = p["grid"]
    cells = np.stack(np.meshgrid(np.arange(G), np.arange(G)), -1).reshape(-1, 2)
    d = ((cells - G // 2 + 0.5) * np.float32(p["cell"])).astype(np.float32)
    d = np.repeat(d, 3, axis=0)
    t = np.full(len(d), p["t0"] + 1.2)
    g = np.full(len(d), 0.95, np.float32)
    e, td = to_dev(records(d, g, np.ones(len(d), bool)), t, torch_dev)
    sam.fill(e, td)
    sig, non, noff, alerts, n_found = sam.search(3, max_alerts=100)
    assert np.all(sig.cpu().numpy() == 0.0)
    assert n_found == 2 * G * G and len(alerts) == 100        # every cell has S = 0 >= -1


def test_bad_parameters_rejected(torch_dev):
    for bad in (dict(P, grid=0), dict(P, r_in=1.0), dict(P, scales=[0]), dict(P, bin_s=0.0),
                dict(P, scales=[P["n_bins"] + 1])):
        with pytest.raises(rta.RTAError):
            make_sam(bad)


def test_full_size_hour_sampled(torch_dev):
    """The measured monitor job: a 1-hour 3 kHz event list (10.8 M events)
    into 64 x 64 cells of 1.5 mrad x 3600 one-second bins, windows of 1 s to
    1 h.  Six sampled time bins of the counts cube against the oracle's
    histogram of the events around them (exact), and the search at the last
    bin against the oracle's search of the same cube: N_on, N_off exact, S to
    rounding, alerts exact."""
    p = {"grid": 64, "cell": 0.0015, "t0": 0.0, "bin_s": 1.0, "n_bins": 3600, "r_on": 1.5, "r_in": 3.5,
         "r_out": 7.0, "gamma_cut": 0.7, "scales": [1, 10, 60, 600, 3600], "sigma_alert": 5.0}
    t, d, g, v = W.sam_events(11, 3600.0, 3000.0, 0.05, [])
    say("alert monitor, full size: %d events" % len(t))
    sam = make_sam(p)
    e, td = to_dev(records(d, g, v), t, torch_dev)
    sam.fill(e, td)
    C = sam.counts().astype(np.int64)
    rng = np.random.default_rng(31)
    for b in [0, 1799, 3599] + [int(x) for x in rng.integers(1, 3599, 3)]:
        m = (t >= b - 1.0) & (t < b + 2.0)
        Cb, _ = osam.histogram(d[m], t[m], g[m], v[m], p)
        assert np.array_equal(C[b], Cb[b]), b
    say("alert monitor, full size: search at bin 3599")
    ref, ref_alerts = osam.search(C, 3599, p)
    sig, non, noff, alerts, n_found = sam.search(3599)
    sig, non, noff = sig.cpu().numpy(), non.cpu().numpy(), noff.cpu().numpy()
    for si, r in enumerate(ref):
        assert np.array_equal(non[si].astype(np.int64), r["N_on"])
        assert np.array_equal(noff[si].astype(np.int64), r["N_off"])
        assert np.allclose(sig[si], r["S"], rtol=1e-12, atol=1e-12)
    near = {(si, x, y) for si, x, y, s in ref_alerts if abs(s - p["sigma_alert"]) < 1e-9}
    got = {(int(a["scale"]), int(a["ix"]), int(a["iy"])) for a in alerts} - near
    assert got == {(si, x, y) for si, x, y, s in ref_alerts} - near and n_found == len(alerts)
