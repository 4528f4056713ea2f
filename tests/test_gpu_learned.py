"""GPU tests of the classification layer and of the learned part.

* features / box cuts / network decisions of rta_classify against the oracle
  (integer decisions bit-exact, except knife-edge rows whose float32 inputs
  sit within rounding of a bin edge, a range edge or the score threshold);
* the per-event pass with an attached network against the oracle's
  size-weighted aggregation;
* the benefit test: trained on the GPU kernels, the network beats the plain
  box cuts in hadron acceptance at equal gamma efficiency (held-out seed).
"""
import numpy as np
import pytest

import dl0sim
import dl0sim.workloads as W
import oracle.boxcut as obox
import paper_1307_6489_amd as rta
from oracle import mlp as omlp
from paper_1307_6489_amd import boxcut, learn

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rta.lib()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def small_model(dev):
    """A network trained on 100k generated images (seed 3, about 780 Adam
    steps) and a held-out set of 20k (seed 4)."""
    cam = dl0sim.camera_c0()
    say("small model: 100k training / 20k held-out images on the 1855-pixel camera")
    tr = learn.image_features(cam, 100_000, 3, dev)
    te = learn.image_features(cam, 20_000, 4, dev)
    net, bc, info = learn.train(tr, dev, epochs=8, batch=1024, lr=2e-3)
    return cam, tr, te, net, bc, info


def rec_tensor(rec, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(rec).view(np.float32).reshape(-1, 16).copy()).to(dev)


def test_features_parity(dev, small_model):
    cam, tr, te, net, bc, info = small_model
    rec = te["rec"][:5000]
    x = rta.features(rec_tensor(rec, dev)).cpu().numpy()
    ref = omlp.features_from_records(rec)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(x), fin)
    assert np.allclose(x[fin], ref[fin], rtol=1e-6, atol=0)


ULP32 = 2.0 ** -23


def knife_edge(bc, feat, score=None, score_tol=1e-3):
    """Rows whose float32 inputs lie within a few float32 ulps of a decision
    edge (log10 size is computed by each side's own log10 and may differ by
    one ulp)."""
    f = np.asarray(feat, np.float64)
    lo, hi = np.array(bc.feat_lo, np.float64), np.array(bc.feat_hi, np.float64)
    tol_lo = 4 * ULP32 * np.abs(lo) + 1e-37
    tol_hi = 4 * ULP32 * np.abs(hi) + 1e-37
    near_range = np.any(np.isfinite(f) & ((np.abs(f - lo) <= tol_lo) | (np.abs(f - hi) <= tol_hi)), 1)
    lgs = np.where(np.isfinite(f[:, 0]), f[:, 0], 0.0)
    near_bin = obox.bin_edge_distance(bc, lgs) < 4 * ULP32 * (np.abs(lgs) + 1.0)
    edge = near_range | near_bin
    if score is not None:
        edge |= np.abs(score - bc.mlp_cut) < score_tol
    return edge


def test_classify_parity_box_only(dev, small_model):
    cam, tr, te, net, bc, info = small_model
    rec = te["rec"]
    out = rta.classify(None, bc, rec_tensor(rec, dev)).cpu().numpy()
    feat = omlp.features_from_records(rec).astype(np.float32)
    s, e, g, fb = obox.classify(bc, feat)
    ok = ~knife_edge(bc, feat)
    assert ok.mean() > 0.99
    assert np.array_equal(out[ok, 2].astype(np.int64), g[ok])
    assert np.all(out[:, 3] == 1)
    fin = ok & np.isfinite(e)
    assert np.allclose(out[fin, 1], e[fin], rtol=1e-5, atol=1e-5)


def test_classify_parity_with_network(dev, small_model):
    """rta_classify with the network against the oracle's decision rule
    applied to the GPU's own features and network outputs, element by
    element: fallback and gamma decisions exact, network scores within 1e-5
    relative (float32 sigmoid), energies equal to the network's output, the
    box-cut rows' scores exact and energies within 1e-5.  The features are
    compared with the oracle's in test_features_parity, the network outputs
    layer by layer in test_gpu_mlp; only rows whose inputs sit within float32
    rounding of a range, bin or score edge are skipped, at most 1 %."""
    import torch
    cam, tr, te, net, bc, info = small_model
    rec = te["rec"]
    R = rec_tensor(rec, dev)
    out = rta.classify(net, bc, R).cpu().numpy().astype(np.float64)
    xg = rta.features(R)
    fin = torch.isfinite(xg).all(1)
    o = np.full((len(rec), 2), np.nan)
    o[fin.cpu().numpy()] = net.forward(xg[fin].contiguous()).cpu().numpy()
    feat = xg.cpu().numpy()
    s, e, g, fb = obox.classify(bc, feat, o[:, 0], o[:, 1])
    ok = ~knife_edge(bc, feat, s, score_tol=1e-6)
    assert ok.mean() > 0.99
    assert np.array_equal(out[ok, 3].astype(np.int64), fb[ok])
    assert np.array_equal(out[ok, 2].astype(np.int64), g[ok])
    net_rows = ok & (fb == 0)
    box_rows = ok & (fb == 1)
    assert net_rows.sum() > 1000 and box_rows.sum() > 10
    assert np.all(np.abs(out[net_rows, 0] - s[net_rows]) <= 1e-5 * s[net_rows] + 1e-7)
    assert np.array_equal(out[net_rows, 1], o[net_rows, 1].astype(np.float32).astype(np.float64))
    assert np.array_equal(out[box_rows, 0], s[box_rows])
    fe = box_rows & np.isfinite(e)
    assert np.all(np.abs(out[fe, 1] - e[fe]) <= 1e-5 * (np.abs(e[fe]) + 1.0))


def test_event_pass_with_network(dev, small_model):
    """Array events through the fused batch with the network attached: event
    gammaness and log10 E are the size-weighted means of rta_classify."""
    import torch
    cam_c0, tr, te, net, bc, info = small_model
    aw = W.array_events(20, seed=8)
    cams = [rta.Camera.from_type(c) for c in aw.pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=True)
    pipe.attach_mlp(net, bc)
    b = pipe.make_batch(torch.from_numpy(aw.pool.blob).to(dev), torch.from_numpy(aw.tel_type).to(dev),
                        torch.from_numpy(aw.tel_off).to(dev), torch.from_numpy(aw.evt_tel_off).to(dev))
    tel, evt = pipe.alloc_outputs(b, dev)
    pipe.process(b, tel, evt)
    cls = rta.classify(net, bc, tel).cpu().numpy()
    rec = rta.records(tel)
    ev = rta.records(evt, rta.EVENT_DTYPE)
    for e in range(len(aw.evt_tel_off) - 1):
        lo, hi = aw.evt_tel_off[e], aw.evt_tel_off[e + 1]
        r = rec[lo:hi]
        c = cls[lo:hi]
        ok = ((r["flags"] & rta.FLAG_HILLAS_INVALID) == 0) & np.isfinite(c[:, 1]) & (r["size"] > 0)
        if ok.sum() == 0:
            assert np.isnan(ev["gammaness"][e])
            continue
        w = r["size"][ok].astype(np.float64)
        assert ev["gammaness"][e] == pytest.approx(np.sum(w * c[ok, 0]) / w.sum(), rel=1e-4, abs=1e-5)
        assert ev["log10_energy"][e] == pytest.approx(np.sum(w * c[ok, 1]) / w.sum(), rel=1e-4, abs=1e-5)
        assert (ev["flags"][e] & rta.EVT_NO_MLP) == 0
        fbk = (r["flags"] & rta.FLAG_MLP_FALLBACK) > 0
        assert np.array_equal(fbk[ok], c[ok, 3] > 0.5)


def test_classification_fused_after_hillas(dev, small_model):
    """Array events with the network attached, each telescope classified in
    the reconstruction kernel right after its Hillas parameters (tel_class
    given): scores and log10 E bit-identical to rta_classify on the same
    records, the same fallback flags, NaN for telescopes without a valid
    image, and every telescope and event record byte-identical to the run
    that classifies in the per-event pass; without stereo the same values."""
    import torch
    cam_c0, tr, te, net, bc, info = small_model
    aw = W.array_events(20, seed=8)
    cams = [rta.Camera.from_type(c) for c in aw.pool.cams]
    blob = torch.from_numpy(aw.pool.blob).to(dev)
    ty, off = torch.from_numpy(aw.tel_type).to(dev), torch.from_numpy(aw.tel_off).to(dev)
    eo = torch.from_numpy(aw.evt_tel_off).to(dev)
    n_tel = len(aw.tel_type)
    pipe = rta.Pipeline(cams, do_stereo=True)
    pipe.attach_mlp(net, bc)
    b1 = pipe.make_batch(blob, ty, off, eo)
    tel1, evt1 = pipe.alloc_outputs(b1, dev)
    pipe.process(b1, tel1, evt1)
    cls = torch.full((n_tel, 2), -7.0, dtype=torch.float32, device=dev)
    b2 = pipe.make_batch(blob, ty, off, eo, tel_class=cls)
    tel2, evt2 = pipe.alloc_outputs(b2, dev)
    pipe.process(b2, tel2, evt2)
    torch.cuda.synchronize()
    assert pipe.status() == 0
    assert torch.equal(tel1.view(torch.int32), tel2.view(torch.int32))
    assert torch.equal(evt1.view(torch.int32), evt2.view(torch.int32))
    rec = rta.records(tel2)
    ref = rta.classify(net, bc, tel2).cpu().numpy()
    c = cls.cpu().numpy()
    valid = (rec["flags"] & rta.FLAG_HILLAS_INVALID) == 0
    assert valid.sum() > 100 and (~valid).sum() > 0
    assert np.array_equal(c[valid].view(np.int32), ref[valid, :2].view(np.int32))
    assert np.all(np.isnan(c[~valid]))
    fb = (rec["flags"] & rta.FLAG_MLP_FALLBACK) > 0
    assert np.array_equal(fb[valid], ref[valid, 3] > 0.5) and not fb[~valid].any()
    # per-telescope classification without the per-event pass, the network
    # given at creation
    pipe_ns = rta.Pipeline(cams, do_stereo=False, mlp=net, boxcut=bc)
    cls3 = torch.full((n_tel, 2), -7.0, dtype=torch.float32, device=dev)
    b3 = pipe_ns.make_batch(blob, ty, off, tel_class=cls3)
    tel3, _ = pipe_ns.alloc_outputs(b3, dev)
    pipe_ns.process(b3, tel3)
    torch.cuda.synchronize()
    assert torch.equal(cls3.view(torch.int32), cls.view(torch.int32))
    assert torch.equal(tel3.view(torch.int32), tel2.view(torch.int32))
    with pytest.raises(rta.RTAError):
        bare = rta.Pipeline(cams, do_stereo=False)
        bare.process(bare.make_batch(blob, ty, off, tel_class=cls3), tel3)
    for kw in ({"mlp": net}, {"boxcut": bc}):  # a network needs its fallback tables and the reverse
        with pytest.raises(rta.RTAError) as e:
            rta.Pipeline(cams, do_stereo=False, **kw)
        assert e.value.status == 1


def test_network_beats_box_cuts_on_gamma_like_hadrons(dev):
    """The harder population: hadrons as single ellipses whose width and
    length overlap the gammas', so the box cuts keep a large hadron
    fraction.  Trained and evaluated on that population (100k / 20k
    images), the network still accepts fewer hadrons at equal gamma
    efficiency, by more than three binomial standard deviations."""
    cam = dl0sim.camera_c0()
    say("gamma-like hadrons: 100k training / 20k held-out images on the 1855-pixel camera")
    tr = learn.image_features(cam, 100_000, 3, dev, hadrons="single")
    te = learn.image_features(cam, 20_000, 4, dev, hadrons="single")
    net, bc, info = learn.train(tr, dev, epochs=8, batch=1024, lr=2e-3)
    res = learn.evaluate(net, bc, te, dev, timing_reps=2)
    say("held-out (gamma-like hadrons):", res)
    assert abs(res["gamma_eff_network"] - res["gamma_eff_box"]) < 0.005
    assert res["hadron_acc_box"] > 0.1   # the box cuts do not separate this population
    diff = res["hadron_acc_box"] - res["hadron_acc_network"]
    assert diff > 3 * np.hypot(res["hadron_acc_box_err"], res["hadron_acc_network_err"])


def test_network_beats_box_cuts(dev, small_model):
    """At equal gamma efficiency on the held-out seed the network accepts
    fewer hadrons than the scaled-width/length box cuts (by more than three
    binomial standard deviations) and estimates log10 E more precisely than
    the size-only fit."""
    cam, tr, te, net, bc, info = small_model
    res = learn.evaluate(net, bc, te, dev, timing_reps=5)
    say("held-out:", res)
    assert abs(res["gamma_eff_network"] - res["gamma_eff_box"]) < 0.005
    diff = res["hadron_acc_box"] - res["hadron_acc_network"]
    assert diff > 3 * np.hypot(res["hadron_acc_box_err"], res["hadron_acc_network_err"])
    assert res["log10e_rms_network"] < res["log10e_rms_linear_fit"]
