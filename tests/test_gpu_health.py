"""GPU parity of the health monitor against the oracle: sums and counts
exact, mean / rms bit-identical (FP64 without contraction on both sides),
the lower median, flags and the verdict exact."""
import numpy as np
import pytest

import dl0sim
import paper_1307_6489_amd as rta
from oracle import health as oh

pytestmark = pytest.mark.gpu
P = {"rms_dead": 0.5, "noisy_factor": 3.0, "ped_tol": 20.0, "sat_frac": 0.01, "bad_frac_max": 0.05}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rta.lib()
    return torch.device("cuda:0")


def check(ct, tr, dev, p=P, cam=None):
    import torch
    cam = cam or rta.Camera.from_type(ct)
    pix, c = rta.health(cam, torch.from_numpy(np.ascontiguousarray(tr)).to(dev), **p)
    rp, rc = oh.health(tr, ct.n_pix, ct.n_gain, ct.ped, ct.hg_switch_adc, p)
    assert np.array_equal(pix["n"].astype(np.int64), rp["n"])
    for k in ("S1", "S2", "n_sat"):
        assert np.array_equal(pix[k.lower()].astype(np.int64), rp[k]), k
    assert np.array_equal(pix["mean"], rp["mean"]) and np.array_equal(pix["rms"], rp["rms"])
    assert np.array_equal(pix["flags"].astype(np.int64), rp["flags"])
    assert np.array_equal(c["median_rms"][:ct.n_gain], rc["median_rms"])
    assert int(c["n_bad"]) == rc["n_bad"] and int(c["verdict"]) == rc["verdict"]
    return pix, c


@pytest.mark.parametrize("ti", [0, 1, 2])
def test_health_generated_events(torch_dev, ti):
    ct = dl0sim.camera_types_c1()[ti]
    say("health:", ct.name, "40 events, seed 17")
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(ct.n_samp), 17, 0, 40)
    sh["size"][::4, 0] = 1e5           # some saturating bright images
    tr = dl0sim.render_traces(ct, sh, 17)
    check(ct, tr, torch_dev)


def test_health_planted_faults_and_many_events(torch_dev):
    """Dead, noisy, shifted and saturating pixels on a single-gain camera,
    3000 events (several events per workgroup); and random 16-bit data at
    the largest shape."""
    ct = dl0sim.CameraType("faulty", 1855, 30, 1, 28.0)
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(30), 18, 0, 3000)
    sh["size"][:, 0] = 0.0
    tr = dl0sim.render_traces(ct, sh, 18)
    tr[:, 0, :, 10] = 301
    tr[:, 0, :, 20] = np.clip(tr[:, 0, :, 20].astype(np.int64) * 5 - 1200, 0, 65535)
    tr[:, 0, :, 30] += 60
    tr[:40, 0, :, 40] = 65535
    say("health: planted faults, 3000 events")
    pix, c = check(ct, tr, torch_dev)
    f = pix["flags"][0]
    assert f[10] & rta.HEALTH_DEAD and f[20] & rta.HEALTH_NOISY and f[30] & rta.HEALTH_PED_SHIFT
    assert f[40] & rta.HEALTH_SATURATING
    big = dl0sim.CameraType("max", 2048, 255, 1, 5.6)
    rng = np.random.default_rng(2)
    tr = rng.integers(0, 65536, size=(5, 1, 255, 2048), dtype=np.uint16)
    say("health: random 2048 x 255")
    check(big, tr, torch_dev)


def test_health_calls_in_a_row_on_one_camera(torch_dev):
    """One camera handle, 300 dual-gain events then 7: the second call's
    totals come from its own workgroups only (the per-workgroup partial
    blocks of the first, larger call are not summed again)."""
    ct = dl0sim.camera_types_c1()[1]
    cam = rta.Camera.from_type(ct)
    for n, seed in ((300, 19), (7, 20)):
        say("health: %d events on one camera handle, seed %d" % (n, seed))
        sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(ct.n_samp), seed, 0, n)
        sh["size"][::5, 0] = 1e5
        check(ct, dl0sim.render_traces(ct, sh, seed), torch_dev, cam=cam)


@pytest.mark.parametrize("n_pix", [1, 7, 100, 1000])
def test_health_small_cameras(torch_dev, n_pix):
    """Cameras far below 2048 pixels: the sort pads the rms with +inf, the
    median is element (N - 1) / 2 of the real pixels.  Dual gain, samples
    around the pedestal, a dead and a noisy pixel where there is room."""
    ct = dl0sim.CameraType("small%d" % n_pix, n_pix, 20, 2, 10.0)
    npad = (n_pix + 7) // 8 * 8
    rng = np.random.default_rng(n_pix)
    tr = rng.integers(281, 322, size=(9, 2, 20, npad), dtype=np.uint16)
    if n_pix > 2:
        tr[:, :, :, 1] = 301
        tr[:, 0, :, 2] = rng.integers(151, 452, size=(9, 20), dtype=np.uint16)
    say("health: %d-pixel dual-gain camera, 9 events" % n_pix)
    pix, c = check(ct, tr, torch_dev)
    if n_pix > 2:
        assert pix["flags"][0][1] & rta.HEALTH_DEAD and pix["flags"][0][2] & rta.HEALTH_NOISY


def test_health_rejects_bad_arguments(torch_dev):
    """Host-side checks: no events, non-finite thresholds, a trace buffer
    that is not 16-byte aligned; nothing is launched for them."""
    import torch
    ct = dl0sim.camera_types_c1()[1]
    cam = rta.Camera.from_type(ct)
    tr = torch.zeros((2 * cam.event_elems + 8,), dtype=torch.uint16, device=torch_dev)
    with pytest.raises(rta.RTAError):
        rta.health(cam, tr[:0])
    with pytest.raises(rta.RTAError):
        rta.health(cam, tr[:2 * cam.event_elems], ped_tol=float("nan"))
    with pytest.raises(rta.RTAError):
        rta.health(cam, tr[1:1 + 2 * cam.event_elems])


def test_health_full_size_sampled(torch_dev):
    """The measured job: 2000 signal-free 2048 x 128 dual-gain events (2.1
    GB, 200 generated events tiled ten times).  64 sampled pixels against
    the oracle on their columns: counts, sums, mean and rms exact, the flags
    that do not involve the camera median exact; the median is the lower
    median of the returned rms values."""
    import torch
    ct = dl0sim.camera_types_c1()[2]
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(ct.n_samp), 21, 0, 200)
    sh["size"][:, 0] = 0.0
    base = dl0sim.render_traces(ct, sh, 21)
    tr = np.tile(base, (10, 1, 1, 1))
    say("health, full size: 2000 x 2048 x 128 x 2")
    cam = rta.Camera.from_type(ct)
    pix, c = rta.health(cam, torch.from_numpy(np.ascontiguousarray(tr)).to(torch_dev), **P)
    idx = np.sort(np.random.default_rng(5).choice(ct.n_pix, 64, replace=False))
    rp, rc = oh.health(np.ascontiguousarray(tr[..., idx]), 64, ct.n_gain, ct.ped[:, idx], ct.hg_switch_adc, P)
    assert np.array_equal(pix["n"][:, idx].astype(np.int64), rp["n"])
    for k in ("S1", "S2", "n_sat"):
        assert np.array_equal(pix[k.lower()][:, idx].astype(np.int64), rp[k]), k
    assert np.array_equal(pix["mean"][:, idx], rp["mean"]) and np.array_equal(pix["rms"][:, idx], rp["rms"])
    keep = rta.HEALTH_DEAD | rta.HEALTH_PED_SHIFT | rta.HEALTH_SATURATING
    assert np.array_equal(pix["flags"][:, idx].astype(np.int64) & keep, rp["flags"] & keep)
    for g in range(ct.n_gain):
        assert c["median_rms"][g] == np.sort(pix["rms"][g])[(ct.n_pix - 1) // 2]
