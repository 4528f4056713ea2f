"""Pins of the health-monitor oracle: sums against a direct loop on a tiny
camera, hand-made dead / noisy / shifted / saturating pixels, the lower
median, constant traces, and the generator's noise (pedestal 301 ADC, rms
sqrt(25 + 100 * 0.1 + 1/12) for the high gain).  CPU only."""
import math

import numpy as np

import dl0sim
from oracle import health as oh

P = {"rms_dead": 0.5, "noisy_factor": 3.0, "ped_tol": 20.0, "sat_frac": 0.01, "bad_frac_max": 0.05}


def test_sums_against_a_direct_loop():
    rng = np.random.default_rng(0)
    tr = rng.integers(0, 65536, size=(3, 2, 5, 8), dtype=np.uint16)
    pix, cam = oh.health(tr, 6, 2, np.zeros((2, 6)), 4000, P)
    for g in range(2):
        for i in range(6):
            vals = [int(tr[e, g, k, i]) for e in range(3) for k in range(5)]
            assert pix["S1"][g, i] == sum(vals) and pix["S2"][g, i] == sum(v * v for v in vals)
            lvl = 4000 if g == 0 else 65535
            assert pix["n_sat"][g, i] == sum(v >= lvl for v in vals) and pix["n"][g, i] == 15
            m = sum(vals) / 15
            assert pix["mean"][g, i] == m
            assert pix["rms"][g, i] == math.sqrt(max(sum(v * v for v in vals) / 15 - m * m, 0.0))


def test_hand_made_bad_pixels():
    rng = np.random.default_rng(1)
    E, T, N = 20, 30, 40
    tr = np.rint(300 + 5 * rng.standard_normal((E, 1, T, 48))).astype(np.uint16)
    tr[:, 0, :, 3] = 300                                   # dead: constant
    tr[:, 0, :, 7] = np.rint(300 + 40 * rng.standard_normal((E, T))).astype(np.uint16)   # noisy
    tr[:, 0, :, 11] += 50                                  # pedestal shifted
    tr[:5, 0, :, 13] = 65535                               # saturating (single gain: 65535)
    pix, cam = oh.health(tr, N, 1, np.full((1, N), 300.0), 4000, P)
    f = pix["flags"][0]
    assert f[3] == oh.DEAD and f[7] & oh.NOISY and f[11] == oh.PED_SHIFT and f[13] & oh.SATURATING
    others = [i for i in range(N) if i not in (3, 7, 11, 13)]
    assert not f[others].any()
    assert cam["n_bad"] == 4 and cam["verdict"] == 1          # 4 > 0.05 * 40
    pix, cam = oh.health(tr, N, 1, np.full((1, N), 300.0), 4000, dict(P, bad_frac_max=0.2))
    assert cam["verdict"] == 0


def test_lower_median():
    tr = np.zeros((1, 1, 2, 8), np.uint16)
    tr[0, 0, 1, :4] = [2, 4, 6, 8]                         # rms = x/2 for samples (0, x)
    pix, cam = oh.health(tr, 4, 1, np.zeros((1, 4)), 4000, P)
    assert list(pix["rms"][0]) == [1.0, 2.0, 3.0, 4.0] and cam["median_rms"][0] == 2.0


def test_generator_noise_is_recovered():
    """Signal-free generated events: mean -> 300 + NSB 0.1 p.e. x 10 ADC and
    rms -> sqrt(5^2 + 10^2 * 0.1 + 1/12) (electronic noise, Poisson NSB,
    rounding) on the high gain; nothing flagged."""
    cam = dl0sim.CameraType("quiet", 1855, 40, 2, 28.0)
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(40), 7, 0, 30)
    sh["size"][:, 0] = 0.0
    tr = dl0sim.render_traces(cam, sh, 7)
    pix, c = oh.health(tr, cam.n_pix, cam.n_gain, cam.ped, cam.hg_switch_adc, P)
    assert abs(pix["mean"][0].mean() - 301.0) < 0.05
    assert abs(np.median(pix["rms"][0]) - math.sqrt(25 + 100 * 0.1 + 1 / 12)) < 0.05
    assert c["n_bad"] == 0 and c["verdict"] == 0
