"""Science alert monitor measured: fill rate, search latency, alert delay.

The paper requires science alerts within 30 s of the triggering events and a
transient search on timescales from seconds to hours, in a source region and
across the field of view (Section 2).  This job measures, on synthetic event
lists (background uniform over the field, flares as point sources):

  fill      events histogrammed per second (device-resident event records);
  search    latency of one search over all timescales for a 64 x 64 and a
            128 x 128 sky grid, 3600 one-second bins, windows of 1 s, 10 s,
            1 min, 10 min and 1 h;
  health    the health monitor's rate over signal-free 2048 x 128 dual-gain
            events (bytes of traces per second);
  alerts    a one-hour event list at 1 kHz with three flares, searched every
            10 s as the data arrive: the delay from each flare's start to its
            first alert at its position.

Run ``python -m paper_1307_6489_amd.monitor``.
"""
from __future__ import annotations

import json
import time

import numpy as np

import paper_1307_6489_amd as rta

SCALES = [1, 10, 60, 600, 3600]


def event_tensors(t, d, g, v, dev):
    import torch
    rec = np.zeros(len(t), rta.EVENT_DTYPE)
    rec["dir_x"], rec["dir_y"], rec["gammaness"] = d[:, 0], d[:, 1], g
    rec["flags"] = np.where(v, 0, rta.EVT_STEREO_INVALID)
    e = torch.from_numpy(rec.view(np.float32).reshape(-1, 8).copy()).to(dev)
    return e, torch.from_numpy(np.ascontiguousarray(t, np.float64)).to(dev)


def make(grid, cell=0.0015):
    return rta.Sam(grid, 3600, 0.0, 1.0, cell, 1.5, 3.5, 7.0, 0.7, 5.0, SCALES)


def fill_and_search_rates(dev, log=None):
    import torch
    import dl0sim.workloads as W
    t, d, g, v = W.sam_events(11, 3600.0, 3000.0, 0.05, [])
    e, td = event_tensors(t, d, g, v, dev)
    out = {"events": int(len(t))}
    for grid in (64, 128):
        sam = make(grid)
        sam.fill(e, td)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            sam.fill(e, td)
        b.record()
        b.synchronize()
        fill_ms = a.elapsed_time(b) / 5
        sam.search(3599, maps=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            sam.search(3599, maps=False)
        search_ms = (time.perf_counter() - t0) / 10 * 1e3
        out["grid%d" % grid] = {"fill_events_per_s": len(t) / (fill_ms * 1e-3), "fill_ms": fill_ms,
                                "search_ms_wall": search_ms, "cells": grid * grid, "scales": SCALES}
        if log:
            log("grid %d: %s" % (grid, out["grid%d" % grid]))
    return out


def alert_delay(dev, log=None):
    import dl0sim.workloads as W
    flares = [(0.010, 0.004, 900.0, 960.0, 5.0, 0.0008),      # one minute, bright
              (-0.018, 0.012, 2000.0, 2600.0, 0.6, 0.0008),  # ten minutes, faint
              (0.0, -0.02, 3000.0, 3004.0, 60.0, 0.0008)]    # four seconds, very bright
    t, d, g, v = W.sam_events(12, 3600.0, 1000.0, 0.05, flares)
    sam = make(64)
    cell = float(np.float32(0.0015))
    first = [None] * len(flares)
    step = 10.0
    lo = 0
    t_now = step
    n_search = 0
    search_s = 0.0
    while t_now <= 3600.0:
        hi = int(np.searchsorted(t, t_now))
        if hi > lo:
            e, td = event_tensors(t[lo:hi], d[lo:hi], g[lo:hi], v[lo:hi], dev)
            sam.fill(e, td)
            lo = hi
        t0 = time.perf_counter()
        _, _, _, alerts, _ = sam.search(int(t_now) - 1, maps=False)
        search_s += time.perf_counter() - t0
        n_search += 1
        for k, (x, y, ta, tb, rate, psf) in enumerate(flares):
            if first[k] is not None or t_now < ta:
                continue
            ix, iy = int(np.floor(x / cell + 32)), int(np.floor(y / cell + 32))
            hit = [a for a in alerts if abs(int(a["ix"]) - ix) <= 1 and abs(int(a["iy"]) - iy) <= 1]
            if hit:
                first[k] = {"t_alert": t_now, "delay_s": t_now - ta, "scales": sorted({SCALES[int(a["scale"])]
                                                                                     for a in hit}),
                            "max_sigma": float(max(a["significance"] for a in hit))}
        t_now += step
    res = {"events": int(len(t)), "search_every_s": step, "searches": n_search,
           "search_ms_mean": search_s / n_search * 1e3,
           "flares": [{"start_s": f[2], "duration_s": f[3] - f[2], "rate_hz": f[4], "first_alert": first[k]}
                      for k, f in enumerate(flares)]}
    if log:
        log("alerts: %s" % json.dumps(res))
    return res


def health_rate(dev, n_evt=2000, log=None):
    """rta_health over n_evt signal-free 2048 x 128 dual-gain events."""
    import torch
    import dl0sim
    ct = dl0sim.camera_types_c1()[2]
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(ct.n_samp), 21, 0, 200)
    sh["size"][:, 0] = 0.0
    base = dl0sim.render_traces(ct, sh, 21)
    tr = torch.from_numpy(np.ascontiguousarray(np.tile(base, (n_evt // 200, 1, 1, 1)))).to(dev)
    cam = rta.Camera.from_type(ct)
    rta.health(cam, tr)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(5):
        rta.health(cam, tr, to_host=False)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / 5
    pix, c = rta.health(cam, tr)
    r = {"events": n_evt, "GB": tr.numel() * 2 / 1e9, "ms": ms, "GBps": tr.numel() * 2 / (ms * 1e-3) / 1e9,
         "hbm_frac": tr.numel() * 2 / (ms * 1e-3) / 8e12, "n_bad": int(c["n_bad"]), "verdict": int(c["verdict"])}
    if log:
        log("health: %s" % r)
    return r


def main():
    import torch
    dev = torch.device("cuda:0")
    say = lambda s: print(s, flush=True)  # noqa: E731
    res = {"rates": fill_and_search_rates(dev, say), "alert_delay": alert_delay(dev, say),
           "health": health_rate(dev, log=say)}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
