"""Signal extractors compared: charge resolution and throughput.

The paper plans to port several signal-extraction algorithms to the GPU and
measure them (Section 5).  This job compares the four extractors of the
library on the mixed dual-gain workload:

  resolution   generated events with their true Cherenkov photo-electron
               counts per pixel; each extractor's charge q is scaled by its
               pulse-containment factor (median q / n_pe of bright pixels) and
               compared with n_pe in bins of n_pe (bias and relative RMS), plus
               the charge of signal-free pixels (mean and RMS, p.e.), where a
               window that searches for the maximum is biased upwards;
  throughput   the fused calibrate -> clean -> Hillas batch on 1e6 camera
               events streamed through a device-resident pool, per extractor,
               with the best launch shape of each (autotuned).

Run ``python -m paper_1307_6489_amd.extractors --help``.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

import paper_1307_6489_amd as rta

NAMES = {rta.EXTRACT_SLIDING: "sliding", rta.EXTRACT_FIXED: "fixed", rta.EXTRACT_GLOBAL_PEAK: "global_peak",
         rta.EXTRACT_NEIGHBOUR_PEAK: "neighbour_peak"}
NPE_BINS = (1, 3, 10, 30, 100, 300, 1000, 3000, 1e9)


def resolution(cams, n_events, dev, seed=31, log=None):
    """Per extractor and camera type: containment factor, bias and relative
    RMS of q/c - n_pe in bins of n_pe, and the signal-free pixel charge."""
    import dl0sim
    out = {}
    for ti, ct in enumerate(cams):
        cam = rta.Camera.from_type(ct)
        sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(ct.n_samp), seed, 1000 * ti, n_events)
        tr, npe = dl0sim.render_traces(ct, sh, seed, event_ids=np.arange(1000 * ti, 1000 * ti + n_events,
                                                                          dtype=np.uint64), want_npe=True)
        import torch
        T = torch.from_numpy(tr).to(dev)
        true = npe.astype(np.float64).reshape(-1)
        per = {}
        for ex, name in NAMES.items():
            q = rta.calibrate(cam, T, outputs=("q",), extractor=ex)["q"].cpu().numpy().astype(np.float64)
            q = q.reshape(-1)
            bright = true > 300
            c = float(np.median(q[bright] / true[bright])) if bright.any() else 1.0
            bins = []
            for lo, hi in zip(NPE_BINS[:-1], NPE_BINS[1:]):
                m = (true >= lo) & (true < hi)
                if m.sum() < 50:
                    continue
                r = (q[m] / c - true[m]) / true[m]
                bins.append({"npe_lo": lo, "npe_hi": hi if hi < 1e8 else None, "pixels": int(m.sum()),
                             "bias": float(np.mean(r)), "rel_rms": float(np.sqrt(np.mean(r * r)))})
            dark = true == 0
            per[name] = {"containment": c, "bins": bins, "signal_free_mean_pe": float(np.mean(q[dark])),
                         "signal_free_rms_pe": float(np.std(q[dark])), "signal_free_pixels": int(dark.sum())}
        out[ct.name] = per
        if log:
            log("resolution %s: %s" % (ct.name, json.dumps({k: (round(v["containment"], 3),
                                                              round(v["signal_free_mean_pe"], 3))
                                                          for k, v in per.items()})))
    return out


def throughput(pool_n, events, dev, steps=5, log=None, only=None):
    """Fused batch per extractor (only: names to run, default all): camera
    events / s, kernel time, the bytes each extractor must read (the fixed
    window reads w samples per pixel; the others the whole high-gain trace)
    and their rate."""
    import torch
    import dl0sim.workloads as W
    from paper_1307_6489_amd import autotune
    pool = W.c1_pool(pool_n, seed=1)
    idx, ty, off = W.stream_order(pool, events, seed=3)
    cams = [rta.Camera.from_type(c) for c in pool.cams]
    blob = torch.from_numpy(pool.blob).to(dev)
    ty_d, off_d = torch.from_numpy(ty).to(dev), torch.from_numpy(off).to(dev)
    stream = torch.cuda.Stream()
    res = {}
    for ex, name in NAMES.items():
        if only and name not in only:
            continue
        pipe = rta.Pipeline(cams, do_stereo=False, extractor=ex)
        b = pipe.make_batch(blob, ty_d, off_d)
        tel, _ = pipe.alloc_outputs(b, dev)
        nt = min(200_000, events)
        tb = pipe.make_batch(blob, ty_d[:nt], off_d[:nt])
        cands = [s for s in rta.list_schedules() if ex == rta.EXTRACT_SLIDING or s[2] == 0]
        best, _ = autotune.tune(pipe, tb, tel[:nt], stream=stream, candidates=cands, use_cache=False)
        with torch.cuda.stream(stream):
            g = pipe.capture(b, tel)
            g.launch(stream)
            stream.synchronize()
            a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(steps):
                g.launch(stream)
            z.record(stream)
            stream.synchronize()
        ms = a.elapsed_time(z) / steps
        if pipe.status():
            raise RuntimeError("device status word set")
        rec = rta.records(tel)
        w = pool.cams[0].window
        N = np.array([c.n_pix for c in pool.cams], np.int64)
        Tn = np.array([c.n_samp for c in pool.cams], np.int64)
        rows = np.full(len(pool.cams), w, np.int64) if ex == rta.EXTRACT_FIXED else Tn
        lg_rows = np.full(len(pool.cams), w, np.int64) if ex != rta.EXTRACT_SLIDING else Tn
        alg = int((N[ty] * rows[ty] * 2).sum() + (rec["n_lowgain"].astype(np.int64) * lg_rows[ty] * 2).sum()
                  + events * 76)
        res[name] = {"camera_events_per_s": events / (ms * 1e-3), "kernel_ms": ms, "schedule": list(best),
                     "alg_bytes": alg, "alg_GBps": alg / (ms * 1e-3) / 1e9,
                     "hbm_frac": alg / (ms * 1e-3) / 8e12}
        if log:
            log("throughput %s: %.2f M camera events/s, %.2f ms, schedule %s"
                % (name, events / (ms * 1e-3) / 1e6, ms, best))
        del g, b, tel, tb, pipe
    return res


def main():
    import torch
    import dl0sim
    ap = argparse.ArgumentParser(description="compare the signal extractors")
    ap.add_argument("--events", type=int, default=400, help="events per camera type for the resolution")
    ap.add_argument("--pool", type=int, default=3000)
    ap.add_argument("--stream", type=int, default=1_000_000)
    ap.add_argument("--only", default="", help="comma-separated extractor names for the throughput "
                    "(%s; default all); with --events 0 the resolution is skipped" % ",".join(NAMES.values()))
    args = ap.parse_args()
    only = [n for n in args.only.split(",") if n]
    for n in only:
        if n not in NAMES.values():
            ap.error("unknown extractor %r" % n)
    dev = torch.device("cuda:0")
    say = lambda s: print(s, flush=True)  # noqa: E731
    t0 = time.time()
    res = {"resolution": resolution(dl0sim.camera_types_c1(), args.events, dev, log=say) if args.events > 0 else {}}
    res["throughput"] = throughput(args.pool, args.stream, dev, log=say, only=only)
    res["seconds"] = time.time() - t0
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
