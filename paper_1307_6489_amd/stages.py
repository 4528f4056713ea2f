"""Unfused stages against the fused kernel: time and bytes per kernel.

The unfused calls (rta_calibrate, rta_clean, rta_hillas) hand per-pixel
intermediates through HBM; the fused batch keeps them in LDS.  This job
times both on one camera type, 2048 pixels x 128 samples, dual gain, 2000
events (200 generated images with a bright third, tiled ten times; 2.1 GB
of traces), and reports for each kernel its time and the bytes it must move:

  calibrate   reads the high-gain trace and the low-gain trace of switched
              pixels; writes S, D (int32), s*, peak, gain (uint8), q, t
              (float32): 19 bytes per pixel;
  clean       reads D and the gain, writes the mask: 6 bytes per pixel;
  hillas      reads D, gain, t and the mask (10 bytes per pixel), writes a
              64-byte record per event;
  fused       the trace reads of calibrate and the 64-byte record.

Run ``python -m paper_1307_6489_amd.stages``.
"""
from __future__ import annotations

import json

import numpy as np

import paper_1307_6489_amd as rta


def timed(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def run(n_evt=2000, reps=5, log=None):
    import torch
    import dl0sim
    dev = torch.device("cuda:0")
    ct = dl0sim.camera_types_c1()[2]
    sh = dl0sim.draw_ellipses(dl0sim.draw_cfg_plain(ct.n_samp), 41, 0, 200)
    sh["size"][::3, 0] *= 10.0
    base = dl0sim.render_traces(ct, sh, 41)
    tr = torch.from_numpy(np.ascontiguousarray(np.tile(base, (n_evt // 200, 1, 1, 1)))).to(dev)
    cam = rta.Camera.from_type(ct)
    N, T = ct.n_pix, ct.n_samp
    out = rta.calibrate(cam, tr)
    mask = rta.clean(cam, out["D"], out["gain"])
    n_sw = int(out["gain"].sum().item())
    trace_bytes = n_evt * N * T * 2 + n_sw * T * 2
    res = {"events": n_evt, "camera": "%dx%dx%d" % (N, T, ct.n_gain), "switched_pixels": n_sw}
    kernels = {
        "calibrate": (lambda: rta.calibrate(cam, tr), trace_bytes + n_evt * N * 19),
        "clean": (lambda: rta.clean(cam, out["D"], out["gain"]), n_evt * N * 6),
        "hillas": (lambda: rta.hillas(cam, out["q"], out["t"], mask, out["gain"]), n_evt * N * 10 + n_evt * 64),
    }
    pipe = rta.Pipeline([cam], do_stereo=False)
    ty = torch.zeros(n_evt, dtype=torch.int32, device=dev)
    off = torch.arange(n_evt, dtype=torch.int64, device=dev) * cam.event_elems
    b = pipe.make_batch(tr.reshape(-1), ty, off)
    tel, _ = pipe.alloc_outputs(b, dev)
    kernels["fused"] = (lambda: pipe.process(b, tel), trace_bytes + n_evt * (64 + 12))
    total_unfused = 0.0
    for name, (fn, nbytes) in kernels.items():
        ms = timed(fn, reps)
        res[name] = {"ms": ms, "bytes": nbytes, "GBps": nbytes / (ms * 1e-3) / 1e9,
                     "hbm_frac": nbytes / (ms * 1e-3) / 8e12}
        if name != "fused":
            total_unfused += ms
        if log:
            log("%s: %s" % (name, res[name]))
    res["unfused_total_ms"] = total_unfused
    res["fused_speedup"] = total_unfused / res["fused"]["ms"]
    return res


def main():
    say = lambda s: print(s, flush=True)  # noqa: E731
    print(json.dumps(run(log=say)), flush=True)


if __name__ == "__main__":
    main()
