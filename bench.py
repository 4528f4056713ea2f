"""Throughput of the fused low-level reconstruction on one MI355X.

Workload (the mixed-camera throughput configuration): dual-gain uint16 traces
of 1855-px x 40-sample, 1764-px x 25-sample and 2048-px x 128-sample cameras
in ratio 1:3:6, plain ellipse images.  A seeded pool of unique camera events
(default 45000, about 32 GB: re-reads of a pool a few times the size of the
256 MB last-level cache still hit it measurably) is made resident in HBM; one step is one pass of calibration -> cleaning ->
Hillas over 1e6 camera events streamed through the pool in a seeded random
order, replayed from a captured HIP graph.  Inputs are resident before the
timed region starts.

Prints one JSON line: camera-events/s (whole job), with input GB/s (full DL0
bytes, both gains), the roofline of the fused kernel (algorithmic HBM bytes:
high-gain trace + low-gain trace of switched pixels + 64-byte record + 12-byte
descriptor per telescope) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

# HBM traffic of the fused kernel from two rocprofv3 --pmc passes (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch) on this workload, each scaled by what the
# counter reads for a plain copy of 2^30 bytes (FETCH_SIZE reads 2^19 KiB:
# factor 2.0; WRITE_SIZE reads 2^20 KiB: factor 1.0).  Valid only for the
# kernel sources, schedule and workload it was taken on; reported as null
# otherwise.
COUNTER_SOURCES = ("paper_1307_6489_amd/csrc/reco.hip", "paper_1307_6489_amd/csrc/rta_internal.h")
MEASURED_TRAFFIC = {
    "sources": "46e85a926f720464", "schedule": (8, 4, 0, 8), "pool_events": 45000, "events": 1_000_000,
    "fetch_kib": 180867876.8, "fetch_factor": 2.0, "write_kib": 62500.0, "write_factor": 1.0,
}


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for rel in COUNTER_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(schedule, pool_n, events):
    m = MEASURED_TRAFFIC
    if m is None or m["sources"] != sources_digest() or list(m["schedule"]) != list(schedule) \
            or m["pool_events"] != pool_n or m["events"] != events:
        return None
    return m["fetch_kib"] * 1024 * m["fetch_factor"] + m["write_kib"] * 1024 * m["write_factor"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pool, ty, off, target_s=10.0, single_s=3.0):
    """The oracle as it stands, on host cores, over a bounded sample of the
    same descriptor stream (time-bounded: chunks of events until about
    target_s seconds of wall time with all threads, then single_s seconds on
    one thread)."""
    import oracle
    ocs = [oracle.Camera.from_type(c) for c in pool.cams]
    threads = max(1, min(16, os.cpu_count() or 1))
    per = np.array([c.dl0_bytes for c in pool.cams], np.int64)

    def run(n_threads, budget, chunk):
        done, t_used, k, nbytes = 0, 0.0, 0, 0
        while t_used < budget and k < len(ty):
            sl = slice(k, min(k + chunk, len(ty)))
            t0 = time.perf_counter()
            oracle.reconstruct_batch(ocs, ty[sl], pool.blob, off[sl], n_threads=n_threads)
            t_used += time.perf_counter() - t0
            done += sl.stop - sl.start
            nbytes += int(per[ty[sl]].sum())
            k = sl.stop
        return done, t_used, nbytes

    done, t_used, nbytes = run(threads, target_s, 1000)
    d1, t1, b1 = run(1, single_s, 50)
    return {"value": done / t_used, "unit": "camera-events/s", "cores": threads, "kind": "oracle",
            "sample": "first %d camera events of the same stream order (C++ FP64 oracle, %d threads, "
                      "%.1f s wall)" % (done, threads, t_used),
            "input_GBps": nbytes / t_used / 1e9,
            "single_thread": {"value": d1 / t1, "events": d1, "seconds": t1, "input_GBps": b1 / t1 / 1e9},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def cpu_baseline_c0(threads):
    """The oracle on the whole plain parity set: 1000 single-gain events of
    the 1855-pixel camera, 30 samples (seed 0), with all threads and with one."""
    import dl0sim
    import oracle
    ct = dl0sim.camera_c0()
    _, tr = dl0sim.plain_events(ct, 0, 1000)
    oc = oracle.Camera.from_type(ct)
    E = len(tr)
    ty = np.zeros(E, np.int32)
    off = np.arange(E, dtype=np.int64) * oc.event_elems
    res = {"events": E, "workload": "1855 px x 30 samples, single gain, 1000 events, seed 0"}
    for name, n_thr in (("threads", threads), ("single_thread", 1)):
        t0 = time.perf_counter()
        oracle.reconstruct_batch([oc], ty, tr.reshape(-1), off, n_threads=n_thr)
        dt = time.perf_counter() - t0
        res[name] = {"cores": n_thr, "camera_events_per_s": E / dt, "seconds": dt,
                     "input_GBps": E * ct.dl0_bytes / dt / 1e9}
    return res


def cpu_baseline_c2(arr, threads, n_evt=2000):
    """The oracle on the first ``n_evt`` array events of the batched job:
    Hillas per telescope (all threads) and stereo per array event."""
    import oracle
    aw, eo, ty, off = arr
    cams = aw.pool.cams
    ocs = [oracle.Camera.from_type(c) for c in cams]
    n_tel = int(eo[n_evt])
    focal = np.array([c.focal_m for c in cams])
    t0 = time.perf_counter()
    rec = oracle.reconstruct_batch(ocs, ty[:n_tel], aw.pool.blob, off[:n_tel], n_threads=threads)
    t1 = time.perf_counter()
    for e in range(n_evt):
        r = rec[eo[e]:eo[e + 1]]
        valid = ((r["flags"] & 1) == 0).astype(np.int32)
        oracle.stereo(r["size"], r["cog_x"], r["cog_y"], r["length"], r["width"], r["psi"], valid,
                      focal[ty[eo[e]:eo[e + 1]]])
    t2 = time.perf_counter()
    dl0 = np.array([c.dl0_bytes for c in cams], np.int64)
    return {"array_events": n_evt, "telescopes": n_tel, "cores": threads, "seconds": t2 - t0,
            "stereo_seconds": t2 - t1, "array_events_per_s": n_evt / (t2 - t0),
            "camera_events_per_s": n_tel / (t2 - t0), "input_GBps": float(dl0[ty[:n_tel]].sum()) / (t2 - t0) / 1e9,
            "workload": "first %d array events of the batched job (multiplicity 2..40, 1:3:6 types)" % n_evt}


def train_network(dev):
    """A gamma/hadron + energy network for the runs with classification:
    2 epochs on 30k generated images of the 1855-pixel camera (seed 3)."""
    import dl0sim
    from paper_1307_6489_amd import learn
    tr = learn.image_features(dl0sim.camera_c0(), 30_000, 3, dev)
    net, bc, info = learn.train(tr, dev, epochs=2, batch=1024, lr=2e-3)
    return net, bc


def latency_run(args, dev, network):
    """Array events with the 2048 x 128 dual-gain type dominating (1:1:8),
    stereo and the gamma/hadron network attached, fed from page-locked host
    memory at a paced rate, cycling through a rendered pool of array events
    until at least --latency-events array events are timed; per-array-event
    latency from device clocks (record write minus the chunk's copy
    completion, and minus the chunk's arrival on the host clock)."""
    import dl0sim.workloads as W
    import paper_1307_6489_amd as rta
    from paper_1307_6489_amd import stream as st
    t0 = time.time()
    net, bc = network
    aw = W.array_events(args.latency_pool, seed=5, weights=(1.0, 1.0, 8.0))
    ps = st.PinnedArrayStream(aw, 8 << 20)
    cams = [rta.Camera.from_type(c) for c in aw.pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=True)
    pipe.set_schedule(*args.latency_schedule)
    pipe.attach_mlp(net, bc)
    warmup = 4
    per = np.array([c[3] - c[2] for c in ps.chunks], np.int64)
    n_chunks, got = 0, 0
    while got < args.latency_events:
        got += int(per[(warmup + n_chunks) % len(per)])
        n_chunks += 1
    r = st.paced_latency(pipe, ps, args.rate, n_chunks, dev, warmup=warmup, classify_after_hillas=True)
    if pipe.status():
        raise RuntimeError("device status word %#x in the latency run" % pipe.status())
    r["pool_array_events"] = args.latency_pool
    r["pool_telescopes"] = int(len(aw.tel_type))
    r["mix"] = ("1855x40 : 1764x25 : 2048x128 = 1:1:8, multiplicity 2..40, network + box-cut fallback "
                "classifying each telescope in the reconstruction kernel after Hillas")
    log("latency run: %s (%.1f s)" % (r, time.time() - t0))
    return r


def array_batch_run(args, dev, stream, network):
    """Batched array events: ragged array events of multiplicity 2..40 over
    the three camera types (1:3:6), replicated from a device-resident pool of
    rendered array events, through one graph-replayed rta_process_batch with
    stereo per array event; schedule from the autotuner on a telescope prefix."""
    import torch
    import dl0sim.workloads as W
    import paper_1307_6489_amd as rta
    from paper_1307_6489_amd import autotune
    t0 = time.time()
    aw = W.array_events(args.array_pool, seed=2)
    eo, ty, off, _ = W.replicate_array_events(aw, args.array_events, seed=9)
    log("array pool: %d array events, %d telescopes, %.2f GB, generated in %.1f s"
        % (args.array_pool, len(aw.tel_type), aw.pool.blob.nbytes / 1e9, time.time() - t0))
    cams = [rta.Camera.from_type(c) for c in aw.pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=True)
    blob_d = torch.from_numpy(aw.pool.blob).to(dev)
    ty_d, off_d, eo_d = (torch.from_numpy(v).to(dev) for v in (ty, off, eo))
    b = pipe.make_batch(blob_d, ty_d, off_d, eo_d)
    tel, evt = pipe.alloc_outputs(b, dev)
    nt = min(args.tune_events, len(ty))
    tb = pipe.make_batch(blob_d, ty_d[:nt], off_d[:nt])
    best, timings = autotune.tune(pipe, tb, tel[:nt], stream=stream, use_cache=False)
    with torch.cuda.stream(stream):
        graph = pipe.capture(b, tel, evt)
        graph.launch(stream)
        stream.synchronize()
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t1 = time.perf_counter()
        a.record(stream)
        for _ in range(args.array_steps):
            graph.launch(stream)
        z.record(stream)
        stream.synchronize()
        wall = time.perf_counter() - t1
    status = pipe.status()
    if status:
        raise RuntimeError("device status word %#x" % status)
    ms = a.elapsed_time(z) / args.array_steps
    # the same job with the network attached: each telescope classified in the
    # reconstruction kernel right after Hillas (per-telescope scores to
    # tel_class), and, for comparison, in the per-event pass
    net_ms = evt_pass_ms = None
    if network is not None:
        pipe.attach_mlp(*network)
        cls = torch.empty((len(ty), 2), dtype=torch.float32, device=dev)
        bf = pipe.make_batch(blob_d, ty_d, off_d, eo_d, tel_class=cls)

        def timed_graph(batch):
            with torch.cuda.stream(stream):
                g2 = pipe.capture(batch, tel, evt)
                g2.launch(stream)
                stream.synchronize()
                a.record(stream)
                for _ in range(args.array_steps):
                    g2.launch(stream)
                z.record(stream)
                stream.synchronize()
            if pipe.status():
                raise RuntimeError("device status word %#x with the network" % pipe.status())
            return a.elapsed_time(z) / args.array_steps

        net_ms = timed_graph(bf)
        evt_pass_ms = timed_graph(b)
        del bf, cls
    dl0 = np.array([c.dl0_bytes for c in aw.pool.cams], np.int64)
    ev = rta.records(evt, rta.EVENT_DTYPE)
    n_evt, n_tel = args.array_events, len(ty)
    r = {"array_events_per_s": n_evt / (wall / args.array_steps), "camera_events_per_s": n_tel / (wall / args.array_steps),
         "dl0_GBps": float(dl0[ty].sum()) / (wall / args.array_steps) / 1e9, "ms_per_step": wall / args.array_steps * 1e3,
         "gpu_ms_per_step": ms, "array_events": n_evt, "telescopes": n_tel, "mean_multiplicity": n_tel / n_evt,
         "stereo_valid_fraction": float(np.mean((ev["flags"] & rta.EVT_STEREO_INVALID) == 0)),
         "pool_array_events": args.array_pool, "pool_GB": aw.pool.blob.nbytes / 1e9,
         "schedule": list(best), "steps": args.array_steps, "graph": True}
    if net_ms is not None:
        r["with_network"] = {
            "classified_after_hillas": {"gpu_ms_per_step": net_ms, "array_events_per_s": n_evt / (net_ms * 1e-3),
                                        "classification_ms_per_step": net_ms - ms,
                                        "classification_ns_per_telescope": (net_ms - ms) * 1e6 / n_tel},
            "classified_in_event_pass": {"gpu_ms_per_step": evt_pass_ms,
                                         "classification_ms_per_step": evt_pass_ms - ms,
                                         "classification_ns_per_telescope": (evt_pass_ms - ms) * 1e6 / n_tel}}
    log("array batch: %s (%.1f s)" % (r, time.time() - t0))
    del graph, blob_d, b, tel, evt, tb
    torch.cuda.empty_cache()
    return r, (aw, eo, ty, off)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pool", type=int, default=45000,
                    help="unique camera events resident in HBM (32 GB: far beyond the 256 MB last-level cache)")
    ap.add_argument("--events", type=int, default=1_000_000, help="camera events per step")
    ap.add_argument("--schedule", type=str, default="",
                    help="pix_per_lane,waves_per_wg,wg_per_cu,chunk (default: autotune before timing)")
    ap.add_argument("--tune-events", type=int, default=200_000,
                    help="camera events of the stream prefix the autotuner times each schedule on")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-graph", action="store_true", help="eager launches instead of graph replay")
    ap.add_argument("--stream-pool", type=int, default=11000,
                    help="unique camera events of the page-locked host pool (~7.8 GB: two 4 GB chunks)")
    ap.add_argument("--stream-chunks", type=int, default=24,
                    help="also stream this many pinned-host chunks of 4 GB through the pipeline (0: skip); "
                         "reported as the PCIe-inclusive rate, never as value")
    ap.add_argument("--latency-events", type=int, default=5000,
                    help="array events timed (1:1:8 mix, network attached) paced from pinned host at --rate GB/s "
                         "for per-event latency (0: skip)")
    ap.add_argument("--latency-pool", type=int, default=400,
                    help="rendered array events of the page-locked pool the paced run cycles through")
    ap.add_argument("--rate", type=float, default=8.0, help="paced DL0 rate for the latency run, GB/s")
    ap.add_argument("--array-events", type=int, default=200_000,
                    help="array events per step of the batched array-event run with stereo (0: skip)")
    ap.add_argument("--array-pool", type=int, default=1000,
                    help="rendered array events resident in HBM for the batched run (~21k telescopes, ~15 GB)")
    ap.add_argument("--array-steps", type=int, default=3)
    ap.add_argument("--copy-probe", action="store_true",
                    help="after timing, run a plain 1 GiB elementwise copy kernel twice (reads and writes "
                         "exactly 2^30 bytes each) to calibrate HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import dl0sim.workloads as W
    import paper_1307_6489_amd as rta

    dev = torch.device("cuda:0")
    t0 = time.time()
    pool = W.c1_pool(args.pool, seed=1)
    idx, ty, off = W.stream_order(pool, args.events, seed=3)
    log("pool: %d events, %.2f GB, generated in %.1f s" % (pool.n, pool.blob.nbytes / 1e9, time.time() - t0))

    cams = [rta.Camera.from_type(c) for c in pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=False)
    blob_d = torch.from_numpy(pool.blob).to(dev)
    ty_d = torch.from_numpy(ty).to(dev)
    off_d = torch.from_numpy(off).to(dev)
    b = pipe.make_batch(blob_d, ty_d, off_d)
    tel, _ = pipe.alloc_outputs(b, dev)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    tune_info = None
    if args.schedule:
        pipe.set_schedule(*[int(v) for v in args.schedule.split(",")])
    else:
        from paper_1307_6489_amd import autotune
        nt = min(args.tune_events, args.events)
        tb = pipe.make_batch(blob_d, ty_d[:nt], off_d[:nt])
        best, timings = autotune.tune(pipe, tb, tel[:nt], stream=stream, use_cache=False, log=log)
        ranked = sorted(timings.items(), key=lambda kv: kv[1])
        tune_info = {"candidates": len(timings), "tune_events": nt, "best": list(best),
                     "best_ms": ranked[0][1], "median_ms": ranked[len(ranked) // 2][1], "worst_ms": ranked[-1][1],
                     "top3": [[list(k), round(v, 4)] for k, v in ranked[:3]]}

    with torch.cuda.stream(stream):
        graph = None if args.no_graph else pipe.capture(b, tel)

        def step():
            if graph is not None:
                graph.launch(stream)
            else:
                pipe.process(b, tel, stream=stream)

        for _ in range(args.warmup):
            step()
        stream.synchronize()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        t0 = time.perf_counter()
        for s in range(args.steps):
            ev[s][0].record(stream)
            step()
            ev[s][1].record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    status = pipe.status()
    if status:
        raise RuntimeError("device status word %#x" % status)

    wall = t1 - t0
    ms_step = wall / args.steps * 1e3
    kern_ms = float(np.mean([a.elapsed_time(bb) for a, bb in ev]))
    n = args.events
    rec = rta.records(tel)
    per_hg = np.array([c.n_pix * c.n_samp * 2 for c in pool.cams], np.int64)
    samp = np.array([c.n_samp for c in pool.cams], np.int64)
    dl0 = np.array([c.dl0_bytes for c in pool.cams], np.int64)
    alg_bytes = int(per_hg[ty].sum() + (rec["n_lowgain"].astype(np.int64) * samp[ty] * 2).sum() + n * (64 + 12))
    dl0_bytes = int(dl0[ty].sum())
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    sched = list(pipe.schedule())
    traffic = measured_traffic(sched, pool.n, n)
    out = {
        "metric": "camera-events/s & input GB/s (calib+clean+Hillas), % of HBM peak",
        "value": n / (ms_step * 1e-3),
        "unit": "camera-events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16/i32/f32",
        "data": "synthetic",
        "input_GBps": dl0_bytes / (ms_step * 1e-3) / 1e9,
        "hbm_frac_algorithmic": achieved / HBM_PEAK_GBPS,
        "config": {
            "workload": "dual-gain camera events, 1855x40 : 1764x25 : 2048x128 = 1:3:6, "
                        "%d per step through a device-resident pool of %d unique events (%.2f GB), "
                        "fused calibrate->clean->Hillas, graph replay" % (n, pool.n, pool.blob.nbytes / 1e9),
            "camera_events_per_step": n,
            "pool_events": pool.n,
            "schedule": sched,
            "autotune": tune_info,
            "graph": graph is not None,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_fused_grid" if sched[2] == 0 else "k_fused",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "traffic_unit": "bytes per launch",
            "alg_bytes_per_launch": alg_bytes,
            "sources": sources_digest(),
            "kernel_ms": kern_ms,
        },
    }
    # free the throughput pool before the optional runs
    del graph, blob_d, b, tel
    torch.cuda.empty_cache()
    if args.stream_chunks > 0:
        from paper_1307_6489_amd import stream as st
        t0 = time.time()
        hpool = W.c1_pool(args.stream_pool, seed=6)
        pinned = st.PinnedPool(hpool, 4 << 30)
        del hpool
        r = st.stream(pipe, pinned, args.stream_chunks, dev)
        r.update(st.copy_bandwidth(1 << 30, dev))
        r["pinned_pool_GB"] = pinned.host.numel() * 2 / 1e9
        out["pinned_stream"] = r
        log("pinned stream: %s (%.1f s)" % (r, time.time() - t0))
        del pinned
    network = train_network(dev) if (args.array_events > 0 or args.latency_events > 0) else None
    arr = None
    if args.array_events > 0:
        out["array_batch"], arr = array_batch_run(args, dev, stream, network)
    if args.latency_events > 0:
        args.latency_schedule = pipe.schedule()
        out["array_latency"] = latency_run(args, dev, network)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu:
        cb = cpu_baseline(pool, ty, off)
        cb["c0_parity_set"] = cpu_baseline_c0(cb["cores"])
        if arr is not None:
            cb["c2_array_events"] = cpu_baseline_c2(arr, cb["cores"])
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
