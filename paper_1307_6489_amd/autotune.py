"""Schedule autotuner for the fused reconstruction kernel.

Times every launch schedule compiled into librta (pixels per lane, waves per
workgroup, persistent workgroups per compute unit, load-chunk depth) on a
caller-supplied batch and keeps the fastest.  Results are cached as JSON keyed
by the device architecture and the camera-type signature (pixels, samples,
gains of every type), so a pipeline over the same camera mix reuses them.
"""
from __future__ import annotations

import json
import os
import time

import paper_1307_6489_amd as rta

CACHE_PATH = os.environ.get("RTA_TUNE_CACHE",
                            os.path.join(os.path.expanduser("~"), ".cache", "rta_mi355x", "schedules.json"))


def cache_key(pipe) -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    sig = ";".join("%dx%dx%d" % (c.n_pix, c.n_samp, c.n_gain) for c in pipe.cams)
    return "%s|%s" % (arch, sig)


def load_cache(path=CACHE_PATH) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(entries: dict, path=CACHE_PATH) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_schedule(pipe, batch, tel_out, sched, stream, reps=3, warmup=1) -> float:
    """Median milliseconds of rta_process_batch under one schedule."""
    import torch
    pipe.set_schedule(*sched)
    for _ in range(warmup):
        pipe.process(batch, tel_out, stream=stream)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        pipe.process(batch, tel_out, stream=stream)
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune(pipe, batch, tel_out, stream=None, candidates=None, reps=3, log=None, use_cache=True, path=CACHE_PATH):
    """Pick the fastest schedule for this pipeline on ``batch`` and apply it.
    Returns (schedule tuple, {schedule: ms})."""
    import torch
    stream = stream or torch.cuda.current_stream()
    key = cache_key(pipe)
    if use_cache:
        hit = load_cache(path).get(key)
        if hit:
            pipe.set_schedule(*hit["schedule"])
            return tuple(hit["schedule"]), {}
    cands = candidates or rta.list_schedules()
    timings = {}
    t0 = time.time()
    for s in cands:
        timings[tuple(s)] = time_schedule(pipe, batch, tel_out, s, stream, reps=reps)
        if log:
            log("  schedule %s: %.3f ms" % (tuple(s), timings[tuple(s)]))
    best = min(timings, key=timings.get)
    pipe.set_schedule(*best)
    if log:
        log("autotune: %d schedules in %.1f s, best %s (%.3f ms)" % (len(cands), time.time() - t0, best,
                                                                      timings[best]))
    if use_cache:
        entries = load_cache(path)
        entries[key] = {"schedule": list(best), "ms": timings[best], "n_tel": int(batch.n_tel),
                        "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
        save_cache(entries, path)
    return best, timings
