"""Schedule autotuner for the fused reconstruction kernel.

A thin front over the library's native tuner: ``rta_pipeline_tune`` times
every launch schedule compiled into librta (pixels per lane, waves per
workgroup, persistent workgroups per compute unit, load-chunk depth) on a
caller-supplied batch with HIP events and applies the fastest; the tune cache
is the library's text file (``rta_tune_cache_lookup`` / ``_store``), keyed by
the device architecture, the extractor and window, and the camera-type
signature (pixels, samples, gains of every type).  A pipeline created with
``tune_cache=path`` reads that file itself.
"""
from __future__ import annotations

import os
import time

import paper_1307_6489_amd as rta

CACHE_PATH = os.environ.get("RTA_TUNE_CACHE",
                            os.path.join(os.path.expanduser("~"), ".cache", "rta_mi355x", "schedules.tsv"))


def tune(pipe, batch, tel_out, stream=None, candidates=None, reps=3, log=None, use_cache=True, path=CACHE_PATH,
         evt_out=None):
    """Pick the fastest schedule for this pipeline on ``batch`` and apply it.
    With use_cache, a cached entry for the pipeline's key is applied without
    timing, and a new result is stored.  Returns (schedule tuple,
    {schedule: median ms}) ({} on a cache hit)."""
    key = pipe.tune_key()
    if use_cache:
        hit = rta.tune_cache_lookup(path, key)
        if hit:
            pipe.set_schedule(*hit[0])
            return hit[0], {}
    t0 = time.time()
    best, timings = pipe.tune(batch, tel_out, evt_out=evt_out, candidates=candidates, reps=reps, stream=stream)
    if log:
        for s, ms in timings.items():
            log("  schedule %s: %.3f ms" % (s, ms))
        log("autotune: %d schedules in %.1f s, best %s (%.3f ms)" % (len(timings), time.time() - t0, best,
                                                                      timings[best]))
    if use_cache:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        rta.tune_cache_store(path, key, best, timings[best])
    return best, timings
