"""DL0 packet ingest measured: decode rate and end-to-end stream rate.

The analysis receives camera events as a telemetry-style packet stream
(Section 5 of the paper: simulated events converted into a byte stream
between the pipeline's processes).  Two measurements on the mixed dual-gain
workload (1855x40 : 1764x25 : 2048x128 = 1:3:6):

  decode      a device-resident packet stream decoded by rta_decode_packets
              (CRC check + big-endian to [G][T][Npad] relayout), HIP-event
              timed; bytes moved = stream read + pool written;
  end to end  page-locked host chunks of whole packets: host framing
              (rta_frame_packets), host-to-device copy on a copy stream,
              decode + fused calibrate -> clean -> Hillas on a compute
              stream, double buffered; camera events / s and stream GB/s.

Run ``python -m paper_1307_6489_amd.ingest --help``.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

import paper_1307_6489_amd as rta


def make_stream(pool_n, seed=1):
    import dl0sim.workloads as W
    from dl0sim import packets
    pool = W.c1_pool(pool_n, seed=seed)
    order = np.random.default_rng(seed + 10).permutation(pool.n)
    st, off = packets.serialize(pool, order, seed=seed + 20)
    return pool, order, st, off


def decode_rate(pool, st, dev, reps=5, log=None):
    import torch
    cams = [rta.Camera.from_type(c) for c in pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=False)
    t0 = time.perf_counter()
    o, t, po, n, used = rta.frame_packets(cams, st)
    frame_s = time.perf_counter() - t0
    data, nb = rta.packet_buffer(st, dev)
    o_d, po_d = torch.from_numpy(o).to(dev), torch.from_numpy(po).to(dev)
    t_src = torch.from_numpy(t).to(dev)
    t_d = t_src.clone()
    pool_d = torch.empty(n, dtype=torch.uint16, device=dev)
    stream = torch.cuda.Stream()

    def one():
        t_d.copy_(t_src)
        rta.decode_packets(pipe, data, o_d, t_d, po_d, n, pool=pool_d, stream=stream, want_rec=False, n_bytes=nb)

    with torch.cuda.stream(stream):
        one()
        stream.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            t_d.copy_(t_src)
            a.record(stream)
            rta.decode_packets(pipe, data, o_d, t_d, po_d, n, pool=pool_d, stream=stream, want_rec=False, n_bytes=nb)
            b.record(stream)
        stream.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    if pipe.status():
        raise RuntimeError("packets rejected")
    moved = st.size + 2 * n
    # reference: a plain device copy of the same number of bytes (read + write)
    src = torch.empty(st.size, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        dst.copy_(src)
        a0, b0 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        for _ in range(reps):
            dst.copy_(src)
        b0.record(stream)
        stream.synchronize()
    copy_ms = a0.elapsed_time(b0) / reps
    del src, dst
    r = {"packets": int(len(o)), "stream_GB": st.size / 1e9, "decode_ms": ms,
         "stream_GBps": st.size / (ms * 1e-3) / 1e9, "camera_events_per_s": len(o) / (ms * 1e-3),
         "bytes_moved_GBps": moved / (ms * 1e-3) / 1e9, "hbm_frac": moved / (ms * 1e-3) / 8e12,
         "host_framing_GBps": st.size / frame_s / 1e9,
         "device_copy_moved_GBps": 2 * st.size / (copy_ms * 1e-3) / 1e9}
    if log:
        log("decode: %s" % r)
    return r


def end_to_end(pool, st, dev, chunk_bytes=1 << 30, n_chunks=24, log=None):
    """Pinned host stream -> frame -> copy -> decode -> fused batch."""
    import torch
    cams = [rta.Camera.from_type(c) for c in pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=False)
    pipe.set_schedule(8, 4, 0, 8)
    host = torch.empty(st.size, dtype=torch.uint8, pin_memory=True)
    host.numpy()[:] = st
    # chunk boundaries at whole packets (found once; the framing itself is
    # repeated and timed per chunk below)
    o_all, _, _, _, _ = rta.frame_packets(cams, st)
    ends = np.append(o_all, st.size)
    chunks = []
    start = 0
    while start < len(o_all):
        stop = start
        while stop < len(o_all) and ends[stop + 1] - ends[start] <= chunk_bytes:
            stop += 1
        stop = max(stop, start + 1)
        chunks.append((int(ends[start]), int(ends[stop])))
        start = stop
    max_bytes = max(b - a for a, b in chunks)
    max_pk = max(int(np.searchsorted(o_all, b) - np.searchsorted(o_all, a)) for a, b in chunks)
    max_elems = max_bytes  # decoded slots never exceed the stream bytes (2 bytes per sample + padding < header)
    copy_s, comp_s = torch.cuda.Stream(), torch.cuda.Stream()
    bufs = [torch.zeros(max_bytes + rta.PACKET_PAD, dtype=torch.uint8, device=dev) for _ in range(2)]
    pools = [torch.empty(max_elems, dtype=torch.uint16, device=dev) for _ in range(2)]
    desc = [[torch.empty(max_pk, dtype=dt, device=dev) for dt in (torch.int64, torch.int32, torch.int64)]
            for _ in range(2)]
    tels = [torch.empty((max_pk, 16), dtype=torch.float32, device=dev) for _ in range(2)]
    hostdesc = [[torch.empty(max_pk, dtype=dt, pin_memory=True) for dt in (torch.int64, torch.int32, torch.int64)]
                for _ in range(2)]
    freed = [torch.cuda.Event() for _ in range(2)]
    for e in freed:
        e.record(comp_s)
    torch.cuda.synchronize()
    frame_s = 0.0
    n_ev = nbytes = 0
    t0 = time.perf_counter()
    for i in range(n_chunks):
        a, b = chunks[i % len(chunks)]
        k = i % 2
        tf = time.perf_counter()
        o, t, po, n, used = rta.frame_packets(cams, host.numpy()[a:b])
        frame_s += time.perf_counter() - tf
        m = len(o)
        freed[k].synchronize()   # the host descriptor buffers of k are free again
        for hd, v in zip(hostdesc[k], (o, t, po)):
            hd.numpy()[:m] = v
        copy_s.wait_event(freed[k])
        with torch.cuda.stream(copy_s):
            bufs[k][:b - a].copy_(host[a:b], non_blocking=True)
            for d, hd in zip(desc[k], hostdesc[k]):
                d[:m].copy_(hd[:m], non_blocking=True)
        copied = torch.cuda.Event()
        copied.record(copy_s)
        comp_s.wait_event(copied)
        rta.decode_packets(pipe, bufs[k], desc[k][0][:m], desc[k][1][:m], desc[k][2][:m], n,
                           pool=pools[k], stream=comp_s, want_rec=False, n_bytes=b - a)
        bt = pipe.make_batch(pools[k][:max(n, 8)], desc[k][1][:m], desc[k][2][:m])
        pipe.process(bt, tels[k][:m], stream=comp_s)
        freed[k].record(comp_s)
        n_ev += m
        nbytes += b - a
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if pipe.status():
        raise RuntimeError("status word set in the end-to-end run")
    r = {"chunks": n_chunks, "chunk_GB_max": max_bytes / 1e9, "camera_events_per_s": n_ev / wall,
         "stream_GBps": nbytes / wall / 1e9, "host_framing_s": frame_s, "wall_s": wall}
    if log:
        log("end to end: %s" % r)
    return r


def main():
    import torch
    ap = argparse.ArgumentParser(description="measure DL0 packet ingest")
    ap.add_argument("--pool", type=int, default=6000, help="camera events serialised (about 4.3 GB)")
    ap.add_argument("--chunks", type=int, default=24)
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    say = lambda s: print(s, flush=True)  # noqa: E731
    t0 = time.time()
    pool, order, st, off = make_stream(args.pool)
    say("stream: %d packets, %.2f GB, built in %.1f s" % (len(off), st.size / 1e9, time.time() - t0))
    res = {"decode": decode_rate(pool, st, dev, log=say)}
    res["end_to_end"] = end_to_end(pool, st, dev, n_chunks=args.chunks, log=say)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
