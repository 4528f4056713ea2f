"""Pinned-host ingest: stream DL0 chunks to the GPU and reconstruct them.

The real-time analysis receives the DL0 stream from the Central Event Builder
and must sustain the array's data rate (the paper quotes 0.5-8 GB/s and
measures host<->GPU copies of page-locked buffers, Section 5).  Here camera
events sit in a page-locked host pool; chunks of whole events are copied to
one of two HBM buffers on a copy stream while the fused kernel reconstructs
the previous chunk on the compute stream (HIP events order the two).  The
figures are end-to-end and PCIe-bound; the HBM roofline of the kernel is
measured separately with a device-resident pool.
"""
from __future__ import annotations

import time

import numpy as np

import paper_1307_6489_amd as rta


class PinnedPool:
    """A page-locked copy of a generator pool with events in a seeded random
    order, cut into chunks of whole events of at most ``chunk_bytes``."""

    def __init__(self, pool, chunk_bytes, seed=5):
        import torch
        rng = np.random.default_rng(seed)
        order = rng.permutation(pool.n)
        elems = np.array([pool.cams[t].event_elems for t in pool.pool_type[order]], np.int64)
        off = np.zeros(len(order), np.int64)
        off[1:] = np.cumsum(elems)[:-1]
        self.host = torch.empty(int(elems.sum()), dtype=torch.uint16, pin_memory=True)
        h = self.host.numpy()
        for k, e in enumerate(order):
            o = int(pool.pool_off[e])
            h[off[k]:off[k] + elems[k]] = pool.blob[o:o + elems[k]]
        self.types = pool.pool_type[order].astype(np.int32)
        self.dl0 = np.array([pool.cams[t].dl0_bytes for t in self.types], np.int64)
        # chunk boundaries: whole events, at most chunk_bytes each
        limit = chunk_bytes // 2
        self.chunks = []
        start = 0
        while start < len(order):
            end = start
            while end < len(order) and off[end] + elems[end] - off[start] <= limit:
                end += 1
            if end == start:
                raise ValueError("chunk smaller than one event")
            self.chunks.append((start, end, int(off[start]), int(off[end - 1] + elems[end - 1] - off[start])))
            start = end
        self.off = off
        self.max_chunk_elems = max(c[3] for c in self.chunks)


def stream(pipe, pinned: PinnedPool, n_chunks, dev, warmup=2, keep_records=False):
    """Reconstruct ``n_chunks`` chunks (cycling through the pinned pool) with
    copy / compute overlap.  Returns throughput figures; with keep_records,
    also "records": per chunk of the pool, the [n][16] float32 device records
    of its last pass."""
    import torch
    copy_s, comp_s = torch.cuda.Stream(), torch.cuda.Stream()
    bufs = [torch.empty(pinned.max_chunk_elems, dtype=torch.uint16, device=dev) for _ in range(2)]
    batches, outs = [], []
    for (s, e, o0, ne) in pinned.chunks:
        ty = torch.from_numpy(pinned.types[s:e].copy()).to(dev)
        off = torch.from_numpy((pinned.off[s:e] - o0).astype(np.int64)).to(dev)
        batches.append((ty, off))
        outs.append(torch.empty((e - s, 16), dtype=torch.float32, device=dev))
    copied = [torch.cuda.Event() for _ in range(2)]
    freed = [torch.cuda.Event() for _ in range(2)]
    for ev in freed:
        ev.record(comp_s)
    torch.cuda.synchronize()

    def run(count, first):
        n_ev = 0
        nbytes = 0
        for i in range(first, first + count):
            c = i % len(pinned.chunks)
            s, e, o0, ne = pinned.chunks[c]
            b = i % 2
            copy_s.wait_event(freed[b])
            with torch.cuda.stream(copy_s):
                bufs[b][:ne].copy_(pinned.host[o0:o0 + ne], non_blocking=True)
            copied[b].record(copy_s)
            comp_s.wait_event(copied[b])
            ty, off = batches[c]
            bt = pipe.make_batch(bufs[b], ty, off)
            pipe.process(bt, outs[c], stream=comp_s)
            freed[b].record(comp_s)
            n_ev += e - s
            nbytes += int(pinned.dl0[s:e].sum())
        return n_ev, nbytes

    run(warmup, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_ev, nbytes = run(n_chunks, warmup)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = {"camera_events_per_s": n_ev / dt, "dl0_GBps": nbytes / dt / 1e9,
           "h2d_payload_GBps": sum(pinned.chunks[(warmup + i) % len(pinned.chunks)][3] * 2
                                   for i in range(n_chunks)) / dt / 1e9,
           "chunks": n_chunks, "chunk_bytes_max": pinned.max_chunk_elems * 2, "seconds": dt}
    if keep_records:
        res["records"] = outs
    return res


def copy_bandwidth(nbytes, dev, reps=5):
    """Page-locked host -> device and device -> host copy rates (GB/s)."""
    import torch
    h = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    res = {}
    for name, fn in (("h2d_GBps", lambda: d.copy_(h, non_blocking=True)),
                     ("d2h_GBps", lambda: h.copy_(d, non_blocking=True))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        res[name] = nbytes * reps / (time.perf_counter() - t0) / 1e9
    return res


class PinnedArrayStream:
    """Page-locked array events cut into chunks of whole array events (at most
    ``chunk_bytes``), with per-chunk descriptors (offsets relative to the chunk)."""

    def __init__(self, aw, chunk_bytes):
        import torch
        pool = aw.pool
        n_tel = len(aw.tel_type)
        elems = np.array([pool.cams[t].event_elems for t in aw.tel_type], np.int64)
        off = np.zeros(n_tel, np.int64)
        off[1:] = np.cumsum(elems)[:-1]
        self.host = torch.empty(int(elems.sum()), dtype=torch.uint16, pin_memory=True)
        h = self.host.numpy()
        for k in range(n_tel):   # telescopes in event order
            o = int(aw.tel_off[k])
            h[off[k]:off[k] + elems[k]] = pool.blob[o:o + elems[k]]
        self.dl0 = np.array([pool.cams[t].dl0_bytes for t in aw.tel_type], np.int64)
        E = len(aw.evt_tel_off) - 1
        limit = chunk_bytes // 2
        self.chunks = []   # (tel_lo, tel_hi, evt_lo, evt_hi, elem_lo, n_elems)
        e0 = 0
        while e0 < E:
            e1 = e0
            t_lo = int(aw.evt_tel_off[e0])
            while e1 < E:
                t_hi = int(aw.evt_tel_off[e1 + 1])
                if off[t_hi - 1] + elems[t_hi - 1] - off[t_lo] > limit and e1 > e0:
                    break
                e1 += 1
            t_hi = int(aw.evt_tel_off[e1])
            self.chunks.append((t_lo, t_hi, e0, e1, int(off[t_lo]), int(off[t_hi - 1] + elems[t_hi - 1] - off[t_lo])))
            e0 = e1
        self.tel_type = aw.tel_type
        self.tel_elem_off = off
        self.evt_tel_off = aw.evt_tel_off
        self.max_chunk_elems = max(c[5] for c in self.chunks)


def clock_pair(stream=None):
    """One reading of the device clock against the host's perf_counter: the
    stamp is taken between two host readings; returns (host seconds at the
    midpoint, device ticks, half-width of the window in seconds)."""
    import torch
    slot = torch.zeros(1, dtype=torch.int64, device="cuda")
    best = None
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rta.device_stamp(slot, stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if best is None or t1 - t0 < best[2] * 2:
            best = (0.5 * (t0 + t1), int(slot.cpu()[0]), 0.5 * (t1 - t0))
    return best


def paced_latency(pipe, ps: PinnedArrayStream, rate_GBps, n_chunks, dev, warmup=4, keep_records=False,
                  classify_after_hillas=False):
    """Submit ``n_chunks`` chunks (cycling through the pinned array events) at
    the paced DL0 rate: a chunk arrives on the host clock when its last byte
    would have arrived at ``rate_GBps``, and is then copied on a copy stream
    and reconstructed (calibration to stereo and classification) on a
    compute stream.  Per array event, two latencies from device clocks:
    "device": its record write minus the completion of its chunk's
    host-to-device copy (both stamped on the device clock); "arrival": its
    record write, mapped to the host clock through clock readings taken
    before and after the run, minus the chunk's arrival (this includes any
    wait behind earlier copies).  p50 / p99 over every array event of the
    timed chunks.  keep_records: also the device records of each chunk's last
    pass ("records": [(tel, evt)] per chunk of the stream).
    classify_after_hillas: with a classifier attached, each telescope is
    classified in the reconstruction kernel (per-telescope scores to a
    tel_class buffer per chunk) rather than in the per-event pass."""
    import torch
    copy_s, comp_s = torch.cuda.Stream(), torch.cuda.Stream()
    nbuf = 3
    bufs = [torch.empty(ps.max_chunk_elems, dtype=torch.uint16, device=dev) for _ in range(nbuf)]
    descs = []
    for (t_lo, t_hi, e_lo, e_hi, o0, ne) in ps.chunks:
        ty = torch.from_numpy(ps.tel_type[t_lo:t_hi].copy()).to(dev)
        off = torch.from_numpy((ps.tel_elem_off[t_lo:t_hi] - o0).astype(np.int64)).to(dev)
        eo = torch.from_numpy((ps.evt_tel_off[e_lo:e_hi + 1] - t_lo).astype(np.int64)).to(dev)
        tel = torch.empty((t_hi - t_lo, 16), dtype=torch.float32, device=dev)
        evt = torch.empty((e_hi - e_lo, 8), dtype=torch.float32, device=dev)
        cls = torch.empty((t_hi - t_lo, 2), dtype=torch.float32, device=dev) if classify_after_hillas else None
        descs.append((ty, off, eo, tel, evt, cls))
    n_inst = n_chunks + warmup
    inst = [i % len(ps.chunks) for i in range(n_inst)]
    n_ev_inst = np.array([ps.chunks[c][3] - ps.chunks[c][2] for c in inst], np.int64)
    ev_base = np.zeros(n_inst + 1, np.int64)
    ev_base[1:] = np.cumsum(n_ev_inst)
    done_clock = torch.zeros(int(ev_base[-1]), dtype=torch.int64, device=dev)
    h2d_clock = torch.zeros(n_inst, dtype=torch.int64, device=dev)
    freed = [torch.cuda.Event() for _ in range(nbuf)]
    for ev in freed:
        ev.record(comp_s)
    torch.cuda.synchronize()
    copied = [torch.cuda.Event() for _ in range(n_inst)]
    sizes = [ps.chunks[c][5] * 2 for c in inst]
    hz = rta.device_clock_hz()
    sync0 = clock_pair()
    arrival = np.zeros(n_inst)
    t_start = time.perf_counter()
    due = t_start
    n_evt = n_tel = nbytes = 0
    for i in range(n_inst):
        c = inst[i]
        t_lo, t_hi, e_lo, e_hi, o0, ne = ps.chunks[c]
        due += sizes[i] / (rate_GBps * 1e9)
        while time.perf_counter() < due:
            pass
        arrival[i] = due
        b = i % nbuf
        copy_s.wait_event(freed[b])
        with torch.cuda.stream(copy_s):
            bufs[b][:ne].copy_(ps.host[o0:o0 + ne], non_blocking=True)
        rta.device_stamp(h2d_clock[i:i + 1], copy_s)
        copied[i].record(copy_s)
        comp_s.wait_event(copied[i])
        ty, off, eo, tel, evt, cls = descs[c]
        bt = pipe.make_batch(bufs[b], ty, off, eo, evt_done_clock=done_clock[ev_base[i]:ev_base[i + 1]],
                             tel_class=cls)
        pipe.process(bt, tel, evt, stream=comp_s)
        freed[b].record(comp_s)
        if i >= warmup:
            n_evt += e_hi - e_lo
            n_tel += t_hi - t_lo
            nbytes += int(ps.dl0[t_lo:t_hi].sum())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    sync1 = clock_pair()
    done = done_clock.cpu().numpy()
    h2d = h2d_clock.cpu().numpy()
    inst_of = np.repeat(np.arange(n_inst), n_ev_inst)
    timed = inst_of >= warmup
    lat_dev = (done - h2d[inst_of])[timed] / hz
    # device ticks -> host seconds: the rate measured between the two readings
    rate = (sync1[1] - sync0[1]) / (sync1[0] - sync0[0])
    host_done = sync0[0] + (done - sync0[1]) / rate
    lat_arr = (host_done - arrival[inst_of])[timed]
    first = ev_base[warmup]
    span = (done[first:].max() - h2d[warmup]) / hz
    res = {"array_events": int(timed.sum()), "array_events_per_s": n_evt / span, "camera_events_per_s": n_tel / span,
           "dl0_GBps": nbytes / span / 1e9, "paced_GBps": rate_GBps,
           "latency_device_ms_p50": float(np.percentile(lat_dev, 50) * 1e3),
           "latency_device_ms_p99": float(np.percentile(lat_dev, 99) * 1e3),
           "latency_device_ms_max": float(lat_dev.max() * 1e3),
           "latency_device_ms_min": float(lat_dev.min() * 1e3),
           "latency_arrival_ms_p50": float(np.percentile(lat_arr, 50) * 1e3),
           "latency_arrival_ms_p99": float(np.percentile(lat_arr, 99) * 1e3),
           "latency_arrival_ms_max": float(lat_arr.max() * 1e3),
           "arrival_minus_device_ms_min": float((lat_arr - lat_dev).min() * 1e3),
           "clock_sync_halfwidth_us": max(sync0[2], sync1[2]) * 1e6,
           "clock_rate_vs_nominal": rate / hz,
           "chunks": n_chunks, "chunk_bytes_mean": float(np.mean(sizes[warmup:])), "wall_s": wall}
    if keep_records:
        res["records"] = [(d[3], d[4]) for d in descs]
    return res
