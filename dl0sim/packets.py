"""DL0 telemetry packet stream (input generator side).

Serialises camera events of a pool into the project's packet format (one
packet per camera event, big-endian fields, CRC-16 trailer; the layout is
documented in dl0sim.c) back to back in one byte stream, the way the event
builder would send them.  Holds no reconstruction arithmetic.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _p, lib

HEADER_BYTES = 32
TRAILER_BYTES = 2


def packet_bytes(cam) -> int:
    return HEADER_BYTES + 2 * cam.n_gain * cam.n_samp * cam.n_pix + TRAILER_BYTES


def serialize(pool, order, seed=0, first_event=0, n_telescopes=100):
    """Packets of pool events ``order`` (indices into the pool), in that
    order.  APIDs (telescope ids), times and event numbers are seeded.
    Returns (stream uint8, packet byte offsets int64)."""
    order = np.asarray(order, np.int64)
    n = len(order)
    rng = np.random.default_rng(seed)
    types = pool.pool_type[order].astype(np.int64)
    size = np.array([packet_bytes(c) for c in pool.cams], np.int64)[types]
    off = np.zeros(n, np.int64)
    if n:
        off[1:] = np.cumsum(size)[:-1]
    meta = np.zeros((n, 8), np.int64)
    meta[:, 0] = types
    meta[:, 1] = [pool.cams[t].n_pix for t in types]
    meta[:, 2] = [pool.cams[t].n_samp for t in types]
    meta[:, 3] = [pool.cams[t].n_gain for t in types]
    meta[:, 4] = [pool.cams[t].n_pix_pad for t in types]
    meta[:, 5] = pool.pool_off[order]
    meta[:, 6] = rng.integers(0, n_telescopes, size=n)
    meta[:, 7] = np.arange(n) & 0x3FFF
    evno = (first_event + np.arange(n)).astype(np.uint64)
    coarse = (1_700_000_000 + np.arange(n) // 1000).astype(np.uint32)
    fine = rng.integers(0, 65536, size=n).astype(np.uint16)
    out = np.zeros(int(size.sum()), np.uint8)
    L = lib()
    L.dl0sim_serialize_packets(ctypes.c_int64(n), _p(meta), _p(evno), _p(coarse), _p(fine),
                               _p(np.ascontiguousarray(pool.blob)), _p(off), _p(out))
    return out, off


def crc16(data) -> int:
    b = np.ascontiguousarray(np.frombuffer(bytes(data), np.uint8) if isinstance(data, (bytes, bytearray))
                             else np.asarray(data, np.uint8))
    return int(lib().dl0sim_crc16(_p(b), ctypes.c_int64(b.size)))
