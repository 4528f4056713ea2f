"""Oracle of the DL0 telemetry packet decode — TEST INFRASTRUCTURE ONLY.

The paper's real-time analysis receives the camera data as a byte stream
formatted like space telemetry source packets (Section 5).  The project's
packet (one per camera event, every multi-byte field big-endian):

    0  u16  packet id: version 0 (3 bits), type 0 (1 bit), secondary header
            flag 1 (1 bit), APID = telescope id (11 bits)
    2  u16  sequence control: flags 0b11 (2 bits), sequence count (14 bits)
    4  u32  packet data length = total packet length - 9
    8  u8   0x10     9  u8  service 210     10  u8  subtype 1
   11  u8   camera type     12  u32  coarse time     16  u16  fine time
   18  u16  n_pix     20  u16  n_samp     22  u8  n_gain     23  u8  spare 0
   24  u64  event number
   32  u16  samples [G][T][N], no padding
  end  u16  CRC-16 (x^16+x^12+x^5+1, register 0xFFFF, MSB first) of every
            byte before it

Framing walks the headers: a packet of total length L = data length + 9
starts where the previous one ended; a packet whose camera type is known
and whose dimensions match that type gets a slot of G*T*Npad elements in
the decoded pool (slots in packet order, each a multiple of 8 elements),
any other packet gets type -1 and no slot.  Decoding checks the header
(version, type and flag bits, service 210/1, spare 0, length =
34 + 2*G*T*N), the type against the framing's and the camera's dimensions,
and the CRC; a packet failing any check keeps type -1.  A good packet's
samples become little-endian uint16 [G][T][Npad] with zero pad columns.

Plain loops and numpy; the CRC is the bitwise C routine oracle_crc16.  Shares
no code with the HIP library.

Parity status: pinned by the CRC's check value, residue and error detection,
a hand-assembled packet and the generator's stream (tests/test_oracle_packets.py,
tests/test_packets_host.py).
"""
from __future__ import annotations

import ctypes
import struct

import numpy as np

from . import _p, lib

HEADER_BAD = 0x1
TYPE_BAD = 0x2
CRC_BAD = 0x4

REC_DTYPE = np.dtype([("event_number", "<u8"), ("coarse_time", "<u4"), ("fine_time", "<u2"), ("apid", "<u2"),
                      ("seq_count", "<u2"), ("cam_type", "<u2"), ("flags", "<u4"), ("crc_stored", "<u2"),
                      ("crc_computed", "<u2"), ("pad_", "<u4")])


def crc16(data) -> int:
    b = np.ascontiguousarray(np.frombuffer(bytes(data), np.uint8) if isinstance(data, (bytes, bytearray))
                             else np.asarray(data, np.uint8))
    return int(lib().oracle_crc16(_p(b), ctypes.c_int64(b.size)))


def frame(stream, types):
    """types: list of (n_pix, n_samp, n_gain).  Returns (packet offsets,
    camera types, pool element offsets, pool elements, bytes consumed)."""
    buf = memoryview(np.ascontiguousarray(stream, np.uint8)).cast("B")
    n = len(buf)
    off, ptype, poff = [], [], []
    pos, pool = 0, 0
    while pos + 8 <= n:
        total = struct.unpack_from(">I", buf, pos + 4)[0] + 9
        if total < 34:
            raise ValueError("framing lost at byte %d" % pos)
        if pos + total > n:
            break
        ty = buf[pos + 11] if pos + 23 <= n else 255
        N, T, G = struct.unpack_from(">HHB", buf, pos + 18)
        ok = ty < len(types) and tuple(types[ty]) == (N, T, G)
        off.append(pos)
        if ok:
            ptype.append(ty)
            poff.append(pool)
            pool += G * T * ((N + 7) // 8 * 8)
        else:
            ptype.append(-1)
            poff.append(0)
        pos += total
    return (np.array(off, np.int64), np.array(ptype, np.int32), np.array(poff, np.int64), pool, pos)


def decode(stream, pkt_off, tel_type, tel_trace_off, pool_elems, types):
    """Decoded pool (uint16), per-packet records and output types."""
    buf = np.ascontiguousarray(stream, np.uint8)
    pool = np.zeros(pool_elems, np.uint16)
    recs = np.zeros(len(pkt_off), REC_DTYPE)
    out_type = np.asarray(tel_type, np.int32).copy()
    for k, po in enumerate(np.asarray(pkt_off, np.int64)):
        po = int(po)
        hdr = bytes(buf[po:po + 32])
        pid, seq, dlen, ver, svc, sub, ty, coarse, fine, N, T, G, spare, evno = struct.unpack(
            ">HHIBBBBIHHHBBQ", hdr)
        total = dlen + 9
        r = recs[k]
        r["event_number"], r["coarse_time"], r["fine_time"] = evno, coarse, fine
        r["apid"], r["seq_count"], r["cam_type"] = pid & 0x7FF, seq & 0x3FFF, ty
        flags = 0
        if (pid >> 11) != 0b00001 or (seq >> 14) != 3 or ver != 0x10 or svc != 210 or sub != 1 or spare != 0 \
                or total != 34 + 2 * G * T * N:
            flags |= HEADER_BAD
        if ty >= len(types) or tuple(types[ty]) != (N, T, G) or tel_type[k] != ty:
            flags |= TYPE_BAD
        if not flags:
            body = 2 * G * T * N
            stored = int(buf[po + 32 + body]) << 8 | int(buf[po + 33 + body])
            comp = crc16(buf[po:po + 32 + body])
            r["crc_stored"], r["crc_computed"] = stored, comp
            if stored != comp:
                flags |= CRC_BAD
            Np = (N + 7) // 8 * 8
            o = int(tel_trace_off[k])
            if o < 0 or o % 8 or o + G * T * Np > pool_elems:
                flags |= TYPE_BAD
            else:
                x = np.frombuffer(buf[po + 32:po + 32 + body].tobytes(), ">u2").reshape(G, T, N)
                ev = np.zeros((G, T, Np), np.uint16)
                ev[:, :, :N] = x
                pool[o:o + G * T * Np] = ev.reshape(-1)
        r["flags"] = flags
        if flags:
            out_type[k] = -1
    return pool, recs, out_type
