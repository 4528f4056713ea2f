"""Pins of the oracle's DL0 packet framing / decode and of its CRC: the
published check value of this CRC, the zero residue of a message followed by
its CRC, detection of every single-bit error and every burst up to 16 bits,
a hand-assembled packet, the generator's serialisation read back exactly,
and the classification of corrupted packets.  CPU only."""
import struct

import numpy as np
import pytest

import dl0sim.workloads as W
from dl0sim import packets as gp
from oracle import packets as op


def test_crc_check_value():
    """CRC-16 with polynomial 0x1021, register 0xFFFF, MSB first, no final
    xor: the catalogue check value over the ASCII digits 1..9 is 0x29B1."""
    assert op.crc16(b"123456789") == 0x29B1
    assert op.crc16(b"") == 0xFFFF


def test_crc_residue_and_agreement_with_the_generator():
    rng = np.random.default_rng(0)
    for n in (1, 2, 7, 64, 1001):
        m = rng.integers(0, 256, n, dtype=np.uint8).tobytes()
        c = op.crc16(m)
        assert op.crc16(m + bytes([c >> 8, c & 0xFF])) == 0
        assert gp.crc16(m) == c          # the generator's own (table-driven) routine


def test_crc_detects_single_bits_and_short_bursts():
    rng = np.random.default_rng(1)
    m = bytearray(rng.integers(0, 256, 40, dtype=np.uint8).tobytes())
    c0 = op.crc16(m)
    for bit in range(8 * len(m)):
        e = bytearray(m)
        e[bit // 8] ^= 0x80 >> (bit % 8)
        assert op.crc16(e) != c0
    for start in range(0, 8 * len(m) - 16, 5):
        for length in (2, 9, 16):
            burst = (1 << (length - 1)) | 1 | int(rng.integers(0, 1 << max(length - 2, 1))) << 1
            burst &= (1 << length) - 1
            e = int.from_bytes(m, "big") ^ (burst << (8 * len(m) - start - length))
            assert op.crc16(e.to_bytes(len(m), "big")) != c0


def hand_packet(apid, seq, ty, coarse, fine, N, T, G, evno, samples, spare=0, version_bits=0b00001):
    body = b"".join(struct.pack(">H", int(v)) for v in np.asarray(samples).reshape(-1))
    total = 32 + len(body) + 2
    hdr = struct.pack(">HHIBBBBIHHHBBQ", (version_bits << 11) | apid, (3 << 14) | seq, total - 9, 0x10, 210, 1,
                      ty, coarse, fine, N, T, G, spare, evno)
    pkt = hdr + body
    c = op.crc16(pkt)
    return pkt + bytes([c >> 8, c & 0xFF])


def test_hand_assembled_packets():
    """Two packets of a 3-pixel, 2-sample, single-gain type and one of a
    9-pixel dual-gain type, assembled here with struct: framing finds them,
    decoding returns the samples little-endian in [G][T][Npad] with zero
    pads, and the header fields."""
    s1 = [[[1, 2, 0x0203], [65535, 0, 0x8001]]]
    s2 = [[[7, 8, 9], [10, 11, 12]]]
    s3 = np.arange(2 * 3 * 9).reshape(2, 3, 9) * 1000
    types = [(3, 2, 1), (9, 3, 2)]
    st = hand_packet(5, 1, 0, 100, 7, 3, 2, 1, 42, s1) + hand_packet(2047, 16383, 0, 101, 8, 3, 2, 1, 43, s2) \
        + hand_packet(0, 2, 1, 102, 9, 9, 3, 2, 2 ** 40, s3)
    off, ty, poff, n, used = op.frame(np.frombuffer(st, np.uint8), types)
    assert list(off) == [0, 46, 92] and list(ty) == [0, 0, 1] and list(poff) == [0, 16, 32] and used == len(st)
    assert n == 16 + 16 + 2 * 3 * 16
    pool, recs, oty = op.decode(np.frombuffer(st, np.uint8), off, ty, poff, n, types)
    assert list(recs["flags"]) == [0, 0, 0] and list(oty) == [0, 0, 1]
    assert list(pool[0:16]) == [1, 2, 0x0203, 0, 0, 0, 0, 0, 65535, 0, 0x8001, 0, 0, 0, 0, 0]
    assert list(pool[16:19]) == [7, 8, 9] and list(pool[24:27]) == [10, 11, 12]
    ev = pool[32:].reshape(2, 3, 16)
    assert np.array_equal(ev[:, :, :9], s3) and not ev[:, :, 9:].any()
    assert list(recs["apid"]) == [5, 2047, 0] and list(recs["seq_count"]) == [1, 16383, 2]
    assert list(recs["event_number"]) == [42, 43, 2 ** 40] and list(recs["coarse_time"]) == [100, 101, 102]
    assert list(recs["fine_time"]) == [7, 8, 9]


def test_generator_stream_reads_back_exactly():
    pool = W.c1_pool(24, seed=1)
    order = np.random.default_rng(3).permutation(pool.n)
    st, off = gp.serialize(pool, order, seed=2)
    types = [(c.n_pix, c.n_samp, c.n_gain) for c in pool.cams]
    o, t, po, n, used = op.frame(st, types)
    assert np.array_equal(o, off) and used == st.size and np.array_equal(t, pool.pool_type[order])
    dec, recs, ot = op.decode(st, o, t, po, n, types)
    assert not recs["flags"].any()
    for k, e in enumerate(order):
        m = pool.cams[t[k]].event_elems
        assert np.array_equal(dec[po[k]:po[k] + m], pool.blob[pool.pool_off[e]:pool.pool_off[e] + m])


def test_corrupted_packets_are_classified():
    pool = W.c1_pool(12, seed=1)
    st, off = gp.serialize(pool, np.arange(pool.n), seed=2)
    types = [(c.n_pix, c.n_samp, c.n_gain) for c in pool.cams]
    bad = st.copy()
    bad[off[1] + 40] ^= 0x10              # payload bit: CRC
    bad[off[2]] |= 0x80                   # version bits: header
    bad[off[3] + 9] = 7                   # service: header
    bad[off[4] + 11] = 9                  # unknown camera type: framing type -1
    bad[off[5] + 19] ^= 1                 # n_pix differs from the type's
    bad[off[6] + 23] = 1                  # spare byte: header
    bad[off[7] + (off[8] - off[7]) - 1] ^= 1   # the CRC field itself
    o, t, po, n, used = op.frame(bad, types)
    assert t[4] == -1 and t[5] == -1 and used == bad.size
    dec, recs, ot = op.decode(bad, o, t, po, n, types)
    f = recs["flags"]
    assert f[1] == op.CRC_BAD and f[7] == op.CRC_BAD
    assert f[2] & op.HEADER_BAD and f[3] & op.HEADER_BAD and f[6] & op.HEADER_BAD
    assert f[4] & op.TYPE_BAD and f[5] & op.TYPE_BAD
    assert f[0] == 0 and f[8] == 0 and all(ot[k] == -1 for k in range(1, 8))


def test_truncated_stream_frames_whole_packets_only():
    pool = W.c1_pool(6, seed=1)
    st, off = gp.serialize(pool, np.arange(pool.n), seed=2)
    types = [(c.n_pix, c.n_samp, c.n_gain) for c in pool.cams]
    cut = st[:off[4] + 100]
    o, t, po, n, used = op.frame(cut, types)
    assert len(o) == 4 and used == off[4]
    with pytest.raises(ValueError):
        garbage = st.copy()
        garbage[4:8] = 0                  # a data length below the smallest packet
        op.frame(garbage, types)
