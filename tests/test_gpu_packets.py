"""GPU parity of the DL0 packet decode (rta_decode_packets) against the
oracle: the decoded pool bit-exact, packet records and rejection flags
exact, rejected packets turned into bad descriptors of the fused batch, and
the reconstruction of a decoded stream identical to that of the original
pool."""
import numpy as np
import pytest

import dl0sim.workloads as W
import paper_1307_6489_amd as rta
from dl0sim import packets as gp
from oracle import packets as op

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rta.lib()
    return torch.device("cuda:0")


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def types_of(pool):
    return [(c.n_pix, c.n_samp, c.n_gain) for c in pool.cams]


def decode_both(pool, st, dev):
    """Frame on the host (C ABI), decode on the GPU and in the oracle."""
    import torch
    cams = [rta.Camera.from_type(c) for c in pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=False)
    o, t, po, n, used = rta.frame_packets(cams, st)
    t_dev = to_dev(t, dev)
    data, nb = rta.packet_buffer(st, dev)
    pool_d, rec = rta.decode_packets(pipe, data, to_dev(o, dev), t_dev, to_dev(po, dev), n, n_bytes=nb)
    torch.cuda.synchronize()
    ref_pool, ref_rec, ref_t = op.decode(st, o, t, po, n, types_of(pool))
    g_rec = rec.cpu().numpy().view(rta.PACKET_DTYPE).reshape(-1)
    return pipe, cams, (o, t, po, n), pool_d, t_dev, g_rec, ref_pool, ref_rec, ref_t


def compare(pool_d, t_dev, g_rec, ref_pool, ref_rec, ref_t, n):
    g_pool = pool_d.cpu().numpy()[:n]
    assert np.array_equal(t_dev.cpu().numpy(), ref_t)
    for f in ("event_number", "coarse_time", "fine_time", "apid", "seq_count", "cam_type", "flags"):
        assert np.array_equal(g_rec[f], ref_rec[f]), f
    good = ref_rec["flags"] == 0
    assert np.array_equal(g_rec["crc_computed"][good], ref_rec["crc_computed"][good])
    return g_pool


@pytest.mark.parametrize("n_pk", [60, 61])
def test_decode_mixed_stream(torch_dev, n_pk):
    """Both stream-length phases: 61 packets leave the stream 2 bytes past a
    4-byte boundary, so the last CRC field ends inside a dword (read through
    the padding after the stream)."""
    pool = W.c1_pool(n_pk, seed=1)
    order = np.random.default_rng(4).permutation(pool.n)
    st, off = gp.serialize(pool, order, seed=2)
    say("decode: %d packets of the 1:3:6 mix, %.1f MB, length mod 4 = %d" % (n_pk, st.size / 1e6, st.size % 4))
    pipe, cams, fr, pool_d, t_dev, g_rec, ref_pool, ref_rec, ref_t = decode_both(pool, st, torch_dev)
    g_pool = compare(pool_d, t_dev, g_rec, ref_pool, ref_rec, ref_t, fr[3])
    assert np.array_equal(g_pool, ref_pool)
    assert not ref_rec["flags"].any() and pipe.status() == 0
    # packet offsets take both 4-byte phases (packets are only 2-byte aligned)
    assert set((off % 4).tolist()) == {0, 2}


def test_decode_corrupted_stream(torch_dev):
    pool = W.c1_pool(30, seed=1)
    st, off = gp.serialize(pool, np.arange(pool.n), seed=2)
    bad = st.copy()
    rng = np.random.default_rng(9)
    for k in (1, 4, 9, 13):                       # single payload bits: CRC
        pos = off[k] + 32 + int(rng.integers(0, off[k + 1] - off[k] - 34))
        bad[pos] ^= 1 << int(rng.integers(0, 8))
    bad[off[2]] |= 0x80                           # version bits
    bad[off[6] + 10] = 2                          # subtype
    bad[off[11] + 11] = 3                         # camera type beyond the pipeline's
    bad[off[15] + 19] ^= 1                        # n_pix differs from the type's
    bad[off[17] + 23] = 5                         # spare byte
    bad[off[20] - 1] ^= 0x40                      # CRC field of packet 19
    say("decode: 30 packets with 10 corrupted")
    pipe, cams, fr, pool_d, t_dev, g_rec, ref_pool, ref_rec, ref_t = decode_both(pool, bad, torch_dev)
    g_pool = compare(pool_d, t_dev, g_rec, ref_pool, ref_rec, ref_t, fr[3])
    f = ref_rec["flags"]
    assert set(np.nonzero(f)[0].tolist()) == {1, 2, 4, 6, 9, 11, 13, 15, 17, 19}
    o, t, po, n = fr
    for k in range(len(o)):
        if f[k] == 0:
            m = pool.cams[t[k]].event_elems
            assert np.array_equal(g_pool[po[k]:po[k] + m], ref_pool[po[k]:po[k] + m])
    assert pipe.status() == rta.STATUS_BAD_PACKET


def test_decode_then_reconstruct_equals_direct(torch_dev):
    """Frame + decode + fused batch gives the records of the fused batch on
    the original pool, byte for byte; rejected packets come out as bad
    descriptors."""
    import torch
    pool = W.c1_pool(90, seed=1)
    order = np.random.default_rng(6).permutation(pool.n)
    st, off = gp.serialize(pool, order, seed=2)
    st[off[10] + 100] ^= 4
    say("decode + reconstruct: 90 packets, one corrupted")
    pipe, cams, fr, pool_d, t_dev, g_rec, ref_pool, ref_rec, ref_t = decode_both(pool, st, torch_dev)
    o, t, po, n = fr
    b = pipe.make_batch(pool_d, t_dev, to_dev(po, torch_dev))
    tel, _ = pipe.alloc_outputs(b, torch_dev)
    pipe.process(b, tel)
    direct = rta.Pipeline(cams, do_stereo=False)
    b2 = direct.make_batch(to_dev(pool.blob, torch_dev), to_dev(pool.pool_type[order].astype(np.int32), torch_dev),
                           to_dev(pool.pool_off[order].astype(np.int64), torch_dev))
    tel2, _ = direct.alloc_outputs(b2, torch_dev)
    direct.process(b2, tel2)
    torch.cuda.synchronize()
    g, r = rta.records(tel), rta.records(tel2)
    for k in range(len(order)):
        if k == 10:
            assert g["flags"][k] & rta.FLAG_BAD_DESCRIPTOR
        else:
            assert g[k].tobytes() == r[k].tobytes()
    assert pipe.status() == rta.STATUS_BAD_PACKET | rta.STATUS_BAD_TYPE


def test_decode_large_stream_sampled(torch_dev):
    """4000 packets (about 2.8 GB of stream) decoded in one launch; 40
    sampled packets against the oracle, every record's CRC verified."""
    import torch
    pool = W.c1_pool(4000, seed=1)
    order = np.random.default_rng(7).permutation(pool.n)
    st, off = gp.serialize(pool, order, seed=2)
    say("decode: 4000 packets, %.2f GB" % (st.size / 1e9))
    cams = [rta.Camera.from_type(c) for c in pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=False)
    o, t, po, n, used = rta.frame_packets(cams, st)
    t_dev = to_dev(t, torch_dev)
    data, nb = rta.packet_buffer(st, torch_dev)
    pool_d, rec = rta.decode_packets(pipe, data, to_dev(o, torch_dev), t_dev, to_dev(po, torch_dev), n, n_bytes=nb)
    torch.cuda.synchronize()
    g_rec = rec.cpu().numpy().view(rta.PACKET_DTYPE).reshape(-1)
    assert not g_rec["flags"].any() and pipe.status() == 0
    rng = np.random.default_rng(8)
    for k in rng.choice(len(o), 40, replace=False):
        m = pool.cams[t[k]].event_elems
        e = order[k]
        got = pool_d[int(po[k]):int(po[k]) + m].cpu().numpy()
        assert np.array_equal(got, pool.blob[pool.pool_off[e]:pool.pool_off[e] + m])
        b = bytes(st[o[k]:o[k] + 32 + 2 * pool.cams[t[k]].n_gain * pool.cams[t[k]].n_samp * pool.cams[t[k]].n_pix])
        assert g_rec["crc_computed"][k] == op.crc16(b)


def test_offsets_outside_the_stream_are_flagged(torch_dev):
    """Packet offsets before the stream, past its end and too close to its
    end for a header read nothing and come back as bad headers (type -1);
    the other packets decode as the oracle says."""
    import torch
    pool = W.c1_pool(12, seed=1)
    st, off = gp.serialize(pool, np.arange(pool.n), seed=2)
    cams = [rta.Camera.from_type(c) for c in pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=False)
    o, t, po, n, used = rta.frame_packets(cams, st)
    ref_pool, ref_rec, ref_t = op.decode(st, o, t, po, n, types_of(pool))
    o2 = o.copy()
    o2[2] = -16
    o2[5] = st.size + 4096
    o2[7] = st.size - 20
    say("decode: 12 packets, 3 offsets outside the stream")
    t_dev = to_dev(t, torch_dev)
    data, nb = rta.packet_buffer(st, torch_dev)
    pool_d, rec = rta.decode_packets(pipe, data, to_dev(o2, torch_dev), t_dev, to_dev(po, torch_dev), n, n_bytes=nb)
    torch.cuda.synchronize()
    g_rec = rec.cpu().numpy().view(rta.PACKET_DTYPE).reshape(-1)
    g_t = t_dev.cpu().numpy()
    g_pool = pool_d.cpu().numpy()
    for k in range(len(o)):
        if k in (2, 5, 7):
            assert g_rec["flags"][k] & rta.PKT_HEADER_BAD and g_t[k] == -1, k
        else:
            assert g_rec["flags"][k] == 0 and g_t[k] == ref_t[k], k
            m = pool.cams[t[k]].event_elems
            assert np.array_equal(g_pool[po[k]:po[k] + m], ref_pool[po[k]:po[k] + m])
    assert pipe.status() == rta.STATUS_BAD_PACKET
