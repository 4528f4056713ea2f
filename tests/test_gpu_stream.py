"""GPU tests of the page-locked host ingest (paper, Section 5: page-locked
host buffers feed the GPU; Section 2.2: the array's DL0 rate): every chunk
reconstructed by the copy / compute overlapped stream, and by the paced
array-event stream with stereo, gives records byte-identical to one
device-resident batch over the same events, and the per-array-event latencies
are ordered as their definitions require."""
import numpy as np
import pytest

import dl0sim.workloads as W
import oracle
import oracle.parity as par
import paper_1307_6489_amd as rta
from paper_1307_6489_amd import stream as st

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


def test_pinned_stream_chunks_equal_device_resident(torch_dev):
    import torch
    pool = W.c1_pool(300, seed=6)
    cams = [rta.Camera.from_type(c) for c in pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=False)
    pinned = st.PinnedPool(pool, 48 << 20)
    n = len(pinned.chunks)
    say("pinned stream: %d events in %d chunks of <= 48 MB, two passes" % (pool.n, n))
    assert n >= 4
    r = st.stream(pipe, pinned, 2 * n + 1, torch_dev, keep_records=True)
    assert pipe.status() == 0
    # the same events, resident in HBM in the pinned pool's order, as one batch
    blob = pinned.host.to(torch_dev)
    b = pipe.make_batch(blob, to_dev(pinned.types, torch_dev), to_dev(pinned.off.astype(np.int64), torch_dev))
    tel, _ = pipe.alloc_outputs(b, torch_dev)
    pipe.process(b, tel)
    torch.cuda.synchronize()
    ref = tel.cpu().view(torch.int32)
    for c, (s, e, o0, ne) in enumerate(pinned.chunks):
        assert torch.equal(r["records"][c].cpu().view(torch.int32), ref[s:e]), c
    # and a sample of the streamed records against the oracle
    g = rta.records(tel)
    host = pinned.host.numpy()
    ocs = [oracle.Camera.from_type(c) for c in pool.cams]
    for k in np.random.default_rng(1).choice(pool.n, 25, replace=False):
        t_, o_ = pinned.types[k], pinned.off[k]
        p, m, h = ocs[t_].reconstruct(host[o_:o_ + pool.cams[t_].event_elems])
        assert not par.hillas_mismatches(g[k], h, pool.cams[t_].geom.x, pool.cams[t_].geom.y, p["q"], p["t"], m), k


def test_paced_array_stream_equals_device_resident(torch_dev):
    import torch
    aw = W.array_events(60, seed=5, weights=(1.0, 1.0, 8.0))
    cams = [rta.Camera.from_type(c) for c in aw.pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=True)
    ps = st.PinnedArrayStream(aw, 8 << 20)
    n = len(ps.chunks)
    say("paced array stream: 60 array events, %d telescopes, %d chunks, 8 GB/s" % (len(aw.tel_type), n))
    r = st.paced_latency(pipe, ps, 8.0, n + 3, torch_dev, keep_records=True)
    assert pipe.status() == 0
    blob = ps.host.to(torch_dev)
    b = pipe.make_batch(blob, to_dev(aw.tel_type.astype(np.int32), torch_dev),
                        to_dev(ps.tel_elem_off.astype(np.int64), torch_dev),
                        to_dev(aw.evt_tel_off.astype(np.int64), torch_dev))
    tel, evt = pipe.alloc_outputs(b, torch_dev)
    pipe.process(b, tel, evt)
    torch.cuda.synchronize()
    tref, eref = tel.cpu().view(torch.int32), evt.cpu().view(torch.int32)
    for c, (t_lo, t_hi, e_lo, e_hi, o0, ne) in enumerate(ps.chunks):
        tc, ec = r["records"][c]
        assert torch.equal(tc.cpu().view(torch.int32), tref[t_lo:t_hi]), c
        assert torch.equal(ec.cpu().view(torch.int32), eref[e_lo:e_hi]), c
    ev = rta.records(evt, rta.EVENT_DTYPE)
    assert np.sum((ev["flags"] & rta.EVT_STEREO_INVALID) == 0) >= 40
    # latencies: every record is written after its chunk's copy completed, and
    # the arrival-based latency includes the device-based one (to within the
    # host / device clock alignment)
    say("latency:", {k: v for k, v in r.items() if k != "records"})
    assert r["array_events"] == sum(ps.chunks[i % n][3] - ps.chunks[i % n][2] for i in range(4, n + 7))
    assert r["latency_device_ms_min"] > 0
    assert r["arrival_minus_device_ms_min"] > -0.2
    assert abs(r["clock_rate_vs_nominal"] - 1.0) < 5e-3
