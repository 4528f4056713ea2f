"""The allocation-free batch call (rta_process_batch_noalloc) against
rta_process_batch on the same batches, through the C ABI: telescope and event
records bit-identical, and the call's own status word.  Two calls in a row,
the second on a smaller batch, in the grid and the persistent (work-queue)
forms of the fused kernel."""
import numpy as np
import pytest

import dl0sim.workloads as W
import paper_1307_6489_amd as rta

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


def both(pipe, blob, ty, off, eo, dev):
    """Records of rta_process_batch and of the allocation-free call on one
    batch, the pipeline's status and the call's status word."""
    import torch
    b = pipe.make_batch(blob, to_dev(ty, dev), to_dev(off, dev), to_dev(eo, dev))
    tel_a, evt_a = pipe.alloc_outputs(b, dev)
    tel_a.fill_(float("nan"))
    evt_a.fill_(float("nan"))
    pipe.process(b, tel_a, evt_a)
    st_a = pipe.status()
    tel_b, evt_b = pipe.alloc_outputs(b, dev)
    tel_b.fill_(float("nan"))
    evt_b.fill_(float("nan"))
    st_b = torch.full((1,), -1, dtype=torch.int32, device=dev)
    pipe.process_noalloc(b, tel_b, evt_b, st_b)
    torch.cuda.synchronize()
    return tel_a, evt_a, st_a, tel_b, evt_b, int(st_b.cpu()[0]) & 0xFFFFFFFF


@pytest.mark.parametrize("sched", [(8, 4, 0, 8), (8, 4, 3, 8)])
def test_noalloc_matches_process_batch(torch_dev, sched):
    import torch
    aw = W.array_events(30, seed=6)
    cams = [rta.Camera.from_type(c) for c in aw.pool.cams]
    pipe = rta.Pipeline(cams, do_stereo=True)
    pipe.set_schedule(*sched)
    blob = to_dev(aw.pool.blob, torch_dev)
    ty = aw.pool.pool_type[aw.tel_pool_idx].astype(np.int32)
    off = aw.pool.pool_off[aw.tel_pool_idx].astype(np.int64)
    eo = aw.evt_tel_off.astype(np.int64)

    say("noalloc call 1: 30 array events, %d telescopes, one type index -1, schedule %s" % (len(ty), sched))
    ty1 = ty.copy()
    ty1[2] = -1
    tel_a, evt_a, st_a, tel_b, evt_b, st_b = both(pipe, blob, ty1, off, eo, torch_dev)
    assert torch.equal(tel_a.view(torch.int32), tel_b.view(torch.int32))
    assert torch.equal(evt_a.view(torch.int32), evt_b.view(torch.int32))
    assert st_a == rta.STATUS_BAD_TYPE and st_b == rta.STATUS_BAD_TYPE
    g = rta.records(tel_b)
    assert g["flags"][2] & rta.FLAG_BAD_DESCRIPTOR
    assert not np.any(np.delete(g["flags"], 2) & rta.FLAG_BAD_DESCRIPTOR)
    assert pipe.status() == 0   # the allocation-free call leaves the pipeline's status word alone

    n_evt = 10
    n_tel = int(eo[n_evt])
    say("noalloc call 2: %d array events, %d telescopes, schedule %s" % (n_evt, n_tel, sched))
    tel_a, evt_a, st_a, tel_b, evt_b, st_b = both(pipe, blob, ty[:n_tel], off[:n_tel], eo[:n_evt + 1], torch_dev)
    assert tel_b.shape[0] == n_tel and evt_b.shape[0] == n_evt
    assert torch.equal(tel_a.view(torch.int32), tel_b.view(torch.int32))
    assert torch.equal(evt_a.view(torch.int32), evt_b.view(torch.int32))
    assert st_a == 0 and st_b == 0       # the scratch status word was cleared
    assert not np.any(rta.records(tel_b)["flags"] & rta.FLAG_BAD_DESCRIPTOR)
    e = rta.records(evt_b, rta.EVENT_DTYPE)
    assert np.sum((e["flags"] & rta.EVT_STEREO_INVALID) == 0) >= 5


def test_noalloc_rejects_bad_arguments(torch_dev):
    import torch
    aw = W.array_events(4, seed=6)
    pipe = rta.Pipeline([rta.Camera.from_type(c) for c in aw.pool.cams], do_stereo=True)
    blob = to_dev(aw.pool.blob, torch_dev)
    ty = aw.pool.pool_type[aw.tel_pool_idx].astype(np.int32)
    off = aw.pool.pool_off[aw.tel_pool_idx].astype(np.int64)
    b = pipe.make_batch(blob, to_dev(ty, torch_dev), to_dev(off, torch_dev),
                        to_dev(aw.evt_tel_off.astype(np.int64), torch_dev))
    tel, evt = pipe.alloc_outputs(b, torch_dev)
    with pytest.raises(rta.RTAError):
        pipe.process_noalloc(b, tel, None)          # stereo needs the event output
    with pytest.raises(rta.RTAError):
        pipe.process_noalloc(b, None, evt)
    torch.cuda.synchronize()
