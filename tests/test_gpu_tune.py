"""Native schedule tuning through the C ABI: rta_pipeline_tune times the
candidates on a batch, applies the fastest and stores it in the pipeline's
tune cache; a pipeline created on a cache without an entry for its key
refuses to process (RTA_E_UNTUNED) until tuned or given a schedule, and one
created on a cache with an entry starts on the cached schedule.  Records are
the same under every schedule."""
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


def test_tune_cache_strict_and_stored(torch_dev, tmp_path):
    import torch
    aw = W.array_events(24, seed=11)
    cams = [rta.Camera.from_type(c) for c in aw.pool.cams]
    path = str(tmp_path / "sched.tsv")
    blob = to_dev(aw.pool.blob, torch_dev)
    ty = to_dev(aw.pool.pool_type[aw.tel_pool_idx].astype(np.int32), torch_dev)
    off = to_dev(aw.pool.pool_off[aw.tel_pool_idx].astype(np.int64), torch_dev)
    eo = to_dev(aw.evt_tel_off.astype(np.int64), torch_dev)

    pipe = rta.Pipeline(cams, do_stereo=True, tune_cache=path)
    key = pipe.tune_key()
    assert key.startswith("gfx") and key.count("|") == 2 and key.endswith(
        ";".join("%dx%dx%d" % (c.n_pix, c.n_samp, c.n_gain) for c in aw.pool.cams))
    b = pipe.make_batch(blob, ty, off, eo)
    tel, evt = pipe.alloc_outputs(b, torch_dev)
    say("untuned pipeline: process must refuse")
    with pytest.raises(rta.RTAError) as e:
        pipe.process(b, tel, evt)
    assert e.value.status == rta.RTA_E_UNTUNED
    with pytest.raises(rta.RTAError) as e:
        pipe.process_noalloc(b, tel, evt)
    assert e.value.status == rta.RTA_E_UNTUNED

    cands = [(8, 4, 0, 8), (4, 4, 0, 16), (8, 4, 2, 8), (2, 8, 1, 8)]
    say("tuning over %d schedules, %d telescopes" % (len(cands), b.n_tel))
    best, ms = pipe.tune(b, tel, evt, candidates=cands, reps=3)
    assert best in cands and set(ms) == set(cands)
    assert all(v > 0 and np.isfinite(v) for v in ms.values())
    assert ms[best] == min(ms.values())
    assert pipe.schedule() == best
    hit = rta.tune_cache_lookup(path, key)
    assert hit is not None and hit[0] == best and hit[1] == pytest.approx(ms[best], rel=1e-5)

    pipe.process(b, tel, evt)
    torch.cuda.synchronize()
    ref_tel, ref_evt = tel.clone(), evt.clone()
    assert pipe.status() == 0

    say("a second pipeline on the same cache starts on the stored schedule")
    pipe2 = rta.Pipeline(cams, do_stereo=True, tune_cache=path)
    assert pipe2.schedule() == best
    tel2, evt2 = pipe2.alloc_outputs(b, torch_dev)
    for s in cands:
        pipe2.set_schedule(*s)
        tel2.fill_(float("nan"))
        evt2.fill_(float("nan"))
        pipe2.process(b, tel2, evt2)
        torch.cuda.synchronize()
        assert torch.equal(tel2.view(torch.int32), ref_tel.view(torch.int32)), s
        assert torch.equal(evt2.view(torch.int32), ref_evt.view(torch.int32)), s

    say("a cache entry for another key leaves a third pipeline untuned until set_schedule")
    pipe3 = rta.Pipeline(cams, do_stereo=True, extractor=rta.EXTRACT_FIXED, tune_cache=path)
    assert pipe3.tune_key() != key
    with pytest.raises(rta.RTAError) as e:
        pipe3.process(b, tel2, evt2)
    assert e.value.status == rta.RTA_E_UNTUNED
    pipe3.set_schedule(8, 4, 0, 8)
    pipe3.process(b, tel2, evt2)
    torch.cuda.synchronize()


def test_tune_without_cache_and_bad_candidates(torch_dev):
    import torch
    aw = W.array_events(6, seed=12)
    pipe = rta.Pipeline([rta.Camera.from_type(c) for c in aw.pool.cams], do_stereo=False)
    blob = to_dev(aw.pool.blob, torch_dev)
    b = pipe.make_batch(blob, to_dev(aw.pool.pool_type[aw.tel_pool_idx].astype(np.int32), torch_dev),
                        to_dev(aw.pool.pool_off[aw.tel_pool_idx].astype(np.int64), torch_dev))
    tel, _ = pipe.alloc_outputs(b, torch_dev)
    say("tuning without a cache; an uncompiled candidate is rejected before any launch")
    with pytest.raises(rta.RTAError) as e:
        pipe.tune(b, tel, candidates=[(8, 4, 0, 8), (3, 4, 0, 8)])
    assert e.value.status == 5
    assert pipe.schedule() == (8, 4, 0, 8)
    with pytest.raises(rta.RTAError):
        pipe.tune(b, tel, candidates=[(8, 4, 0, 8)], reps=0)
    best, ms = pipe.tune(b, tel, candidates=[(8, 4, 0, 8), (8, 8, 0, 16)], reps=1)
    assert pipe.schedule() == best and len(ms) == 2
    torch.cuda.synchronize()
