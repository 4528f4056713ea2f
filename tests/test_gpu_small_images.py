"""Images around the single-wavefront limit of the islands / Hillas phases.

Images of at most 64 mask pixels take their union-find and Hillas sums in
one wavefront; larger ones in the whole workgroup.  Plain traces (constant
pedestal, no noise) with pulses in exactly the chosen pixels, grown as
separate clusters of at least two neighbours, give masks of exactly n pixels
in several islands for n on both sides of 64.  The fused and unfused GPU
paths are compared with the oracle on every record (the oracle's own pixel
count confirms each construction), and with each other bit for bit outside
the time regression.
"""
import numpy as np
import pytest

import dl0sim
import oracle
import paper_1307_6489_amd as rta
from test_gpu_parity import check_records, oracle_events, say, to_dev, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu

SIZES = [0, 2, 3, 17, 63, 64, 65, 66, 127, 128, 129, 300]


def grow_clusters(nbr, n_pix, n, rng):
    """Pixel set of exactly n pixels made of separate clusters (no two
    clusters adjacent), each connected and of at least two pixels."""
    if n == 0:
        return np.zeros(0, np.int64)
    k = 1 if n < 8 else int(rng.integers(2, 5))
    sizes = [n // k + (1 if i < n % k else 0) for i in range(k)]
    chosen, blocked = [], np.zeros(n_pix, bool)
    for size in sizes:
        for _ in range(200):
            seed = int(rng.integers(n_pix))
            if blocked[seed]:
                continue
            cl, front, inside = [seed], [seed], {seed}
            while front and len(cl) < size:
                p = front.pop(0)
                for m in rng.permutation(nbr[p]):
                    m = int(m)
                    if m < 0 or m in inside or blocked[m]:
                        continue
                    inside.add(m)
                    cl.append(m)
                    front.append(m)
                    if len(cl) == size:
                        break
            if len(cl) == size:
                break
        else:
            raise RuntimeError("could not place a cluster of %d pixels" % size)
        chosen += cl
        for p in cl:
            blocked[p] = True
            blocked[nbr[p][nbr[p] >= 0]] = True
    return np.array(chosen, np.int64)


def traces_with_masks(ct, sizes, seed):
    """uint16 [E][G][T][Npad] traces: the rounded pedestal everywhere, plus a
    pulse in the chosen pixels of each event (amplitude 150..1500 ADC in the
    high gain, start following x so the images have a time gradient)."""
    rng = np.random.default_rng(seed)
    G, T, N, Np = ct.n_gain, ct.n_samp, ct.n_pix, ct.n_pix_pad
    x = ct.geom.x.astype(np.float64)
    shape = np.array([0.3, 1.0, 0.6, 0.2])
    tr = np.zeros((len(sizes), G, T, Np), np.uint16)
    base = np.rint(ct.ped).astype(np.int64)  # [G][N]
    for e, n in enumerate(sizes):
        for g in range(G):
            tr[e, g, :, :N] = base[g][None, :]
        pix = grow_clusters(ct.geom.nbr, N, n, rng)
        for i in pix:
            amp = rng.uniform(150.0, 1500.0)
            s0 = 6 + int(round(4.0 * (x[i] - x.min()) / (x.max() - x.min())))
            for k in range(4):
                tr[e, 0, s0 + k, i] += np.uint16(round(amp * shape[k]))
    return tr


@pytest.mark.parametrize("which", ["c0", "1764x25"])
def test_images_around_the_wave_limit(torch_dev, which):
    import torch
    ct = dl0sim.camera_c0() if which == "c0" else dl0sim.camera_types_c1()[1]
    say("small images: %s, mask sizes %s, seed 41" % (ct.name, SIZES))
    tr = traces_with_masks(ct, SIZES, 41)
    oc = oracle.Camera.from_type(ct)
    E = len(SIZES)
    offs = np.arange(E, dtype=np.int64) * oc.event_elems
    pixes, masks, recs = oracle_events([oc], np.zeros(E, np.int64), tr.reshape(-1), offs)
    got_n = [int(r["n_pix"]) for r in recs]
    assert got_n == SIZES, got_n
    assert max(int(r["n_islands"]) for r in recs) >= 3

    cam = rta.Camera.from_type(ct)
    out = rta.calibrate(cam, to_dev(tr, torch_dev))
    mask = rta.clean(cam, out["D"], out["gain"])
    assert np.array_equal(mask.cpu().numpy(), np.stack(masks))
    unfused = rta.hillas(cam, out["q"], out["t"], mask, out["gain"]).cpu()
    check_records(rta.records(unfused), recs, pixes, masks, lambda k: ct, "unfused", t_input_f32=True)

    pipe = rta.Pipeline([cam], do_stereo=False)
    b = pipe.make_batch(to_dev(tr.reshape(-1), torch_dev), torch.zeros(E, dtype=torch.int32, device=torch_dev),
                        to_dev(offs, torch_dev))
    for sched in [(8, 4, 0, 8), (4, 8, 0, 8), (8, 4, 2, 8), (2, 8, 3, 16)]:
        say("fused, schedule", sched)
        pipe.set_schedule(*sched)
        tel, _ = pipe.alloc_outputs(b, torch_dev)
        tel.fill_(float("nan"))
        pipe.process(b, tel)
        got = tel.cpu()
        check_records(rta.records(got), recs, pixes, masks, lambda k: ct, "fused %s" % (sched,))
        if sched[1] == 4:  # 256 threads: the unfused kernels' reduction order
            same = [k for k in range(16) if k not in (8, 9)]
            assert torch.equal(got.view(torch.int32)[:, same], unfused.view(torch.int32)[:, same])
    assert pipe.status() == 0
