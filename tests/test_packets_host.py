"""Host framing of the DL0 packet stream through the C ABI (rta_frame_packets
runs on the host only, so these run without a GPU) against the oracle's
framing: whole streams, corrupted headers, truncation and lost framing."""
import numpy as np
import pytest

import dl0sim.workloads as W
import paper_1307_6489_amd as rta
from dl0sim import packets as gp
from oracle import packets as op


@pytest.fixture(scope="module")
def stream():
    pool = W.c1_pool(30, seed=1)
    order = np.random.default_rng(4).permutation(pool.n)
    st, off = gp.serialize(pool, order, seed=2)
    return pool, order, st, off


def types_of(pool):
    return [(c.n_pix, c.n_samp, c.n_gain) for c in pool.cams]


def test_framing_matches_the_oracle(stream):
    pool, order, st, off = stream
    o, t, po, n, used = rta.frame_packets(pool.cams, st)
    ro, rt, rpo, rn, rused = op.frame(st, types_of(pool))
    assert np.array_equal(o, ro) and np.array_equal(t, rt) and np.array_equal(po, rpo)
    assert n == rn and used == rused == st.size
    assert np.array_equal(o, off) and np.array_equal(t, pool.pool_type[order])


def test_framing_of_corrupted_and_truncated_streams(stream):
    pool, order, st, off = stream
    bad = st.copy()
    bad[off[2] + 11] = 200                # unknown camera type
    bad[off[5] + 21] ^= 3                 # n_samp differs from the type's
    bad[off[7] + 40] ^= 0xFF              # payload: framing does not look at it
    o, t, po, n, used = rta.frame_packets(pool.cams, bad)
    ro, rt, rpo, rn, rused = op.frame(bad, types_of(pool))
    assert np.array_equal(t, rt) and np.array_equal(po, rpo) and n == rn
    assert t[2] == -1 and t[5] == -1 and t[7] >= 0
    cut = st[:off[9] + 77]
    o, t, po, n, used = rta.frame_packets(pool.cams, cut)
    assert len(o) == 9 and used == off[9]
    o, t, po, n, used = rta.frame_packets(pool.cams, st, cap=4)
    assert len(o) == 4 and used == off[4]


def test_lost_framing_is_an_error(stream):
    pool, order, st, off = stream
    bad = st.copy()
    bad[off[3] + 4:off[3] + 8] = 0        # data length below the smallest packet
    with pytest.raises(rta.RTAError):
        rta.frame_packets(pool.cams, bad)
    with pytest.raises(ValueError):
        op.frame(bad, types_of(pool))
