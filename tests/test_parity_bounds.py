"""The parity bound for Hillas records computed from float32 peak times (the
unfused Hillas call's input) covers the effect of that rounding: on oracle
events, the least-squares slope and intercept of the times rounded to float32
differ from those of the FP64 times by no more than the extra allowance of
hillas_mismatches(t_input_f32=True), and the allowance is needed (the plain
1e-5 scale alone is exceeded on some events).  CPU only."""
import math

import numpy as np

import dl0sim
import oracle
import oracle.parity as par


def test_float32_time_rounding_is_covered():
    ct = dl0sim.camera_c0()
    _, tr = dl0sim.plain_events(ct, 0, 700)
    oc = oracle.Camera.from_type(ct)
    exceeded = 0
    for e in range(len(tr)):
        p, m, h = oc.reconstruct(tr[e])
        if int(h["flags"]) & 3:
            continue
        mm = m.astype(bool)
        x, y = ct.geom.x[mm].astype(np.float64), ct.geom.y[mm].astype(np.float64)
        psi = float(h["psi"])
        l = (x - h["cog_x"]) * math.cos(psi) + (y - h["cog_y"]) * math.sin(psi)
        t32 = p["t"][mm].astype(np.float32).astype(np.float64)
        lb = l - l.mean()
        slope = float(np.sum(lb * (t32 - t32.mean())) / np.sum(lb * lb))
        icpt = float(t32.mean() - slope * l.mean())
        g = h.copy()
        g["time_gradient"], g["time_intercept"] = slope, icpt
        assert not par.hillas_mismatches(g, h, ct.geom.x, ct.geom.y, p["q"], p["t"], m, t_input_f32=True), e
        exceeded += bool(par.hillas_mismatches(g, h, ct.geom.x, ct.geom.y, p["q"], p["t"], m))
    assert exceeded >= 1
