"""Seeded workload recipes built from the generator (inputs only).

A *pool* is one uint16 blob holding camera events grouped by type (all events
of type 0, then type 1, ...); a *descriptor list* gives the processing order:
for every telescope its type and the element offset of its trace block in the
pool.  Offsets are multiples of 8 elements (16 bytes), as the reconstruction
requires.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import (C1_WEIGHTS, CameraType, camera_types_c1, draw_array, draw_cfg_plain, draw_ellipses,
               mix_types, render_traces)


@dataclass
class Pool:
    cams: list               # CameraType per type index
    blob: np.ndarray         # uint16 [total]
    pool_type: np.ndarray    # int32 [n_pool] type of each pool entry
    pool_off: np.ndarray     # int64 [n_pool] element offset of each pool entry
    showers: np.ndarray      # generator truth per pool entry

    @property
    def n(self):
        return len(self.pool_type)

    def dl0_bytes(self, idx=None):
        per = np.array([c.dl0_bytes for c in self.cams], np.int64)
        t = self.pool_type if idx is None else self.pool_type[idx]
        return int(per[t].sum())


def render_pool(cams, counts, seed, first_event=0, showers_per_type=None, n_threads=None) -> Pool:
    """Render ``counts[t]`` camera events of each type ``t``, grouped by type.
    ``showers_per_type`` (optional) gives the image parameters per type;
    otherwise plain ellipses are drawn with the counter of each entry."""
    counts = np.asarray(counts, np.int64).reshape(len(cams))
    pool_type = np.repeat(np.arange(len(cams), dtype=np.int32), counts)
    sizes = np.array([cams[t].event_elems for t in pool_type], np.int64)
    pool_off = np.zeros(len(pool_type), np.int64)
    if len(sizes):
        pool_off[1:] = np.cumsum(sizes)[:-1]
    blob = np.empty(int(sizes.sum()), np.uint16)
    from . import SHOWER_DTYPE
    showers = np.zeros(len(pool_type), SHOWER_DTYPE)
    start = 0
    for ty, cam in enumerate(cams):
        n = int(counts[ty])
        if n == 0:
            continue
        ids = np.arange(first_event + start, first_event + start + n, dtype=np.uint64)
        if showers_per_type is not None:
            sh = showers_per_type[ty]
        else:
            sh = draw_ellipses(draw_cfg_plain(cam.n_samp), seed, first_event + start, n)
        o0 = int(pool_off[start])
        render_traces(cam, sh, seed, event_ids=ids, out=blob[o0:o0 + n * cam.event_elems], n_threads=n_threads)
        showers[start:start + n] = sh
        start += n
    return Pool(list(cams), blob, pool_type, pool_off, showers)


def c1_pool(n_unique: int, seed: int = 1, cams=None, n_threads=None) -> Pool:
    """The mixed dual-gain throughput workload: 1855x40, 1764x25 and 2048x128
    cameras in ratio 1:3:6 (exact proportions), plain ellipse images."""
    cams = cams or camera_types_c1()
    types = mix_types(n_unique, seed, C1_WEIGHTS)
    counts = np.bincount(types, minlength=len(cams))
    return render_pool(cams, counts, seed, n_threads=n_threads)


def stream_order(pool: Pool, n_events: int, seed: int):
    """Descriptor list of ``n_events`` camera events cycling through the pool
    in a seeded random order (each pass a new permutation)."""
    rng = np.random.default_rng(seed)
    idx = np.concatenate([rng.permutation(pool.n) for _ in range((n_events + pool.n - 1) // max(pool.n, 1))])
    idx = idx[:n_events]
    return idx, pool.pool_type[idx].astype(np.int32), pool.pool_off[idx].astype(np.int64)


@dataclass
class ArrayWorkload:
    pool: Pool
    evt_tel_off: np.ndarray   # int64 [E+1]
    tel_type: np.ndarray      # int32 [n_tel]
    tel_off: np.ndarray       # int64 [n_tel]
    tel_pool_idx: np.ndarray  # int64 [n_tel]
    src_nominal: np.ndarray   # float64 [E][2]


def array_events(n_evt: int, seed: int = 2, cams=None, weights=C1_WEIGHTS, mult=(2, 40), n_threads=None):
    """Ragged array events with consistent stereo geometry: every telescope has
    its own rendered image whose major axis points at the event's source."""
    cams = cams or camera_types_c1()
    ad = draw_array(draw_cfg_plain(40), seed, 0, n_evt, cams, weights, mult)
    n_tel = len(ad.tel_type)
    # group the telescopes by type in the pool, keep event order in descriptors
    order = np.argsort(ad.tel_type, kind="stable")
    counts = np.bincount(ad.tel_type, minlength=len(cams))
    per_type = []
    start = 0
    for ty, cam in enumerate(cams):
        sh = ad.showers[order[start:start + counts[ty]]].copy()
        # pulse timing centred for this camera's trace length
        sh["t0"][:, 0] = sh["t0"][:, 0] - 20.0 + cam.n_samp / 2.0
        per_type.append(sh)
        start += counts[ty]
    pool = render_pool(cams, counts, seed, first_event=10_000_000, showers_per_type=per_type, n_threads=n_threads)
    pool_idx = np.empty(n_tel, np.int64)
    pool_idx[order] = np.arange(n_tel)
    return ArrayWorkload(pool, ad.evt_tel_off, ad.tel_type.astype(np.int32), pool.pool_off[pool_idx], pool_idx,
                         ad.src_nominal)


def replicate_array_events(aw: ArrayWorkload, n_evt: int, seed: int):
    """Descriptors of ``n_evt`` array events that cycle through the rendered
    array events of ``aw`` (each pass a new seeded permutation), so a batch of
    any size references a fixed device pool.  Returns (evt_tel_off int64
    [n_evt+1], tel_type int32, tel_off int64, source array event index)."""
    rng = np.random.default_rng(seed)
    n_src = len(aw.evt_tel_off) - 1
    src = np.concatenate([rng.permutation(n_src) for _ in range((n_evt + n_src - 1) // max(n_src, 1))])[:n_evt]
    lo = aw.evt_tel_off[src]
    mult = aw.evt_tel_off[src + 1] - lo
    evt_tel_off = np.zeros(n_evt + 1, np.int64)
    evt_tel_off[1:] = np.cumsum(mult)
    # telescope k of output event e is telescope lo[e] + (k - evt_tel_off[e]) of the pool event
    rel = np.arange(evt_tel_off[-1], dtype=np.int64) - np.repeat(evt_tel_off[:-1], mult)
    tel_src = np.repeat(lo, mult) + rel
    return evt_tel_off, aw.tel_type[tel_src].astype(np.int32), aw.tel_off[tel_src].astype(np.int64), src


def sam_events(seed: int, duration_s: float, bkg_rate_hz: float, fov_rad: float, sources=(),
               gamma_frac_bkg: float = 0.1, invalid_frac: float = 0.02):
    """Synthetic event list for the alert monitor: background events uniform
    in time and in a disc of radius fov_rad, with a gamma-like fraction
    gamma_frac_bkg; sources = [(x, y, t_start, t_end, rate_hz, psf_rad)]
    add gamma-like events around (x, y) (Gaussian spread psf_rad) during
    [t_start, t_end).  Returns (time float64, dir float32 [n][2], gammaness
    float32, stereo-valid bool), sorted by time."""
    rng = np.random.default_rng(seed)
    nb = rng.poisson(bkg_rate_hz * duration_s)
    t = [rng.uniform(0.0, duration_s, nb)]
    r = fov_rad * np.sqrt(rng.uniform(0.0, 1.0, nb))
    ph = rng.uniform(0.0, 2.0 * np.pi, nb)
    d = [np.stack([r * np.cos(ph), r * np.sin(ph)], 1)]
    g = [np.where(rng.uniform(0.0, 1.0, nb) < gamma_frac_bkg, rng.uniform(0.7, 1.0, nb), rng.uniform(0.0, 0.5, nb))]
    for (x, y, t_a, t_b, rate, psf) in sources:
        ns = rng.poisson(rate * (t_b - t_a))
        t.append(rng.uniform(t_a, t_b, ns))
        d.append(np.stack([x + psf * rng.standard_normal(ns), y + psf * rng.standard_normal(ns)], 1))
        g.append(rng.uniform(0.75, 1.0, ns))
    t = np.concatenate(t)
    d = np.concatenate(d).astype(np.float32)
    g = np.concatenate(g).astype(np.float32)
    valid = rng.uniform(0.0, 1.0, len(t)) >= invalid_frac
    order = np.argsort(t, kind="stable")
    return t[order], d[order], g[order], valid[order]
