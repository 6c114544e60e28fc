"""Ray casting of an INR's level set by range analysis (App. A; the ray caster
of the range-analysis work it follows).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Per ray o + t d, t in [t_near, t_far]: the segment [t, t + de] with
de = min(step, t_far - t) is bounded by the method (UP and RA-UA: the soft
bound centre -/+ k spread; AA and RA-Fixed: the hard range).  If the bound
excludes the iso-value the ray advances to t + de and the step doubles (up
to step_max), missing once t >= t_far; otherwise it hits at t + de / 2 when
de <= step_min, or halves the step (to de / 2).  Ray state is float64; the
segment's centre o + d (t + de / 2) and half-vector d de / 2 are formed in
float64 (product, then sum) and rounded to float32, the precision in which
the library takes them.  Parameters given as float32 (iso, k, steps) are
widened from their float32 values.
"""

from __future__ import annotations

import numpy as np

from .propagate import AA, RAFIXED, propagate_segments


def cast(layers, origins, dirs, tnear, tfar, method: str, k: float, iso: float, step0: float, step_min: float,
         step_max: float, max_iter: int, act: str = "relu"):
    """Returns (t_hit float32 [n] (NaN: no hit), steps int32 [n], the
    smallest |endpoint - iso| over each ray's decisions [n] float64)."""
    org = np.asarray(origins, dtype=np.float32).astype(np.float64)
    dr = np.asarray(dirs, dtype=np.float32).astype(np.float64)
    tn = np.asarray(tnear, dtype=np.float32).astype(np.float64)
    tf = np.asarray(tfar, dtype=np.float32).astype(np.float64)
    f32 = lambda x: float(np.float32(x))
    k = 1.0 if method in (AA, RAFIXED) else f32(k)
    iso, step0, step_min, step_max = f32(iso), f32(step0), f32(step_min), f32(step_max)
    n = org.shape[0]
    t = tn.copy()
    dt = np.full(n, step0)
    thit = np.full(n, np.nan, dtype=np.float32)
    steps = np.zeros(n, dtype=np.int32)
    margin = np.full(n, np.inf)
    active = tn < tf
    for _ in range(max_iter):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        te, d = t[idx], dt[idx]
        de = np.minimum(d, tf[idx] - te)
        h = de * 0.5
        tm = te + h
        c = (org[idx] + dr[idx] * tm[:, None]).astype(np.float32)
        v = (dr[idx] * h[:, None]).astype(np.float32)
        mu, sp = propagate_segments(layers, c, v, method, act=act)
        ks = k * sp
        lo, hi = mu - ks, mu + ks
        margin[idx] = np.minimum(margin[idx], np.minimum(np.abs(lo - iso), np.abs(hi - iso)))
        steps[idx] += 1
        excl = (lo > iso) | (hi < iso)
        adv = idx[excl]
        t[adv] = te[excl] + de[excl]
        dt[adv] = np.minimum(2.0 * d[excl], step_max)
        active[adv[t[adv] >= tf[adv]]] = False
        keep = ~excl
        hit = keep & (de <= step_min)
        thit[idx[hit]] = (te[hit] + 0.5 * de[hit]).astype(np.float32)
        active[idx[hit]] = False
        ref = keep & ~hit
        dt[idx[ref]] = 0.5 * de[ref]
    return thit, steps, margin
