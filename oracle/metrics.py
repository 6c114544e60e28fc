"""Error rates and parity helpers, float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""

from __future__ import annotations

import numpy as np


def fpr_fnr(predicted, truth):
    """False-positive and false-negative rates of an active-cell prediction
    (Sec. V-A-3): FPR = FP/(FP+TN), FNR = FN/(FN+TP); boolean arrays over the
    same cells.  A rate with an empty denominator is reported as 0."""
    predicted = np.asarray(predicted, dtype=bool)
    truth = np.asarray(truth, dtype=bool)
    fp = np.sum(predicted & ~truth)
    tn = np.sum(~predicted & ~truth)
    fn = np.sum(~predicted & truth)
    tp = np.sum(predicted & truth)
    fpr = fp / (fp + tn) if fp + tn else 0.0
    fnr = fn / (fn + tp) if fn + tp else 0.0
    return float(fpr), float(fnr)


def set_recall(predicted_ids, reference_ids):
    """|predicted & reference| / |reference| over id sets."""
    ref = np.unique(np.asarray(reference_ids))
    if ref.size == 0:
        return 1.0
    hit = np.intersect1d(np.unique(np.asarray(predicted_ids)), ref).size
    return hit / ref.size


def rel_err(got, ref, scale):
    """|got - ref| / max(|ref|, scale), elementwise."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(got - ref) / np.maximum(np.abs(ref), scale)


def margin(centre, spread, k, isos):
    """Distance of the nearest bound endpoint to the nearest iso-value:
    min_j min(|centre - k spread - c_j|, |centre + k spread - c_j|)."""
    isos = np.asarray(isos, dtype=np.float64)
    lo = (centre - k * spread)[:, None]
    hi = (centre + k * spread)[:, None]
    return np.minimum(np.abs(lo - isos[None, :]), np.abs(hi - isos[None, :])).min(axis=1)
