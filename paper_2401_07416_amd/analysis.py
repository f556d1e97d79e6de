"""Analysis of a database of trajectories (arXiv 2401.07416 section 3.2).

Eq. (16) runs on the GPU (``tdse.dissimilarity``); this module holds the
host-side pieces around it: the time-quadrature weights of eq. (16) over the
record frames, and the cluster statistics of eqs. (17)-(18) and their medians
over a 2D embedding with cluster labels (the embedding and the clustering
themselves are out of scope).
"""
from __future__ import annotations

import numpy as np


def frame_weights(times, t0: float, t1: float):
    """Frames inside [t0, t1] and their weights for eq. (16)'s time average:
    the trapezoid rule over those frames divided by the span they cover.
    Returns (indices, weights).  The window is taken at the record times it
    contains (the records are the only samples of the density)."""
    times = np.asarray(times, dtype=np.float64)
    idx = np.nonzero((times >= t0) & (times <= t1))[0]
    if idx.size == 0:
        raise ValueError("no frame inside [t0, t1]")
    if idx.size == 1:
        return idx, np.ones(1)
    t = times[idx]
    w = np.zeros(idx.size)
    dt = np.diff(t)
    w[:-1] += 0.5 * dt
    w[1:] += 0.5 * dt
    return idx, w / (t[-1] - t[0])


def _centres(xy, labels):
    xy = np.asarray(xy, dtype=np.float64).reshape(-1, 2)
    labels = np.asarray(labels)
    clusters = np.unique(labels)
    centres = np.stack([xy[labels == c].mean(axis=0) for c in clusters])
    return xy, labels, clusters, centres


def cluster_dispersion(xy, labels) -> dict:
    """acd (eq. 17): mean distance of the cluster centres from the sample
    centre; aicd (eq. 18): mean distance of the points from their cluster
    centre; mcd and micd: the medians of the same distances."""
    xy, labels, clusters, centres = _centres(xy, labels)
    centre = xy.mean(axis=0)
    dc = np.sqrt(np.sum((centres - centre) ** 2, axis=1))
    pos = np.searchsorted(clusters, labels)
    dp = np.sqrt(np.sum((xy - centres[pos]) ** 2, axis=1))
    return {"acd": float(dc.mean()), "aicd": float(dp.sum() / xy.shape[0]),
            "mcd": float(np.median(dc)), "micd": float(np.median(dp))}
