"""Clustering quality against planted ground-truth communities.

The quality experiments of the paper (Sec. 4 setup, Sec. 4.3) score a
clustering against ground-truth communities by average precision and recall:
each community c is matched to the cluster c' that shares the most vertices
with it (a cluster may be matched by several communities or by none), and
precision |c & c'| / |c'| and recall |c & c'| / |c| are averaged over the
communities.  Here the ground truth is the generator's planted communities
(the paper's SNAP ground truth is not available), and ties for the largest
intersection go to the smallest cluster label so the score is deterministic.

Host-side bookkeeping on labels the GPU returned; nothing here is on the
clustering path.
"""
from __future__ import annotations

import numpy as np


def precision_recall(labels, communities, top: int = 0):
    """Average precision and recall of a clustering against communities.

    labels: int[n] cluster label of every vertex; communities: int[n]
    community of every vertex (-1 = in none).  top > 0 keeps only the `top`
    largest communities (ties by smaller id), as the paper keeps the 5000
    largest SNAP communities.  Returns (precision, recall, communities used).
    """
    labels = np.asarray(labels, dtype=np.int64)
    comm = np.asarray(communities, dtype=np.int64)
    if labels.shape != comm.shape:
        raise ValueError("labels and communities must have one entry per vertex")
    inside = comm >= 0
    if not inside.any():
        return 0.0, 0.0, 0
    cids, csize = np.unique(comm[inside], return_counts=True)
    if top > 0 and len(cids) > top:
        order = np.lexsort((cids, -csize))[:top]
        keep_ids = np.sort(cids[order])
    else:
        keep_ids = cids
    sel = inside & np.isin(comm, keep_ids)
    L = labels.max() + 1 if labels.size else 1
    # intersections |c & c'| for every (community, cluster) pair that meets
    key = comm[sel] * L + labels[sel]
    pair, inter = np.unique(key, return_counts=True)
    pc, pl = pair // L, pair % L
    # per community: the largest intersection, ties to the smallest label
    # (pairs are sorted by community then label, so a stable sort by
    # descending count keeps the smallest label first)
    order = np.lexsort((pl, -inter, pc))
    first = np.ones(len(order), dtype=bool)
    first[1:] = pc[order][1:] != pc[order][:-1]
    best = order[first]
    m_comm, m_label, m_inter = pc[best], pl[best], inter[best]
    cl_size = np.bincount(labels, minlength=L)
    size_of = dict(zip(cids.tolist(), csize.tolist()))
    c_size = np.array([size_of[c] for c in m_comm.tolist()], dtype=np.float64)
    prec = m_inter / cl_size[m_label]
    rec = m_inter / c_size
    return float(prec.mean()), float(rec.mean()), int(len(m_comm))
