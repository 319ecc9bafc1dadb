"""Truth matching of reconstructed tracks against the generator's Monte-Carlo labels.

Evaluation only (used on the oracle's and on the GPU library's outputs alike).

Definitions:
  * a (MC track, sector) segment is findable if it has >= min_hits clusters in that sector;
  * a track's label is the MC id holding most of its clusters (ties: smaller id); its
    purity is the fraction of its clusters carrying that label;
  * a track is fake if purity < 0.9 or its label is noise (-1);
  * found = a non-fake track whose (label, sector) is findable; further such tracks of the
    same (label, sector) are clones;
  * efficiency = found / findable, fake rate = fakes / tracks, clone rate = clones / tracks.
"""
from __future__ import annotations

import numpy as np

N_ROWS = 152


def cluster_sector(row_off, n_sectors=36, n_rows=N_ROWS):
    counts = np.diff(np.asarray(row_off))
    g = np.repeat(np.arange(counts.shape[0]), counts)
    return g // n_rows


def match(label, row_off, hit_off, hit_ids, track_sector, min_hits=20, purity_min=0.9):
    label = np.asarray(label)
    sec_of = cluster_sector(row_off)
    # findable segments
    sig = label >= 0
    key = label[sig].astype(np.int64) * 64 + sec_of[sig]
    uk, cnt = np.unique(key, return_counts=True)
    findable = set(uk[cnt >= min_hits].tolist())
    T = len(hit_off) - 1
    labels = np.full(T, -1, np.int64)
    purity = np.zeros(T)
    fake = np.zeros(T, bool)
    for t in range(T):
        h = hit_ids[hit_off[t]:hit_off[t + 1]]
        lab = label[h]
        vals, c = np.unique(lab, return_counts=True)
        best = np.flatnonzero(c == c.max())
        lt = vals[best].min()
        labels[t] = lt
        purity[t] = c.max() / max(1, len(h))
        fake[t] = (lt < 0) or (purity[t] < purity_min)
    seen = set()
    found = 0
    clones = 0
    for t in range(T):
        if fake[t]:
            continue
        k = int(labels[t]) * 64 + int(track_sector[t])
        if k not in findable:
            continue
        if k in seen:
            clones += 1
        else:
            seen.add(k)
            found += 1
    nf = len(findable)
    return dict(findable=nf, found=found, clones=clones, fakes=int(fake.sum()), tracks=T,
                efficiency=found / nf if nf else 1.0,
                fake_rate=fake.sum() / T if T else 0.0,
                clone_rate=clones / T if T else 0.0,
                labels=labels, purity=purity, fake=fake)
