"""Pins of the oracle's hit removal for compression strategy B (keep only the clusters
near good tracks) against hand-worked geometry, the generator's closed-form helices, brute
force and Monte-Carlo truth.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import truthmatch
from paper_2009_07515_amd import synth

W = 1.0          # the default vicinity half-width (cm)


def _frame_from_rows(rows_y_z, n_sectors=36, n_rows=152):
    """Clusters given as {(sector, row): [(y, z), ...]} -> (y, z, row_off), in that order."""
    y, z, counts = [], [], np.zeros(n_sectors * n_rows, np.int64)
    for g in range(n_sectors * n_rows):
        for (yy, zz) in rows_y_z.get((g // n_rows, g % n_rows), []):
            y.append(yy)
            z.append(zz)
            counts[g] += 1
    ro = np.zeros(n_sectors * n_rows + 1, np.int64)
    np.cumsum(counts, out=ro[1:])
    return np.array(y, np.float32), np.array(z, np.float32), ro


def _one_track(x_ref, p, sector, hit_ids):
    return dict(n_tracks=1, n_hits=len(hit_ids), params=np.array([p], np.float64),
                x_ref=np.array([x_ref]), sector=np.array([sector], np.int32),
                hit_off=np.array([0, len(hit_ids)], np.int64), hit_ids=np.array(hit_ids, np.int64))


# --------------------------------------------------------------------------------------
# Hand-worked window on a straight track (B = 0): y = y0 + (x - x0) tan(phi),
# z = z0 + (x - x0) tan(lambda) / cos(phi).  Probes just inside and just outside the 1 cm
# vicinity at rows inside the track's row span, a probe on the track beyond its span and one
# in the neighbouring sector.
# --------------------------------------------------------------------------------------
def test_reject_window_hand_example(row_x):
    o = oracle.Oracle(row_x, bz=0.0)
    X = row_x.astype(np.float64)
    sphi, tl = 0.1, 0.2
    tphi, c = sphi / math.sqrt(1 - sphi * sphi), math.sqrt(1 - sphi * sphi)
    y0, z0, r0, r1 = 1.0, 10.0, 5, 120

    def on_track(r):
        return y0 + (X[r] - X[r0]) * tphi, z0 + (X[r] - X[r0]) * tl / c

    rows = {}
    for r in range(r0, r1 + 1):
        rows[(3, r)] = [on_track(r)]
    probes = []   # (sector, row, dy, dz, expected)
    for r in (40, 80):
        for dy, dz, exp in ((0.999, 0.0, 1), (1.001, 0.0, 0), (0.0, -0.999, 1), (0.0, -1.001, 0),
                            (0.7, 0.7, 1), (-0.999, 0.999, 1)):
            probes.append((3, r, dy, dz, exp))
    probes.append((3, r0, 0.5, 0.0, 1))         # the first and last rows of the span
    probes.append((3, r1, -0.5, 0.3, 1))
    probes.append((3, r1 + 1, 0.0, 0.0, 0))     # just outside the span
    probes.append((3, r0 - 1, 0.0, 0.0, 0))
    probes.append((3, 130, 0.0, 0.0, 0))        # beyond the outermost cluster's row
    probes.append((3, 2, 0.0, 0.0, 0))          # below the innermost cluster's row
    probes.append((4, 80, 0.0, 0.0, 0))         # another sector
    for s, r, dy, dz, _ in probes:
        yy, zz = on_track(r)
        rows.setdefault((s, r), []).append((yy + dy, zz + dz))
    y, z, ro = _frame_from_rows(rows)
    hits = [int(ro[3 * 152 + r]) for r in range(r0, r1 + 1)]
    trk = _one_track(X[r0], [y0, z0, sphi, tl, 1.0], 3, hits)
    keep, k = o.reject_frame(y, z, ro, trk)
    assert np.all(keep[hits] == 1)
    seen = {}
    for s, r, dy, dz, exp in probes:
        g = s * 152 + r
        j = seen.get(g, 1 if (s == 3 and r0 <= r <= r1) else 0)
        seen[g] = j + 1
        assert keep[ro[g] + j] == exp, (s, r, dy, dz)
    assert k == len(hits) + sum(e for *_, e in probes)


# --------------------------------------------------------------------------------------
# The pT threshold: |q/pT| * pT_min <= 1 is good.  A bad track keeps nothing, not even
# its own clusters.
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("qpt,good", [(19.99, True), (-19.99, True), (20.01, False), (-20.01, False)])
def test_reject_pt_threshold(row_x, qpt, good):
    o = oracle.Oracle(row_x, bz=0.0)
    X = row_x.astype(np.float64)
    rows = {(0, r): [(0.0, 5.0)] for r in range(10, 40)}
    y, z, ro = _frame_from_rows(rows)
    hits = [int(ro[r]) for r in range(10, 40)]
    keep, k = o.reject_frame(y, z, ro, _one_track(X[10], [0.0, 5.0, 0.0, 0.0, qpt], 0, hits))
    assert k == (30 if good else 0)


# --------------------------------------------------------------------------------------
# Curved tracks: the vicinity follows the helix.  For noise-free helices (B = 0.5 T) the
# generator's closed-form crossing of a middle row, shifted by 0.999 cm in y or z, is kept,
# and shifted by 1.001 cm is removed (no other track nearby in the tiny event).
# --------------------------------------------------------------------------------------
def test_reject_vicinity_follows_the_helix(row_x):
    o = oracle.Oracle(row_x)
    f = synth.config1_single_sector(seed=5, n_tracks=12, sigma=0.0, noise_frac=0.0)
    r = o.track_frame(f.y, f.z, f.row_off)
    assert r["n_tracks"] >= 3
    X = row_x.astype(np.float64)
    rows_of = np.repeat(np.arange(152), np.diff(f.row_off[:153]))
    n_checked = 0
    for t in range(r["n_tracks"]):
        h = r["hit_ids"][r["hit_off"][t]:r["hit_off"][t + 1]]
        mid = h[len(h) // 2]
        rr = rows_of[mid]
        for dy, dz, exp in ((0.999, 0, 1), (1.001, 0, 0), (0, 0.999, 1), (0, -1.001, 0)):
            rows = {(0, q): [(float(f.y[i]), float(f.z[i])) for i in range(f.row_off[q], f.row_off[q + 1])]
                    for q in range(152)}
            rows[(0, rr)].append((f.truth_y[mid] + dy, f.truth_z[mid] + dz))
            y, z, ro = _frame_from_rows(rows)
            # the same clusters, one probe appended at the end of row rr
            remap = np.arange(f.n_clusters) + (np.arange(f.n_clusters) >= f.row_off[rr + 1])
            trk = dict(r, hit_ids=remap[r["hit_ids"]])
            keep, _ = o.reject_frame(y, z, ro, trk)
            probe = ro[rr + 1] - 1
            others = [tt for tt in range(r["n_tracks"]) if tt != t]
            near = any(abs(o.propagate(r["x_ref"][tt], X[rr], r["params"][tt])[1][0] - y[probe]) < 3
                       for tt in others)
            if near:
                continue
            assert keep[probe] == exp, (t, dy, dz)
            n_checked += 1
    assert n_checked >= 8


# --------------------------------------------------------------------------------------
# The y-sorted window scan equals the all-clusters definition.
# --------------------------------------------------------------------------------------
def test_reject_sorted_scan_equals_brute_force(small_pbpb_frame, row_x):
    f = small_pbpb_frame
    o = oracle.Oracle(row_x)
    r = o.track_frame(f.y, f.z, f.row_off)
    a, ka = o.reject_frame(f.y, f.z, f.row_off, r)
    b, kb = o.reject_frame(f.y, f.z, f.row_off, r, brute=True)
    assert ka == kb and np.array_equal(a, b)


# --------------------------------------------------------------------------------------
# Monte-Carlo truth on the Pb-Pb event: clusters of found track segments survive, noise
# and clusters of segments the tracking did not find are mostly removed (the caveat of
# strategy B, Sec. 4).
# --------------------------------------------------------------------------------------
def test_reject_statistics_on_pbpb_event(cfg2_frame, row_x):
    f = cfg2_frame
    o = oracle.Oracle(row_x)
    r = o.track_frame(f.y, f.z, f.row_off)
    keep, k = o.reject_frame(f.y, f.z, f.row_off, r)
    sec = truthmatch.cluster_sector(f.row_off)
    found = set()
    for t in range(r["n_tracks"]):
        h = r["hit_ids"][r["hit_off"][t]:r["hit_off"][t + 1]]
        v, c = np.unique(f.label[h], return_counts=True)
        j = int(np.argmax(c))
        if v[j] >= 0 and c[j] >= 0.9 * len(h):
            found.add(int(v[j]) * 64 + int(r["sector"][t]))
    key = f.label.astype(np.int64) * 64 + sec
    sig = f.label >= 0
    in_found = sig & np.isin(key, np.array(sorted(found), np.int64))
    assert keep[in_found].mean() >= 0.999
    assert keep[sig & ~in_found].mean() <= 0.3
    assert keep[~sig].mean() <= 0.1
    assert k == int(keep.sum())
    print(f"kept {k} of {f.n_clusters}: found segments {keep[in_found].mean():.5f}, "
          f"other signal {keep[sig & ~in_found].mean():.3f}, noise {keep[~sig].mean():.3f}")
