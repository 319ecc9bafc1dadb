"""Pins of the oracle's follow rule and selection against hand-worked cases (CPU only).

Follow (tracklet construction, R8): at each row beyond the chain the state is propagated
and the least-chi2 cluster inside |dy| <= min(win_y, nsig * sqrt(S_yy)) (z alike) is taken
if chi2 <= chi2_max; the pass stops after more than max_miss consecutive rows without a
cluster.  The frames below are straight tracks at B = 0 along the sector axis (y = 0,
z = 10 cm, exactly representable), so the filtered state stays exactly on the line and
the predicted covariance is that of a straight-line least-squares fit with the C0 prior:
an independent textbook computation fixes S_yy, and with it which side of a cut a
displaced cluster lies on.

Selection (R9): weight w = (n << 32) | (2^32 - 1 - rank); each cluster keeps the largest
weight; a tracklet keeps the clusters carrying its own weight; one pass.
"""
import numpy as np
import pytest

import oracle
from paper_2009_07515_amd import synth

ROWS = synth.row_x()
NR = len(ROWS)
SIGMA = 0.1
Z0 = 10.0


def _frame(rows, extra=None):
    """One sector: a cluster at (0, Z0) on each row of `rows`, plus extra {row: [(y, z)]}."""
    per = {r: [(0.0, Z0)] for r in rows}
    for r, cl in (extra or {}).items():
        per.setdefault(r, []).extend(cl)
    ys, zs, cnt = [], [], np.zeros(NR, np.int64)
    for r in range(NR):
        for y, z in per.get(r, []):
            ys.append(y)
            zs.append(z)
        cnt[r] = len(per.get(r, []))
    off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    return np.array(ys, np.float32), np.array(zs, np.float32), off


def _track(frame, **params):
    o = oracle.Oracle(ROWS, bz=0.0, n_sectors=1, params=params)
    r = o.track_frame(*frame, debug=True)
    d = r["debug"]
    sizes = [int(n) for n in d["tl_nhits"] if n > 0]
    return sizes, [int(n) for n in r["nhits"]]


# --------------------------------------------------------------------------------------
# Consecutive misses
# --------------------------------------------------------------------------------------
def test_gap_of_max_miss_rows_is_bridged_and_one_more_stops():
    # rows 10..40 and 45..70: a gap of 4 empty rows (41..44).  Each segment's chain starts
    # one row above its lowest cluster; both tracklets bridge the gap and hold all 57.
    sizes, tracks = _track(_frame(list(range(10, 41)) + list(range(45, 71))))
    assert sizes == [57, 57]
    assert tracks == [57]
    # a gap of 5 (41..45): neither follow crosses it
    sizes, tracks = _track(_frame(list(range(10, 41)) + list(range(46, 72))))
    assert sizes == [31, 26]
    assert tracks == [31, 26]


def test_misses_are_counted_consecutively():
    # two gaps of 3 rows each: 3 + 3 > max_miss, but the counter restarts at each cluster
    sizes, _ = _track(_frame(list(range(10, 41)) + list(range(44, 61)) + list(range(64, 81))))
    assert sizes[0] == 31 + 17 + 17


@pytest.mark.parametrize("max_miss,gap,bridged", [(2, 2, True), (2, 3, False), (0, 1, False), (6, 6, True),
                                                  (6, 7, False)])
def test_max_miss_parameter(max_miss, gap, bridged):
    rows = list(range(10, 41)) + list(range(41 + gap, 41 + gap + 25))
    sizes, _ = _track(_frame(rows), max_miss=max_miss)
    assert (sizes[0] == len(rows)) == bridged, sizes


# --------------------------------------------------------------------------------------
# Window clamp and chi2 cut at a displaced cluster two rows beyond the chain
# --------------------------------------------------------------------------------------
def _predicted_S(used_rows, at_row, c0_pos=1.0, c0_slope=1.0):
    """S = sigma^2 + variance of the straight-line prediction at row `at_row` from a
    least-squares fit of the clusters on `used_rows` with the prior diag(c0_pos, c0_slope)
    on (position, slope) at the first used row.  At phi = 0 and B = 0 the y and z parts of
    the 5-parameter state are two such independent fits (d y/d sin(phi) = dx and
    d z/d tan(lambda) = dx there)."""
    x = ROWS.astype(np.float64)
    x0 = x[used_rows[0]]
    H = np.stack([np.ones(len(used_rows)), x[used_rows] - x0], axis=1)
    info = np.diag([1.0 / c0_pos, 1.0 / c0_slope]) + H.T @ H / SIGMA ** 2
    h = np.array([1.0, x[at_row] - x0])
    return SIGMA ** 2 + h @ np.linalg.solve(info, h)


# the chain of rows 10..40 runs over rows 11..39 and the outward follow takes row 40; row
# 41 is empty; the displaced cluster sits on row 42
USED = list(range(11, 41))
S42 = _predicted_S(USED, 42)


def _displaced(dy=0.0, dz=0.0, **params):
    f = _frame(list(range(10, 41)), extra={42: [(dy, Z0 + dz)]})
    sizes, _ = _track(f, **params)
    return sizes[0]


def _chi2(dy_f32, dz_f32=0.0):
    return (dy_f32 ** 2 + dz_f32 ** 2) / S42


def test_independent_prediction_is_in_the_expected_range():
    # two rows beyond a 30-cluster line fit: a little above the cluster variance
    assert 0.0101 < S42 < 0.0125


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_chi2_cut_at_chi2_max(sign):
    below = np.float32(sign * np.sqrt(16.0 * (1 - 1e-5) * S42))
    above = np.float32(sign * np.sqrt(16.0 * (1 + 1e-5) * S42))
    assert _chi2(float(below)) < 16.0 < _chi2(float(above))
    assert _displaced(dy=float(below)) == 32
    assert _displaced(dy=float(above)) == 31
    # the same cluster against a lower cut
    assert _displaced(dy=float(below), chi2_max=15.0) == 31


def test_window_clamp_is_nsig_times_predicted_error():
    s = np.sqrt(S42)
    d3 = float(np.float32(3.0 * s))        # chi2 = 9 < 16: only a window can refuse it
    assert _displaced(dy=d3) == 32          # 3 sigma inside the 5-sigma window
    assert _displaced(dy=d3, nsig=1.0) == 31  # outside the 1-sigma window (3 cm alone admits it)
    assert _displaced(dy=d3, nsig=3.1) == 32
    assert _displaced(dy=d3, nsig=2.9) == 31
    d09 = float(np.float32(0.9 * s))
    assert _displaced(dy=d09, nsig=1.0) == 32   # a window of nsig * S (not its root) would refuse it
    # the same in z
    assert _displaced(dz=d3) == 32
    assert _displaced(dz=d3, nsig=1.0) == 31


def test_window_clamp_is_min_of_fixed_window_and_predicted_error():
    s = np.sqrt(S42)
    d2 = float(np.float32(2.0 * s))        # chi2 = 4, inside 5 sigma
    assert _displaced(dy=d2) == 32
    assert _displaced(dy=d2, win_y=float(1.5 * s)) == 31   # the fixed window is the smaller one
    assert _displaced(dy=d2, win_y=float(2.5 * s)) == 32
    assert _displaced(dz=d2, win_z=float(1.5 * s)) == 31


def test_least_chi2_cluster_wins_within_the_window():
    s = np.sqrt(S42)
    near, far = float(np.float32(1.0 * s)), float(np.float32(-2.0 * s))
    o = oracle.Oracle(ROWS, bz=0.0, n_sectors=1)
    # the far cluster first in the row: the choice must not depend on the in-row order
    f = _frame(list(range(10, 41)), extra={42: [(far, Z0), (near, Z0)]})
    r = o.track_frame(*f, debug=True)
    d = r["debug"]
    k = int(np.flatnonzero(d["tl_nhits"] > 0)[0])
    assert d["tl_hits"][k][42] == 1        # in-row index of the nearer cluster
    # equal chi2 (mirror images): the smaller in-row index
    f = _frame(list(range(10, 41)), extra={42: [(near, Z0), (-near, Z0)]})
    r = o.track_frame(*f, debug=True)
    d = r["debug"]
    k = int(np.flatnonzero(d["tl_nhits"] > 0)[0])
    assert d["tl_hits"][k][42] == 0


# --------------------------------------------------------------------------------------
# Selection (orc_select) on hand-built tracklets
# --------------------------------------------------------------------------------------
def _tl(rows_ids):
    h = np.full(NR, -1, np.int32)
    for r, c in rows_ids:
        h[r] = c
    return h


def _select(tls, ranks, n_clusters=1000, seed=0):
    o = oracle.Oracle(ROWS)
    hits = np.stack(tls)
    n = (hits >= 0).sum(axis=1)
    return o.select(n_clusters, n, ranks, hits, shuffle_seed=seed)


def _w(n, rank):
    return np.uint64((n << 32) | (0xFFFFFFFF - rank))


A30 = _tl([(r, r) for r in range(0, 30)])                                          # clusters 0..29
B30 = _tl([(r, r) for r in range(15, 30)] + [(r, 100 + r) for r in range(30, 45)])  # shares 15..29
B31 = _tl([(r, r) for r in range(15, 30)] + [(r, 100 + r) for r in range(30, 46)])


@pytest.mark.parametrize("seed", [0, 1, 99])
def test_equal_length_smaller_rank_wins(seed):
    W, wt, kept = _select([A30, B30], [0, 1], seed=seed)
    assert list(kept) == [30, 15]
    assert wt[0] == _w(30, 0) and wt[1] == _w(30, 1)
    assert W[20] == _w(30, 0) and W[135] == _w(30, 1) and W[5] == _w(30, 0)
    W, wt, kept = _select([A30, B30], [7, 3], seed=seed)
    assert list(kept) == [15, 30]
    assert W[20] == _w(30, 3)


@pytest.mark.parametrize("seed", [0, 5])
def test_longer_tracklet_wins_whatever_its_rank(seed):
    W, wt, kept = _select([A30, B31], [0, 1], seed=seed)
    assert list(kept) == [15, 31]
    assert W[20] == _w(31, 1)


def test_short_tracklets_take_no_part():
    C19 = _tl([(r, r) for r in range(0, 19)])
    W, wt, kept = _select([A30, C19], [5, 0])
    assert wt[1] == 0 and kept[1] == 0
    assert kept[0] == 30 and W[3] == _w(30, 5)
    W, _, _ = _select([C19], [0])
    assert not W.any()


@pytest.mark.parametrize("seed", [0, 3, 12345])
def test_one_pass_no_redistribution(seed):
    A = _tl([(r, r) for r in range(0, 40)])                                              # n 40, rank 2
    B = _tl([(r, r) for r in range(25, 40)] + [(r, 200 + r) for r in range(40, 55)])     # n 30, rank 0
    C = _tl([(r, 200 + r) for r in range(45, 55)] + [(r, 300 + r) for r in range(55, 70)])  # n 25, rank 1
    W, wt, kept = _select([A, B, C], [2, 0, 1], seed=seed)
    # A takes the 15 it shares with B; B keeps 15 and is rejected, yet still holds the 10
    # clusters it shares with C, so C keeps only its own 15 and is rejected too
    assert list(kept) == [40, 15, 15]
    assert W[250] == _w(30, 0) and W[360] == _w(25, 1) and W[30] == _w(40, 2)
