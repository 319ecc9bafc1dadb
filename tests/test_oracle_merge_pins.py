"""Pins of the oracle's merging across sector boundaries and of its refit across sector
frames, against facts that do not come from the oracle: the generator's closed-form
plane crossings in two sector frames, finite differences, the inverse rotation, noise-free
helices, the chi2 distribution of independent Gaussian estimates, and Monte-Carlo truth.
CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_2009_07515_amd import synth

W = math.pi / 9.0          # azimuth step between neighbouring sectors


def _orc(row_x, **kw):
    return oracle.Oracle(row_x, **kw)


def _majority(label, hit_off, hit_ids):
    lab = np.empty(len(hit_off) - 1, np.int64)
    pur = np.empty(len(hit_off) - 1)
    for t in range(len(hit_off) - 1):
        v, c = np.unique(label[hit_ids[hit_off[t]:hit_off[t + 1]]], return_counts=True)
        k = int(np.argmax(c))
        lab[t], pur[t] = v[k], c[k] / c.sum()
    return lab, pur


# --------------------------------------------------------------------------------------
# Rotation into the next sector's frame, then propagation in that frame, lands on the
# generator's closed-form crossing of the other sector's row plane.
# --------------------------------------------------------------------------------------
def test_rotation_matches_generator_closed_form(row_x):
    o = _orc(row_x)
    X = row_x.astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(11))
    n_checked = 0
    for _ in range(200):
        s = int(rng.integers(0, 18))
        a0, a1 = (s + 0.5) * W, (s + 1.5) * W
        phi0 = a0 + rng.uniform(-0.1, 0.15)
        pt = rng.uniform(0.15, 2.0)
        q = rng.choice([-1.0, 1.0])
        kappa = -synth.C_B * synth.B_Z * q / pt
        tgl = rng.uniform(-1, 1)
        zv = np.zeros(1)
        r1, r2 = sorted(rng.choice(152, 2, replace=False))
        ok1, y1, z1, sp1, _ = synth.plane_crossing(zv, zv, zv, np.array([phi0]), np.array([kappa]),
                                                   np.array([tgl]), a0, X[r1])
        ok2, y2, z2, sp2, _ = synth.plane_crossing(zv, zv, zv, np.array([phi0]), np.array([kappa]),
                                                   np.array([tgl]), a1, X[r2])
        if not (ok1[0] and ok2[0]) or abs(sp1[0]) > 0.9 or abs(sp2[0]) > 0.9:
            continue
        p = [y1[0], z1[0], sp1[0], tgl, q / pt]
        ok, xr, pr, _, _ = o.rotate(W, X[r1], p)
        if not ok:
            continue
        okp, p2, _, _ = o.propagate(xr, X[r2], pr)
        assert okp
        assert abs(p2[0] - y2[0]) < 1e-9 and abs(p2[1] - z2[0]) < 1e-9
        assert abs(p2[2] - sp2[0]) < 1e-12
        assert p2[3] == tgl and p2[4] == q / pt
        n_checked += 1
    assert n_checked > 40


# --------------------------------------------------------------------------------------
# Rotation Jacobian: rotating back is the inverse map, so the product of the two
# Jacobians is the identity; and propagate(rotate(p)) to a fixed plane differentiates to
# J_prop J_rot (central differences of the maps themselves).
# --------------------------------------------------------------------------------------
def test_rotation_jacobian_inverse_and_finite_differences(row_x):
    o = _orc(row_x)
    rng = np.random.Generator(np.random.PCG64(12))
    n_checked = 0
    for _ in range(200):
        p = np.array([rng.uniform(-30, 30), rng.uniform(-100, 100), rng.uniform(-0.7, 0.7),
                      rng.uniform(-1, 1), rng.uniform(-6, 6)])
        x = rng.uniform(90, 240)
        d = rng.choice([-W, W])
        ok, xr, pr, _, J = o.rotate(d, x, p)
        if not ok:
            continue
        okb, xb, pb, _, Jb = o.rotate(-d, xr, pr)
        assert okb
        assert abs(xb - x) < 1e-10 and np.allclose(pb, p, rtol=0, atol=1e-10)
        np.testing.assert_allclose(Jb @ J, np.eye(5), atol=1e-10)
        X1 = xr + rng.uniform(1.0, 8.0)
        okp, _, _, Jp = o.propagate(xr, X1, pr)
        if not okp:
            continue
        for j in range(5):
            eps = 1e-6 * max(1.0, abs(p[j]))
            f = []
            for sgn in (1, -1):
                q = p.copy()
                q[j] += sgn * eps
                okq, xq, pq, _, _ = o.rotate(d, x, q)
                okf, pf, _, _ = o.propagate(xq, X1, pq)
                assert okq and okf
                f.append(pf)
            fd = (f[0] - f[1]) / (2 * eps)
            np.testing.assert_allclose((Jp @ J)[:, j], fd, rtol=1e-6, atol=1e-7)
        n_checked += 1
    assert n_checked > 100


# --------------------------------------------------------------------------------------
# Fit across sector frames.  Noise-free helices that cross sector edges give back the
# generated state at their innermost cluster; with one sector the fit is the sector fit.
# --------------------------------------------------------------------------------------
def _noise_free_event(seed=77, n_primary=1500):
    return synth.config2_pbpb_event(seed=seed, n_primary=n_primary, sigma=0.0, noise_frac=0.0)


def _clusters_by_track(f):
    g = np.repeat(np.arange(36 * 152), np.diff(f.row_off))
    return g // 152, g % 152


def test_fit_across_sectors_recovers_truth(row_x):
    f = _noise_free_event()
    o = _orc(row_x)
    X = row_x.astype(np.float64)
    sec, row = _clusters_by_track(f)
    n_checked = 0
    for lab in np.unique(f.label[f.label >= 0])[:600]:
        idx = np.flatnonzero(f.label == lab)
        secs = np.unique(sec[idx])
        if len(secs) < 2 or len(np.unique(secs // 18)) > 1 or np.any(np.abs(f.truth_sphi[idx]) > 0.9):
            continue
        if min(np.sum(sec[idx] == s) for s in secs) < 10 or f.trk_secondary[lab]:
            continue
        rho = np.hypot(X[row[idx]], f.y[idx].astype(np.float64))
        idx = idx[np.argsort(rho)]
        ok, p, _, _ = o.fit_hits_sectors(X[row[idx]], f.y[idx], f.z[idx], sec[idx])
        assert ok
        i0 = idx[0]
        truth = [f.truth_y[i0], f.truth_z[i0], f.truth_sphi[i0], f.trk_tgl[lab], f.trk_qpt[lab]]
        assert abs(p[0] - truth[0]) < 2e-5 and abs(p[1] - truth[1]) < 2e-5
        assert abs(p[2] - truth[2]) < 2e-6 and abs(p[3] - truth[3]) < 2e-6
        assert abs(p[4] - truth[4]) < 1e-4 * max(1.0, abs(truth[4]))
        n_checked += 1
    assert n_checked > 50


def test_fit_in_one_sector_is_the_sector_fit(small_pbpb_frame, row_x):
    f = small_pbpb_frame
    o = _orc(row_x)
    r = o.track_frame(f.y, f.z, f.row_off)
    X = row_x.astype(np.float64)
    _, row = _clusters_by_track(f)
    for t in range(0, r["n_tracks"], 7):
        h = r["hit_ids"][r["hit_off"][t]:r["hit_off"][t + 1]]
        ok, p, Cv, chi2 = o.fit_hits_sectors(X[row[h]], f.y[h], f.z[h], np.full(len(h), r["sector"][t]))
        assert ok
        assert np.array_equal(p, r["params"][t]) and np.array_equal(Cv, r["cov"][t])
        assert chi2 == r["chi2"][t]


# --------------------------------------------------------------------------------------
# Merging on noise-free events: the segments of a helix split by a sector edge are joined
# (chi2 of the link near 0) and the merged fit returns the generated state.
# --------------------------------------------------------------------------------------
def test_merge_joins_noise_free_split_tracks(row_x):
    f = _noise_free_event()
    o = _orc(row_x)
    r = o.track_frame(f.y, f.z, f.row_off)
    m = o.merge_frame(f.y, f.z, f.row_off, r)
    lab, pur = _majority(f.label, r["hit_off"], r["hit_ids"])
    links = np.flatnonzero(m["next"] >= 0)
    assert len(links) > 500
    assert np.all(lab[links] == lab[m["next"][links]])
    assert np.all(m["link_chi2"][links] < 1.0)
    # MC tracks in several sector tracks of one side
    sec = r["sector"]
    split = 0
    joined = 0
    for L in np.unique(lab[pur == 1.0]):
        ts = np.flatnonzero((lab == L) & (pur == 1.0))
        if len(ts) < 2 or len(np.unique(sec[ts] // 18)) > 1:
            continue
        split += 1
        joined += len(np.unique(m["track_merged"][ts])) == 1
    assert split > 300 and joined >= 0.99 * split
    # merged fits equal the truth at the innermost cluster
    X = row_x.astype(np.float64)
    for k in np.flatnonzero(m["n_segments"] >= 2)[:200]:
        i0 = m["hit_ids"][m["hit_off"][k]]
        L = f.label[i0]
        p = m["params"][k]
        if np.any(np.abs(f.truth_sphi[f.label == L]) > 0.9) or f.trk_secondary[L]:
            continue
        assert abs(p[0] - f.truth_y[i0]) < 2e-5 and abs(p[1] - f.truth_z[i0]) < 2e-5
        assert abs(p[2] - f.truth_sphi[i0]) < 2e-6 and abs(p[3] - f.trk_tgl[L]) < 2e-6
        assert abs(p[4] - f.trk_qpt[L]) < 1e-4 * max(1.0, abs(f.trk_qpt[L]))
        assert m["x_ref"][k] == X[f.row_off.searchsorted(i0, side="right") - 1 - 152 * m["sector"][k]]


# --------------------------------------------------------------------------------------
# Structure of the merged output: a partition of the input tracks in chain order, merged
# tracks ordered by the index of their first (innermost) segment, single segments
# unchanged.
# --------------------------------------------------------------------------------------
def test_merge_output_invariants(small_pbpb_frame, row_x):
    f = small_pbpb_frame
    o = _orc(row_x)
    r = o.track_frame(f.y, f.z, f.row_off)
    m = o.merge_frame(f.y, f.z, f.row_off, r)
    T, M = r["n_tracks"], m["n_merged"]
    tm = m["track_merged"]
    assert np.all((tm >= 0) & (tm < M))
    assert np.array_equal(np.bincount(tm, minlength=M), m["n_segments"])
    assert m["n_hits"] == r["n_hits"] and np.sum(m["nhits"]) == r["n_hits"]
    assert np.array_equal(np.sort(m["hit_ids"]), np.sort(r["hit_ids"]))
    nxt = m["next"]
    # the first segment of each merged track: the member that no other member links to
    # (links of a chain whose refit failed stay in `next`, its segments stay apart)
    first = []
    for k in range(M):
        ts = np.flatnonzero(tm == k)
        first.append([t for t in ts if not np.any(nxt[ts] == t)][0])
    first = np.array(first)
    assert np.all(np.diff(first) > 0)
    for k in range(M):
        ts = np.flatnonzero(tm == k)
        # the chain from the first track, in link order, holds exactly these tracks
        chain = [first[k]]
        while nxt[chain[-1]] >= 0 and len(chain) < len(ts):
            chain.append(nxt[chain[-1]])
        assert sorted(chain) == ts.tolist()
        h = np.concatenate([r["hit_ids"][r["hit_off"][t]:r["hit_off"][t + 1]] for t in chain])
        assert np.array_equal(m["hit_ids"][m["hit_off"][k]:m["hit_off"][k + 1]], h)
        assert m["sector"][k] == r["sector"][chain[0]] and m["x_ref"][k] == r["x_ref"][chain[0]]
        assert m["ndf"][k] == 2 * m["nhits"][k] - 5
        if len(chain) == 1:
            assert np.array_equal(m["params"][k], r["params"][chain[0]])
            assert m["chi2"][k] == r["chi2"][chain[0]]
        for a, b in zip(chain[:-1], chain[1:]):
            assert r["sector"][b] // 18 == r["sector"][a] // 18
            assert (r["sector"][b] - r["sector"][a]) % 18 in (1, 17)
        assert abs(m["z_beam"][k] - o.beamline_z(m["x_ref"][k], m["params"][k])) == 0.0


# --------------------------------------------------------------------------------------
# Merging on the Pb-Pb event with noise: the chi2 of true links follows the chi2
# distribution of 5 degrees of freedom (mean 5, median 4.35), which needs correct
# covariances for the rotated outer state and the inner state; split tracks are
# rejoined and almost no link joins different particles.
# --------------------------------------------------------------------------------------
def test_merge_statistics_on_pbpb_event(cfg2_frame, row_x):
    f = cfg2_frame
    o = _orc(row_x)
    r = o.track_frame(f.y, f.z, f.row_off)
    m = o.merge_frame(f.y, f.z, f.row_off, r)
    lab, pur = _majority(f.label, r["hit_off"], r["hit_ids"])
    links = np.flatnonzero(m["next"] >= 0)
    true = (lab[links] == lab[m["next"][links]]) & (lab[links] >= 0)
    assert np.sum(~true) <= 0.002 * len(links)
    c = m["link_chi2"][links][true]
    assert 4.5 < c.mean() < 6.0 and 3.9 < np.median(c) < 5.2
    sec = r["sector"]
    split = joined = 0
    for L in np.unique(lab[(pur >= 0.9) & (lab >= 0)]):
        ts = np.flatnonzero((lab == L) & (pur >= 0.9))
        if len(ts) < 2 or len(np.unique(sec[ts] // 18)) > 1:
            continue
        split += 1
        joined += len(np.unique(m["track_merged"][ts])) == 1
    assert split > 3000 and joined >= 0.97 * split
    print(f"links {len(links)}, wrong {np.sum(~true)}, chi2 mean {c.mean():.2f} median {np.median(c):.2f}, "
          f"split {split}, rejoined {joined}")


# --------------------------------------------------------------------------------------
# Selection among competing links, on hand-built inputs: two copies of the inner segment
# of a split noise-free helix compete for its outer segment.  The copy whose outer state
# is displaced by 0.1 cm in y (a worse chi2) loses to the exact one whatever the order;
# two exact copies tie and the smaller index wins.
# --------------------------------------------------------------------------------------
def test_merge_keeps_the_best_of_competing_tracks(row_x):
    f = _noise_free_event()
    o = _orc(row_x)
    r = o.track_frame(f.y, f.z, f.row_off)
    m = o.merge_frame(f.y, f.z, f.row_off, r)
    a = int(np.flatnonzero((m["next"] >= 0) & (m["next"][np.maximum(m["next"], 0)] < 0))[0])
    b = int(m["next"][a])

    def build(order, shift):
        tr = {k: [] for k in ("params", "cov", "x_ref", "chi2", "ndf", "nhits", "sector",
                              "params_outer", "cov_outer")}
        hits, off = [], [0]
        for t, dy in zip(order, shift):
            for k in tr:
                tr[k].append(np.array(r[k][t], copy=True))
            tr["params_outer"][-1][0] += dy
            h = r["hit_ids"][r["hit_off"][t]:r["hit_off"][t + 1]]
            hits.append(h)
            off.append(off[-1] + len(h))
        tr = {k: np.array(v) for k, v in tr.items()}
        tr.update(n_tracks=len(order), n_hits=off[-1], hit_off=np.array(off, np.int64),
                  hit_ids=np.concatenate(hits))
        return o.merge_frame(f.y, f.z, f.row_off, tr)

    # displaced copy first, exact copy second, outer segment last
    mm = build([a, a, b], [0.1, 0.0, 0.0])
    assert list(mm["next"]) == [-1, 2, -1]
    assert mm["n_merged"] == 2 and list(mm["n_segments"]) == [1, 2]
    # exact copy first
    mm = build([a, a, b], [0.0, 0.1, 0.0])
    assert list(mm["next"]) == [2, -1, -1]
    # two exact copies: equal chi2, the smaller index wins
    mm = build([a, a, b], [0.0, 0.0, 0.0])
    assert list(mm["next"]) == [2, -1, -1]
