"""Parity of the HIP merge (tpcsf_merge through the C ABI) with the oracle's merge.

Contract: the links between sector tracks, the merged tracks' composition, order and hit
lists, and the input-to-merged map are identical to the oracle's; merged parameters are
within 1e-4 of the oracle's, |dp_i| <= 1e-4 * max(|p_i|, f_i) with floors
f = (10 cm, 10 cm, 0.1, 0.1, 0.1 c/GeV), covariance diagonals alike, chi2 to 1e-6.

The gate and chi2 cuts are binary64 decisions whose operands the GPU rounds in its own
order, so a pair lying within rounding of a cut may be decided the other way.  Such a
link difference is accepted, and counted, only if the oracle itself takes the GPU's
decision for that outer end once its cuts move by a small relative band (1e-12 when both
merge the same tracks; 1e-8 when the oracle merges its own tracks, whose parameters
differ from the GPU's by ~1e-9); the merged tracks holding those ends are then left out
of the element-wise comparison.
"""
import numpy as np
import pytest

import oracle
from conftest import CFG3_TUNING
from paper_2009_07515_amd import synth

pytestmark = pytest.mark.gpu

FLOORS = np.array([10.0, 10.0, 0.1, 0.1, 0.1])


def _np(res):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items()}


def _gpu_tracks_and_merge(f, n_tf=1, trk=None, cap_merged=None, hit_rec=False):
    from paper_2009_07515_amd import tpcsf
    trk = trk or tpcsf.Tracker(synth.row_x())
    fr = tpcsf.DeviceFrame.from_numpy(f.y, f.z, f.row_off, n_tf=n_tf) if n_tf > 1 else \
        tpcsf.DeviceFrame.from_numpy(f.y, f.z, f.row_off)
    tb = tpcsf.TrackBuffers(fr.n_clusters, outer=True, hit_rec=hit_rec)
    tracks = _np(trk.track(fr, out=tb))
    out = None
    if cap_merged is not None:
        out = tpcsf.MergedBuffers(tb)
        out.cap_merged = cap_merged
    merged = _np(trk.merge(fr, tb, out=out))
    return trk, tracks, merged


def _close(a, b):
    tol = 1e-4 * np.maximum(np.abs(b), FLOORS)
    err = np.abs(a - b)
    assert np.all(err <= tol), (err / tol).max(axis=0)


def _members(m):
    """Input tracks of every merged track, in chain order (head first)."""
    T = len(m["track_merged"])
    nxt = np.asarray(m["next"])
    has_prev = np.zeros(T, bool)
    has_prev[nxt[nxt >= 0]] = True
    chains = {}
    for h in np.flatnonzero(~has_prev):
        c, t = [], int(h)
        while t >= 0:
            c.append(t)
            t = int(nxt[t])
        chains[int(m["track_merged"][h])] = tuple(c)
    return chains


def _borderline_links(g, o, frame, tracks, row_x, band):
    """Outer ends whose GPU link differs from the oracle's; each must be reproduced by the
    oracle with its gate window or chi2 cut moved by `band` relative."""
    diff = np.flatnonzero(g["next"] != o["next"])
    if diff.size == 0:
        return diff
    p = oracle.DEFAULT_PARAMS
    alt = []
    for key in ("merge_window", "merge_chi2"):
        for f in (1 - band, 1 + band):
            oo = oracle.Oracle(row_x, params={key: p[key] * f})
            alt.append(oo.merge_frame(frame.y, frame.z, frame.row_off, tracks)["next"])
    for a in diff:
        assert any(n[a] == g["next"][a] for n in alt), f"outer end {a}: link {g['next'][a]} vs {o['next'][a]}"
    return diff


def _check_same_merge(g, o, label="", frame=None, tracks=None, row_x=None, band=1e-12):
    diff = np.zeros(0, np.int64)
    if frame is not None and not np.array_equal(g["next"], o["next"]):
        diff = _borderline_links(g, o, frame, tracks, row_x, band)
    print(f"{label}: {diff.size} link decisions within rounding of a cut")
    if diff.size == 0:
        assert g["n_merged"] == o["n_merged"], label
        assert np.array_equal(g["next"], o["next"]), label
        assert np.array_equal(g["track_merged"], o["track_merged"]), label
        assert np.array_equal(g["hit_off"], o["hit_off"]), label
        assert np.array_equal(g["hit_ids"].astype(np.int64), o["hit_ids"]), label
        gi = oi = np.arange(g["n_merged"])
    else:
        # compare the merged tracks made of the same input tracks, none of them touched
        touched = set(int(a) for a in diff)
        for a in diff:
            touched.update(int(v) for v in (g["next"][a], o["next"][a]) if v >= 0)
        cg, co = _members(g), _members(o)
        by_members = {c: k for k, c in co.items()}
        gi, oi = [], []
        for k in sorted(cg):
            c = cg[k]
            if touched.isdisjoint(c):
                assert c in by_members, (label, c)
                gi.append(k)
                oi.append(by_members[c])
        gi, oi = np.array(gi, np.int64), np.array(oi, np.int64)
        assert len(gi) >= len(cg) - 4 * diff.size
        for kg, ko in zip(gi, oi):
            hg = g["hit_ids"][g["hit_off"][kg]:g["hit_off"][kg + 1]].astype(np.int64)
            ho = o["hit_ids"][o["hit_off"][ko]:o["hit_off"][ko + 1]]
            assert np.array_equal(hg, ho), label
    for k in ("n_segments", "sector", "nhits", "ndf"):
        assert np.array_equal(g[k][gi], o[k][oi]), (label, k)
    assert np.array_equal(g["x_ref"][gi], o["x_ref"][oi])
    _close(g["params"][gi], o["params"][oi])
    sg, so = np.sqrt(g["cov"][gi][:, [0, 2, 5, 9, 14]]), np.sqrt(o["cov"][oi][:, [0, 2, 5, 9, 14]])
    assert np.all(np.abs(sg - so) <= 1e-4 * so)
    assert np.allclose(g["chi2"][gi], o["chi2"][oi], rtol=1e-6, atol=1e-9)
    zg, zo = g["z_beam"][gi], o["z_beam"][oi]
    assert np.all(np.abs(zg - zo) <= 1e-4 * np.maximum(np.abs(zo), 10.0))
    links = (o["next"] >= 0) & (g["next"] == o["next"])
    assert np.allclose(g["link_chi2"][links], o["link_chi2"][links], rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("which,rec", [("small", False), ("small", True), ("cfg2", True)])
def test_merge_parity_with_oracle(which, rec, small_pbpb_frame, cfg2_frame, row_x):
    """rec: the refit reads the tracking call's per-hit records instead of the clusters."""
    f = {"small": small_pbpb_frame, "cfg2": cfg2_frame}[which]
    _, tracks, merged = _gpu_tracks_and_merge(f, hit_rec=rec)
    o = oracle.Oracle(row_x)
    r = o.track_frame(f.y, f.z, f.row_off)
    assert tracks["n_tracks"] == r["n_tracks"]
    _close(tracks["params_outer"], r["params_outer"])
    so = np.sqrt(r["cov_outer"][:, [0, 2, 5, 9, 14]])
    assert np.all(np.abs(np.sqrt(tracks["cov_outer"][:, [0, 2, 5, 9, 14]]) - so) <= 1e-4 * so)
    m = o.merge_frame(f.y, f.z, f.row_off, r)
    # the oracle merges its own tracks, whose parameters differ from the GPU's by ~1e-9
    _check_same_merge(merged, m, which, f, r, row_x, band=1e-8)
    n_multi = int(np.sum(merged["n_segments"] >= 2))
    print(f"{which}: {tracks['n_tracks']} sector tracks -> {merged['n_merged']} merged, {n_multi} of several")
    assert n_multi > 0


def test_merge_of_the_full_time_frame_equals_oracle_merge_of_the_same_tracks(cfg3_frame, row_x):
    """The 2 ms Pb-Pb frame (27M clusters) in the benchmark's configuration: the oracle
    merges the GPU's own sector tracks (its tracking of this frame takes minutes), and the
    GPU merge must equal that merge."""
    from paper_2009_07515_amd import tpcsf
    f = cfg3_frame
    trk = tpcsf.Tracker(synth.row_x(), tuning=CFG3_TUNING)
    _, tracks, merged = _gpu_tracks_and_merge(f, trk=trk, hit_rec=True)
    o = oracle.Oracle(row_x)
    m = o.merge_frame(f.y, f.z, f.row_off, tracks)
    _check_same_merge(merged, m, "cfg3", f, tracks, row_x)
    print(f"cfg3: {tracks['n_tracks']} sector tracks -> {merged['n_merged']} merged")


def test_merge_of_a_batch_equals_frames_alone():
    frames = [synth.config2_pbpb_event(seed=700 + i, n_primary=300 + 500 * i) for i in range(3)]
    y, z, ro = synth.concat_frames(frames)
    batch = type("F", (), dict(y=y, z=z, row_off=ro))
    trk, tb, mb = _gpu_tracks_and_merge(batch, n_tf=3)
    base_t = base_m = base_c = 0
    for i, f in enumerate(frames):
        _, t1, m1 = _gpu_tracks_and_merge(f, trk=trk)
        sel = np.flatnonzero(mb["tf"] == i)
        assert len(sel) == m1["n_merged"]
        for k in ("params", "cov", "chi2", "n_segments", "nhits", "sector", "z_beam"):
            assert np.array_equal(mb[k][sel], m1[k]), (i, k)
        h = np.concatenate([mb["hit_ids"][mb["hit_off"][j]:mb["hit_off"][j + 1]] for j in sel])
        assert np.array_equal(h - base_c, m1["hit_ids"])
        tm = mb["track_merged"][base_t:base_t + t1["n_tracks"]]
        assert np.array_equal(tm - base_m, m1["track_merged"])
        base_t += t1["n_tracks"]
        base_m += m1["n_merged"]
        base_c += f.n_clusters


def test_merge_capacity_and_invalid_input(small_pbpb_frame):
    from paper_2009_07515_amd import tpcsf
    f = small_pbpb_frame
    trk, tracks, full = _gpu_tracks_and_merge(f)
    with pytest.raises(tpcsf.TpcsfError) as e:
        _gpu_tracks_and_merge(f, trk=trk, cap_merged=5)
    assert e.value.status == tpcsf.E_CAPACITY
    # tracks out of (time frame, sector) order are rejected on the device
    fr = tpcsf.DeviceFrame.from_numpy(f.y, f.z, f.row_off)
    tb = tpcsf.TrackBuffers(fr.n_clusters, outer=True)
    trk.track(fr, out=tb)
    T = int(tb.n_tracks.item())
    tb.sector[:T] = tb.sector[:T].flip(0)
    with pytest.raises(tpcsf.TpcsfError) as e:
        trk.merge(fr, tb)
    assert e.value.status == tpcsf.E_INVALID
    # outer states are required
    tb2 = tpcsf.TrackBuffers(fr.n_clusters)
    trk.track(fr, out=tb2)
    with pytest.raises(tpcsf.TpcsfError) as e:
        trk.merge(fr, tb2, out=tpcsf.MergedBuffers(tb2))
    assert e.value.status == tpcsf.E_INVALID
    # the context keeps working
    _, _, again = _gpu_tracks_and_merge(f, trk=trk)
    assert np.array_equal(again["hit_ids"], full["hit_ids"])
