"""Parity of the HIP merge (tpcsf_merge through the C ABI) with the oracle's merge.

Contract: the links between sector tracks, the merged tracks' composition, order and hit
lists, and the input-to-merged map are identical to the oracle's; merged parameters are
within 1e-4 of the oracle's, |dp_i| <= 1e-4 * max(|p_i|, f_i) with floors
f = (10 cm, 10 cm, 0.1, 0.1, 0.1 c/GeV), covariance diagonals alike, chi2 to 1e-6.
"""
import numpy as np
import pytest

import oracle
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


def _check_same_merge(g, o, label=""):
    assert g["n_merged"] == o["n_merged"], label
    assert np.array_equal(g["next"], o["next"]), label
    assert np.array_equal(g["track_merged"], o["track_merged"]), label
    assert np.array_equal(g["hit_off"], o["hit_off"]), label
    assert np.array_equal(g["hit_ids"].astype(np.int64), o["hit_ids"]), label
    for k in ("n_segments", "sector", "nhits", "ndf"):
        assert np.array_equal(g[k], o[k]), (label, k)
    assert np.array_equal(g["x_ref"], o["x_ref"])
    _close(g["params"], o["params"])
    sg, so = np.sqrt(g["cov"][:, [0, 2, 5, 9, 14]]), np.sqrt(o["cov"][:, [0, 2, 5, 9, 14]])
    assert np.all(np.abs(sg - so) <= 1e-4 * so)
    assert np.allclose(g["chi2"], o["chi2"], rtol=1e-6, atol=1e-9)
    assert np.all(np.abs(g["z_beam"] - o["z_beam"]) <= 1e-4 * np.maximum(np.abs(o["z_beam"]), 10.0))
    links = o["next"] >= 0
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
    _check_same_merge(merged, m, which)
    n_multi = int(np.sum(merged["n_segments"] >= 2))
    print(f"{which}: {tracks['n_tracks']} sector tracks -> {merged['n_merged']} merged, {n_multi} of several")
    assert n_multi > 0


def test_merge_of_the_full_time_frame_equals_oracle_merge_of_the_same_tracks(row_x):
    """The 2 ms Pb-Pb frame (27M clusters) in the benchmark's configuration: the oracle
    merges the GPU's own sector tracks (its tracking of this frame takes minutes), and the
    GPU merge must equal that merge."""
    from paper_2009_07515_amd import tpcsf
    f = synth.config3_time_frame()
    trk = tpcsf.Tracker(synth.row_x(), tuning=dict(bin_y=2.0, bin_z=4.0, cap_mul=4, block=512, tl_block=256,
                                                    chunk=2))
    _, tracks, merged = _gpu_tracks_and_merge(f, trk=trk, hit_rec=True)
    o = oracle.Oracle(row_x)
    m = o.merge_frame(f.y, f.z, f.row_off, tracks)
    _check_same_merge(merged, m, "cfg3")
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
