"""Parity of the HIP path (libtpcsf through its C ABI) with the reference oracle.

Contract:
  * grid tables (extents, bin sizes, ny/nz, bin_start, perm) and the raw and cleaned
    neighbour links are bit-exact with the oracle (both are defined in binary32);
  * chain bottoms (starts) and their rank order are identical;
  * tracks: same hit lists as the FP64 oracle, and parameters within 1e-4 relative of the
    FP64 oracle refit on the GPU's own hit lists, |dp_i| <= 1e-4 * max(|p_i|, f_i) with
    floors f = (10 cm, 10 cm, 0.1, 0.1, 0.1 c/GeV); covariance diagonals alike;
  * efficiency and fake rate within 0.001 (absolute) of the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
import truthmatch
from paper_2009_07515_amd import synth

pytestmark = pytest.mark.gpu

FLOORS = np.array([10.0, 10.0, 0.1, 0.1, 0.1])


def _tracker(**kw):
    from paper_2009_07515_amd import tpcsf
    return tpcsf.Tracker(synth.row_x(), **kw)


def _frame(f):
    from paper_2009_07515_amd import tpcsf
    return tpcsf.DeviceFrame.from_numpy(f.y, f.z, f.row_off)


def _np(res):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items()}


def _check_grid_and_links(f, dbg, ref):
    d = ref["debug"]
    R = 36 * 152
    assert np.array_equal(dbg["row_lo"][:, 0], d["g_ylo"]) and np.array_equal(dbg["row_lo"][:, 1], d["g_zlo"])
    assert np.array_equal(dbg["row_bin"][:, 0], d["g_by"]) and np.array_equal(dbg["row_bin"][:, 1], d["g_bz"])
    assert np.array_equal(dbg["row_nb"][:, 0], d["g_ny"]) and np.array_equal(dbg["row_nb"][:, 1], d["g_nz"])
    assert np.array_equal(dbg["perm"], d["perm"])
    # bin_start: per row at the library's own base, vs the oracle's concatenation
    bb = 2 * f.row_off[:R] + 65 * np.arange(R)
    for g in range(R):
        nb = int(d["g_ny"][g]) * int(d["g_nz"][g]) + 1
        a = dbg["bin_start"][bb[g]:bb[g] + nb]
        b = d["bin_start"][d["g_bin_base"][g]:d["g_bin_base"][g] + nb]
        assert np.array_equal(a, b), g
    for k in ("up", "dn", "cup", "cdn"):
        assert np.array_equal(dbg[k], d[k]), k
    starts = np.flatnonzero(d["start"])
    gpu_starts = f.row_off[dbg["start_row"]] + dbg["start_idx"]
    assert np.array_equal(gpu_starts, starts)


def _check_tracks(f, res, ref, o64, label_check=True):
    T = res["n_tracks"]
    assert T == ref["n_tracks"]
    assert np.array_equal(res["hit_off"], ref["hit_off"])
    assert np.array_equal(res["hit_ids"].astype(np.int64), ref["hit_ids"])
    assert np.array_equal(res["cluster_track"], ref["cluster_track"])
    assert np.array_equal(res["sector"], ref["sector"])
    assert np.array_equal(res["nhits"], ref["nhits"]) and np.array_equal(res["ndf"], ref["ndf"])
    assert np.array_equal(res["x_ref"], ref["x_ref"])
    p, q = res["params"], ref["params"]
    tol = 1e-4 * np.maximum(np.abs(q), FLOORS)
    err = np.abs(p - q)
    assert np.all(err <= tol), (err / tol).max(axis=0)
    sg, sr = np.sqrt(res["cov"][:, [0, 2, 5, 9, 14]]), np.sqrt(ref["cov"][:, [0, 2, 5, 9, 14]])
    assert np.all(np.abs(sg - sr) <= 1e-4 * sr)
    assert np.allclose(res["chi2"], ref["chi2"], rtol=1e-6, atol=1e-9)
    _check_zbeam(res, ref)
    return err / np.maximum(np.abs(q), FLOORS)


def _check_zbeam(res, ref, orc=None):
    """z at the beam line: the oracle's function of the GPU's own (x_ref, params) to rounding
    (both FP64; atan2 and sqrt may differ by an ulp, which the arc length 1/kappa scales
    to well below 1e-7 cm); and the oracle's own estimate within the tolerance of the z
    parameter, 1e-4 * max(|z|, 10 cm)."""
    zg, zo = res["z_beam"], ref["z_beam"]
    assert zg.shape == zo.shape and np.all(np.isfinite(zg))
    assert np.all(np.abs(zg - zo) <= 1e-4 * np.maximum(np.abs(zo), 10.0)), np.abs(zg - zo).max()
    orc = orc or oracle.Oracle(synth.row_x())
    own = np.array([orc.beamline_z(res["x_ref"][t], res["params"][t]) for t in range(len(zg))])
    assert np.all(np.abs(zg - own) <= 1e-7 + 1e-12 * np.abs(own)), np.abs(zg - own).max()


@pytest.mark.parametrize("which", ["cfg1", "small", "cfg2"])
def test_parity_with_oracle(which, cfg1_frame, small_pbpb_frame, cfg2_frame, row_x):
    f = {"cfg1": cfg1_frame, "small": small_pbpb_frame, "cfg2": cfg2_frame}[which]
    trk = _tracker()
    fr = _frame(f)
    res = _np(trk.track(fr, mode="batch"))
    dbg = trk.debug(fr)
    ref = oracle.Oracle(row_x).track_frame(f.y, f.z, f.row_off, debug=True)
    _check_grid_and_links(f, dbg, ref)
    # tracklet sizes per start (FP64 on both sides: identical decisions)
    assert np.array_equal(dbg["tl_nhits"], ref["debug"]["tl_nhits"])
    # the same Kalman steps: propagations and updates of the tracklets and of the final
    # fit, chi2 evaluations; clusters inside the follow windows (a window edge computed from
    # covariances that differ by rounding may, rarely, take or leave one cluster)
    w_g, w_o = dbg["work"], ref["debug"]["work"]
    assert np.array_equal(w_g[[0, 1, 3, 4, 5]], w_o[[0, 1, 3, 4, 5]]), (w_g, w_o)
    assert abs(int(w_g[2]) - int(w_o[2])) <= 1e-6 * w_o[2] + 2, (w_g, w_o)
    rel = _check_tracks(f, res, ref, None)
    print(f"{which}: {res['n_tracks']} tracks, max rel param err per parameter {rel.max(axis=0)}")
    m_g = truthmatch.match(f.label, f.row_off, res["hit_off"], res["hit_ids"], res["sector"])
    m_o = truthmatch.match(f.label, f.row_off, ref["hit_off"], ref["hit_ids"], ref["sector"])
    assert abs(m_g["efficiency"] - m_o["efficiency"]) <= 1e-3
    assert abs(m_g["fake_rate"] - m_o["fake_rate"]) <= 1e-3


def test_params_match_fp64_refit_of_gpu_hits(small_pbpb_frame, row_x):
    """Independent of decisions: refit each GPU track's own clusters with the FP64 oracle."""
    f = small_pbpb_frame
    res = _np(_tracker().track(_frame(f)))
    o = oracle.Oracle(row_x)
    X = row_x.astype(np.float64)
    g_of = np.repeat(np.arange(36 * 152), np.diff(f.row_off))
    worst = np.zeros(5)
    for t in range(res["n_tracks"]):
        h = res["hit_ids"][res["hit_off"][t]:res["hit_off"][t + 1]]
        ok, p, c, chi2, _ = o.fit_hits(X[g_of[h] % 152], f.y[h], f.z[h])
        assert ok
        rel = np.abs(res["params"][t] - p) / np.maximum(np.abs(p), FLOORS)
        worst = np.maximum(worst, rel)
    assert np.all(worst <= 1e-4), worst
    print("max relative parameter error vs FP64 refit:", worst)


def test_plain_equals_batch_and_is_deterministic(small_pbpb_frame):
    f = small_pbpb_frame
    trk = _tracker()
    fr = _frame(f)
    a = _np(trk.track(fr, mode="plain"))
    b = _np(trk.track(fr, mode="batch"))
    c = _np(trk.track(fr, mode="batch"))
    for k in ("hit_off", "hit_ids", "params", "cov", "chi2", "cluster_track", "sector", "tf", "z_beam"):
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(b[k], c[k]), k
    # the optional outputs (outer states, per-hit records) in both forms
    from paper_2009_07515_amd import tpcsf
    opt = []
    for mode in ("plain", "batch"):
        ob = tpcsf.TrackBuffers(fr.n_clusters, outer=True, hit_rec=True)
        res = _np(trk.track(fr, mode=mode, out=ob))
        opt.append((res, ob.hit_rec[:res["n_hits"]].cpu().numpy()))
    for k in ("params_outer", "cov_outer", "hit_ids", "params"):
        assert np.array_equal(opt[0][0][k], opt[1][0][k]), k
    assert np.array_equal(opt[0][1], opt[1][1])
    assert np.array_equal(opt[1][0]["params"], b["params"])
    # the optional per-hit records: the clusters' coordinates, row planes and indices
    tb = tpcsf.TrackBuffers(fr.n_clusters, hit_rec=True)
    d = _np(trk.track(fr, out=tb))
    H = d["n_hits"]
    rec = tb.hit_rec[:H].cpu().numpy()
    h = d["hit_ids"]
    assert np.array_equal(rec[:, 3].view(np.int32), h)
    assert np.array_equal(rec[:, 0], f.y[h]) and np.array_equal(rec[:, 1], f.z[h])
    g = np.repeat(np.arange(len(f.row_off) - 1), np.diff(f.row_off))
    assert np.array_equal(rec[:, 2], synth.row_x()[g[h] % 152])
    assert np.array_equal(d["hit_ids"], b["hit_ids"])


def test_multi_frame_batch_equals_frames_alone():
    from paper_2009_07515_amd import tpcsf
    frames = [synth.config2_pbpb_event(seed=900 + i, n_primary=300 + 400 * i) for i in range(3)]
    y, z, ro = synth.concat_frames(frames)
    trk = _tracker()
    both = _np(trk.track(tpcsf.DeviceFrame.from_numpy(y, z, ro, n_tf=3)))
    base_c, base_t = 0, 0
    for i, f in enumerate(frames):
        one = _np(trk.track(_frame(f)))
        sel = both["tf"] == i
        assert sel.sum() == one["n_tracks"]
        idx = np.flatnonzero(sel)
        assert np.array_equal(both["params"][idx], one["params"])
        assert np.array_equal(both["z_beam"][idx], one["z_beam"])
        for t in range(one["n_tracks"]):
            hb = both["hit_ids"][both["hit_off"][idx[t]]:both["hit_off"][idx[t] + 1]]
            ho = one["hit_ids"][one["hit_off"][t]:one["hit_off"][t + 1]]
            assert np.array_equal(hb - base_c, ho)
        ct = both["cluster_track"][base_c:base_c + f.n_clusters]
        assert np.array_equal(np.where(ct >= 0, ct - base_t, -1), one["cluster_track"])
        base_c += f.n_clusters
        base_t += one["n_tracks"]


@pytest.mark.parametrize("tun", [dict(bin_y=0.5, bin_z=0.5, block=64, tl_block=64, chunk=4),
                                 dict(bin_y=7.0, bin_z=30.0, cap_mul=1, cap_add=8, block=1024, tl_block=128),
                                 dict(bin_y=1.0, bin_z=4.0, cap_mul=4, chunk=2)])
def test_tuning_does_not_change_tracks(small_pbpb_frame, tun):
    f = small_pbpb_frame
    fr = _frame(f)
    ref = _np(_tracker().track(fr))
    got = _np(_tracker(tuning=tun).track(fr))
    for k in ("hit_off", "hit_ids", "params", "cov", "cluster_track", "z_beam"):
        assert np.array_equal(ref[k], got[k]), k


def test_edge_cases(row_x):
    from paper_2009_07515_amd import tpcsf
    trk = _tracker()
    R = 36 * 152
    # empty frame
    res = _np(trk.track(tpcsf.DeviceFrame.from_numpy(np.zeros(0), np.zeros(0), np.zeros(R + 1, np.int64))))
    assert res["n_tracks"] == 0 and res["n_hits"] == 0
    # single clusters, all in one row, and a frame of pure noise
    rng = np.random.Generator(np.random.PCG64(3))
    # a row too large for the grid's on-chip tables, and rows with a crowded bin
    # (hundreds of identical clusters, and a handful of duplicates) beside ordinary rows
    big = np.eye(1, R, 200, dtype=np.int64)[0] * 40000
    crowd = rng.integers(0, 6, R)
    crowd[300:303] = 700
    for counts in (np.ones(R, np.int64), np.eye(1, R, 77, dtype=np.int64)[0] * 3000,
                   rng.integers(0, 6, R), big, crowd):
        n = int(counts.sum())
        ro = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        y = rng.uniform(-15, 15, n).astype(np.float32)
        z = rng.uniform(-250, 250, n).astype(np.float32)
        if counts is big:
            z *= 10.0        # 40000 bins: more than the on-chip tables hold
        if counts is crowd:
            for g, k in ((300, 500), (301, 60), (302, 66)):
                y[ro[g]:ro[g] + k] = 1.25
                z[ro[g]:ro[g] + k] = -7.5
        res = _np(trk.track(tpcsf.DeviceFrame.from_numpy(y, z, ro)))
        dbg = trk.debug(tpcsf.DeviceFrame.from_numpy(y, z, ro))
        ref = oracle.Oracle(row_x).track_frame(y, z, ro, debug=True)
        assert res["n_tracks"] == ref["n_tracks"]
        for k in ("up", "dn", "cup", "cdn", "perm"):
            assert np.array_equal(dbg[k], ref["debug"][k])


def test_selection_in_a_row_beyond_the_on_chip_weights(small_pbpb_frame, row_x):
    """A row of 13,000 clusters (more than the selection kernel reduces in LDS, so its
    weights take the global-atomics path) that the tracks of the event cross: the same
    tracks, hit lists and parameters as the oracle."""
    from paper_2009_07515_amd import tpcsf
    f = small_pbpb_frame
    g = 60                                   # sector 0, row 60
    a, b = int(f.row_off[g]), int(f.row_off[g + 1])
    rng = np.random.Generator(np.random.PCG64(17))
    n_add = 13000 - (b - a)
    x = float(row_x[60])
    ya = rng.uniform(-x * np.tan(np.pi / 18), x * np.tan(np.pi / 18), n_add).astype(np.float32)
    za = rng.uniform(0.0, 250.0, n_add).astype(np.float32)
    y = np.concatenate([f.y[:b], ya, f.y[b:]]).astype(np.float32)
    z = np.concatenate([f.z[:b], za, f.z[b:]]).astype(np.float32)
    ro = f.row_off.copy()
    ro[g + 1:] += n_add
    assert ro[g + 1] - ro[g] == 13000
    trk = _tracker()
    res = _np(trk.track(tpcsf.DeviceFrame.from_numpy(y, z, ro)))
    ref = oracle.Oracle(row_x).track_frame(y, z, ro)
    in_row = int(((res["hit_ids"] >= ro[g]) & (res["hit_ids"] < ro[g + 1])).sum())
    assert res["n_tracks"] > 100 and in_row > 10
    print(f"{res['n_tracks']} tracks, {in_row} of their clusters in the 13,000-cluster row", flush=True)
    _check_tracks(None, res, ref, None)


def test_capacity_and_invalid_inputs(small_pbpb_frame):
    from paper_2009_07515_amd import tpcsf
    f = small_pbpb_frame
    trk = _tracker()
    fr = _frame(f)
    full = _np(trk.track(fr))
    assert full["n_tracks"] > 5
    small = tpcsf.TrackBuffers(f.n_clusters, cap_tracks=3)
    with pytest.raises(tpcsf.TpcsfError) as e:
        trk.track(fr, out=small)
    assert e.value.status == tpcsf.E_CAPACITY
    assert int(small.n_tracks.item()) == full["n_tracks"]          # required size reported
    # the context keeps working afterwards
    again = _np(trk.track(fr))
    assert np.array_equal(again["hit_ids"], full["hit_ids"])
    # non-finite coordinates are reported at sync
    y = f.y.copy()
    y[10] = np.nan
    with pytest.raises(tpcsf.TpcsfError) as e:
        trk.track(tpcsf.DeviceFrame.from_numpy(y, f.z, f.row_off))
    assert e.value.status == tpcsf.E_INVALID
    # malformed offsets are rejected before any launch
    ro = f.row_off.copy()
    ro[5], ro[6] = ro[6], ro[5] + 1
    with pytest.raises(tpcsf.TpcsfError) as e:
        trk.track(tpcsf.DeviceFrame.from_numpy(f.y, f.z, ro))
    assert e.value.status == tpcsf.E_INVALID
    # budget smaller than the scratch of one frame
    tight = _tracker(hbm_budget=1 << 20)
    with pytest.raises(tpcsf.TpcsfError) as e:
        tight.track(fr)
    assert e.value.status == tpcsf.E_NOMEM
