"""The uneven batch: 64 time frames, pp-like (0.5 ms at 500 kHz) and Pb-Pb-like (0.5-2 ms
at 50 kHz) alternating, about 0.6G clusters with a per-sector occupancy spread of more
than 20x, tracked in one batched call (one launch per stage over all 64 x 36 sectors, the
tracklet stage from the persistent work queue, the sequence replayed from a HIP graph).

Contract: every frame's tracks, hit lists, cluster map and parameters in the batch are
byte-identical to that frame tracked alone; a pp frame and the smallest Pb-Pb frame match
the FP64 oracle (same hit lists, parameters within |dp_i| <= 1e-4 max(|p_i|, f_i),
efficiency and fake rate within 0.001)."""
import numpy as np
import pytest

import oracle_sectors
import truthmatch
from conftest import CFG3_GRID, CFG3_TUNING
from paper_2009_07515_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]

FLOORS = np.array([10.0, 10.0, 0.1, 0.1, 0.1])


def _np(res):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items()}


def test_uneven_batch_of_64_frames(cfg4_frames, row_x):
    import torch
    from paper_2009_07515_amd import tpcsf
    frames = cfg4_frames
    sizes = np.array([f.n_clusters for f in frames])
    y, z, ro = synth.concat_frames(frames)
    n = int(y.shape[0])
    sec = np.diff(ro[::152])
    print(f"cfg4: {len(frames)} frames, {n} clusters (frames {sizes.min()}..{sizes.max()}, sectors "
          f"{sec.min()}..{sec.max()})", flush=True)
    torch.cuda.empty_cache()
    trk = tpcsf.Tracker(row_x, tuning=CFG3_TUNING)
    trk.reserve(n, len(frames))
    print(f"arena {trk.arena_bytes(n, len(frames)) / 2**30:.1f} GiB", flush=True)
    fr = tpcsf.DeviceFrame.from_numpy(y, z, ro, n_tf=len(frames))
    res = _np(trk.track(fr, mode="batch"))
    again = _np(trk.track(fr, mode="batch"))           # graph replay
    for k in ("hit_ids", "params", "cluster_track"):
        assert np.array_equal(res[k], again[k]), k
    del again
    print(f"batch: {res['n_tracks']} tracks", flush=True)

    single = tpcsf.Tracker(row_x, tuning=CFG3_TUNING)
    base_c = base_t = 0
    alone = {}
    for i, f in enumerate(frames):
        r1 = _np(single.track(tpcsf.DeviceFrame.from_numpy(f.y, f.z, f.row_off)))
        T1 = r1["n_tracks"]
        sel = slice(base_t, base_t + T1)
        assert np.all(res["tf"][sel] == i), i
        for k in ("params", "cov", "chi2", "x_ref", "z_beam", "nhits", "ndf", "sector"):
            assert np.array_equal(res[k][sel], r1[k]), (i, k)
        h0, h1 = res["hit_off"][base_t], res["hit_off"][base_t + T1]
        assert np.array_equal(res["hit_ids"][h0:h1] - base_c, r1["hit_ids"]), i
        assert np.array_equal(res["hit_off"][base_t:base_t + T1 + 1] - h0, r1["hit_off"]), i
        ct = res["cluster_track"][base_c:base_c + f.n_clusters]
        assert np.array_equal(np.where(ct >= 0, ct - base_t, -1), r1["cluster_track"]), i
        if i in (0, 1) or f.n_clusters == sizes[1::2].min():
            alone[i] = r1
        base_c += f.n_clusters
        base_t += T1
    assert base_t == res["n_tracks"] and base_c == n
    print("every frame of the batch equals the frame alone", flush=True)

    # the oracle on a pp frame and on the smallest Pb-Pb frame
    for i in (0, int(1 + 2 * np.argmin(sizes[1::2]))):
        f, r1 = frames[i], alone[i]
        ref = oracle_sectors.track_frame_parallel(row_x, f.y, f.z, f.row_off, grid=CFG3_GRID, debug=False)
        assert r1["n_tracks"] == ref["n_tracks"], i
        assert np.array_equal(r1["hit_off"], ref["hit_off"]), i
        assert np.array_equal(r1["hit_ids"].astype(np.int64), ref["hit_ids"]), i
        err = np.abs(r1["params"] - ref["params"]) / np.maximum(np.abs(ref["params"]), FLOORS)
        assert np.all(err <= 1e-4), err.max(axis=0)
        m_g = truthmatch.match(f.label, f.row_off, r1["hit_off"], r1["hit_ids"], r1["sector"])
        m_o = truthmatch.match(f.label, f.row_off, ref["hit_off"], ref["hit_ids"], ref["sector"])
        assert abs(m_g["efficiency"] - m_o["efficiency"]) <= 1e-3
        assert abs(m_g["fake_rate"] - m_o["fake_rate"]) <= 1e-3
        print(f"frame {i} ({f.n_clusters} clusters, {r1['n_tracks']} tracks): hit lists identical to the oracle, "
              f"max rel. param error {err.max(axis=0)}, efficiency {m_g['efficiency']:.4f}", flush=True)
    trk.close()
    single.close()
