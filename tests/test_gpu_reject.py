"""Parity of the HIP hit removal for compression strategy B (tpcsf_reject through the C
ABI) with the oracle's: the keep flags are identical (binary64 decisions on both sides)."""
import numpy as np
import pytest

import oracle
from conftest import CFG3_TUNING
from paper_2009_07515_amd import synth

pytestmark = pytest.mark.gpu


def _np(res):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items()}


def _gpu(f, n_tf=1, trk=None, tuning=None):
    from paper_2009_07515_amd import tpcsf
    trk = trk or tpcsf.Tracker(synth.row_x(), tuning=tuning)
    fr = tpcsf.DeviceFrame.from_numpy(f.y, f.z, f.row_off, n_tf=n_tf)
    tb = tpcsf.TrackBuffers(fr.n_clusters)
    tracks = _np(trk.track(fr, out=tb))
    keep, k = trk.reject(fr, tb)
    return trk, tracks, keep.cpu().numpy(), k


@pytest.mark.parametrize("which", ["cfg1", "small", "cfg2"])
def test_reject_parity_with_oracle(which, cfg1_frame, small_pbpb_frame, cfg2_frame, row_x):
    f = {"cfg1": cfg1_frame, "small": small_pbpb_frame, "cfg2": cfg2_frame}[which]
    _, tracks, keep, k = _gpu(f)
    o = oracle.Oracle(row_x)
    r = o.track_frame(f.y, f.z, f.row_off)
    ko, kk = o.reject_frame(f.y, f.z, f.row_off, r)
    assert k == kk and np.array_equal(keep, ko)
    print(f"{which}: kept {k} of {f.n_clusters} ({k / max(f.n_clusters, 1):.3f})")


def test_reject_of_the_full_time_frame_equals_oracle(cfg3_frame, row_x):
    """The 2 ms Pb-Pb frame in the benchmark's tuning: the oracle removes hits around the
    GPU's own sector tracks (its tracking of this frame takes minutes)."""
    f = cfg3_frame
    _, tracks, keep, k = _gpu(f, tuning=CFG3_TUNING)
    ko, kk = oracle.Oracle(row_x).reject_frame(f.y, f.z, f.row_off, tracks)
    assert k == kk and np.array_equal(keep, ko)
    print(f"cfg3: kept {k} of {f.n_clusters} ({k / f.n_clusters:.3f})")


def test_reject_of_a_batch_equals_frames_alone():
    frames = [synth.config2_pbpb_event(seed=800 + i, n_primary=200 + 400 * i) for i in range(3)]
    y, z, ro = synth.concat_frames(frames)
    batch = type("F", (), dict(y=y, z=z, row_off=ro))
    trk, _, kb, nb = _gpu(batch, n_tf=3)
    c0 = 0
    tot = 0
    for f in frames:
        _, _, k1, n1 = _gpu(f, trk=trk)
        assert np.array_equal(kb[c0:c0 + f.n_clusters], k1)
        c0 += f.n_clusters
        tot += n1
    assert nb == tot


def test_reject_needs_the_last_frame(small_pbpb_frame, cfg1_frame):
    from paper_2009_07515_amd import tpcsf
    trk = tpcsf.Tracker(synth.row_x())
    fa = tpcsf.DeviceFrame.from_numpy(small_pbpb_frame.y, small_pbpb_frame.z, small_pbpb_frame.row_off)
    fb = tpcsf.DeviceFrame.from_numpy(cfg1_frame.y, cfg1_frame.z, cfg1_frame.row_off)
    ta = tpcsf.TrackBuffers(fa.n_clusters)
    tbb = tpcsf.TrackBuffers(fb.n_clusters)
    trk.track(fa, out=ta)
    trk.track(fb, out=tbb)
    with pytest.raises(tpcsf.TpcsfError) as e:
        trk.reject(fa, ta)
    assert e.value.status == tpcsf.E_INVALID
    keep, k = trk.reject(fb, tbb)
    assert k > 0


def test_reject_of_a_row_larger_than_the_flag_table(cfg1_frame, row_x):
    """A row of more than 20,000 clusters (dense noise added to row 60 of sector 0): more
    than one pass of the row kernel's on-chip flag table, whose slices must together give
    the oracle's keep flags."""
    f = cfg1_frame
    g = 60
    rng = np.random.Generator(np.random.PCG64(11))
    m = 20000
    half = float(row_x[g]) * np.tan(np.pi / 18)
    ny = rng.uniform(-half, half, m).astype(np.float32)
    nz = rng.uniform(-250.0, 250.0, m).astype(np.float32)
    at = int(f.row_off[g + 1])
    y = np.insert(f.y, at, ny)
    z = np.insert(f.z, at, nz)
    ro = f.row_off.copy()
    ro[g + 1:] += m
    frame = type("F", (), dict(y=y, z=z, row_off=ro))
    assert ro[g + 1] - ro[g] > 16384
    _, tracks, keep, k = _gpu(frame)
    ko, kk = oracle.Oracle(row_x).reject_frame(y, z, ro, tracks)
    assert k == kk and np.array_equal(keep, ko)
    row_keep = keep[ro[g]:ro[g + 1]]
    own = np.zeros(ro[g + 1] - ro[g], bool)
    own[tracks["cluster_track"][ro[g]:ro[g + 1]] >= 0] = True
    # clusters kept for lying in a track's window only, not for being a track's own
    assert int(row_keep[~own].sum()) > 20
    print(f"row of {ro[g + 1] - ro[g]} clusters: {int(row_keep.sum())} kept, {tracks['n_tracks']} tracks")


def test_reject_reports_tracks_outside_their_sector(small_pbpb_frame):
    from paper_2009_07515_amd import tpcsf
    f = small_pbpb_frame
    trk = tpcsf.Tracker(synth.row_x())
    fr = tpcsf.DeviceFrame.from_numpy(f.y, f.z, f.row_off)
    tb = tpcsf.TrackBuffers(fr.n_clusters)
    trk.track(fr, out=tb)
    keep0, k0 = trk.reject(fr, tb)
    s0 = int(tb.sector[0].item())
    tb.sector[0] = (s0 + 1) % 36          # its clusters now lie outside its sector
    with pytest.raises(tpcsf.TpcsfError) as e:
        trk.reject(fr, tb)
    assert e.value.status == tpcsf.E_INVALID
    tb.sector[0] = s0
    keep1, k1 = trk.reject(fr, tb)        # the context keeps working
    assert k1 == k0 and torch_equal(keep1, keep0)


def torch_equal(a, b):
    return bool((a == b).all().item())
