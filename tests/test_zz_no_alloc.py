"""tpcsf_track_batch_noalloc (scratch in the fixed per-GPU array, no allocation) against
tpcsf_track_batch on the same frames: identical outputs, on two calls in a row, the second
with a smaller frame; a frame whose scratch exceeds the array is refused before launch."""
import numpy as np
import pytest

from paper_2009_07515_amd import synth

pytestmark = pytest.mark.gpu

KEYS_EXACT = ("n_tracks", "n_hits", "hit_off", "hit_ids", "cluster_track", "nhits", "ndf", "sector", "tf",
              "params", "cov", "x_ref", "chi2", "z_beam")


def _np(res):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items()}


def _same(a, b, label):
    for k in KEYS_EXACT:
        if k in a:
            assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (label, k)


def test_noalloc_equals_batch_on_two_calls_in_a_row(small_pbpb_frame, cfg1_frame, cfg2_frame):
    from paper_2009_07515_amd import tpcsf
    trk = tpcsf.Tracker(synth.row_x())
    ref = tpcsf.Tracker(synth.row_x())
    big = tpcsf.DeviceFrame.from_numpy(small_pbpb_frame.y, small_pbpb_frame.z, small_pbpb_frame.row_off)
    small = tpcsf.DeviceFrame.from_numpy(cfg1_frame.y, cfg1_frame.z, cfg1_frame.row_off)
    assert trk.arena_bytes(big.n_clusters) <= tpcsf.NOALLOC_SCRATCH_BYTES
    print(f"frames of {big.n_clusters} and {small.n_clusters} clusters, scratch "
          f"{trk.arena_bytes(big.n_clusters)} of {tpcsf.NOALLOC_SCRATCH_BYTES} bytes", flush=True)
    r_big = _np(ref.track(big, mode="batch"))
    r_small = _np(ref.track(small, mode="batch"))
    n_big = _np(trk.track(big, mode="noalloc"))
    n_small = _np(trk.track(small, mode="noalloc"))
    assert n_big["n_tracks"] > 100 and n_small["n_tracks"] > 5
    _same(n_big, r_big, "first call")
    _same(n_small, r_small, "second, smaller call")
    # the same context's batched form, after the no-alloc calls, still agrees
    _same(_np(trk.track(small, mode="batch")), r_small, "batched after no-alloc")
    # a frame whose scratch exceeds the fixed array is refused before any launch
    huge = tpcsf.DeviceFrame.from_numpy(cfg2_frame.y, cfg2_frame.z, cfg2_frame.row_off)
    assert trk.arena_bytes(huge.n_clusters) > tpcsf.NOALLOC_SCRATCH_BYTES
    with pytest.raises(tpcsf.TpcsfError) as e:
        trk.track(huge, mode="noalloc")
    assert e.value.status == tpcsf.E_NOMEM
    _same(_np(trk.track(small, mode="noalloc")), r_small, "after the refused call")
