"""Parity of the HIP track-model compression (tpcsf_compress / tpcsf_decompress through the
C ABI) with the oracle's: rows identical; residual codes identical except where the
oracle's unrounded residual lies within 1e-6 of a rounding tie (binary64 positions that
differ by rounding may round such a value either way); decoded clusters within half a step
of the originals and within 1e-5 cm of the oracle's decoding (the GPU and oracle track
parameters agree to ~1e-9 relative, which moves a far row's position by ~1e-7 cm)."""
import numpy as np
import pytest

import oracle
from conftest import CFG3_TUNING
from paper_2009_07515_amd import synth

pytestmark = pytest.mark.gpu

STEP = 0.01


def _np(res):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items()}


def _gpu(f, n_tf=1, trk=None, tuning=None, hit_rec=False):
    from paper_2009_07515_amd import tpcsf
    trk = trk or tpcsf.Tracker(synth.row_x(), tuning=tuning)
    fr = tpcsf.DeviceFrame.from_numpy(f.y, f.z, f.row_off, n_tf=n_tf)
    tb = tpcsf.TrackBuffers(fr.n_clusters, hit_rec=hit_rec)
    tracks = _np(trk.track(fr, out=tb))
    codes, rows = trk.compress(fr, tb)
    yz = trk.decompress(tb, codes, rows)
    return trk, tracks, codes.cpu().numpy(), rows.cpu().numpy(), yz.cpu().numpy()


def _check(f, tracks, codes, rows, yz, o_codes, o_resid, o_pred, label):
    h = tracks["hit_ids"]
    g = np.repeat(np.arange(len(f.row_off) - 1), np.diff(f.row_off))
    assert np.array_equal(rows, (g[h] % 152).astype(np.uint8)), label
    diff = codes != o_codes
    if diff.any():
        frac = np.abs(o_resid[diff] - np.floor(o_resid[diff]) - 0.5)
        assert np.all(frac < 1e-6), (label, int(diff.sum()))
    assert np.all(np.abs(yz[:, 0] - f.y[h]) <= STEP / 2 + 1e-9)
    assert np.all(np.abs(yz[:, 1] - f.z[h]) <= STEP / 2 + 1e-9)
    same = ~diff.any(axis=1)
    # the positions follow the track parameters, which agree to ~1e-9 relative: far from
    # x_ref that is ~1e-7 cm
    dev = np.abs(yz[same] - (o_pred + o_codes * STEP)[same]).max(initial=0.0)
    assert dev < 1e-5, dev
    print(f"{label}: {len(h)} clusters, {int(diff.sum())} codes at a rounding tie, decode deviation {dev:.2e} cm")


@pytest.mark.parametrize("which,rec", [("cfg1", False), ("small", False), ("small", True), ("cfg2", True)])
def test_compress_parity_with_oracle(which, rec, cfg1_frame, small_pbpb_frame, cfg2_frame, row_x):
    """rec: the encoder reads the tracking call's per-hit records instead of the clusters."""
    f = {"cfg1": cfg1_frame, "small": small_pbpb_frame, "cfg2": cfg2_frame}[which]
    _, tracks, codes, rows, yz = _gpu(f, hit_rec=rec)
    o = oracle.Oracle(row_x)
    r = o.track_frame(f.y, f.z, f.row_off)
    assert np.array_equal(r["hit_ids"], tracks["hit_ids"].astype(np.int64))
    oc, ores, opred = o.compress_frame(f.y, f.z, f.row_off, r)
    _check(f, tracks, codes, rows, yz, oc, ores, opred, which)


def test_compress_of_the_full_time_frame_equals_oracle(cfg3_frame, row_x):
    """The 2 ms Pb-Pb frame: the oracle compresses the GPU's own tracks."""
    f = cfg3_frame
    _, tracks, codes, rows, yz = _gpu(f, tuning=CFG3_TUNING, hit_rec=True)
    oc, ores, opred = oracle.Oracle(row_x).compress_frame(f.y, f.z, f.row_off, tracks)
    _check(f, tracks, codes, rows, yz, oc, ores, opred, "cfg3")


def test_compress_of_a_batch_equals_frames_alone():
    frames = [synth.config2_pbpb_event(seed=600 + i, n_primary=200 + 300 * i) for i in range(3)]
    y, z, ro = synth.concat_frames(frames)
    batch = type("F", (), dict(y=y, z=z, row_off=ro))
    trk, tb, cb, rb, yb = _gpu(batch, n_tf=3)
    h0 = 0
    for f in frames:
        _, t1, c1, r1, y1 = _gpu(f, trk=trk)
        n = len(c1)
        assert np.array_equal(cb[h0:h0 + n], c1) and np.array_equal(rb[h0:h0 + n], r1)
        assert np.array_equal(yb[h0:h0 + n], y1)
        h0 += n
    assert h0 == len(cb)
