"""Pins of the oracle's track-model compression (residuals of the attached clusters to the
track's helix, quantised) against noise-free helices, a hand-worked straight track, the
decoding error bound and the residual distribution of Gaussian clusters.  CPU only."""
import math

import numpy as np

import oracle
from paper_2009_07515_amd import synth

STEP = 0.01     # the default quantisation step (cm)


def _entropy(q):
    _, k = np.unique(q, return_counts=True)
    p = k / k.sum()
    return float(-(p * np.log2(p)).sum())


# --------------------------------------------------------------------------------------
# Noise-free helices: the clusters lie on the fitted helix to ~1e-5 cm, so every residual
# code is 0 (a wrong prediction - sign, arc length, row plane - would move them by many
# steps).
# --------------------------------------------------------------------------------------
def test_noise_free_tracks_have_zero_codes(row_x):
    o = oracle.Oracle(row_x)
    f = synth.config2_pbpb_event(seed=77, n_primary=500, sigma=0.0, noise_frac=0.0)
    r = o.track_frame(f.y, f.z, f.row_off)
    codes, resid, _ = o.compress_frame(f.y, f.z, f.row_off, r)
    assert codes.shape[0] == r["n_hits"] > 10000
    assert np.all(codes == 0)
    assert np.abs(resid).max() < 0.05


# --------------------------------------------------------------------------------------
# Hand-worked codes on a straight track (B = 0): clusters at known offsets from the line
# y = y0 + (x - x0) tan(phi), z = z0 + (x - x0) tan(lambda) / cos(phi).
# --------------------------------------------------------------------------------------
def test_codes_hand_example(row_x):
    o = oracle.Oracle(row_x, bz=0.0)
    X = row_x.astype(np.float64)
    sphi, tl, y0, z0 = -0.2, 0.5, 3.0, -40.0
    c = math.sqrt(1 - sphi * sphi)
    offs = [(0.0, 0.0, 0, 0), (0.0349, -0.0151, 3, -2), (-0.0049, 0.0051, 0, 1), (0.1234, 0.987, 12, 99),
            (-1.0, 2.5, -100, 250)]
    rows = [7, 30, 31, 90, 140]
    y, z, counts = [], [], np.zeros(36 * 152, np.int64)
    for r, (dy, dz, _, _) in zip(rows, offs):
        y.append(y0 + (X[r] - X[rows[0]]) * sphi / c + dy)
        z.append(z0 + (X[r] - X[rows[0]]) * tl / c + dz)
        counts[5 * 152 + r] += 1
    ro = np.zeros(36 * 152 + 1, np.int64)
    np.cumsum(counts, out=ro[1:])
    y = np.array(y, np.float32)
    z = np.array(z, np.float32)
    trk = dict(n_tracks=1, n_hits=5, params=np.array([[y[0], z[0], sphi, tl, 0.0]]), x_ref=np.array([X[rows[0]]]),
               sector=np.array([5], np.int32), hit_off=np.array([0, 5]), hit_ids=np.arange(5))
    codes, _, pred = o.compress_frame(y, z, ro, trk)
    assert [tuple(v) for v in codes] == [(cy, cz) for *_, cy, cz in offs]


# --------------------------------------------------------------------------------------
# Decoding: y_p + q * step reproduces every attached cluster within half a step; with
# clusters smeared by 0.1 cm the residuals are that Gaussian (robust width), and their
# codes carry far fewer bits than the absolute coordinates at the same step.
# --------------------------------------------------------------------------------------
def test_decoding_bound_and_residual_distribution(cfg2_frame, row_x):
    f = cfg2_frame
    o = oracle.Oracle(row_x)
    r = o.track_frame(f.y, f.z, f.row_off)
    codes, resid, pred = o.compress_frame(f.y, f.z, f.row_off, r)
    h = r["hit_ids"]
    dec = pred + codes * STEP
    assert np.all(np.abs(dec[:, 0] - f.y[h]) <= STEP / 2 + 1e-9)
    assert np.all(np.abs(dec[:, 1] - f.z[h]) <= STEP / 2 + 1e-9)
    assert np.array_equal(codes, np.floor(resid + 0.5).astype(np.int32))
    for k in range(2):
        mad = np.median(np.abs(resid[:, k] * STEP - np.median(resid[:, k] * STEP))) * 1.4826
        assert 0.085 < mad < 0.105, mad
    h_res = _entropy(codes[:, 0]), _entropy(codes[:, 1])
    h_abs = _entropy(np.floor(f.y[h] / STEP)), _entropy(np.floor(f.z[h] / STEP))
    assert h_res[0] < h_abs[0] - 6 and h_res[1] < h_abs[1] - 8
    print(f"bits per coordinate: residual codes {h_res[0]:.2f}, {h_res[1]:.2f}; absolute {h_abs[0]:.2f}, "
          f"{h_abs[1]:.2f}")
