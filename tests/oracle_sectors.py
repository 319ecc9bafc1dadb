"""The oracle on a whole frame, one sector per task in a thread pool (test infrastructure).

Sectors are tracked independently by the method (grid, links, chains, tracklets, selection
and final fit never look across a sector), so the oracle's run on a one-sector slice of
the frame is its run on that sector of the whole frame.  The ctypes calls release the
interpreter lock, so the sectors run in parallel.  The per-sector results are put back
together in the layout of oracle.Oracle.track_frame(debug=True) on the whole frame: track
order (sector, rank), frame cluster indices, the grid's bin tables concatenated row by row.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle

N_ROWS = 152


def _one(args):
    row_x, grid, params, y, z, off, debug = args
    o = oracle.Oracle(row_x, n_sectors=1, grid=grid, params=params)
    return o.track_frame(y, z, off, debug=debug)


def track_frame_parallel(row_x, y, z, row_off, n_sectors=36, grid=None, params=None, debug=True, sectors=None,
                         workers=None):
    """Oracle result of the given sectors (all by default) of one frame.  With `sectors`,
    the result covers only those sectors: tracks, hit_ids and cluster_track refer to the
    frame's cluster indices, and debug arrays are given per sector in 'per_sector'."""
    row_off = np.asarray(row_off, dtype=np.int64)
    secs = list(range(n_sectors)) if sectors is None else list(sectors)
    tasks = []
    for s in secs:
        ro = row_off[s * N_ROWS:(s + 1) * N_ROWS + 1]
        b, e = int(ro[0]), int(ro[-1])
        tasks.append((row_x, grid, params, y[b:e], z[b:e], ro - b, debug))
    workers = workers or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        parts = list(ex.map(_one, tasks))
    n = int(row_off[-1])
    T = sum(p["n_tracks"] for p in parts)
    out = dict(n_tracks=T, n_hits=sum(p["n_hits"] for p in parts), sectors=secs, per_sector=parts)
    cat = lambda k: np.concatenate([p[k] for p in parts]) if parts else np.zeros(0)  # noqa: E731
    for k in ("params", "cov", "x_ref", "chi2", "ndf", "nhits", "z_beam", "params_outer", "cov_outer"):
        out[k] = cat(k)
    out["sector"] = np.concatenate([np.full(p["n_tracks"], s, np.int32) for s, p in zip(secs, parts)])
    hit_ids, hit_off, base_h = [], [np.zeros(1, np.int64)], 0
    ct = np.full(n, -1, np.int32)
    base_t = 0
    for s, p in zip(secs, parts):
        b = int(row_off[s * N_ROWS])
        hit_ids.append(p["hit_ids"] + b)
        hit_off.append(p["hit_off"][1:] + base_h)
        base_h += int(p["n_hits"])
        c = p["cluster_track"]
        e = b + c.shape[0]
        ct[b:e] = np.where(c >= 0, c + base_t, -1)
        base_t += int(p["n_tracks"])
    out["hit_ids"] = np.concatenate(hit_ids) if hit_ids else np.zeros(0, np.int64)
    out["hit_off"] = np.concatenate(hit_off)
    out["cluster_track"] = ct
    if debug and sectors is None:
        d = {}
        dbg = [p["debug"] for p in parts]
        for k in ("g_ylo", "g_zlo", "g_by", "g_bz", "g_ny", "g_nz", "perm", "up", "dn", "cup", "cdn", "start",
                  "W", "tl_nhits"):
            d[k] = np.concatenate([x[k] for x in dbg])
        bases, acc, bs = [], 0, []
        for x in dbg:
            used = int(x["g_bin_base"][-1] + x["g_ny"][-1].astype(np.int64) * x["g_nz"][-1] + 1)
            bases.append(x["g_bin_base"] + acc)
            bs.append(x["bin_start"][:used])
            acc += used
        d["g_bin_base"] = np.concatenate(bases)
        d["bin_start"] = np.concatenate(bs)
        d["tl_start"] = np.concatenate([x["tl_start"] + int(row_off[s * N_ROWS]) for s, x in zip(secs, dbg)])
        d["work"] = np.sum([x["work"] for x in dbg], axis=0)
        out["debug"] = d
    return out
