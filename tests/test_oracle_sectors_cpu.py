"""The per-sector parallel run of the oracle (tests/oracle_sectors.py) equals the oracle's
whole-frame run: same tracks, hit lists, cluster map, grid tables, links and tracklet
sizes (the method never looks across a sector)."""
import numpy as np

import oracle
import oracle_sectors


def test_parallel_sectors_equal_whole_frame(small_pbpb_frame, row_x):
    f = small_pbpb_frame
    grid = dict(bin_y=2.0, bin_z=4.0, cap_mul=4, cap_add=64)
    whole = oracle.Oracle(row_x, grid=grid).track_frame(f.y, f.z, f.row_off, debug=True)
    par = oracle_sectors.track_frame_parallel(row_x, f.y, f.z, f.row_off, grid=grid, workers=4)
    for k in ("n_tracks", "n_hits"):
        assert whole[k] == par[k], k
    for k in ("params", "cov", "x_ref", "chi2", "ndf", "nhits", "sector", "hit_off", "hit_ids", "cluster_track",
              "z_beam", "params_outer", "cov_outer"):
        assert np.array_equal(whole[k], par[k]), k
    for k in ("g_ylo", "g_zlo", "g_by", "g_bz", "g_ny", "g_nz", "g_bin_base", "perm", "up", "dn", "cup", "cdn",
              "start", "tl_start", "tl_nhits", "work"):
        assert np.array_equal(whole["debug"][k], par["debug"][k]), k
    used = int(whole["debug"]["g_bin_base"][-1] + whole["debug"]["g_ny"][-1] * whole["debug"]["g_nz"][-1] + 1)
    assert np.array_equal(whole["debug"]["bin_start"][:used], par["debug"]["bin_start"])
    # selection weights differ only by the rank offset of each sector's first start
    assert np.array_equal(whole["debug"]["W"] >> np.uint64(32), par["debug"]["W"] >> np.uint64(32))
