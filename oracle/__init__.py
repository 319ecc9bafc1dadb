"""Reference oracle for TPC sector track finding: ctypes wrapper around liborc_{f64,f32}.so.

Test infrastructure only.  The test suite, the smoke check and the CPU baseline of the
benchmark may use it; the GPU library never does.  The C source (orc.c) states the
method step by step with the readings it takes where the paper (arXiv:2009.07515,
Sec. 6) is silent.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

# Method constants (they define the result).  The GPU library carries its own copy of
# these defaults; tests pass identical explicit values to both sides.
DEFAULT_PARAMS = dict(
    win_y=3.0, win_z=3.0, kink_max=1.0,
    sigma_y=0.1, sigma_z=0.1, chi2_max=16.0, sinphi_max=0.99, nsig=5.0,
    c0=(1.0, 1.0, 1.0, 1.0, 100.0),
    min_chain=5, min_track_hits=20, max_miss=4,
    merge_edge=6.0, merge_window=5.0, merge_chi2=30.0,
    reject_pt_min=0.05, reject_window=1.0,
    resid_step=0.01,
)
# Grid tuning (changes the grid tables, never links or tracks).
DEFAULT_GRID = dict(bin_y=2.0, bin_z=2.0, cap_mul=2, cap_add=64)


class _Cfg(C.Structure):
    _fields_ = [
        ("n_sectors", C.c_int32), ("n_rows", C.c_int32), ("row_x", C.POINTER(C.c_float)),
        ("bz", C.c_double),
        ("win_y", C.c_float), ("win_z", C.c_float), ("kink_max", C.c_float),
        ("sigma_y", C.c_double), ("sigma_z", C.c_double), ("chi2_max", C.c_double),
        ("sinphi_max", C.c_double), ("nsig", C.c_double), ("c0", C.c_double * 5),
        ("min_chain", C.c_int32), ("min_track_hits", C.c_int32), ("max_miss", C.c_int32),
        ("bin_y", C.c_float), ("bin_z", C.c_float), ("cap_mul", C.c_int32), ("cap_add", C.c_int32),
        ("merge_edge", C.c_double), ("merge_window", C.c_double), ("merge_chi2", C.c_double),
        ("reject_pt_min", C.c_double), ("reject_window", C.c_double),
        ("resid_step", C.c_double),
    ]


class _Tracks(C.Structure):
    _fields_ = [
        ("cap_tracks", C.c_int64), ("cap_hits", C.c_int64),
        ("n_tracks", C.c_int64), ("n_hits", C.c_int64),
        ("params", C.c_void_p), ("cov", C.c_void_p), ("x_ref", C.c_void_p), ("chi2", C.c_void_p),
        ("ndf", C.c_void_p), ("nhits", C.c_void_p), ("sector", C.c_void_p),
        ("hit_off", C.c_void_p), ("hit_ids", C.c_void_p), ("cluster_track", C.c_void_p),
        ("z_beam", C.c_void_p), ("params_outer", C.c_void_p), ("cov_outer", C.c_void_p),
    ]


class _Merged(C.Structure):
    _fields_ = [
        ("cap_merged", C.c_int64), ("cap_hits", C.c_int64),
        ("n_merged", C.c_int64), ("n_hits", C.c_int64),
        ("params", C.c_void_p), ("cov", C.c_void_p), ("x_ref", C.c_void_p), ("chi2", C.c_void_p),
        ("z_beam", C.c_void_p), ("ndf", C.c_void_p), ("nhits", C.c_void_p), ("sector", C.c_void_p),
        ("n_segments", C.c_void_p), ("hit_off", C.c_void_p), ("hit_ids", C.c_void_p),
        ("track_merged", C.c_void_p), ("next", C.c_void_p), ("link_chi2", C.c_void_p),
    ]


class _Debug(C.Structure):
    _fields_ = [
        ("g_ylo", C.c_void_p), ("g_zlo", C.c_void_p), ("g_by", C.c_void_p), ("g_bz", C.c_void_p),
        ("g_ny", C.c_void_p), ("g_nz", C.c_void_p), ("g_bin_base", C.c_void_p),
        ("bin_start", C.c_void_p), ("bin_start_cap", C.c_int64), ("perm", C.c_void_p),
        ("up", C.c_void_p), ("dn", C.c_void_p), ("cup", C.c_void_p), ("cdn", C.c_void_p),
        ("start", C.c_void_p),
        ("cap_tracklets", C.c_int64), ("n_tracklets", C.c_int64),
        ("tl_start", C.c_void_p), ("tl_nhits", C.c_void_p), ("tl_hits", C.c_void_p),
        ("W", C.c_void_p), ("work", C.c_int64 * 6),
    ]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


_LIBS = {}


def _lib(mode):
    if mode not in _LIBS:
        path = _build.lib_path(mode)
        if not os.path.exists(path):
            _build.build()
        lib = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        lib.orc_track_frame.argtypes = [C.POINTER(_Cfg), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.POINTER(_Tracks), C.POINTER(_Debug), C.c_uint64]
        lib.orc_grid_row.argtypes = [C.POINTER(_Cfg), C.c_int64, C.c_void_p, C.c_void_p,
                                     C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_float),
                                     C.POINTER(C.c_float), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.c_void_p, C.c_int64, C.c_void_p]
        lib.orc_links_sector.argtypes = [C.POINTER(_Cfg), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                         C.c_void_p, C.c_void_p]
        lib.orc_propagate.argtypes = [C.POINTER(_Cfg), C.c_double, C.c_double, dp, dp, dp]
        lib.orc_seed.argtypes = [C.POINTER(_Cfg), dp, dp, dp, dp]
        lib.orc_update.argtypes = [C.POINTER(_Cfg), C.c_double, C.c_double, dp, dp]
        lib.orc_update.restype = C.c_double
        lib.orc_beamline_z.argtypes = [C.POINTER(_Cfg), C.c_double, dp]
        lib.orc_beamline_z.restype = C.c_double
        lib.orc_fit_hits.argtypes = [C.POINTER(_Cfg), C.c_int32, dp, dp, dp, dp, dp, dp, dp]
        lib.orc_rotate.argtypes = [C.POINTER(_Cfg), C.c_double, dp, dp, dp, dp]
        lib.orc_fit_hits_sectors.argtypes = [C.POINTER(_Cfg), C.c_int32, dp, dp, dp, C.c_void_p, dp, dp, dp]
        lib.orc_reject_frame.argtypes = [C.POINTER(_Cfg), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.POINTER(_Tracks), C.c_int, C.c_void_p]
        lib.orc_reject_frame.restype = C.c_int64
        lib.orc_compress_frame.argtypes = [C.POINTER(_Cfg), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.POINTER(_Tracks), C.c_void_p, C.c_void_p, C.c_void_p]
        lib.orc_select.argtypes = [C.POINTER(_Cfg), C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.orc_select.restype = None
        lib.orc_merge_frame.argtypes = [C.POINTER(_Cfg), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.POINTER(_Tracks), C.POINTER(_Merged)]
        _LIBS[mode] = lib
    return _LIBS[mode]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Oracle:
    """One configured oracle.  mode 'f64' (reference for parameters and efficiency) or
    'f32' (Kalman in float).  Grid and links are binary32 in both modes."""

    def __init__(self, row_x, bz=0.5, n_sectors=36, mode="f64", params=None, grid=None):
        self.mode = mode
        self.lib = _lib(mode)
        self.row_x = np.ascontiguousarray(row_x, dtype=np.float32)
        self.n_rows = int(self.row_x.shape[0])
        self.n_sectors = n_sectors
        self.params = dict(DEFAULT_PARAMS, **(params or {}))
        self.grid = dict(DEFAULT_GRID, **(grid or {}))
        p, g = self.params, self.grid
        self.cfg = _Cfg(n_sectors, self.n_rows, self.row_x.ctypes.data_as(C.POINTER(C.c_float)), bz,
                        p["win_y"], p["win_z"], p["kink_max"], p["sigma_y"], p["sigma_z"],
                        p["chi2_max"], p["sinphi_max"], p["nsig"], (C.c_double * 5)(*p["c0"]),
                        p["min_chain"], p["min_track_hits"], p["max_miss"],
                        g["bin_y"], g["bin_z"], g["cap_mul"], g["cap_add"],
                        p["merge_edge"], p["merge_window"], p["merge_chi2"],
                        p["reject_pt_min"], p["reject_window"], p["resid_step"])

    # -- whole frame ----------------------------------------------------------------
    def track_frame(self, y, z, row_off, debug=False, shuffle_seed=0):
        y = np.ascontiguousarray(y, dtype=np.float32)
        z = np.ascontiguousarray(z, dtype=np.float32)
        row_off = np.ascontiguousarray(row_off, dtype=np.int64)
        n = int(y.shape[0])
        cap_t = max(16, n // 8)
        cap_h = max(16, n)
        o = dict(params=np.zeros((cap_t, 5)), cov=np.zeros((cap_t, 15)), x_ref=np.zeros(cap_t),
                 chi2=np.zeros(cap_t), ndf=np.zeros(cap_t, np.int32), nhits=np.zeros(cap_t, np.int32),
                 sector=np.zeros(cap_t, np.int32), hit_off=np.zeros(cap_t + 1, np.int64),
                 hit_ids=np.zeros(cap_h, np.int64), cluster_track=np.zeros(max(n, 1), np.int32),
                 z_beam=np.zeros(cap_t), params_outer=np.zeros((cap_t, 5)), cov_outer=np.zeros((cap_t, 15)))
        tr = _Tracks(cap_t, cap_h, 0, 0, *[_ptr(o[k]) for k in
                                            ("params", "cov", "x_ref", "chi2", "ndf", "nhits", "sector",
                                             "hit_off", "hit_ids", "cluster_track", "z_beam",
                                             "params_outer", "cov_outer")])
        dbg = None
        d = {}
        if debug:
            nrows = self.n_sectors * self.n_rows
            bcap = int(self.grid["cap_mul"]) * n + (int(self.grid["cap_add"]) + 1) * nrows + 1
            d = dict(g_ylo=np.zeros(nrows, np.float32), g_zlo=np.zeros(nrows, np.float32),
                     g_by=np.zeros(nrows, np.float32), g_bz=np.zeros(nrows, np.float32),
                     g_ny=np.zeros(nrows, np.int32), g_nz=np.zeros(nrows, np.int32),
                     g_bin_base=np.zeros(nrows, np.int64), bin_start=np.zeros(bcap, np.uint32),
                     perm=np.zeros(max(n, 1), np.uint32),
                     up=np.zeros(max(n, 1), np.int32), dn=np.zeros(max(n, 1), np.int32),
                     cup=np.zeros(max(n, 1), np.int32), cdn=np.zeros(max(n, 1), np.int32),
                     start=np.zeros(max(n, 1), np.uint8),
                     tl_start=np.zeros(max(n, 1), np.int64), tl_nhits=np.zeros(max(n, 1), np.int32),
                     W=np.zeros(max(n, 1), np.uint64))
            # tracklet hit tables only for modest frames (n_rows ints per start)
            cap_tl = max(n, 1)
            d["tl_hits"] = np.full((cap_tl, self.n_rows), -1, np.int32) if n <= 200_000 else None
            dbg = _Debug(_ptr(d["g_ylo"]), _ptr(d["g_zlo"]), _ptr(d["g_by"]), _ptr(d["g_bz"]),
                         _ptr(d["g_ny"]), _ptr(d["g_nz"]), _ptr(d["g_bin_base"]), _ptr(d["bin_start"]),
                         bcap, _ptr(d["perm"]), _ptr(d["up"]), _ptr(d["dn"]), _ptr(d["cup"]),
                         _ptr(d["cdn"]), _ptr(d["start"]), cap_tl, 0, _ptr(d["tl_start"]),
                         _ptr(d["tl_nhits"]), _ptr(d["tl_hits"]), _ptr(d["W"]))
        rc = self.lib.orc_track_frame(C.byref(self.cfg), n, _ptr(y), _ptr(z), _ptr(row_off),
                                      C.byref(tr), C.byref(dbg) if dbg is not None else None,
                                      shuffle_seed)
        if rc != 0:
            raise RuntimeError(f"orc_track_frame failed with {rc}")
        T, H = tr.n_tracks, tr.n_hits
        res = dict(n_tracks=T, n_hits=H, params=o["params"][:T], cov=o["cov"][:T], x_ref=o["x_ref"][:T],
                   chi2=o["chi2"][:T], ndf=o["ndf"][:T], nhits=o["nhits"][:T], sector=o["sector"][:T],
                   hit_off=o["hit_off"][:T + 1], hit_ids=o["hit_ids"][:H],
                   cluster_track=o["cluster_track"][:n], z_beam=o["z_beam"][:T],
                   params_outer=o["params_outer"][:T], cov_outer=o["cov_outer"][:T])
        if debug:
            K = dbg.n_tracklets
            for k in ("tl_start", "tl_nhits"):
                d[k] = d[k][:K]
            if d["tl_hits"] is not None:
                d["tl_hits"] = d["tl_hits"][:K]
            for k in ("perm", "up", "dn", "cup", "cdn", "start", "W"):
                d[k] = d[k][:n]
            d["work"] = np.array(list(dbg.work), np.int64)
            res["debug"] = d
        return res

    def merge_frame(self, y, z, row_off, trk):
        """Merge one frame's sector tracks (a track_frame result) across sector edges and
        refit the merged tracks (orc_merge_frame)."""
        y = np.ascontiguousarray(y, dtype=np.float32)
        z = np.ascontiguousarray(z, dtype=np.float32)
        row_off = np.ascontiguousarray(row_off, dtype=np.int64)
        n = int(y.shape[0])
        T = int(trk["n_tracks"])
        H = int(trk["n_hits"]) if "n_hits" in trk else int(len(trk["hit_ids"]))
        conv = dict(params=np.float64, cov=np.float64, x_ref=np.float64, chi2=np.float64, ndf=np.int32,
                    nhits=np.int32, sector=np.int32, hit_off=np.int64, hit_ids=np.int64,
                    params_outer=np.float64, cov_outer=np.float64)
        keep = {k: np.ascontiguousarray(np.asarray(trk[k]), dtype=t) for k, t in conv.items()}
        tr = _Tracks(T, H, T, H,
                     *[_ptr(keep[k]) if k in keep else None for k in
                       ("params", "cov", "x_ref", "chi2", "ndf", "nhits", "sector", "hit_off", "hit_ids",
                        "cluster_track", "z_beam", "params_outer", "cov_outer")])
        cm, ch = max(T, 1), max(H, 1)
        o = dict(params=np.zeros((cm, 5)), cov=np.zeros((cm, 15)), x_ref=np.zeros(cm), chi2=np.zeros(cm),
                 z_beam=np.zeros(cm), ndf=np.zeros(cm, np.int32), nhits=np.zeros(cm, np.int32),
                 sector=np.zeros(cm, np.int32), n_segments=np.zeros(cm, np.int32),
                 hit_off=np.zeros(cm + 1, np.int64), hit_ids=np.zeros(ch, np.int64),
                 track_merged=np.full(cm, -1, np.int32), next=np.full(cm, -1, np.int32),
                 link_chi2=np.zeros(cm))
        mo = _Merged(cm, ch, 0, 0, *[_ptr(o[k]) for k in
                                     ("params", "cov", "x_ref", "chi2", "z_beam", "ndf", "nhits", "sector",
                                      "n_segments", "hit_off", "hit_ids", "track_merged", "next",
                                      "link_chi2")])
        rc = self.lib.orc_merge_frame(C.byref(self.cfg), n, _ptr(y), _ptr(z), _ptr(row_off),
                                      C.byref(tr), C.byref(mo))
        if rc != 0:
            raise RuntimeError(f"orc_merge_frame failed with {rc}")
        M, Hm = mo.n_merged, mo.n_hits
        res = {k: v[:M] for k, v in o.items() if k not in ("hit_off", "hit_ids", "track_merged", "next",
                                                          "link_chi2")}
        res.update(n_merged=M, n_hits=Hm, hit_off=o["hit_off"][:M + 1], hit_ids=o["hit_ids"][:Hm],
                   track_merged=o["track_merged"][:T], next=o["next"][:T], link_chi2=o["link_chi2"][:T])
        return res

    def reject_frame(self, y, z, row_off, trk, brute=False):
        """Hit removal, strategy B (orc_reject_frame): keep flags (uint8) and the kept count."""
        y = np.ascontiguousarray(y, dtype=np.float32)
        z = np.ascontiguousarray(z, dtype=np.float32)
        row_off = np.ascontiguousarray(row_off, dtype=np.int64)
        n = int(y.shape[0])
        T = int(trk["n_tracks"])
        H = int(trk["n_hits"]) if "n_hits" in trk else int(len(trk["hit_ids"]))
        conv = dict(params=np.float64, x_ref=np.float64, sector=np.int32, hit_off=np.int64, hit_ids=np.int64)
        keep_arr = {k: np.ascontiguousarray(np.asarray(trk[k]), dtype=t) for k, t in conv.items()}
        tr = _Tracks(T, H, T, H, *[_ptr(keep_arr[k]) if k in keep_arr else None for k in
                                   ("params", "cov", "x_ref", "chi2", "ndf", "nhits", "sector", "hit_off",
                                    "hit_ids", "cluster_track", "z_beam", "params_outer", "cov_outer")])
        keep = np.zeros(max(n, 1), np.uint8)
        k = self.lib.orc_reject_frame(C.byref(self.cfg), n, _ptr(y), _ptr(z), _ptr(row_off), C.byref(tr),
                                      int(bool(brute)), _ptr(keep))
        if k < 0:
            raise RuntimeError("orc_reject_frame failed")
        return keep[:n], int(k)

    def compress_frame(self, y, z, row_off, trk):
        """Track-model compression (orc_compress_frame): residual codes [H, 2] (int32),
        unrounded residuals in steps [H, 2] and predicted positions [H, 2]."""
        y = np.ascontiguousarray(y, dtype=np.float32)
        z = np.ascontiguousarray(z, dtype=np.float32)
        row_off = np.ascontiguousarray(row_off, dtype=np.int64)
        n = int(y.shape[0])
        T = int(trk["n_tracks"])
        H = int(trk["n_hits"]) if "n_hits" in trk else int(len(trk["hit_ids"]))
        conv = dict(params=np.float64, x_ref=np.float64, sector=np.int32, hit_off=np.int64, hit_ids=np.int64)
        a = {k: np.ascontiguousarray(np.asarray(trk[k]), dtype=t) for k, t in conv.items()}
        tr = _Tracks(T, H, T, H, *[_ptr(a[k]) if k in a else None for k in
                                   ("params", "cov", "x_ref", "chi2", "ndf", "nhits", "sector", "hit_off",
                                    "hit_ids", "cluster_track", "z_beam", "params_outer", "cov_outer")])
        codes = np.zeros((max(H, 1), 2), np.int32)
        resid = np.zeros((max(H, 1), 2))
        pred = np.zeros((max(H, 1), 2))
        rc = self.lib.orc_compress_frame(C.byref(self.cfg), n, _ptr(y), _ptr(z), _ptr(row_off), C.byref(tr),
                                         _ptr(codes), _ptr(resid), _ptr(pred))
        if rc != 0:
            raise RuntimeError("orc_compress_frame failed")
        return codes[:H], resid[:H], pred[:H]

    # -- single steps ----------------------------------------------------------------
    def select(self, n_clusters, tl_n, rank, hits, shuffle_seed=0):
        """Selection among one sector's tracklets (orc_select).  hits: [K, n_rows] cluster
        index per row (-1 none).  Returns (W [n_clusters] uint64, weights [K] uint64,
        kept [K] int32)."""
        tl_n = np.ascontiguousarray(tl_n, dtype=np.int32)
        rank = np.ascontiguousarray(rank, dtype=np.int64)
        hits = np.ascontiguousarray(hits, dtype=np.int32)
        K = int(tl_n.shape[0])
        assert hits.shape == (K, self.n_rows)
        W = np.zeros(max(n_clusters, 1), np.uint64)
        wt = np.zeros(max(K, 1), np.uint64)
        kept = np.zeros(max(K, 1), np.int32)
        self.lib.orc_select(C.byref(self.cfg), int(n_clusters), K, _ptr(tl_n), _ptr(rank), _ptr(hits),
                            int(shuffle_seed), _ptr(W), _ptr(wt), _ptr(kept))
        return W[:n_clusters], wt[:K], kept[:K]

    def grid_row(self, y, z):
        y = np.ascontiguousarray(y, dtype=np.float32)
        z = np.ascontiguousarray(z, dtype=np.float32)
        n = int(y.shape[0])
        cap = int(self.grid["cap_mul"]) * n + int(self.grid["cap_add"]) + 1
        bs = np.zeros(cap, np.uint32)
        perm = np.zeros(max(n, 1), np.uint32)
        f = [C.c_float() for _ in range(4)]
        i = [C.c_int32() for _ in range(2)]
        rc = self.lib.orc_grid_row(C.byref(self.cfg), n, _ptr(y), _ptr(z), *[C.byref(v) for v in f],
                                   *[C.byref(v) for v in i], _ptr(bs), cap, _ptr(perm))
        if rc != 0:
            raise RuntimeError("orc_grid_row failed")
        ny, nz = i[0].value, i[1].value
        return dict(ylo=f[0].value, zlo=f[1].value, by=f[2].value, bz=f[3].value, ny=ny, nz=nz,
                    bin_start=bs[:ny * nz + 1], perm=perm[:n])

    def links_sector(self, y, z, row_off_sector, brute=False):
        y = np.ascontiguousarray(y, dtype=np.float32)
        z = np.ascontiguousarray(z, dtype=np.float32)
        ro = np.ascontiguousarray(row_off_sector, dtype=np.int64)
        n = int(ro[-1] - ro[0])
        up = np.zeros(max(n, 1), np.int32)
        dn = np.zeros(max(n, 1), np.int32)
        self.lib.orc_links_sector(C.byref(self.cfg), _ptr(y), _ptr(z), _ptr(ro), int(bool(brute)),
                                  _ptr(up), _ptr(dn))
        return up[:n], dn[:n]

    def propagate(self, x0, x1, p, Cov=None):
        p = np.array(p, dtype=np.float64)
        Cv = np.zeros(15) if Cov is None else np.array(Cov, dtype=np.float64)
        J = np.zeros(25)
        rc = self.lib.orc_propagate(C.byref(self.cfg), x0, x1, _dp(p), _dp(Cv), _dp(J))
        return rc == 0, p, Cv, J.reshape(5, 5)

    def rotate(self, delta, x, p, Cov=None):
        """State (x, p, C) in the frame of a sector at azimuth larger by delta."""
        xx = np.array([x], dtype=np.float64)
        p = np.array(p, dtype=np.float64)
        Cv = np.zeros(15) if Cov is None else np.array(Cov, dtype=np.float64)
        J = np.zeros(25)
        rc = self.lib.orc_rotate(C.byref(self.cfg), float(delta), _dp(xx), _dp(p), _dp(Cv), _dp(J))
        return rc == 0, float(xx[0]), p, Cv, J.reshape(5, 5)

    def fit_hits_sectors(self, x, y, z, sec):
        x, y, z = (np.ascontiguousarray(v, dtype=np.float64) for v in (x, y, z))
        sec = np.ascontiguousarray(sec, dtype=np.int32)
        p = np.zeros(5)
        Cv = np.zeros(15)
        chi2 = np.zeros(1)
        rc = self.lib.orc_fit_hits_sectors(C.byref(self.cfg), int(x.shape[0]), _dp(x), _dp(y), _dp(z),
                                           _ptr(sec), _dp(p), _dp(Cv), _dp(chi2))
        return rc == 0, p, Cv, float(chi2[0])

    def beamline_z(self, x0, p):
        """z at the beam line of the helix of state p at plane x0 (continuous-readout z estimate, Sec. 6)."""
        p = np.array(p, dtype=np.float64)
        return float(self.lib.orc_beamline_z(C.byref(self.cfg), float(x0), _dp(p)))

    def seed(self, x, y, z):
        x, y, z = (np.array(v, dtype=np.float64) for v in (x, y, z))
        p = np.zeros(5)
        rc = self.lib.orc_seed(C.byref(self.cfg), _dp(x), _dp(y), _dp(z), _dp(p))
        return rc == 0, p

    def update(self, my, mz, p, Cov):
        p = np.array(p, dtype=np.float64)
        Cv = np.array(Cov, dtype=np.float64)
        chi2 = self.lib.orc_update(C.byref(self.cfg), my, mz, _dp(p), _dp(Cv))
        return chi2, p, Cv

    def fit_hits(self, x, y, z):
        x, y, z = (np.ascontiguousarray(v, dtype=np.float64) for v in (x, y, z))
        p = np.zeros(5)
        Cv = np.zeros(15)
        chi2 = np.zeros(1)
        po = np.zeros(5)
        rc = self.lib.orc_fit_hits(C.byref(self.cfg), int(x.shape[0]), _dp(x), _dp(y), _dp(z),
                                   _dp(p), _dp(Cv), _dp(chi2), _dp(po))
        return rc == 0, p, Cv, float(chi2[0]), po


def lower_to_full(c15):
    """15-element lower triangle (row-major) -> symmetric 5x5."""
    c15 = np.asarray(c15)
    M = np.zeros(c15.shape[:-1] + (5, 5))
    k = 0
    for i in range(5):
        for j in range(i + 1):
            M[..., i, j] = c15[..., k]
            M[..., j, i] = c15[..., k]
            k += 1
    return M
