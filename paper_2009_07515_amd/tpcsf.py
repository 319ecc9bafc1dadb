"""Python binding of libtpcsf (include/tpcsf.h): argument marshalling only.

Every step of the tracking runs in the HIP kernels of libtpcsf.so; this module passes
torch device pointers, sizes and the current HIP stream through the C ABI, and wraps the
results as torch tensors.  There is no CPU fallback: if the library is missing or no GPU
is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpcsf.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "tpcsf.h")

OK, E_INVALID, E_NOMEM, E_CAPACITY, E_HIP, E_BUSY, E_TIMEOUT = 0, -1, -2, -3, -4, -5, -6
NOALLOC_SCRATCH_BYTES = 256 << 20   # TPCSF_NOALLOC_SCRATCH_BYTES of the header
_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_CAPACITY", -4: "E_HIP", -5: "E_BUSY",
          -6: "E_TIMEOUT"}


class TpcsfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tpcsf {_NAMES.get(status, status)}: {msg}")
        self.status = status


class Geometry(C.Structure):
    _fields_ = [("n_sectors", C.c_int32), ("n_rows", C.c_int32), ("row_x", C.c_void_p), ("bz", C.c_double)]


class Params(C.Structure):
    _fields_ = [("win_y", C.c_float), ("win_z", C.c_float), ("kink_max", C.c_float),
                ("sigma_y", C.c_double), ("sigma_z", C.c_double), ("chi2_max", C.c_double),
                ("sinphi_max", C.c_double), ("nsig", C.c_double), ("c0", C.c_double * 5),
                ("min_chain", C.c_int32), ("min_track_hits", C.c_int32), ("max_miss", C.c_int32),
                ("merge_edge", C.c_double), ("merge_window", C.c_double), ("merge_chi2", C.c_double),
                ("reject_pt_min", C.c_double), ("reject_window", C.c_double), ("resid_step", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["c0"] = tuple(self.c0)
        return d


class Tuning(C.Structure):
    _fields_ = [("bin_y", C.c_float), ("bin_z", C.c_float), ("cap_mul", C.c_int32), ("cap_add", C.c_int32),
                ("block", C.c_int32), ("tl_block", C.c_int32), ("chunk", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FrameDesc(C.Structure):
    _fields_ = [("n_tf", C.c_int32), ("n_clusters", C.c_int64), ("y", C.c_void_p), ("z", C.c_void_p),
                ("row_offsets", C.c_void_p), ("row_offsets_host", C.c_void_p)]


class TracksDesc(C.Structure):
    _fields_ = [("cap_tracks", C.c_int64), ("cap_hits", C.c_int64), ("n_tracks", C.c_void_p),
                ("n_hits", C.c_void_p), ("params", C.c_void_p), ("cov", C.c_void_p), ("x_ref", C.c_void_p),
                ("chi2", C.c_void_p), ("ndf", C.c_void_p), ("nhits", C.c_void_p), ("sector", C.c_void_p),
                ("tf", C.c_void_p), ("hit_off", C.c_void_p), ("hit_ids", C.c_void_p),
                ("cluster_track", C.c_void_p), ("z_beam", C.c_void_p), ("params_outer", C.c_void_p),
                ("cov_outer", C.c_void_p), ("hit_rec", C.c_void_p)]


class MergedDesc(C.Structure):
    _fields_ = [("cap_merged", C.c_int64), ("cap_hits", C.c_int64), ("n_merged", C.c_void_p),
                ("n_hits", C.c_void_p)] + [(k, C.c_void_p) for k in
                                           ("params", "cov", "x_ref", "chi2", "z_beam", "ndf", "nhits", "sector",
                                            "tf", "n_segments", "hit_off", "hit_ids", "track_merged", "next",
                                            "link_chi2")]


class HostTracks(C.Structure):
    _fields_ = [("cap_tracks", C.c_int64), ("cap_hits", C.c_int64), ("n_tracks", C.c_int64), ("n_hits", C.c_int64),
                ("params", C.c_void_p), ("cov", C.c_void_p), ("x_ref", C.c_void_p), ("chi2", C.c_void_p),
                ("ndf", C.c_void_p), ("nhits", C.c_void_p), ("sector", C.c_void_p), ("hit_off", C.c_void_p),
                ("hit_ids", C.c_void_p), ("cluster_track", C.c_void_p), ("z_beam", C.c_void_p)]


class DebugView(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("row_lo", "row_bin", "row_nb", "bin_start", "perm", "up", "dn",
                                           "cup", "cdn", "n_starts", "start_row", "start_idx", "tl_nhits",
                                           "work")]


_lib = None


def load():
    """Load libtpcsf.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2009_07515_amd.build` first")
    # torch ships its own HIP runtime under the same soname; load it first so that the
    # library and torch's allocator and streams share one runtime in this process
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.tpcsf_default_params.argtypes = [C.POINTER(Params)]
    lib.tpcsf_default_params.restype = None
    lib.tpcsf_default_tuning.argtypes = [C.POINTER(Tuning)]
    lib.tpcsf_default_tuning.restype = None
    lib.tpcsf_create.argtypes = [C.POINTER(Geometry), C.POINTER(Params), C.POINTER(Tuning), C.c_size_t,
                                 C.POINTER(vp)]
    lib.tpcsf_create.restype = C.c_int
    lib.tpcsf_destroy.argtypes = [vp]
    lib.tpcsf_destroy.restype = C.c_int
    lib.tpcsf_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
    lib.tpcsf_set_tuning.restype = C.c_int
    lib.tpcsf_arena_bytes.argtypes = [vp, C.c_int64, C.c_int32]
    lib.tpcsf_arena_bytes.restype = C.c_size_t
    for fn in ("tpcsf_track_plain", "tpcsf_track_batch", "tpcsf_track_batch_noalloc"):
        getattr(lib, fn).argtypes = [vp, C.POINTER(FrameDesc), C.POINTER(TracksDesc), vp]
        getattr(lib, fn).restype = C.c_int
    lib.tpcsf_merge.argtypes = [vp, C.POINTER(FrameDesc), C.POINTER(TracksDesc), C.POINTER(MergedDesc), vp]
    lib.tpcsf_merge.restype = C.c_int
    lib.tpcsf_merge_work.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.tpcsf_reject.argtypes = [vp, C.POINTER(FrameDesc), C.POINTER(TracksDesc), vp, vp, vp]
    lib.tpcsf_reject.restype = C.c_int
    lib.tpcsf_compress.argtypes = [vp, C.POINTER(FrameDesc), C.POINTER(TracksDesc), vp, vp, vp]
    lib.tpcsf_compress.restype = C.c_int
    lib.tpcsf_decompress.argtypes = [vp, C.POINTER(TracksDesc), vp, vp, vp, vp]
    lib.tpcsf_decompress.restype = C.c_int
    lib.tpcsf_merge_work.restype = C.c_int
    lib.tpcsf_sync.argtypes = [vp, vp]
    lib.tpcsf_sync.restype = C.c_int
    lib.tpcsf_debug.argtypes = [vp, C.POINTER(DebugView)]
    lib.tpcsf_debug.restype = C.c_int
    lib.tpcsf_set_stage_timing.argtypes = [vp, C.c_int32]
    lib.tpcsf_set_stage_timing.restype = C.c_int
    lib.tpcsf_stage_count.argtypes = []
    lib.tpcsf_stage_count.restype = C.c_int32
    lib.tpcsf_stage_name.argtypes = [C.c_int32]
    lib.tpcsf_stage_name.restype = C.c_char_p
    lib.tpcsf_stage_times.argtypes = [vp, C.POINTER(C.c_float), C.c_int32]
    lib.tpcsf_stage_times.restype = C.c_int
    lib.tpcsf_last_error.argtypes = [vp]
    lib.tpcsf_last_error.restype = C.c_char_p
    lib.tpcsf_reserve.argtypes = [vp, C.c_int64, C.c_int32]
    lib.tpcsf_reserve.restype = C.c_int
    lib.tpcsf_autotune.argtypes = [vp, C.POINTER(FrameDesc), C.POINTER(TracksDesc), C.POINTER(Tuning), C.c_int32,
                                   C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_int32), vp]
    lib.tpcsf_autotune.restype = C.c_int
    lib.tpcsf_server_create.argtypes = [C.POINTER(Geometry), C.POINTER(Params), C.POINTER(Tuning), C.c_int32,
                                        C.c_size_t, C.POINTER(vp)]
    lib.tpcsf_server_create.restype = C.c_int
    lib.tpcsf_server_destroy.argtypes = [vp]
    lib.tpcsf_server_destroy.restype = C.c_int
    lib.tpcsf_server_submit.argtypes = [vp, vp, vp, vp, C.c_int64, C.POINTER(C.c_uint64)]
    lib.tpcsf_server_submit.restype = C.c_int
    lib.tpcsf_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int32)]
    lib.tpcsf_server_poll.restype = C.c_int
    lib.tpcsf_server_wait.argtypes = [vp, C.c_uint64, C.c_int64]
    lib.tpcsf_server_wait.restype = C.c_int
    lib.tpcsf_server_result.argtypes = [vp, C.c_uint64, C.POINTER(HostTracks)]
    lib.tpcsf_server_result.restype = C.c_int
    lib.tpcsf_server_bytes_used.argtypes = [vp]
    lib.tpcsf_server_bytes_used.restype = C.c_size_t
    lib.tpcsf_server_last_error.argtypes = [vp]
    lib.tpcsf_server_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def header_symbols():
    """Function names declared in include/tpcsf.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(tpcsf_[a-z_]+)\s*\(", txt)))


def default_params():
    p = Params()
    load().tpcsf_default_params(C.byref(p))
    return p


def default_tuning():
    t = Tuning()
    load().tpcsf_default_tuning(C.byref(t))
    return t


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class DeviceFrame:
    """A batch of time frames resident in device memory (torch tensors) plus the host copy
    of the row offsets the library validates."""

    def __init__(self, y, z, row_off, row_off_host, n_tf):
        self.y, self.z, self.row_off = y, z, row_off
        self.row_off_host = np.ascontiguousarray(row_off_host, dtype=np.int64)
        self.n_tf = int(n_tf)

    @property
    def n_clusters(self):
        return int(self.y.shape[0])

    @classmethod
    def from_numpy(cls, y, z, row_off, n_tf=1, device="cuda"):
        import torch
        y = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(device)
        z = torch.from_numpy(np.ascontiguousarray(z, dtype=np.float32)).to(device)
        ro = np.ascontiguousarray(row_off, dtype=np.int64)
        return cls(y, z, torch.from_numpy(ro).to(device), ro, n_tf)

    def desc(self):
        d = FrameDesc()
        d.n_tf = self.n_tf
        d.n_clusters = self.n_clusters
        d.y = _ptr(self.y) if self.n_clusters else None
        d.z = _ptr(self.z) if self.n_clusters else None
        d.row_offsets = _ptr(self.row_off)
        d.row_offsets_host = self.row_off_host.ctypes.data_as(C.c_void_p)
        return d


class TrackBuffers:
    """Caller-owned output buffers (device).  Default capacities are exact upper bounds:
    a track keeps >= min_track_hits clusters and no cluster is in two tracks."""

    def __init__(self, n_clusters, cap_tracks=None, cap_hits=None, min_track_hits=20, device="cuda",
                 outer=False, hit_rec=False):
        import torch
        n = int(n_clusters)
        self.cap_tracks = int(cap_tracks if cap_tracks is not None else n // max(1, min_track_hits) + 1)
        self.cap_hits = int(cap_hits if cap_hits is not None else n)
        T, H = self.cap_tracks, self.cap_hits
        kw = dict(device=device)
        self.n_tracks = torch.zeros(1, dtype=torch.int64, **kw)
        self.n_hits = torch.zeros(1, dtype=torch.int64, **kw)
        self.params = torch.empty((max(T, 1), 5), dtype=torch.float64, **kw)
        self.cov = torch.empty((max(T, 1), 15), dtype=torch.float64, **kw)
        self.x_ref = torch.empty(max(T, 1), dtype=torch.float64, **kw)
        self.chi2 = torch.empty(max(T, 1), dtype=torch.float64, **kw)
        self.ndf = torch.empty(max(T, 1), dtype=torch.int32, **kw)
        self.nhits = torch.empty(max(T, 1), dtype=torch.int32, **kw)
        self.sector = torch.empty(max(T, 1), dtype=torch.int32, **kw)
        self.tf = torch.empty(max(T, 1), dtype=torch.int32, **kw)
        self.hit_off = torch.zeros(T + 1, dtype=torch.int64, **kw)
        self.hit_ids = torch.empty(max(H, 1), dtype=torch.int32, **kw)
        self.cluster_track = torch.empty(max(n, 1), dtype=torch.int32, **kw)
        self.z_beam = torch.empty(max(T, 1), dtype=torch.float64, **kw)
        # outer states (input of the merge) only on request
        self.params_outer = torch.empty((max(T, 1), 5), dtype=torch.float64, **kw) if outer else None
        self.cov_outer = torch.empty((max(T, 1), 15), dtype=torch.float64, **kw) if outer else None
        # per-hit cluster records (y, z, row plane x, index bits), read by merge and compress
        self.hit_rec = torch.empty((max(H, 1), 4), dtype=torch.float32, **kw) if hit_rec else None

    def desc(self):
        d = TracksDesc()
        d.cap_tracks, d.cap_hits = self.cap_tracks, self.cap_hits
        for k in ("n_tracks", "n_hits", "params", "cov", "x_ref", "chi2", "ndf", "nhits", "sector", "tf",
                  "hit_off", "hit_ids", "cluster_track", "z_beam"):
            setattr(d, k, _ptr(getattr(self, k)))
        if self.params_outer is not None:
            d.params_outer, d.cov_outer = _ptr(self.params_outer), _ptr(self.cov_outer)
        if self.hit_rec is not None:
            d.hit_rec = _ptr(self.hit_rec)
        return d

    def result(self, n_clusters):
        """Slices of the buffers holding the last call's tracks (after a sync)."""
        T = int(self.n_tracks.item())
        H = int(self.n_hits.item())
        return dict(n_tracks=T, n_hits=H, params=self.params[:T], cov=self.cov[:T], x_ref=self.x_ref[:T],
                    chi2=self.chi2[:T], ndf=self.ndf[:T], nhits=self.nhits[:T], sector=self.sector[:T],
                    tf=self.tf[:T], hit_off=self.hit_off[:T + 1], hit_ids=self.hit_ids[:H],
                    cluster_track=self.cluster_track[:n_clusters], z_beam=self.z_beam[:T],
                    **({} if self.params_outer is None else
                       dict(params_outer=self.params_outer[:T], cov_outer=self.cov_outer[:T])))


class MergedBuffers:
    """Caller-owned output of the merge (device).  Default capacities hold every input
    track as its own merged track."""

    def __init__(self, tracks: "TrackBuffers", device="cuda"):
        import torch
        T, H = tracks.cap_tracks, tracks.cap_hits
        self.cap_merged, self.cap_hits = T, H
        kw = dict(device=device)
        f64 = dict(dtype=torch.float64, **kw)
        i32 = dict(dtype=torch.int32, **kw)
        self.n_merged = torch.zeros(1, dtype=torch.int64, **kw)
        self.n_hits = torch.zeros(1, dtype=torch.int64, **kw)
        self.params = torch.empty((max(T, 1), 5), **f64)
        self.cov = torch.empty((max(T, 1), 15), **f64)
        self.x_ref = torch.empty(max(T, 1), **f64)
        self.chi2 = torch.empty(max(T, 1), **f64)
        self.z_beam = torch.empty(max(T, 1), **f64)
        self.ndf = torch.empty(max(T, 1), **i32)
        self.nhits = torch.empty(max(T, 1), **i32)
        self.sector = torch.empty(max(T, 1), **i32)
        self.tf = torch.empty(max(T, 1), **i32)
        self.n_segments = torch.empty(max(T, 1), **i32)
        self.hit_off = torch.zeros(T + 1, dtype=torch.int64, **kw)
        self.hit_ids = torch.empty(max(H, 1), **i32)
        self.track_merged = torch.empty(max(T, 1), **i32)
        self.next = torch.empty(max(T, 1), **i32)
        self.link_chi2 = torch.empty(max(T, 1), **f64)

    def desc(self):
        d = MergedDesc()
        d.cap_merged, d.cap_hits = self.cap_merged, self.cap_hits
        for k, _ in MergedDesc._fields_[2:]:
            setattr(d, k, _ptr(getattr(self, k)))
        return d

    def result(self, n_tracks):
        """Slices holding the last merge's output (after a sync); n_tracks input tracks."""
        M = int(self.n_merged.item())
        H = int(self.n_hits.item())
        out = {k: getattr(self, k)[:M] for k in ("params", "cov", "x_ref", "chi2", "z_beam", "ndf", "nhits",
                                                  "sector", "tf", "n_segments")}
        out.update(n_merged=M, n_hits=H, hit_off=self.hit_off[:M + 1], hit_ids=self.hit_ids[:H],
                   track_merged=self.track_merged[:n_tracks], next=self.next[:n_tracks],
                   link_chi2=self.link_chi2[:n_tracks])
        return out


class Tracker:
    """A tpcsf context on the current HIP device."""

    def __init__(self, row_x, bz=0.5, n_sectors=36, params=None, tuning=None, hbm_budget=0):
        lib = load()
        self.lib = lib
        self.row_x = np.ascontiguousarray(row_x, dtype=np.float32)
        self.n_sectors = int(n_sectors)
        self.n_rows = int(self.row_x.shape[0])
        geo = Geometry(self.n_sectors, self.n_rows, self.row_x.ctypes.data_as(C.c_void_p), float(bz))
        p = default_params()
        for k, v in (params or {}).items():
            if k == "c0":
                p.c0 = (C.c_double * 5)(*v)
            else:
                setattr(p, k, v)
        t = default_tuning()
        for k, v in (tuning or {}).items():
            setattr(t, k, v)
        self.params, self.tuning = p, t
        h = C.c_void_p()
        st = lib.tpcsf_create(C.byref(geo), C.byref(p), C.byref(t), int(hbm_budget), C.byref(h))
        if st != OK:
            raise TpcsfError(st, "tpcsf_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.tpcsf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != OK:
            raise TpcsfError(st, self.lib.tpcsf_last_error(self.h).decode())

    def set_tuning(self, **kw):
        t = Tuning.from_buffer_copy(self.tuning)
        for k, v in kw.items():
            setattr(t, k, v)
        self._check(self.lib.tpcsf_set_tuning(self.h, C.byref(t)))
        self.tuning = t

    def arena_bytes(self, n_clusters, n_tf=1):
        return int(self.lib.tpcsf_arena_bytes(self.h, int(n_clusters), int(n_tf)))

    @staticmethod
    def _stream(stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        return C.c_void_p(s.cuda_stream)

    def launch(self, frame: DeviceFrame, out: TrackBuffers, mode="batch", stream=None):
        """Enqueue one tracking call (no sync)."""
        fd, od = frame.desc(), out.desc()
        fn = {"batch": self.lib.tpcsf_track_batch, "plain": self.lib.tpcsf_track_plain,
              "noalloc": self.lib.tpcsf_track_batch_noalloc}[mode]
        self._check(fn(self.h, C.byref(fd), C.byref(od), self._stream(stream)))

    def sync(self, stream=None):
        self._check(self.lib.tpcsf_sync(self.h, self._stream(stream)))

    def track(self, frame: DeviceFrame, mode="batch", out=None, stream=None):
        """Track a batch and return the result tensors (synchronises)."""
        if out is None:
            out = TrackBuffers(frame.n_clusters, min_track_hits=self.params.min_track_hits)
        self.launch(frame, out, mode, stream)
        self.sync(stream)
        return out.result(frame.n_clusters)

    def launch_merge(self, frame: DeviceFrame, tracks: TrackBuffers, out: "MergedBuffers", stream=None):
        """Enqueue the merge of a batch's sector tracks (no sync)."""
        fd, td, md = frame.desc(), tracks.desc(), out.desc()
        self._check(self.lib.tpcsf_merge(self.h, C.byref(fd), C.byref(td), C.byref(md), self._stream(stream)))

    def merge(self, frame: DeviceFrame, tracks: TrackBuffers, out=None, stream=None):
        """Merge the sector tracks of the last tracking call on `frame` (held in `tracks`,
        made with outer=True) across sector edges and refit; returns the merged tracks."""
        if out is None:
            out = MergedBuffers(tracks)
        self.launch_merge(frame, tracks, out, stream)
        self.sync(stream)
        return out.result(int(tracks.n_tracks.item()))

    def launch_reject(self, frame: DeviceFrame, tracks: TrackBuffers, keep, n_kept, stream=None):
        """Enqueue the strategy-B hit removal for the last tracking call (no sync)."""
        fd, td = frame.desc(), tracks.desc()
        self._check(self.lib.tpcsf_reject(self.h, C.byref(fd), C.byref(td), _ptr(keep), _ptr(n_kept),
                                          self._stream(stream)))

    def reject(self, frame: DeviceFrame, tracks: TrackBuffers, stream=None):
        """Keep flags (uint8, input order) and kept count of the strategy-B hit removal for
        the sector tracks of the last tracking call on `frame` (synchronises)."""
        import torch
        keep = torch.empty(max(frame.n_clusters, 1), dtype=torch.uint8, device=frame.y.device)
        n_kept = torch.zeros(1, dtype=torch.int64, device=frame.y.device)
        self.launch_reject(frame, tracks, keep, n_kept, stream)
        self.sync(stream)
        return keep[:frame.n_clusters], int(n_kept.item())

    def launch_compress(self, frame: DeviceFrame, tracks: TrackBuffers, codes, rows, stream=None):
        fd, td = frame.desc(), tracks.desc()
        self._check(self.lib.tpcsf_compress(self.h, C.byref(fd), C.byref(td), _ptr(codes), _ptr(rows),
                                            self._stream(stream)))

    def launch_decompress(self, tracks: TrackBuffers, codes, rows, yz, stream=None):
        td = tracks.desc()
        self._check(self.lib.tpcsf_decompress(self.h, C.byref(td), _ptr(codes), _ptr(rows), _ptr(yz),
                                              self._stream(stream)))

    def compress(self, frame: DeviceFrame, tracks: TrackBuffers, stream=None):
        """Residual codes [H, 2] (int32) and rows [H] (uint8) of the tracks' clusters, in
        hit-list order (synchronises)."""
        import torch
        H = max(tracks.cap_hits, 1)
        codes = torch.empty((H, 2), dtype=torch.int32, device=frame.y.device)
        rows = torch.empty(H, dtype=torch.uint8, device=frame.y.device)
        self.launch_compress(frame, tracks, codes, rows, stream)
        self.sync(stream)
        n = int(tracks.n_hits.item())
        return codes[:n], rows[:n]

    def decompress(self, tracks: TrackBuffers, codes, rows, stream=None):
        """Decoded cluster positions [H, 2] (float64) from the codes and rows (synchronises)."""
        import torch
        H = max(tracks.cap_hits, 1)
        c = torch.zeros((H, 2), dtype=torch.int32, device=codes.device)
        r = torch.zeros(H, dtype=torch.uint8, device=codes.device)
        c[:codes.shape[0]] = codes
        r[:rows.shape[0]] = rows
        yz = torch.empty((H, 2), dtype=torch.float64, device=codes.device)
        self.launch_decompress(tracks, c, r, yz, stream)
        self.sync(stream)
        return yz[:codes.shape[0]]

    def merge_work(self):
        w = (C.c_int64 * 6)()
        self._check(self.lib.tpcsf_merge_work(self.h, w))
        return np.array(list(w), np.int64)

    def reserve(self, max_clusters, max_tf=1):
        """Fix the scratch layout to this capacity (one graph then serves smaller batches)."""
        self._check(self.lib.tpcsf_reserve(self.h, int(max_clusters), int(max_tf)))

    def autotune(self, frame: DeviceFrame, points=None, reps=3, out=None, stream=None):
        """Time the batched form at each tuning point, check that all give the same result,
        and keep the fastest.  Returns (best index, ms per point, tuning points)."""
        pts = [dict(self.tuning.as_dict(), **p) for p in (points or default_sweep())]
        arr = (Tuning * len(pts))()
        for i, p in enumerate(pts):
            for k, v in p.items():
                setattr(arr[i], k, v)
        if out is None:
            out = TrackBuffers(frame.n_clusters, min_track_hits=self.params.min_track_hits)
        ms = (C.c_float * len(pts))()
        best = C.c_int32(-1)
        fd, od = frame.desc(), out.desc()
        self._check(self.lib.tpcsf_autotune(self.h, C.byref(fd), C.byref(od), arr, len(pts), int(reps), ms,
                                            C.byref(best), self._stream(stream)))
        self.tuning = Tuning.from_buffer_copy(arr[best.value])
        return best.value, [float(v) for v in ms], pts

    def set_stage_timing(self, on=True):
        self._check(self.lib.tpcsf_set_stage_timing(self.h, 1 if on else 0))

    def stage_names(self):
        return [self.lib.tpcsf_stage_name(i).decode() for i in range(self.lib.tpcsf_stage_count())]

    def stage_times(self):
        """{stage: ms} of the last timed batched call (after a sync)."""
        n = self.lib.tpcsf_stage_count()
        buf = (C.c_float * n)()
        self._check(self.lib.tpcsf_stage_times(self.h, buf, n))
        return dict(zip(self.stage_names(), [float(v) for v in buf]))

    def debug(self, frame: DeviceFrame):
        """Copies of the last call's intermediate arrays (grid, links, starts)."""
        import torch
        v = DebugView()
        self._check(self.lib.tpcsf_debug(self.h, C.byref(v)))
        n, R = frame.n_clusters, frame.n_tf * self.n_sectors * self.n_rows

        torch.cuda.synchronize()

        def dev(ptr, count, dtype):
            buf = np.empty(count, dtype=dtype)
            if count:
                _memcpy_d2h(buf.ctypes.data, ptr, buf.nbytes)
            return buf

        ns = int(dev(v.n_starts, 1, np.int64)[0])
        res = dict(row_lo=dev(v.row_lo, 2 * R, np.float32).reshape(R, 2),
                   row_bin=dev(v.row_bin, 2 * R, np.float32).reshape(R, 2),
                   row_nb=dev(v.row_nb, 2 * R, np.int32).reshape(R, 2),
                   perm=dev(v.perm, n, np.uint32), up=dev(v.up, n, np.int32), dn=dev(v.dn, n, np.int32),
                   cup=dev(v.cup, n, np.int32), cdn=dev(v.cdn, n, np.int32), n_starts=ns,
                   start_row=dev(v.start_row, ns, np.int32), start_idx=dev(v.start_idx, ns, np.int32),
                   tl_nhits=dev(v.tl_nhits, ns, np.int32), work=dev(v.work, 6, np.int64))
        t = self.tuning
        nb_total = int(t.cap_mul) * n + (int(t.cap_add) + 1) * R
        res["bin_start"] = dev(v.bin_start, nb_total, np.uint32)
        return res


def default_sweep():
    """Tuning points of the autotuner: grid bin sizes and bin cap crossed with launch
    shapes (row-kernel block, tracklet block, work-queue chunk)."""
    bins = [dict(bin_y=1.0, bin_z=2.0, cap_mul=2), dict(bin_y=2.0, bin_z=2.0, cap_mul=2),
            dict(bin_y=4.0, bin_z=4.0, cap_mul=2), dict(bin_y=2.0, bin_z=4.0, cap_mul=4),
            dict(bin_y=3.0, bin_z=3.0, cap_mul=8), dict(bin_y=16.0, bin_z=1.0, cap_mul=4),
            # one y-bin per row: a window's z-bins form one contiguous range
            dict(bin_y=1000.0, bin_z=0.5, cap_mul=2), dict(bin_y=1000.0, bin_z=1.0, cap_mul=2),
            dict(bin_y=1000.0, bin_z=2.0, cap_mul=2)]
    shapes = [dict(block=256, tl_block=256, chunk=1), dict(block=128, tl_block=128, chunk=1),
              dict(block=256, tl_block=64, chunk=1), dict(block=512, tl_block=256, chunk=2),
              dict(block=1024, tl_block=256, chunk=1)]
    return [dict(b, **sh) for b in bins for sh in shapes]


class Server:
    """Continuous-batching server of the library (see tpcsf_server_* in the header)."""

    def __init__(self, row_x, bz=0.5, n_sectors=36, params=None, tuning=None, n_slots=4, hbm_budget=0):
        lib = load()
        self.lib = lib
        self.row_x = np.ascontiguousarray(row_x, dtype=np.float32)
        self.n_sectors, self.n_rows = int(n_sectors), int(self.row_x.shape[0])
        geo = Geometry(self.n_sectors, self.n_rows, self.row_x.ctypes.data_as(C.c_void_p), float(bz))
        p = default_params()
        for k, v in (params or {}).items():
            if k == "c0":
                p.c0 = (C.c_double * 5)(*v)
            else:
                setattr(p, k, v)
        t = default_tuning()
        for k, v in (tuning or {}).items():
            setattr(t, k, v)
        self.params = p
        h = C.c_void_p()
        st = lib.tpcsf_server_create(C.byref(geo), C.byref(p), C.byref(t), int(n_slots), int(hbm_budget), C.byref(h))
        if st != OK:
            raise TpcsfError(st, "tpcsf_server_create failed")
        self.h = h
        self._inputs = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.tpcsf_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != OK:
            raise TpcsfError(st, self.lib.tpcsf_server_last_error(self.h).decode())

    def submit(self, y, z, row_off):
        """Admit a frame (numpy arrays; pinned memory makes the upload asynchronous).
        Returns a ticket, or None if the server is busy (an admission stall)."""
        y = np.ascontiguousarray(y, dtype=np.float32)
        z = np.ascontiguousarray(z, dtype=np.float32)
        ro = np.ascontiguousarray(row_off, dtype=np.int64)
        t = C.c_uint64()
        st = self.lib.tpcsf_server_submit(self.h, y.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p),
                                          ro.ctypes.data_as(C.c_void_p), int(y.shape[0]), C.byref(t))
        if st == E_BUSY:
            return None
        self._check(st)
        self._inputs[t.value] = (y, z, ro)      # keep the host arrays alive until done
        return t.value

    def poll(self, ticket):
        d = C.c_int32()
        self._check(self.lib.tpcsf_server_poll(self.h, ticket, C.byref(d)))
        return bool(d.value)

    def wait(self, ticket, timeout_s=-1.0):
        st = self.lib.tpcsf_server_wait(self.h, ticket, int(timeout_s * 1e6) if timeout_s >= 0 else -1)
        if st == E_TIMEOUT:
            return False
        self._check(st)
        return True

    def release(self, ticket):
        """Release a completed frame's slot without copying its tracks."""
        st = self.lib.tpcsf_server_result(self.h, ticket, None)
        del self._inputs[ticket]
        self._check(st)

    def result(self, ticket):
        """Tracks of a completed frame as numpy arrays; releases its slot."""
        y, _, _ = self._inputs[ticket]
        n = int(y.shape[0])
        T = n // max(1, self.params.min_track_hits) + 1
        o = dict(params=np.zeros((T, 5)), cov=np.zeros((T, 15)), x_ref=np.zeros(T), chi2=np.zeros(T),
                 ndf=np.zeros(T, np.int32), nhits=np.zeros(T, np.int32), sector=np.zeros(T, np.int32),
                 hit_off=np.zeros(T + 1, np.int64), hit_ids=np.zeros(max(n, 1), np.int32),
                 cluster_track=np.zeros(max(n, 1), np.int32), z_beam=np.zeros(T))
        ht = HostTracks(T, n, 0, 0, *[o[k].ctypes.data_as(C.c_void_p) for k in
                                      ("params", "cov", "x_ref", "chi2", "ndf", "nhits", "sector", "hit_off",
                                       "hit_ids", "cluster_track", "z_beam")])
        st = self.lib.tpcsf_server_result(self.h, ticket, C.byref(ht))
        del self._inputs[ticket]
        self._check(st)
        Tn, Hn = ht.n_tracks, ht.n_hits
        res = {k: v[:Tn] for k, v in o.items() if k not in ("hit_off", "hit_ids", "cluster_track")}
        res.update(n_tracks=Tn, n_hits=Hn, hit_off=o["hit_off"][:Tn + 1], hit_ids=o["hit_ids"][:Hn],
                   cluster_track=o["cluster_track"][:n])
        return res

    def bytes_used(self):
        return int(self.lib.tpcsf_server_bytes_used(self.h))


_hip = None


def _memcpy_d2h(dst, src, nbytes):
    """hipMemcpy device-to-host (used only to read the debug view of the arena)."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    rc = _hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(src), C.c_size_t(nbytes), 2)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
