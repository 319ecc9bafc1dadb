#!/usr/bin/env python3
"""Benchmark of TPC sector track finding on one MI355X.

Workload (the headline `value`): one 2 ms continuous-readout Pb-Pb time frame (Poisson
50 kHz collisions, Exp(1500) primaries each, 10% secondaries, 5% noise, z shifted by the
drift velocity times the collision time), all 36 sectors x 152 rows, generated with a
fixed seed.  The paper's Run 3 time frames are not available; this synthetic frame has
their shape.

A step is one batched tracking call over the whole time frame (every stage, every
sector, one HIP graph replay) with the clusters already resident in HBM.  The plain form
(every stage launched per sector) is timed beside it on the same input.  Besides the
step: the uneven batch of 64 time frames (pp-like and Pb-Pb-like) in one batched call,
autotuned on itself; the serving run (frames of that mix arriving by a Poisson process at
80% of the measured capacity for 60 s, admitted under a 64 GiB budget); the next stages
(merge, hit removal, compression); and the reference oracle on the host cores.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TPC clusters tracked/sec on 1 MI355X (batched vs plain) + p99 time-frame latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6      # MI355X binary64 vector peak (TFLOP/s)


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def stage_bytes(c):
    """Algorithmic HBM bytes of each stage: every stage-boundary array written once and
    read once where a later stage needs it (no re-reads, no atomics' extra traffic, no
    candidate scans).  c holds the counts of the measured input: N clusters, R rows, B bin
    entries, C clusters on cleaned chains, S starts, K tracklets, H_t tracklet clusters,
    H_c clusters of tracklets in the selection, F track candidates, H_a accepted clusters,
    T tracks, nr rows per sector."""
    N, R, B, C, S, K, Ht, Hc, F, Ha, T, nr = (c[k] for k in ("N", "R", "B", "C", "S", "K", "Ht", "Hc", "F", "Ha",
                                                             "T", "nr"))
    return {
        "reset": 0,
        # read y, z; write sorted (y, z), perm, inverse perm, bin table
        "grid": 8 * N + 16 * N + 4 * B,
        # read sorted (y, z), perm, bin tables; write up, dn
        "links": 12 * N + 4 * B + 8 * N,
        # read up, dn; write cleaned links; per-row start counts
        "clean": 16 * N + 8 * R,
        "row_scan": 16 * R,
        # read cleaned links and the inverse perm; write (row, position, rank) of every start
        "starts": 12 * N + 12 * S,
        # read starts and the chain links; write chain rows of the hit table, lengths
        "walk": 8 * S + 4 * C + 2 * C + 8 * S,
        # read start, chain coordinates (twice: fit and refit); write the hit table rows
        # outside the chain and the tracklet record with its selection weight
        "tracklets": 20 * K + 16 * Ht + 2 * nr * K,
        # read every tracklet's weight and row range, the hit-table entries of the
        # tracklets in the selection; write the weight of every cluster
        "claim": 8 * K + 2 * Hc + 4 * N,
        # read records, tables and weights; write kept masks and the candidate list
        "keep": 12 * K + 2 * nr * K + 4 * Hc + 40 * F,
        # read candidates, masks, kept coordinates (twice); write the fit results
        "fit": 44 * F + 16 * Ha + 2 * Ha + 176 * F,
        "track_scan": 24 * S,
        # read fit results, hit table entries and perm; write track records (with z at the
        # beam line) and hit lists
        "emit": 176 * T + 208 * T + 10 * Ha,
        # read inverse perm and weights, per assigned cluster its track's flag, index and
        # hit range (once per track); write the cluster->track map
        "assign": 12 * N + 24 * T,
    }


def coarse_bytes(c):
    """The same stages under the byte model of the method's stage-boundary arrays written
    once and read once in their minimal form (8-byte (y, z), 4-byte links, indices and
    weights): K1 grid 8N read + 8N sorted + 4N perm + 4B; K2 links 8N + 4B read, 8N links;
    K3 cleaning 16N; K4 starts 8N + 4S; K5 tracklets 12 per chain cluster + 8 per
    follow-window cluster + 4 per tracklet cluster + 80 per tracklet; K6 selection 4 per
    tracklet cluster + 8N weights + N flags; K7 final fit and emit 16 per accepted
    cluster + 100 per track + 4N cluster map."""
    N, B, S, K, Ht, Ha, T, C = (c[k] for k in ("N", "B", "S", "K", "Ht", "Ha", "T", "C"))
    W = c["work"]["tl_window_clusters"]
    return {"grid": 20 * N + 4 * B, "links": 16 * N + 4 * B, "clean": 16 * N, "starts": 8 * N + 4 * S,
            "tracklets": 12 * C + 8 * W + 4 * Ht + 80 * K, "selection": 4 * Ht + 9 * N,
            "fit_emit": 16 * Ha + 100 * T + 4 * N}


def counts_from(trk, frame, res, nr):
    d = trk.debug(frame)
    nb = d["row_nb"].astype(np.int64)
    tl = d["tl_nhits"].astype(np.int64)
    linked = int(((d["cup"] >= 0) | (d["cdn"] >= 0)).sum())
    w = [int(v) for v in d["work"]]
    return dict(N=frame.n_clusters, R=int(nb.shape[0]), B=int((nb[:, 0] * nb[:, 1] + 1).sum()), C=linked,
                S=int(d["n_starts"]), K=int((tl > 0).sum()), Ht=int(tl.sum()), Hc=int(tl[tl >= 20].sum()),
                F=int(res["n_tracks"]), Ha=int(res["n_hits"]), T=int(res["n_tracks"]), nr=nr,
                work=dict(tl_propagations=w[0], tl_updates=w[1], tl_window_clusters=w[2],
                          fit_propagations=w[3], fit_updates=w[4], fit_chi2=w[5]))


# binary64 floating-point operations of one step, counted from the formulas (an FMA is
# two, a division or square root one): helix propagation with its Jacobian and the
# covariance transport J C J^T; Kalman update with the 2x2 gain; chi2 of a cluster
# inside a follow window; chi2 of a cluster in the final fit
FLOPS_PROPAGATE, FLOPS_UPDATE, FLOPS_WINDOW, FLOPS_CHI2 = 182, 121, 12, 17
# the coarser per-step model of the method's description (propagation ~120, update ~130,
# window cluster ~20), reported beside it
COARSE_PROPAGATE, COARSE_UPDATE, COARSE_WINDOW = 120, 130, 20


def stage_flops(c):
    """Algorithmic binary64 operations of the Kalman stages, from the step counts of the
    call (the same counts the oracle takes for this input)."""
    w = c["work"]
    return {"tracklets": FLOPS_PROPAGATE * w["tl_propagations"] + FLOPS_UPDATE * w["tl_updates"]
            + FLOPS_WINDOW * w["tl_window_clusters"],
            "fit": FLOPS_PROPAGATE * w["fit_propagations"] + FLOPS_UPDATE * w["fit_updates"]
            + FLOPS_CHI2 * w["fit_chi2"]}


def kernel_source_sha():
    """sha256 over the tracking kernels' sources (kernels, then the shared Kalman code)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("tpcsf_kernels.hip", "tpcsf_kalman.h"):
        h.update(open(os.path.join(ROOT, "paper_2009_07515_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` (calibrated FETCH_SIZE + WRITE_SIZE) from the
    committed rocprofv3 summary, or None if the kernels changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "tpcsf_cfg3_counters.txt")
    if not os.path.exists(path):
        return None
    sha = kernel_source_sha()
    rec = {}
    for ln in open(path):
        f = ln.split()
        if f and f[0] == "source_sha256" and f[1] != sha:
            return None
        if f and f[0] == "kernel":
            rec[f[1]] = dict(zip(f[2::2], map(float, f[3::2])))
    r = rec.get("k_" + kernel)
    return None if r is None else r["fetch_bytes"] + r["write_bytes"]


def cpu_model():
    """CPU model name and the cores this process may run on (the machine's CPU share)."""
    name = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                name = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return name, avail, os.cpu_count() or 1


# sectors of the oracle samples, alternating between the two sides of the TPC
SECTOR_SAMPLE = [0, 18, 9, 27, 4, 22, 13, 31, 2, 20, 11, 29, 6, 24, 15, 33, 1, 19, 10, 28]


def cpu_threads(f, threads, n_sectors):
    """The FP64 oracle on a sample of whole sectors of the frame (about 2 s of CPU work
    each), one sector per task on `threads` host threads (the oracle's C calls release
    the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    from paper_2009_07515_amd import synth
    rx = synth.row_x()
    secs = SECTOR_SAMPLE[:n_sectors]

    def one(s):
        a, b = int(f.row_off[s * 152]), int(f.row_off[(s + 1) * 152])
        ro = f.row_off[s * 152:(s + 1) * 152 + 1] - a
        return oracle.Oracle(rx, n_sectors=1).track_frame(f.y[a:b], f.z[a:b], ro)["n_tracks"]

    n_cl = int(sum(f.row_off[(s + 1) * 152] - f.row_off[s * 152] for s in secs))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        n_tracks = sum(ex.map(one, secs))
    wall = time.perf_counter() - t0
    return dict(value=n_cl / wall, seconds=wall, tracks=int(n_tracks), threads=threads, sectors=secs, clusters=n_cl)


def cpu_baseline(f, budget_s, max_sectors):
    """The FP64 oracle on whole sectors of the same frame until ~budget_s of CPU time."""
    import oracle
    from paper_2009_07515_amd import synth
    o = oracle.Oracle(synth.row_x())
    R = 36 * 152
    counts = np.diff(f.row_off)
    done_cl, done_t, sectors = 0, 0.0, []
    for s in SECTOR_SAMPLE[:max_sectors]:
        sub = np.zeros(R, np.int64)
        sub[s * 152:(s + 1) * 152] = counts[s * 152:(s + 1) * 152]
        a, b = f.row_off[s * 152], f.row_off[(s + 1) * 152]
        ro = np.concatenate([[0], np.cumsum(sub)]).astype(np.int64)
        t0 = time.perf_counter()
        o.track_frame(f.y[a:b], f.z[a:b], ro)
        done_t += time.perf_counter() - t0
        done_cl += int(b - a)
        sectors.append(s)
        log(f"oracle sector {s}: {b - a} clusters, cumulative {done_t:.1f} s")
        if done_t >= budget_s:
            break
    return dict(value=done_cl / done_t, unit="clusters/s", cores=1, kind="oracle",
                sample=f"FP64 oracle, 1 thread, sectors {sectors} of the same time frame "
                       f"({done_cl} clusters, {done_t:.1f} s)")


def cpu_next_stages(f):
    """The oracle's merge, hit removal and compression timed on sectors 0 and 1 of the same
    frame (two neighbours, so that tracks cross their shared edge), after its tracking."""
    import oracle
    from paper_2009_07515_amd import synth
    o = oracle.Oracle(synth.row_x())
    R = 36 * 152
    counts = np.diff(f.row_off)
    sub = np.zeros(R, np.int64)
    sub[:2 * 152] = counts[:2 * 152]
    b = int(f.row_off[2 * 152])
    ro = np.concatenate([[0], np.cumsum(sub)]).astype(np.int64)
    y, z = f.y[:b], f.z[:b]
    t0 = time.perf_counter()
    r = o.track_frame(y, z, ro)
    t_track = time.perf_counter() - t0
    out = {}
    t0 = time.perf_counter()
    m = o.merge_frame(y, z, ro, r)
    t = time.perf_counter() - t0
    out["merge"] = {"value": r["n_tracks"] / t, "unit": "sector tracks/s", "seconds": t,
                    "merged_of_several": int((m["n_segments"] >= 2).sum())}
    t0 = time.perf_counter()
    o.reject_frame(y, z, ro, r)
    t = time.perf_counter() - t0
    out["reject"] = {"value": b / t, "unit": "clusters/s", "seconds": t}
    t0 = time.perf_counter()
    o.compress_frame(y, z, ro, r)
    t = time.perf_counter() - t0
    out["compress"] = {"value": r["n_hits"] / t, "unit": "attached clusters/s", "seconds": t}
    out["sample"] = (f"FP64 oracle, 1 thread, sectors 0 and 1 of the same time frame ({b} clusters, "
                     f"{r['n_tracks']} tracks; tracking them took {t_track:.1f} s, not counted)")
    out["cores"] = 1
    log(f"oracle next stages on sectors 0-1: merge {out['merge']['seconds']:.2f} s, reject "
        f"{out['reject']['seconds']:.2f} s, compress {out['compress']['seconds']:.2f} s")
    return out


def config4_sweep():
    """Tuning points of the uneven batch: grid bins (at most 4n + 64 bins per row, so that
    the layout reserved for the batch holds every point) crossed with launch shapes and
    work-queue chunks."""
    bins = [dict(bin_y=2.0, bin_z=2.0, cap_mul=2), dict(bin_y=2.0, bin_z=4.0, cap_mul=4),
            dict(bin_y=4.0, bin_z=4.0, cap_mul=2), dict(bin_y=1000.0, bin_z=1.0, cap_mul=2)]
    shapes = [dict(block=256, tl_block=256, chunk=1), dict(block=512, tl_block=256, chunk=2),
              dict(block=1024, tl_block=256, chunk=1), dict(block=256, tl_block=128, chunk=4)]
    return [dict(b, **sh) for b in bins for sh in shapes]


def bench_config4(frames, steps, plain_steps, autotune=True):
    """The uneven batch of 64 time frames in one batched call (one launch per stage over
    all 64 x 36 sectors, the tracklet stage from the persistent work queue, one graph),
    autotuned on itself; beside it the plain per-sector form and the frames tracked one
    call each (batched form per frame)."""
    import torch
    from paper_2009_07515_amd import synth, tpcsf
    y, z, ro = synth.concat_frames(frames)
    n, n_tf = int(y.shape[0]), len(frames)
    sizes = np.array([f.n_clusters for f in frames])
    sec = np.diff(ro[::152])
    stream = torch.cuda.current_stream()
    trk = tpcsf.Tracker(synth.row_x(), tuning=dict(bin_y=2.0, bin_z=4.0, cap_mul=4, block=512, tl_block=256,
                                                   chunk=2))
    trk.reserve(n, n_tf)
    fr = tpcsf.DeviceFrame.from_numpy(y, z, ro, n_tf=n_tf, device="cuda:0")
    out = tpcsf.TrackBuffers(n)
    tune = None
    if autotune:
        t0 = time.perf_counter()
        best, tms, pts = trk.autotune(fr, points=config4_sweep(), reps=2, out=out)
        tune = {"points": len(pts), "best": pts[best], "best_ms": tms[best], "worst_ms": max(tms),
                "seconds": time.perf_counter() - t0}
        log(f"config4 autotune: {len(pts)} points in {tune['seconds']:.1f} s, best {pts[best]} {tms[best]:.2f} ms "
            f"(slowest {max(tms):.2f} ms)")
    res = trk.track(fr, out=out, mode="batch")
    T, H = res["n_tracks"], res["n_hits"]
    for _ in range(2):
        trk.launch(fr, out, "batch")
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        trk.launch(fr, out, "batch")
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    trk.sync()
    assert int(out.n_tracks.item()) == T
    per = np.array([a.elapsed_time(b) for a, b in ev])
    log(f"config4 batched: {n} clusters in {n_tf} frames, {wall * 1e3:.2f} ms/step, {n / wall / 1e9:.3f} G clusters/s")
    plain = None
    if plain_steps > 0:
        trk.track(fr, out=out, mode="plain")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(plain_steps):
            trk.launch(fr, out, "plain")
        torch.cuda.synchronize()
        wp = (time.perf_counter() - t0) / plain_steps
        trk.sync()
        assert int(out.n_tracks.item()) == T
        plain = {"ms_per_step": wp * 1e3, "clusters_per_s": n / wp, "steps": plain_steps}
        log(f"config4 plain: {wp * 1e3:.1f} ms/step, {n / wp / 1e9:.3f} G clusters/s")
    # the frames one call each (batched form per frame, inputs already on the device)
    one = tpcsf.Tracker(synth.row_x(), tuning=trk.tuning.as_dict())
    one.reserve(int(sizes.max()), 1)
    t_one = 0.0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    base = 0
    for f in frames:
        rof = torch.from_numpy(f.row_off).to("cuda:0")
        fi = tpcsf.DeviceFrame(fr.y[base:base + f.n_clusters], fr.z[base:base + f.n_clusters], rof,
                               np.ascontiguousarray(f.row_off), 1)
        oi = tpcsf.TrackBuffers(f.n_clusters)
        one.launch(fi, oi, "batch")          # captures this frame's graph
        e0.record(stream)
        one.launch(fi, oi, "batch")
        e1.record(stream)
        torch.cuda.synchronize()
        t_one += e0.elapsed_time(e1) * 1e-3
        base += f.n_clusters
    one.sync()
    one.close()
    log(f"config4 frames one call each: {t_one * 1e3:.1f} ms in total, {n / t_one / 1e9:.3f} G clusters/s")
    tuning = trk.tuning.as_dict()
    del out, fr
    trk.close()
    torch.cuda.empty_cache()
    return {"workload": "64 time frames, even pp-like (0.5 ms at 500 kHz, Exp(30) tracks), odd Pb-Pb-like "
                        "(0.5-2 ms at 50 kHz, Exp(1500) tracks), in one batched call",
            "clusters": n, "time_frames": n_tf, "tracks": T, "assigned_clusters": H,
            "frame_clusters": {"min": int(sizes.min()), "max": int(sizes.max()), "mean": float(sizes.mean())},
            "sector_clusters": {"min": int(sec.min()), "max": int(sec.max())},
            "value": n / wall, "unit": "clusters/s", "ms_per_step": wall * 1e3, "steps": steps,
            "step_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99))},
            "plain": plain, "frames_one_call_each": {"ms": t_one * 1e3, "clusters_per_s": n / t_one},
            "autotune": tune, "tuning": tuning}


def serve(frames, tuning, seconds, n_slots, cap_seconds, budget_gib=64):
    """Serving run over the frames of the uneven mix.  The server (n_slots slots, a
    64 GiB HBM budget) first runs closed-loop with every slot kept busy, which gives its
    capacity; then frames arrive by a Poisson process at 80% of that capacity for
    `seconds` and are admitted first come, first served.  One host thread submits, a
    second one polls the admitted frames (polling drives the download of each finished
    frame's tracks) and releases them.  Per frame: arrival, admission and completion
    (tracks on the host) times.  An admission stall is an arrival that found no slot
    free or no budget left and had to wait."""
    import threading
    import torch
    from paper_2009_07515_amd import synth, tpcsf

    def pinned(a):
        return torch.from_numpy(np.ascontiguousarray(a)).pin_memory().numpy()

    t0 = time.perf_counter()
    pool = [(pinned(f.y), pinned(f.z), pinned(f.row_off)) for f in frames]
    sizes = np.array([f.n_clusters for f in frames], dtype=np.float64)
    log(f"serving pool: {len(pool)} frames pinned in {time.perf_counter() - t0:.1f} s")
    srv = tpcsf.Server(synth.row_x(), tuning=tuning, n_slots=n_slots, hbm_budget=budget_gib << 30)
    # grow the slots before timing: the largest frames, as many at once as the budget admits
    big = list(np.argsort(-sizes)[:n_slots])
    tks = [t for t in (srv.submit(*pool[i]) for i in big) if t is not None]
    for t in tks:
        srv.wait(t)
        srv.release(t)
    log(f"serving: {len(tks)} slots grown, {srv.bytes_used() / 2**30:.1f} GiB of device memory")

    lock = threading.Lock()
    inflight = {}           # ticket -> record
    done = []
    stop = threading.Event()

    def completer():
        while not stop.is_set() or inflight:
            with lock:
                items = list(inflight.items())
            for t, rec in items:
                if srv.poll(t):
                    rec["done"] = time.perf_counter()
                    srv.release(t)
                    with lock:
                        del inflight[t]
                        done.append(rec)
            time.sleep(5e-5)

    rng = np.random.Generator(np.random.PCG64(1005))

    # capacity: closed loop, every slot kept busy with frames drawn from the pool
    th = threading.Thread(target=completer)
    th.start()
    t_start = time.perf_counter()
    while time.perf_counter() - t_start < cap_seconds:
        w = int(rng.integers(0, len(pool)))
        while True:
            t = srv.submit(*pool[w])
            if t is not None:
                break
            time.sleep(5e-5)
        with lock:
            inflight[t] = {"w": w, "admit": time.perf_counter()}
    stop.set()
    th.join()
    cap_wall = time.perf_counter() - t_start
    capacity = sum(sizes[r["w"]] for r in done) / cap_wall
    log(f"serving capacity (closed loop, {n_slots} slots, {cap_wall:.1f} s, {len(done)} frames): "
        f"{capacity / 1e9:.3f} G clusters/s")

    # open loop: Poisson arrivals at 80% of that capacity, first come first served
    lam = 0.8 * capacity / sizes.mean()
    arrivals = np.cumsum(rng.exponential(1.0 / lam, int(seconds * lam * 1.5) + 16))
    arrivals = arrivals[arrivals < seconds]
    which = rng.integers(0, len(pool), arrivals.shape[0])
    done.clear()
    stop.clear()
    th = threading.Thread(target=completer)
    th.start()
    t_start = time.perf_counter()
    for a, w in zip(arrivals, which):
        ta = t_start + a
        while time.perf_counter() < ta:
            time.sleep(min(2e-4, max(0.0, ta - time.perf_counter())))
        busy = False
        while True:
            ts = time.perf_counter()
            t = srv.submit(*pool[int(w)])
            te = time.perf_counter()
            if t is not None:
                break
            busy = True
            time.sleep(5e-5)
        with lock:
            inflight[t] = {"w": int(w), "arrive": ta, "admit": te, "busy": busy, "submit": te - ts}
    stop.set()
    th.join()
    wall = time.perf_counter() - t_start
    srv_bytes = srv.bytes_used()
    srv.close()
    arr = np.array([r["arrive"] for r in done])
    adm = np.array([r["admit"] for r in done])
    fin = np.array([r["done"] for r in done])
    cl = np.array([sizes[r["w"]] for r in done])
    lat, wait, svc = (fin - arr) * 1e3, (adm - arr) * 1e3, (fin - adm) * 1e3
    sub = np.array([r["submit"] for r in done]) * 1e3
    # a stall: the first admission attempt found no free slot or no budget (E_BUSY)
    busy = np.array([r["busy"] for r in done])
    stalled = int(busy.sum())

    def pct(v):
        return {"p50": float(np.percentile(v, 50)), "p99": float(np.percentile(v, 99)), "max": float(v.max())}

    res = {"seconds": wall, "frames": int(len(done)), "arrival_rate_hz": lam, "load": 0.8, "slots": n_slots,
           "hbm_budget_gib": budget_gib, "device_bytes": srv_bytes,
           "capacity_clusters_per_s": capacity, "capacity_window_s": cap_wall,
           "clusters_per_s_incl_pcie": float(cl.sum()) / wall,
           "latency_ms": pct(lat), "admission_wait_ms": pct(wait), "service_ms": pct(svc),
           "admission_stalls": stalled, "admission_wait_s": float(wait.sum() * 1e-3),
           "stalled_wait_ms": pct(wait[busy]) if stalled else None,
           # host time of the admitting call itself (checks, upload enqueue, graph launch)
           "submit_call_ms": pct(sub),
           "pool": {"frames": len(pool), "clusters_min": int(sizes.min()), "clusters_max": int(sizes.max()),
                    "clusters_mean": float(sizes.mean())}}
    log(f"serving: {res['frames']} frames in {wall:.1f} s, latency p50 {res['latency_ms']['p50']:.1f} ms, p99 "
        f"{res['latency_ms']['p99']:.1f} ms, {stalled} arrivals stalled (admission wait p99 "
        f"{res['admission_wait_ms']['p99']:.1f} ms, submit call p50 {res['submit_call_ms']['p50']:.2f} ms), "
        f"service p50 {res['service_ms']['p50']:.1f} ms")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--tf-us", type=float, default=2000.0, help="time-frame length (us)")
    ap.add_argument("--cpu-budget", type=float, default=6.0, help="seconds of single-thread oracle time")
    ap.add_argument("--cpu-sectors", type=int, default=3, help="at most this many sectors in the single-thread run")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tuning", type=str, default="", help="JSON dict of tuning overrides")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tuning")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the serving run (Poisson arrivals at 80%% of capacity); 0 skips it")
    ap.add_argument("--serve-slots", type=int, default=6)
    ap.add_argument("--serve-cap-seconds", type=float, default=10.0,
                    help="length of the closed-loop capacity measurement before the serving run")
    ap.add_argument("--config4-steps", type=int, default=5,
                    help="timed batched calls of the 64-frame uneven batch (0 skips it)")
    ap.add_argument("--config4-frames", type=int, default=64)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the multi-core oracle run (0: the cores available, at most 16)")
    ap.add_argument("--compress-steps", type=int, default=20,
                    help="timed calls of the track-model compression (0: skip)")
    ap.add_argument("--reject-steps", type=int, default=20,
                    help="timed calls of the strategy-B hit removal (0: skip)")
    ap.add_argument("--merge-steps", type=int, default=20,
                    help="timed calls of the merge across sector edges (0: skip)")
    ap.add_argument("--size-curve", type=str, default="100,250,500,1000",
                    help="shorter Pb-Pb frame lengths (us) timed in both forms, besides the main frame; 'none' skips")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this size (for byte-counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py: this build measures one GPU only; --gpus must be 1 "
                  "(time frames are independent and would shard across GPUs without communication)",
                  file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2009_07515_amd import synth, tpcsf

    log("generating the time frame")
    t0 = time.perf_counter()
    f = synth.config3_time_frame(length_us=args.tf_us)
    N = f.n_clusters
    log(f"{N} clusters, {f.n_events} collisions, generated in {time.perf_counter() - t0:.1f} s")
    frames4 = None
    if args.config4_steps > 0 or args.serve_seconds > 0:
        # before the GPU is touched: worker processes generate the uneven batch
        t0 = time.perf_counter()
        frames4 = synth.config4_batch(args.config4_frames)
        log(f"uneven batch: {len(frames4)} frames, {sum(x.n_clusters for x in frames4)} clusters, generated in "
            f"{time.perf_counter() - t0:.1f} s")

    torch.cuda.set_device(0)
    frame = tpcsf.DeviceFrame.from_numpy(f.y, f.z, f.row_off, device="cuda:0")
    tuning = json.loads(args.tuning) if args.tuning else None
    trk = tpcsf.Tracker(synth.row_x(), tuning=tuning)
    out = tpcsf.TrackBuffers(N)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    # autotuner: bin sizes, bin cap and launch shapes on this input, result-invariance checked
    tune = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        best, tms, pts = trk.autotune(frame, reps=2, out=out)
        tune = {"points": len(pts), "best": pts[best], "best_ms": tms[best], "default_ms": tms[0],
                "seconds": time.perf_counter() - t0}
        log(f"autotune: {len(pts)} points in {tune['seconds']:.1f} s, best {pts[best]} "
            f"{tms[best]:.3f} ms (first point {tms[0]:.3f} ms)")

    # reference result of this input (also warms the graph)
    res0 = trk.track(frame, out=out, mode="batch")
    T0, H0 = res0["n_tracks"], res0["n_hits"]
    log(f"{T0} tracks, {H0} assigned clusters")
    for _ in range(args.warmup):
        trk.launch(frame, out, "batch")
    torch.cuda.synchronize()

    # timed region: K batched steps back to back
    K = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        ev[k][0].record(stream)
        trk.launch(frame, out, "batch")
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    trk.sync()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    ms = wall * 1e3 / K
    value = N / (wall / K)
    assert int(out.n_tracks.item()) == T0 and int(out.n_hits.item()) == H0
    log(f"batched: {ms:.3f} ms/step, {value / 1e9:.3f} G clusters/s")

    # plain per-sector form on the same input
    plain = None
    if args.plain_steps > 0:
        trk.track(frame, out=out, mode="plain")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            trk.launch(frame, out, "plain")
        torch.cuda.synchronize()
        wall_p = time.perf_counter() - t0
        trk.sync()
        assert int(out.n_tracks.item()) == T0 and int(out.n_hits.item()) == H0
        ms_p = wall_p * 1e3 / args.plain_steps
        plain = {"value": N / (wall_p / args.plain_steps), "ms_per_step": ms_p, "steps": args.plain_steps}
        log(f"plain: {ms_p:.3f} ms/step, {plain['value'] / 1e9:.3f} G clusters/s")

    # clusters/s against the frame length, both forms: Pb-Pb frames of the same recipe
    # (50 kHz, 0.1 ms up to the main frame's length), each tracked with the tuning above
    size_curve = None
    lengths = [] if args.size_curve.strip().lower() in ("", "none") else \
        [float(x) for x in args.size_curve.split(",") if x.strip()]
    if lengths:
        size_curve = []
        for L in lengths:
            fs = synth.config3_time_frame(length_us=L)
            ns = fs.n_clusters
            frs = tpcsf.DeviceFrame.from_numpy(fs.y, fs.z, fs.row_off, device="cuda:0")
            outs = tpcsf.TrackBuffers(ns)
            rs = trk.track(frs, out=outs, mode="batch")
            for _ in range(2):
                trk.launch(frs, outs, "batch")
            torch.cuda.synchronize()
            ks = max(5, args.steps // 2)
            t0 = time.perf_counter()
            for _ in range(ks):
                trk.launch(frs, outs, "batch")
            torch.cuda.synchronize()
            wb = (time.perf_counter() - t0) / ks
            trk.sync()
            assert int(outs.n_tracks.item()) == rs["n_tracks"]
            pt = {"tf_us": L, "clusters": ns, "tracks": rs["n_tracks"], "batch_ms": wb * 1e3,
                  "batch_clusters_per_s": ns / wb}
            if args.plain_steps > 0:
                trk.track(frs, out=outs, mode="plain")
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.plain_steps):
                    trk.launch(frs, outs, "plain")
                torch.cuda.synchronize()
                wp = (time.perf_counter() - t0) / args.plain_steps
                trk.sync()
                assert int(outs.n_tracks.item()) == rs["n_tracks"]
                pt.update({"plain_ms": wp * 1e3, "plain_clusters_per_s": ns / wp})
            size_curve.append(pt)
            log(f"frame {L:.0f} us: {ns} clusters, batched {wb * 1e3:.3f} ms ({ns / wb / 1e9:.3f} G/s)"
                + (f", plain {pt['plain_ms']:.3f} ms ({pt['plain_clusters_per_s'] / 1e9:.3f} G/s)" if "plain_ms" in pt
                   else ""))
            del frs, outs
        main_pt = {"tf_us": args.tf_us, "clusters": N, "tracks": T0, "batch_ms": ms, "batch_clusters_per_s": value}
        if plain:
            main_pt.update({"plain_ms": plain["ms_per_step"], "plain_clusters_per_s": plain["value"]})
        size_curve.append(main_pt)

    # the uneven batch of 64 time frames in one call, autotuned on itself
    config4 = None
    if args.config4_steps > 0:
        config4 = bench_config4(frames4, args.config4_steps, min(1, args.plain_steps),
                                autotune=not args.no_autotune)

    # calibration copy for hardware byte counters: one device copy of a known size
    if args.calib_copy_mib > 0:
        n_el = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n_el, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB read + {args.calib_copy_mib} MiB written")
        del a, b

    # stage timing: event nodes inside the same graph, K more timed replays
    trk.set_stage_timing(True)
    trk.track(frame, out=out, mode="batch")
    acc = None
    for _ in range(K):
        trk.launch(frame, out, "batch")
        trk.sync()
        st = trk.stage_times()
        acc = st if acc is None else {k: acc[k] + st[k] for k in st}
    stages = {k: v / K for k, v in acc.items()}
    res = out.result(N)
    cnt = counts_from(trk, frame, res, 152)
    sb = stage_bytes(cnt)
    sf = stage_flops(cnt)
    dom = max((k for k in stages if k != "reset"), key=lambda k: stages[k])
    hbm_gbs = sb[dom] / (stages[dom] * 1e-3) / 1e9
    path_bytes = sum(sb.values())
    if dom in sf:
        # a Kalman stage: bound by binary64 vector arithmetic
        achieved = sf[dom] / (stages[dom] * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                    "frac": achieved / FP64_PEAK_TFS, "traffic": profiled_traffic(dom),
                    "algorithmic_flops_per_launch": sf[dom], "launch_ms": stages[dom],
                    "hbm": {"algorithmic_bytes_per_launch": sb[dom], "achieved_GBs": hbm_gbs,
                            "frac": hbm_gbs / HBM_PEAK_GBS}}
    else:
        roofline = {"bound": "hbm", "kernel": dom, "achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": hbm_gbs / HBM_PEAK_GBS, "traffic": profiled_traffic(dom),
                    "algorithmic_bytes_per_launch": sb[dom], "launch_ms": stages[dom]}
    kalman = {k: {"TFLOPs": sf[k] / (stages[k] * 1e-3) / 1e12, "frac_fp64_peak": sf[k] / (stages[k] * 1e-3) / 1e12
                  / FP64_PEAK_TFS} for k in sf}
    w = cnt["work"]
    sv = (COARSE_PROPAGATE * w["tl_propagations"] + COARSE_UPDATE * w["tl_updates"]
          + COARSE_WINDOW * w["tl_window_clusters"])
    kalman["tracklets"]["coarse_model"] = {"flops_per_launch": sv,
                                           "frac_fp64_peak": sv / (stages["tracklets"] * 1e-3) / 1e12 / FP64_PEAK_TFS}
    log("stages (ms): " + ", ".join(f"{k} {v:.3f}" for k, v in stages.items()))
    trk.set_stage_timing(False)

    # track-model compression of the attached clusters: timed encode calls, one decode,
    # and the bits per coordinate of the codes against absolute coordinates at the same step
    compress = None
    if args.compress_steps > 0:
        # the tracks with their per-hit records, which the encoder reads
        out_r = tpcsf.TrackBuffers(N, hit_rec=True)
        trk.track(frame, out=out_r)
        out = out_r
        H = int(out.n_hits.item())
        codes = torch.empty((max(out.cap_hits, 1), 2), dtype=torch.int32, device="cuda:0")
        rows = torch.empty(max(out.cap_hits, 1), dtype=torch.uint8, device="cuda:0")
        yz = torch.empty((max(out.cap_hits, 1), 2), dtype=torch.float64, device="cuda:0")
        trk.launch_compress(frame, out, codes, rows)
        trk.launch_decompress(out, codes, rows, yz)
        trk.sync()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        for _ in range(args.compress_steps):
            trk.launch_compress(frame, out, codes, rows)
        e1.record(stream)
        for _ in range(args.compress_steps):
            trk.launch_decompress(out, codes, rows, yz)
        e2.record(stream)
        torch.cuda.synchronize()
        trk.sync()
        c_ms, d_ms = e0.elapsed_time(e1) / args.compress_steps, e1.elapsed_time(e2) / args.compress_steps
        step = trk.params.resid_step
        q = codes[:H].cpu().numpy()
        hid = out.hit_ids[:H].cpu().numpy()
        dec = yz[:H].cpu().numpy()
        err = max(float(np.abs(dec[:, 0] - f.y[hid]).max()), float(np.abs(dec[:, 1] - f.z[hid]).max()))

        def entropy(v):
            _, k = np.unique(v, return_counts=True)
            pr = k / k.sum()
            return float(-(pr * np.log2(pr)).sum())

        # encode, per launch: per cluster the hit index (4 B), y and z (8 B), the codes (8 B)
        # and the row (1 B); per track its state, x_ref, sector, time frame, hit range (72 B)
        enc_bytes = 21 * H + 72 * T0
        enc_gbs = enc_bytes / (c_ms * 1e-3) / 1e9
        compress = {"roofline": {"bound": "hbm", "kernel": "c_encode", "achieved": enc_gbs, "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": enc_gbs / HBM_PEAK_GBS, "traffic": profiled_traffic("c_encode"),
                                 "algorithmic_bytes_per_launch": enc_bytes, "launch_ms": c_ms},
                    "encode_ms": c_ms, "decode_ms": d_ms, "calls": args.compress_steps, "clusters": H,
                    "clusters_per_s": H / (c_ms * 1e-3), "step_cm": step, "max_decode_error_cm": err,
                    "bits_residual": [entropy(q[:, 0]), entropy(q[:, 1])],
                    "bits_absolute": [entropy(np.floor(f.y[hid] / step)), entropy(np.floor(f.z[hid] / step))]}
        log(f"compress: {H} clusters, encode {c_ms:.3f} ms, decode {d_ms:.3f} ms, bits/coordinate "
            f"{compress['bits_residual'][0]:.2f}/{compress['bits_residual'][1]:.2f} vs absolute "
            f"{compress['bits_absolute'][0]:.2f}/{compress['bits_absolute'][1]:.2f}, max error {err:.4f} cm")

    # hit removal for compression, strategy B: timed calls on the tracks of the last
    # tracking call (it reuses that call's grids).  Not part of the step above.
    reject = None
    if args.reject_steps > 0:
        trk.track(frame, out=out)
        keep = torch.empty(N, dtype=torch.uint8, device="cuda:0")
        n_kept = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        trk.launch_reject(frame, out, keep, n_kept)
        trk.sync()
        kept = int(n_kept.item())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.reject_steps):
            trk.launch_reject(frame, out, keep, n_kept)
        e1.record(stream)
        torch.cuda.synchronize()
        trk.sync()
        r_ms = e0.elapsed_time(e1) / args.reject_steps
        assert int(n_kept.item()) == kept
        # per call: y, z, bin-order position, cluster->track map and keep flag of every
        # cluster (17 B); per track its state and hit range (64 B); the hit list (4 B a hit)
        rej_bytes = 17 * N + 64 * T0 + 4 * H0
        rej_gbs = rej_bytes / (r_ms * 1e-3) / 1e9
        reject = {"roofline": {"bound": "hbm", "kernel": "r_span + r_fill + r_rows", "achieved": rej_gbs,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": rej_gbs / HBM_PEAK_GBS,
                               "traffic": None, "algorithmic_bytes_per_launch": rej_bytes, "launch_ms": r_ms},
                  "ms_per_call": r_ms, "calls": args.reject_steps, "clusters": N, "kept": kept,
                  "kept_fraction": kept / N, "clusters_per_s": N / (r_ms * 1e-3)}
        log(f"reject: kept {kept} of {N} ({kept / N:.3f}) in {r_ms:.3f} ms")

    # merging across sector edges and refit across sector frames (the stage after sector
    # tracking): timed calls on this frame's sector tracks, tracked with the outer states
    # the merge needs.  Not part of the step above.
    merge = None
    if args.merge_steps > 0:
        tb = tpcsf.TrackBuffers(N, outer=True, hit_rec=True)
        trk.track(frame, out=tb)
        mb = tpcsf.MergedBuffers(tb)
        mres = trk.merge(frame, tb, out=mb)
        M = mres["n_merged"]
        n_multi = int((mres["n_segments"] >= 2).sum().item())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.merge_steps):
            trk.launch_merge(frame, tb, mb)
        e1.record(stream)
        torch.cuda.synchronize()
        trk.sync()
        m_ms = e0.elapsed_time(e1) / args.merge_steps
        assert int(mb.n_merged.item()) == M
        w = trk.merge_work()
        # binary64 operations: per gate pair a propagation (182) and a 5x5 chi2 (155); per
        # refit rotation 60, propagation 182, update 121
        m_flops = 337 * int(w[0]) + 60 * int(w[3]) + 182 * int(w[4]) + 121 * int(w[5])
        m_tfs = m_flops / (m_ms * 1e-3) / 1e12
        merge = {"roofline": {"bound": "alu", "kernel": "merge (all kernels)", "achieved": m_tfs,
                              "peak": FP64_PEAK_TFS, "unit": "TFLOP/s", "frac": m_tfs / FP64_PEAK_TFS,
                              "traffic": None, "algorithmic_flops_per_launch": m_flops, "launch_ms": m_ms},
                 "ms_per_call": m_ms, "calls": args.merge_steps, "sector_tracks": T0, "merged_tracks": M,
                 "merged_of_several": n_multi, "tracks_per_s": T0 / (m_ms * 1e-3),
                 "work": {"gate_pairs": int(w[0]), "match_propagations": int(w[1]), "match_chi2": int(w[2]),
                          "fit_rotations": int(w[3]), "fit_propagations": int(w[4]), "fit_updates": int(w[5])}}
        log(f"merge: {T0} sector tracks -> {M} ({n_multi} of several) in {m_ms:.3f} ms")

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "clusters/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+fp64",
        "data": "synthetic",
        "config": {"workload": f"one {args.tf_us / 1000:g} ms continuous-readout Pb-Pb time frame, 36 sectors x 152 rows",
                   "clusters": N, "collisions": f.n_events, "tracks": T0, "batch_time_frames": 1,
                   "tuning": trk.tuning.as_dict()},
        "plain": plain,
        # per-step event times of the back-to-back graph replays (device-resident frame)
        "graph_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                     "max": float(lat.max())},
        "stages_ms": stages,
        "counts": cnt,
        "roofline": roofline,
        "kalman_stages": kalman,
        "merge": merge,
        "reject": reject,
        "compress": compress,
        "size_curve": size_curve,
        "path_hbm": {"bytes_per_cluster": path_bytes / N,
                     "achieved_GBs": path_bytes / (ms * 1e-3) / 1e9,
                     "frac": path_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "coarse_model": {"bytes_per_cluster": sum(coarse_bytes(cnt).values()) / N,
                                      "achieved_GBs": sum(coarse_bytes(cnt).values()) / (ms * 1e-3) / 1e9,
                                      "frac": sum(coarse_bytes(cnt).values()) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
                     "io_floor_bytes_per_cluster": 16},
        "config4": config4,
    }
    line["autotune"] = tune
    # time-frame latency: arrival to tracks on the host, from the serving run
    line["latency_ms"] = None
    if args.serve_seconds > 0:
        del out, frame
        trk.close()
        torch.cuda.empty_cache()
        line["serving"] = serve(frames4, line["config"]["tuning"], args.serve_seconds, args.serve_slots,
                                args.serve_cap_seconds)
        line["latency_ms"] = line["serving"]["latency_ms"]
    if not args.no_cpu:
        name, avail, total = cpu_model()
        threads = args.cpu_threads or min(16, avail)
        single = cpu_baseline(f, args.cpu_budget, args.cpu_sectors)
        multi = cpu_threads(f, threads, threads)
        log(f"oracle on {threads} threads: {len(multi['sectors'])} sectors in {multi['seconds']:.1f} s, "
            f"{multi['value'] / 1e6:.2f} M clusters/s")
        line["cpu_baseline"] = {"value": multi["value"], "unit": "clusters/s", "cores": threads, "kind": "oracle",
                                "sample": f"FP64 oracle on {len(multi['sectors'])} whole sectors {multi['sectors']} of "
                                          f"the same time frame ({multi['clusters']} clusters, one sector per task "
                                          f"on {threads} threads, {multi['seconds']:.1f} s wall)",
                                "cpu": name, "cores_available": avail, "cores_host": total,
                                "single_thread": single, "next_stages": cpu_next_stages(f)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
