"""Seeded synthetic TPC workloads: helix tracks, clusters, noise and Monte-Carlo truth.

This module is input generation only.  It simulates what the detector would record
(charged helices in a solenoid field crossing the pad-row planes of the 36 TPC sectors,
Gaussian cluster smearing, uniform noise, continuous-readout drift shift) and returns
structure-of-arrays frames.  It contains none of the tracking method's arithmetic: the
crossings are solved in closed form on the global circle, independently of the tracker's
row-to-row propagation.

The workload shapes follow the paper's setting: 36 sectors of 152 pad rows, minimum-bias
Pb-Pb collisions read out continuously at 50 kHz and grouped into time frames
(Sec. 2 and Sec. 7.1 of arXiv:2009.07515), with z shifted by the unknown collision time
(Sec. 2, loss of absolute z in continuous readout).

Conventions (shared by every consumer as *input* conventions, not as method code):
  * sector s in [0, 36): s < 18 is the A side (physical z > 0), s >= 18 the C side;
    the sector's centre azimuth is alpha = ((s mod 18) + 0.5) * pi / 9, half-opening pi / 18.
  * local frame: x = X cos(alpha) + Y sin(alpha), y = -X sin(alpha) + Y cos(alpha), z = z.
  * pad row r is the plane x = X_r, X_r = float32(85 + r * 160 / 151) cm (the float32
    value is the geometry; every consumer uses it exactly).
  * curvature kappa = -C_B * B_z * (q / pT) [1/cm]; d(phi)/ds = kappa along the transverse
    arc length s; dz/ds = tan(lambda) = sinh(eta).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

N_SECTORS = 36
N_ROWS = 152
C_B = 0.00299792458          # cm^-1 T^-1 GeV
B_Z = 0.5                    # T
V_DRIFT = 2.58               # cm / us
Z_MAX = 250.0                # cm, drift length
HALF_OPEN = math.pi / 18.0


def row_x() -> np.ndarray:
    """Pad-row plane positions X_r (cm) as float32 values."""
    r = np.arange(N_ROWS, dtype=np.float64)
    return (85.0 + r * 160.0 / 151.0).astype(np.float32)


def sector_alpha(s: int) -> float:
    return ((s % 18) + 0.5) * math.pi / 9.0


@dataclasses.dataclass
class Frame:
    """One time frame (or one event) in SoA layout, grouped by (sector, row).

    y, z      float32[N]   local cluster coordinates (cm); z is the drift-shifted z
    row_off   int64[36*152+1]  CSR offsets; clusters of (sector s, row r) are
                           row_off[s*152+r] : row_off[s*152+r+1]
    label     int32[N]     Monte-Carlo track id, -1 for noise
    truth_*   float64[N]   noise-free local state at the crossing (y, z_shifted, sin(phi));
                           NaN for noise
    trk_*     per MC track: q/pT, tan(lambda), is_secondary, event id, vertex z, t0
    """
    y: np.ndarray
    z: np.ndarray
    row_off: np.ndarray
    label: np.ndarray
    truth_y: np.ndarray
    truth_z: np.ndarray
    truth_sphi: np.ndarray
    trk_qpt: np.ndarray
    trk_tgl: np.ndarray
    trk_secondary: np.ndarray
    trk_event: np.ndarray
    n_events: int
    tf_length_us: float
    trk_vz: np.ndarray = None        # per MC track: vertex z (cm, physical)
    trk_t0: np.ndarray = None        # per MC track: collision time in the frame (us)

    @property
    def n_clusters(self) -> int:
        return int(self.y.shape[0])


@dataclasses.dataclass
class Tracks:
    """Generated helices in global coordinates."""
    xv: np.ndarray
    yv: np.ndarray
    zv: np.ndarray
    pt: np.ndarray
    eta: np.ndarray
    phi: np.ndarray
    q: np.ndarray
    secondary: np.ndarray
    t0_us: np.ndarray          # collision time inside the frame
    event: np.ndarray

    def __len__(self):
        return int(self.pt.shape[0])


def _concat_tracks(parts):
    return Tracks(*[np.concatenate([getattr(p, f.name) for p in parts])
                    for f in dataclasses.fields(Tracks)])


def sample_event(rng, n_primary, pt_mean, sec_frac, eta_max=0.9, phi_range=None,
                 t0_us=0.0, event=0, vertex_sigma_z=1.0):
    """Kinematics of one collision: primaries at (0, 0, N(0, sigma_z)) plus secondaries."""
    n_sec = int(round(sec_frac * n_primary))
    n = n_primary + n_sec
    # Exp(mean m) conditioned on pT > 0.1 equals 0.1 + Exp(m) (memorylessness)
    pt = 0.1 + rng.exponential(pt_mean, n)
    eta = rng.uniform(-eta_max, eta_max, n)
    if phi_range is None:
        phi = rng.uniform(0.0, 2 * math.pi, n)
    else:
        phi = rng.uniform(phi_range[0], phi_range[1], n)
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    zv0 = rng.normal(0.0, vertex_sigma_z)
    xv = np.zeros(n)
    yv = np.zeros(n)
    zv = np.full(n, zv0)
    secondary = np.zeros(n, dtype=bool)
    if n_sec:
        r = 30.0 * np.sqrt(rng.random(n_sec))
        a = rng.uniform(0, 2 * math.pi, n_sec)
        xv[n_primary:] = r * np.cos(a)
        yv[n_primary:] = r * np.sin(a)
        zv[n_primary:] = zv0 + rng.uniform(-30.0, 30.0, n_sec)
        secondary[n_primary:] = True
    return Tracks(xv, yv, zv, pt, eta, phi, q, secondary,
                  np.full(n, t0_us), np.full(n, event, dtype=np.int64))


def _exit_azimuth(xv, yv, phi0, kappa, rho):
    """Azimuth of the first point where each helix (projected) leaves the cylinder of
    radius rho around the beam axis; NaN if it never gets there.  Circle-circle
    intersection in the transverse plane."""
    out = np.full(xv.shape, np.nan)
    straight = np.abs(kappa) < 1e-12
    # straight lines: solve |P + t d| = rho, t > 0
    if straight.any():
        dx, dy = np.cos(phi0[straight]), np.sin(phi0[straight])
        px, py = xv[straight], yv[straight]
        b = px * dx + py * dy
        c = px * px + py * py - rho * rho
        disc = b * b - c
        t = -b + np.sqrt(np.maximum(disc, 0.0))
        az = np.arctan2(py + t * dy, px + t * dx)
        out[straight] = np.where(disc >= 0, az, np.nan)
    cur = ~straight
    if cur.any():
        k = kappa[cur]
        R = 1.0 / np.abs(k)
        # centre of curvature: position + (1/kappa) * (-sin phi, cos phi)
        cx = xv[cur] - np.sin(phi0[cur]) / k
        cy = yv[cur] + np.cos(phi0[cur]) / k
        d = np.hypot(cx, cy)
        a = (d * d + rho * rho - R * R) / (2.0 * d)
        h2 = rho * rho - a * a
        ok = h2 >= 0
        h = np.sqrt(np.maximum(h2, 0.0))
        ux, uy = cx / d, cy / d
        bx, by = a * ux, a * uy
        p1x, p1y = bx - h * uy, by + h * ux
        p2x, p2y = bx + h * uy, by - h * ux
        # sweep angle from the vertex around the centre, in the direction of motion
        a0 = np.arctan2(yv[cur] - cy, xv[cur] - cx)
        sgn = np.sign(k)
        sw1 = np.mod(sgn * (np.arctan2(p1y - cy, p1x - cx) - a0), 2 * math.pi)
        sw2 = np.mod(sgn * (np.arctan2(p2y - cy, p2x - cx) - a0), 2 * math.pi)
        first1 = sw1 <= sw2
        px_ = np.where(first1, p1x, p2x)
        py_ = np.where(first1, p1y, p2y)
        out[cur] = np.where(ok, np.arctan2(py_, px_), np.nan)
    return out


def plane_crossing(xv, yv, zv, phi0, kappa, tgl, alpha, X):
    """First crossing of the plane x_local = X of the sector with centre azimuth alpha,
    moving outward (cos(phi_local) > 0) within the first half turn.

    Returns (ok, y_local, z_phys, sin(phi_local), s)."""
    ca, sa = np.cos(alpha), np.sin(alpha)
    d0 = xv * ca + yv * sa
    e0 = -xv * sa + yv * ca
    psi0 = phi0 - alpha
    sp0, cp0 = np.sin(psi0), np.cos(psi0)
    straight = np.abs(kappa) < 1e-12
    ks = np.where(straight, 1.0, kappa)
    v = sp0 + kappa * (X - d0)
    okv = np.abs(v) < 1.0
    vv = np.clip(v, -1.0, 1.0)
    delta = np.arcsin(vv) - psi0
    turn = np.where(kappa > 0, np.mod(delta, 2 * math.pi), -np.mod(-delta, 2 * math.pi))
    s_cur = turn / ks
    y_cur = e0 - (np.sqrt(1.0 - vv * vv) - cp0) / ks
    ok_cur = okv & (np.abs(turn) <= math.pi) & (s_cur >= 0)
    # straight lines
    cps = np.where(cp0 > 0, cp0, 1.0)
    s_str = (X - d0) / cps
    y_str = e0 + s_str * sp0
    ok_str = (cp0 > 0) & (s_str >= 0)
    ok = np.where(straight, ok_str, ok_cur)
    s = np.where(straight, s_str, s_cur)
    y = np.where(straight, y_str, y_cur)
    sphi = np.where(straight, sp0, vv)
    z = zv + tgl * s
    return ok, y, z, sphi, s


def _azimuth_range(tr: Tracks, kappa):
    """Azimuth interval (lo, hi) swept by each track's position between the inner and
    outer radius of the pad-row polygon.  For a vertex on the beam axis the position
    azimuth at radius rho is phi0 + asin(kappa * rho / 2) (half the turning angle), which
    is monotone in rho."""
    X = row_x().astype(np.float64)
    r_in = X[0]
    r_out = X[-1] / math.cos(HALF_OPEN)
    primary = (tr.xv == 0) & (tr.yv == 0)
    a_in = np.clip(kappa * r_in / 2, -1.0, 1.0)
    a_out = np.clip(kappa * r_out / 2, -1.0, 1.0)
    t_in = tr.phi + np.arcsin(a_in)
    t_out = tr.phi + np.arcsin(a_out)
    lo = np.minimum(t_in, t_out)
    hi = np.maximum(t_in, t_out)
    # displaced vertices: the position azimuth need not be monotone in radius, so every
    # sector is a candidate (exact, at 18x the cost for those tracks)
    sec = ~primary
    lo[sec] = 0.0
    hi[sec] = 2 * math.pi - 1e-9
    return lo, hi


def crossings(tr: Tracks, bz=B_Z, sectors=None, z_max=Z_MAX, chunk=1 << 22):
    """All recorded (noise-free) clusters of a set of tracks.

    A cluster is recorded where a helix first crosses a row plane of a sector moving
    outward, within the first half turn, inside the sector's acceptance
    |y| <= X tan(pi/18) and |z_phys| < z_max.  The sector side follows the sign of the
    physical z.  Returns dict of arrays (track, sector, row, y, z_phys, sphi)."""
    n = len(tr)
    kappa = -C_B * bz * tr.q / tr.pt
    tgl = np.sinh(tr.eta)
    X = row_x().astype(np.float64)
    tan_half = math.tan(HALF_OPEN)
    w = math.pi / 9.0
    lo, hi = _azimuth_range(tr, kappa)
    k_lo = np.floor(lo / w).astype(np.int64)
    k_hi = np.floor(hi / w).astype(np.int64)
    nk = np.minimum(k_hi - k_lo + 1, 18)
    pair_trk = np.repeat(np.arange(n), nk)
    first = np.repeat(np.cumsum(nk) - nk, nk)
    pair_k = np.mod(k_lo[pair_trk] + (np.arange(pair_trk.shape[0]) - first), 18)
    out = {k: [] for k in ("track", "sector", "row", "y", "z", "sphi")}
    rows = np.arange(N_ROWS)
    per = max(1, chunk // N_ROWS)
    for c0 in range(0, pair_trk.shape[0], per):
        t = pair_trk[c0:c0 + per]
        k = pair_k[c0:c0 + per]
        alpha = (k + 0.5) * w
        ok, y, z, sphi, _ = plane_crossing(tr.xv[t, None], tr.yv[t, None], tr.zv[t, None],
                                           tr.phi[t, None], kappa[t, None], tgl[t, None],
                                           alpha[:, None], X[None, :])
        ok &= (np.abs(y) <= X[None, :] * tan_half) & (np.abs(z) < z_max)
        pi_, ri = np.nonzero(ok)
        sec = np.where(z[pi_, ri] > 0, k[pi_], k[pi_] + 18)
        keep = np.isin(sec, sectors) if sectors is not None else slice(None)
        out["track"].append(t[pi_][keep])
        out["sector"].append(sec[keep])
        out["row"].append(rows[ri][keep])
        out["y"].append(y[pi_, ri][keep])
        out["z"].append(z[pi_, ri][keep])
        out["sphi"].append(sphi[pi_, ri][keep])
    if not out["track"]:
        return {k: np.zeros(0, dtype=np.int64 if k in ("track", "sector", "row") else np.float64)
                for k in out}
    return {k: np.concatenate(v) for k, v in out.items()}


def assemble(rng, tr: Tracks, cl, sigma, noise_frac, tf_length_us, sectors=None,
             n_events=1, shuffle_rows=True) -> Frame:
    """Smear, drift-shift, add noise, and sort clusters into (sector, row) CSR order."""
    n_sig = cl["track"].shape[0]
    t0 = tr.t0_us[cl["track"]]
    zphys = cl["z"]
    zshift = zphys - np.sign(zphys) * V_DRIFT * t0
    y_true = cl["y"]
    y = y_true + (rng.normal(0.0, sigma, n_sig) if sigma > 0 else 0.0)
    z = zshift + (rng.normal(0.0, sigma, n_sig) if sigma > 0 else 0.0)
    sector = cl["sector"]
    row = cl["row"]
    label = cl["track"].astype(np.int64)
    n_noise = int(round(noise_frac * n_sig))
    if n_noise:
        secs = np.asarray(sectors if sectors is not None else np.arange(N_SECTORS))
        ns = secs[rng.integers(0, secs.shape[0], n_noise)]
        nr = rng.integers(0, N_ROWS, n_noise)
        X = row_x().astype(np.float64)[nr]
        ny = rng.uniform(-1.0, 1.0, n_noise) * X * math.tan(HALF_OPEN)
        shift = V_DRIFT * tf_length_us
        a_side = ns < 18
        nz = np.where(a_side, rng.uniform(-shift, Z_MAX, n_noise), rng.uniform(-Z_MAX, shift, n_noise))
        if tf_length_us == 0:
            nz = np.where(a_side, rng.uniform(0.0, Z_MAX, n_noise), rng.uniform(-Z_MAX, 0.0, n_noise))
        y = np.concatenate([y, ny])
        z = np.concatenate([z, nz])
        sector = np.concatenate([sector, ns])
        row = np.concatenate([row, nr])
        label = np.concatenate([label, np.full(n_noise, -1)])
        y_true = np.concatenate([y_true, np.full(n_noise, np.nan)])
        zshift = np.concatenate([zshift, np.full(n_noise, np.nan)])
        sphi = np.concatenate([cl["sphi"], np.full(n_noise, np.nan)])
    else:
        sphi = cl["sphi"]
    key = (sector * N_ROWS + row).astype(np.int16)
    if shuffle_rows:
        # random order inside each row: shuffle, then a stable (radix) sort by row key
        perm = rng.permutation(key.shape[0])
        order = perm[np.argsort(key[perm], kind="stable")]
    else:
        order = np.argsort(key, kind="stable")
    counts = np.bincount(key, minlength=N_SECTORS * N_ROWS)
    row_off = np.zeros(N_SECTORS * N_ROWS + 1, dtype=np.int64)
    np.cumsum(counts, out=row_off[1:])
    return Frame(
        y=np.ascontiguousarray(y[order], dtype=np.float32),
        z=np.ascontiguousarray(z[order], dtype=np.float32),
        row_off=row_off,
        label=label[order].astype(np.int32),
        truth_y=y_true[order], truth_z=zshift[order], truth_sphi=sphi[order],
        trk_qpt=tr.q / tr.pt, trk_tgl=np.sinh(tr.eta), trk_secondary=tr.secondary,
        trk_event=tr.event, n_events=n_events, tf_length_us=tf_length_us,
        trk_vz=np.asarray(tr.zv, dtype=np.float64), trk_t0=np.asarray(tr.t0_us, dtype=np.float64))


# ----------------------------------------------------------------------------------------
# The five workloads.  Config k uses base seed 1000 + k; time frame i of config k uses
# seed (1000 + k) * 10**6 + i (numpy PCG64).
# ----------------------------------------------------------------------------------------

def seed_for(config: int, tf_index: int = 0) -> int:
    return (1000 + config) * 10 ** 6 + tf_index


def config1_single_sector(seed=None, n_tracks=50, sigma=0.1, noise_frac=0.02, bz=B_Z):
    """One pp-like event in sector 0: 50 helices, pT = 0.1 + Exp(0.5) GeV, 0 < eta < 0.9,
    phi uniform inside the sector, vertex z ~ N(0, 1 cm), 2% noise."""
    rng = np.random.Generator(np.random.PCG64(seed_for(1) if seed is None else seed))
    tr = sample_event(rng, n_tracks, 0.5, 0.0, phi_range=(0.0, 2 * HALF_OPEN))
    tr.eta = np.abs(tr.eta)
    cl = crossings(tr, bz=bz, sectors=[0])
    return assemble(rng, tr, cl, sigma, noise_frac, 0.0, sectors=[0])


def config2_pbpb_event(seed=None, n_primary=8000, sigma=0.1, noise_frac=0.05, bz=B_Z):
    """One central Pb-Pb-like event, full TPC: 8000 primaries, pT = 0.1 + Exp(0.6),
    |eta| < 0.9, +10% secondaries from displaced vertices (r < 30 cm), 5% noise."""
    rng = np.random.Generator(np.random.PCG64(seed_for(2) if seed is None else seed))
    tr = sample_event(rng, n_primary, 0.6, 0.1)
    cl = crossings(tr, bz=bz)
    return assemble(rng, tr, cl, sigma, noise_frac, 0.0)


def time_frame(seed, length_us, rate_khz=50.0, mult_mean=1500.0, pt_mean=0.6, sec_frac=0.1,
               noise_frac=0.05, sigma=0.1, bz=B_Z):
    """Continuous-readout time frame: Poisson(rate * length) collisions at uniform times,
    each with Exp(mult_mean) primaries; clusters clipped at physical |z| < 250 cm and
    shifted in z by the drift velocity times the collision time."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_ev = int(rng.poisson(rate_khz * 1e-3 * length_us))
    parts = []
    for e in range(n_ev):
        t0 = rng.uniform(0.0, length_us)
        m = int(round(rng.exponential(mult_mean)))
        if m == 0:
            continue
        parts.append(sample_event(rng, m, pt_mean, sec_frac, t0_us=t0, event=e))
    if not parts:
        parts.append(sample_event(rng, 0, pt_mean, 0.0))
    tr = _concat_tracks(parts)
    cl = crossings(tr, bz=bz)
    return assemble(rng, tr, cl, sigma, noise_frac, length_us, n_events=n_ev)


def config3_time_frame(seed=None, length_us=2000.0):
    """Poisson(50 kHz) minimum-bias Pb-Pb collisions over 2 ms, multiplicity per event
    Exp(mean 1500), Pb-Pb kinematics (pT mean 0.6, 10% secondaries, 5% noise)."""
    return time_frame(seed_for(3) if seed is None else seed, length_us)


def config4_frame(i, seed=None):
    """Time frame i of the uneven 64-frame batch: even i pp-like (Poisson 500 kHz,
    Exp(30) tracks, 0.5 ms, 2% noise, no secondaries, pT mean 0.5), odd i Pb-Pb-like
    (config-3 recipe with a uniform 0.5-2 ms length)."""
    s = seed_for(4, i) if seed is None else seed
    if i % 2 == 0:
        return time_frame(s, 500.0, rate_khz=500.0, mult_mean=30.0, pt_mean=0.5, sec_frac=0.0,
                          noise_frac=0.02)
    length = float(np.random.Generator(np.random.PCG64(s ^ 0x5EED)).uniform(500.0, 2000.0))
    return time_frame(s, length)


@dataclasses.dataclass
class LightFrame:
    """A frame without its per-cluster truth beyond the labels (batches of many frames)."""
    y: np.ndarray
    z: np.ndarray
    row_off: np.ndarray
    label: np.ndarray
    tf_length_us: float
    n_events: int

    @property
    def n_clusters(self) -> int:
        return int(self.y.shape[0])


def _config4_light(i: int) -> LightFrame:
    f = config4_frame(i)
    return LightFrame(f.y, f.z, f.row_off, f.label, f.tf_length_us, f.n_events)


def config4_batch(n_tf: int = 64, workers: int | None = None) -> list:
    """Frames 0..n_tf-1 of the uneven batch (config4_frame), generated in worker processes
    started afresh (spawned interpreters that import only this module, so that the caller
    may already drive a GPU).  The frames are those of config4_frame, without the
    per-cluster truth other than the labels."""
    import multiprocessing
    import os
    from concurrent.futures import ProcessPoolExecutor
    workers = workers or min(16, os.cpu_count() or 1, n_tf)
    if workers <= 1:
        return [_config4_light(i) for i in range(n_tf)]
    # Pb-Pb frames (odd indices) first: the long tasks start early
    order = sorted(range(n_tf), key=lambda i: (i % 2 == 0, i))
    with ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn")) as ex:
        got = dict(zip(order, ex.map(_config4_light, order)))
    return [got[i] for i in range(n_tf)]


def concat_frames(frames):
    """Concatenate frames into one batch: y, z, label concatenated, row offsets chained."""
    offs = [np.int64(0)]
    ys, zs, ro = [], [], [np.zeros(1, dtype=np.int64)]
    base = 0
    for f in frames:
        ys.append(f.y)
        zs.append(f.z)
        ro.append(f.row_off[1:] + base)
        base += f.n_clusters
    return (np.concatenate(ys) if ys else np.zeros(0, np.float32),
            np.concatenate(zs) if zs else np.zeros(0, np.float32),
            np.concatenate(ro))
