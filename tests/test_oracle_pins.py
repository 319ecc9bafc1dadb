"""Pins of the reference oracle against facts that do not come from the oracle itself:
closed-form helices, an independent ODE integration, finite differences, the textbook
Gaussian posterior, nonlinear least squares, brute force on tiny inputs, hand-worked
examples and graph invariants.  CPU only."""
import math

import numpy as np
import pytest
from scipy.optimize import least_squares

import oracle
import truthmatch
from paper_2009_07515_amd import synth

C_B = 0.00299792458


def _orc(row_x, mode="f64", **kw):
    return oracle.Oracle(row_x, mode=mode, **kw)


# --------------------------------------------------------------------------------------
# Generator: closed-form circle/plane crossing vs RK4 integration of the equations of
# motion (dX/ds = cos phi, dY/ds = sin phi, dphi/ds = kappa, dz/ds = tan lambda).
# --------------------------------------------------------------------------------------
def _rk4_step(st, h, kappa, tgl):
    def f(s):
        return np.array([math.cos(s[2]), math.sin(s[2]), kappa, tgl])
    k1 = f(st)
    k2 = f(st + 0.5 * h * k1)
    k3 = f(st + 0.5 * h * k2)
    k4 = f(st + h * k3)
    return st + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)


def test_generator_crossings_match_rk4():
    rng = np.random.Generator(np.random.PCG64(11))
    tr = synth.sample_event(rng, 6, 0.5, 0.5)
    cl = synth.crossings(tr)
    X = synth.row_x().astype(np.float64)
    kappa = -C_B * synth.B_Z * tr.q / tr.pt
    tgl = np.sinh(tr.eta)
    checked = 0
    for t in range(len(tr)):
        sel = np.flatnonzero(cl["track"] == t)
        if sel.size == 0:
            continue
        pick = sel[np.linspace(0, sel.size - 1, min(4, sel.size)).astype(int)]
        for i in pick:
            k = cl["sector"][i] % 18
            a = (k + 0.5) * math.pi / 9
            Xr = X[cl["row"][i]]
            st = np.array([tr.xv[t], tr.yv[t], tr.phi[t], tr.zv[t]])
            h = 0.05
            xl = st[0] * math.cos(a) + st[1] * math.sin(a)
            # march until the local x passes the plane while moving outward
            for _ in range(200000):
                nx = _rk4_step(st, h, kappa[t], tgl[t])
                nxl = nx[0] * math.cos(a) + nx[1] * math.sin(a)
                if xl < Xr <= nxl and math.cos(nx[2] - a) > 0:
                    break
                st, xl = nx, nxl
            lo, hi = 0.0, h
            for _ in range(60):
                mid = 0.5 * (lo + hi)
                m = _rk4_step(st, mid, kappa[t], tgl[t])
                if m[0] * math.cos(a) + m[1] * math.sin(a) < Xr:
                    lo = mid
                else:
                    hi = mid
            m = _rk4_step(st, 0.5 * (lo + hi), kappa[t], tgl[t])
            yl = -m[0] * math.sin(a) + m[1] * math.cos(a)
            assert abs(yl - cl["y"][i]) < 1e-6
            assert abs(m[3] - cl["z"][i]) < 1e-6
            assert abs(math.sin(m[2] - a) - cl["sphi"][i]) < 1e-8
            checked += 1
    assert checked >= 12


# --------------------------------------------------------------------------------------
# Propagation: the true state at one row, propagated with the oracle's helix step,
# lands on the generator's closed-form crossing of another row.
# --------------------------------------------------------------------------------------
def _noise_free_sector0(n_tracks=60, seed=77, bz=synth.B_Z):
    return synth.config1_single_sector(seed=seed, n_tracks=n_tracks, sigma=0.0, noise_frac=0.0, bz=bz)


def test_propagation_reproduces_generator_crossings(row_x):
    f = _noise_free_sector0()
    o = _orc(row_x)
    X = row_x.astype(np.float64)
    rows = np.repeat(np.arange(152), np.diff(f.row_off[:153]))
    n_checked = 0
    for lab in np.unique(f.label)[:30]:
        idx = np.flatnonzero(f.label == lab)
        idx = idx[np.argsort(rows[idx])]
        good = idx[np.abs(f.truth_sphi[idx]) < 0.95]
        if good.size < 10:
            continue
        a, b = good[0], good[-1]
        for i0, i1 in ((a, b), (b, a), (good[3], good[7])):
            p = [f.truth_y[i0], f.truth_z[i0], f.truth_sphi[i0], f.trk_tgl[lab], f.trk_qpt[lab]]
            ok, p1, _, _ = o.propagate(X[rows[i0]], X[rows[i1]], p)
            assert ok
            assert abs(p1[0] - f.truth_y[i1]) < 1e-9
            assert abs(p1[1] - f.truth_z[i1]) < 1e-9
            assert abs(p1[2] - f.truth_sphi[i1]) < 1e-12
            n_checked += 1
    assert n_checked > 20


# --------------------------------------------------------------------------------------
# Jacobian of the propagation vs central finite differences of the propagation itself.
# --------------------------------------------------------------------------------------
def test_jacobian_matches_finite_differences(row_x):
    o = _orc(row_x)
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(200):
        p = np.array([rng.uniform(-20, 20), rng.uniform(-100, 100), rng.uniform(-0.8, 0.8),
                      rng.uniform(-1, 1), rng.uniform(-8, 8)])
        x0 = rng.uniform(85, 240)
        x1 = x0 + rng.choice([-1, 1]) * rng.uniform(0.5, 6.0)
        ok, _, _, J = o.propagate(x0, x1, p)
        if not ok:
            continue
        for j in range(5):
            eps = 1e-6 * max(1.0, abs(p[j]))
            pp, pm = p.copy(), p.copy()
            pp[j] += eps
            pm[j] -= eps
            okp, fp, _, _ = o.propagate(x0, x1, pp)
            okm, fm, _, _ = o.propagate(x0, x1, pm)
            assert okp and okm
            fd = (fp - fm) / (2 * eps)
            np.testing.assert_allclose(J[:, j], fd, rtol=1e-6, atol=1e-7)


# --------------------------------------------------------------------------------------
# Covariance transport: C1 = J C0 J^T against explicit numpy algebra on a random C0.
# --------------------------------------------------------------------------------------
def test_covariance_transport_is_jcjt(row_x):
    o = _orc(row_x)
    rng = np.random.Generator(np.random.PCG64(8))
    A = rng.normal(size=(5, 5))
    Cf = A @ A.T + np.eye(5)
    c15 = np.array([Cf[i, j] for i in range(5) for j in range(i + 1)])
    ok, _, c1, J = o.propagate(120.0, 124.2, [3.0, 10.0, 0.3, 0.5, 2.0], c15)
    assert ok
    np.testing.assert_allclose(oracle.lower_to_full(c1), J @ Cf @ J.T, rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------------------
# Kalman update vs the textbook Gaussian posterior in information form.
# --------------------------------------------------------------------------------------
def test_update_equals_gaussian_posterior(row_x):
    o = _orc(row_x)
    rng = np.random.Generator(np.random.PCG64(9))
    H = np.zeros((2, 5))
    H[0, 0] = H[1, 1] = 1
    R = np.diag([0.1 ** 2, 0.1 ** 2])
    for _ in range(20):
        A = rng.normal(size=(5, 5))
        Cf = A @ A.T + 0.1 * np.eye(5)
        c15 = np.array([Cf[i, j] for i in range(5) for j in range(i + 1)])
        p = rng.normal(size=5)
        m = p[:2] + rng.normal(size=2)
        chi2, p1, c1 = o.update(m[0], m[1], p, c15)
        P = np.linalg.inv(np.linalg.inv(Cf) + H.T @ np.linalg.inv(R) @ H)
        mean = P @ (np.linalg.solve(Cf, p) + H.T @ np.linalg.solve(R, m))
        r = m - p[:2]
        np.testing.assert_allclose(p1, mean, rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(oracle.lower_to_full(c1), P, rtol=1e-8, atol=1e-10)
        assert chi2 == pytest.approx(r @ np.linalg.solve(Cf[:2, :2] + R, r), rel=1e-10)


# --------------------------------------------------------------------------------------
# Seed: three points on an exact helix give its parameters.
# --------------------------------------------------------------------------------------
def test_seed_is_exact_on_a_helix(row_x):
    f = _noise_free_sector0()
    o = _orc(row_x)
    X = row_x.astype(np.float64)
    rows = np.repeat(np.arange(152), np.diff(f.row_off[:153]))
    done = 0
    for lab in np.unique(f.label)[:30]:
        idx = np.flatnonzero(f.label == lab)
        idx = idx[np.argsort(rows[idx])]
        idx = idx[np.abs(f.truth_sphi[idx]) < 0.95]
        if idx.size < 5:
            continue
        s = [idx[0], idx[idx.size // 2], idx[-1]]
        ok, p = o.seed(X[rows[s]], f.truth_y[s], f.truth_z[s])
        assert ok
        truth = [f.truth_y[s[0]], f.truth_z[s[0]], f.truth_sphi[s[0]], f.trk_tgl[lab], f.trk_qpt[lab]]
        np.testing.assert_allclose(p, truth, rtol=1e-9, atol=1e-9)
        done += 1
    assert done > 15


# --------------------------------------------------------------------------------------
# End to end on noise-free helices: every findable segment is found once, with only its
# own clusters, and the fitted parameters equal the generated ones (up to the binary32
# rounding of the cluster coordinates).
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("bz", [synth.B_Z, 0.0])
def test_noise_free_helices_recover_truth(row_x, bz):
    f = _noise_free_sector0(n_tracks=120, seed=91, bz=bz)
    o = _orc(row_x, bz=bz)
    r = o.track_frame(f.y, f.z, f.row_off)
    m = truthmatch.match(f.label, f.row_off, r["hit_off"], r["hit_ids"], r["sector"])
    assert m["fakes"] == 0 and m["clones"] == 0
    assert np.all(m["purity"] == 1.0)
    assert m["found"] == m["findable"] and m["findable"] > 30
    rows = np.repeat(np.arange(152), np.diff(f.row_off[:153]))
    for t in range(r["n_tracks"]):
        h = r["hit_ids"][r["hit_off"][t]:r["hit_off"][t + 1]]
        lab = f.label[h[0]]
        seg = np.flatnonzero(f.label == lab)
        # every cluster of the segment away from the turning point is on the track
        inner = seg[np.abs(f.truth_sphi[seg]) < 0.9]
        assert set(inner.tolist()) <= set(h.tolist())
        assert np.all(np.diff(rows[h]) > 0)
        i0 = h[0]
        truth = np.array([f.truth_y[i0], f.truth_z[i0], f.truth_sphi[i0], f.trk_tgl[lab],
                          f.trk_qpt[lab] if bz != 0 else 0.0])
        p = r["params"][t]
        assert abs(p[0] - truth[0]) < 2e-5 and abs(p[1] - truth[1]) < 2e-5
        assert abs(p[2] - truth[2]) < 2e-6 and abs(p[3] - truth[3]) < 2e-6
        assert abs(p[4] - truth[4]) < 1e-4 * max(1.0, abs(truth[4]))
        if bz == 0:
            assert p[4] == 0.0
        assert r["x_ref"][t] == row_x[rows[i0]]


# --------------------------------------------------------------------------------------
# Step counts of the method on one straight track through all rows (B = 0).  Rows 0 and
# 151 carry no links, so the chain covers rows 1..150: 149 propagations and 150 updates.
# The outward follow takes row 151 (1 propagation, 1 cluster in the window, 1 update),
# the refit covers rows 151..1 and starts with a propagation to its own outermost row
# (151 propagations and updates), the inward follow takes row 0 (1, 1, 1).  The final fit
# takes 151 propagations and 152 updates per pass and evaluates chi2 on the inward pass.
# --------------------------------------------------------------------------------------
def test_step_counts_of_one_straight_track(row_x):
    o = _orc(row_x, bz=0.0)
    x = np.asarray(row_x, np.float64)
    y = (1.0 + 0.05 * x).astype(np.float32)
    z = (-3.0 + 0.2 * x).astype(np.float32)
    counts = np.zeros(36 * 152, np.int64)
    counts[:152] = 1
    ro = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    r = o.track_frame(y, z, ro, debug=True)
    assert r["n_tracks"] == 1 and r["nhits"][0] == 152
    assert list(r["debug"]["work"]) == [149 + 1 + 151 + 1, 150 + 1 + 151 + 1, 2, 151 + 151, 152 + 152, 152]


# --------------------------------------------------------------------------------------
# z at the beam line (Sec. 6): hand-worked straight lines; invariance of the result
# when the state is moved along its own helix (a wrong circle centre, sign or branch
# would change it); and noise-free primaries, whose tracks must point back to the
# vertex z (the generator's, t0 = 0).
# --------------------------------------------------------------------------------------
def test_beamline_z_straight_line_closed_form(row_x):
    o = _orc(row_x, bz=0.0)
    # the line through (100, 0) with direction (0.8, 0.6) is closest to the axis 80 cm back
    assert abs(o.beamline_z(100.0, [0.0, 10.0, 0.6, 0.5, 0.0]) - (10.0 - 0.5 * 80.0)) < 1e-12
    # through (120, 15) with direction (0.96, -0.28): 111 cm back
    assert abs(o.beamline_z(120.0, [15.0, -4.0, -0.28, -0.25, 0.0]) - (-4.0 + 0.25 * 111.0)) < 1e-12


def test_beamline_z_is_invariant_along_the_helix(row_x):
    o = _orc(row_x)
    rng = np.random.default_rng(5)
    n = 0
    for _ in range(300):
        x0, x1 = rng.uniform(85, 140), rng.uniform(150, 245)
        p = [rng.uniform(-10, 10), rng.uniform(-200, 200), rng.uniform(-0.5, 0.5), rng.uniform(-1, 1),
             rng.uniform(-2, 2)]
        ok, p1, _, _ = o.propagate(x0, x1, p)
        if not ok:
            continue
        assert abs(o.beamline_z(x0, p) - o.beamline_z(x1, p1)) < 1e-8
        n += 1
    assert n > 200


@pytest.mark.parametrize("bz", [synth.B_Z, 0.0])
def test_beamline_z_of_noise_free_primaries_is_the_vertex(row_x, bz):
    f = synth.config1_single_sector(seed=93, n_tracks=80, sigma=0.0, noise_frac=0.0, bz=bz)
    o = _orc(row_x, bz=bz)
    r = o.track_frame(f.y, f.z, f.row_off)
    n = 0
    for t in range(r["n_tracks"]):
        lab = f.label[r["hit_ids"][r["hit_off"][t]]]
        if f.trk_secondary[lab]:
            continue
        assert abs(r["z_beam"][t] - f.trk_vz[lab]) < 1e-3
        n += 1
    assert n > 30


# --------------------------------------------------------------------------------------
# Final fit vs nonlinear least squares: the inward pass starts at the outermost cluster
# from the outward estimate with covariance C0, so it estimates the minimiser of
#   sum_i |m_i - h_i(q)|^2 / sigma^2 + (q - p_outer)^T C0^-1 (q - p_outer)
# over the state q at the outermost cluster, with h_i the exact helix (circle geometry).
# An extended Kalman filter reaches that minimiser up to linearisation error, which
# shrinks in proportion to the cluster noise; a wrong Jacobian entry, a dropped term or a
# wrong sign would leave an O(sigma) gap at any noise.  Hence the check at 1e-4 cm.
# --------------------------------------------------------------------------------------
def _circle_predict(q, xa, xs, bz):
    y, z, s, t, k = q
    kap = -C_B * bz * k
    if abs(kap) < 1e-14:
        c = math.sqrt(1 - s * s)
        return y + (xs - xa) * s / c, z + t * (xs - xa) / c
    phia = math.asin(s)
    xc = xa - s / kap
    yc = y + math.cos(phia) / kap
    sinp = kap * (xs - xc)
    phi = np.arcsin(np.clip(sinp, -1, 1))
    return yc - np.cos(phi) / kap, z + t * (phi - phia) / kap


@pytest.mark.parametrize("bz", [synth.B_Z, 0.0])
def test_final_fit_matches_nonlinear_least_squares(row_x, bz):
    sg = 1e-4
    f = synth.config1_single_sector(seed=123, n_tracks=40, sigma=0.0, noise_frac=0.0, bz=bz)
    o = _orc(row_x, bz=bz, params=dict(sigma_y=sg, sigma_z=sg))
    X = row_x.astype(np.float64)
    rows = np.repeat(np.arange(152), np.diff(f.row_off[:153]))
    c0 = np.array(oracle.DEFAULT_PARAMS["c0"])
    rng = np.random.Generator(np.random.PCG64(17))
    done = 0
    for lab in np.unique(f.label):
        idx = np.flatnonzero(f.label == lab)
        idx = idx[np.argsort(rows[idx])]
        idx = idx[np.abs(f.truth_sphi[idx]) < 0.9]
        if idx.size < 30:
            continue
        xs = X[rows[idx]]
        ys = f.truth_y[idx] + rng.normal(0, sg, idx.size)
        zs = f.truth_z[idx] + rng.normal(0, sg, idx.size)
        ok, p_in, c_in, chi2, p_out = o.fit_hits(xs, ys, zs)
        assert ok
        xa = xs[-1]

        def resid(q):
            py, pz = _circle_predict(q, xa, xs, bz)
            q = np.asarray(q)
            return np.concatenate([(ys - py) / sg, (zs - pz) / sg, (q - p_out) / np.sqrt(c0)])

        sol = least_squares(resid, p_out, xtol=1e-15, ftol=1e-15, gtol=1e-15, method="lm")
        q = sol.x
        # the NLS optimum transported to the innermost cluster
        py, pz = _circle_predict(q, xa, xs[:1], bz)
        kap = -C_B * bz * q[4]
        s_in = q[2] + kap * (xs[0] - xa)
        sig = np.sqrt(np.diag(oracle.lower_to_full(c_in)))
        got = np.array([py[0], pz[0], s_in, q[3], q[4]])
        for i in range(5 if bz != 0 else 4):
            assert abs(p_in[i] - got[i]) < 0.01 * sig[i], (lab, i, p_in[i], got[i], sig[i])
        assert chi2 == pytest.approx(np.sum(sol.fun ** 2), rel=0.02, abs=0.5)
        done += 1
    assert done >= 5


def test_fit_pulls_are_standard_normal(row_x):
    """Statistical check of the covariance at the real cluster noise: pulls of the fitted
    parameters against the generated ones have mean ~0 and width ~1."""
    f = synth.config1_single_sector(seed=321, n_tracks=600, sigma=0.1, noise_frac=0.0)
    o = _orc(row_x)
    X = row_x.astype(np.float64)
    rows = np.repeat(np.arange(152), np.diff(f.row_off[:153]))
    pulls = []
    for lab in np.unique(f.label):
        idx = np.flatnonzero(f.label == lab)
        idx = idx[np.argsort(rows[idx])]
        idx = idx[np.abs(f.truth_sphi[idx]) < 0.9]
        if idx.size < 40:
            continue
        ok, p, c, chi2, _ = o.fit_hits(X[rows[idx]], f.y[idx], f.z[idx])
        assert ok
        i0 = idx[0]
        truth = np.array([f.truth_y[i0], f.truth_z[i0], f.truth_sphi[i0], f.trk_tgl[lab], f.trk_qpt[lab]])
        pulls.append((p - truth) / np.sqrt(np.diag(oracle.lower_to_full(c))))
    pulls = np.array(pulls)
    assert pulls.shape[0] > 150
    assert np.all(np.abs(pulls.mean(axis=0)) < 0.15)
    rms = pulls.std(axis=0)
    assert np.all((rms > 0.8) & (rms < 1.25)), rms


# --------------------------------------------------------------------------------------
# Grid: hand-worked example, cap rule and bijection invariants.
# --------------------------------------------------------------------------------------
def test_grid_hand_example(row_x):
    o = _orc(row_x, grid=dict(bin_y=2.0, bin_z=2.0, cap_mul=2, cap_add=64))
    g = o.grid_row(np.array([3.9, 0.0, 1.5], np.float32), np.array([10.0, 0.0, 0.0], np.float32))
    # extents y in [0, 3.9] -> ny = 1 + trunc(1.95) = 2; z in [0, 10] -> nz = 1 + 5 = 6
    assert (g["ylo"], g["zlo"], g["ny"], g["nz"], g["by"], g["bz"]) == (0.0, 0.0, 2, 6, 2.0, 2.0)
    # bins: c0 -> iy = min(1, 1) = 1, iz = min(5, 5) = 5 -> 11; c1 -> 0; c2 -> iy 0 -> 0
    assert g["perm"].tolist() == [1, 2, 0]
    expect = [0] + [2] * 11 + [3]
    assert g["bin_start"].tolist() == expect


def test_grid_cap_doubles_bins(row_x):
    o = _orc(row_x, grid=dict(bin_y=1.0, bin_z=1.0, cap_mul=2, cap_add=0))
    # 4 clusters spanning 0..3 in y and 0..100 in z: 4 * 101 bins > 8 -> bz doubles until
    # ny * nz <= 8: bz = 64 gives nz = 1 + trunc(100/64) = 2, 4 * 2 = 8
    y = np.array([0, 1, 2, 3], np.float32)
    z = np.array([0, 30, 60, 100], np.float32)
    g = o.grid_row(y, z)
    assert (g["ny"], g["nz"], g["bz"], g["by"]) == (4, 2, 64.0, 1.0)
    # when nz reaches 1 the y bin doubles: 4 clusters in y 0..30, cap 4 -> by 8 -> ny 4
    o2 = _orc(row_x, grid=dict(bin_y=1.0, bin_z=1.0, cap_mul=1, cap_add=0))
    g2 = o2.grid_row(np.array([0, 10, 20, 30], np.float32), np.zeros(4, np.float32))
    assert (g2["nz"], g2["ny"], g2["by"]) == (1, 4, 8.0)


def test_grid_invariants(small_pbpb_frame, row_x):
    f = small_pbpb_frame
    for grid in (dict(bin_y=0.5, bin_z=0.5), dict(bin_y=2.0, bin_z=2.0), dict(bin_y=7.0, bin_z=13.0)):
        o = _orc(row_x, grid=dict(oracle.DEFAULT_GRID, **grid))
        d = o.track_frame(f.y, f.z, f.row_off, debug=True)["debug"]
        for g in range(0, 36 * 152, 97):
            a, b = f.row_off[g], f.row_off[g + 1]
            n = b - a
            ny, nz = d["g_ny"][g], d["g_nz"][g]
            assert ny * nz <= 2 * n + 64
            perm = d["perm"][a:b].astype(np.int64)
            assert sorted(perm.tolist()) == list(range(n))
            bs = d["bin_start"][d["g_bin_base"][g]:d["g_bin_base"][g] + ny * nz + 1].astype(np.int64)
            assert bs[0] == 0 and bs[-1] == n and np.all(np.diff(bs) >= 0)
            ys, zs = f.y[a:b][perm], f.z[a:b][perm]
            iy = np.minimum(ny - 1, ((ys - np.float32(d["g_ylo"][g])) / np.float32(d["g_by"][g])).astype(np.int32))
            iz = np.minimum(nz - 1, ((zs - np.float32(d["g_zlo"][g])) / np.float32(d["g_bz"][g])).astype(np.int32))
            bins = iz * ny + iy
            assert np.all(np.diff(bins) >= 0)
            same = np.diff(bins) == 0
            assert np.all(np.diff(perm)[same] > 0)
            assert np.array_equal(np.bincount(bins, minlength=ny * nz), np.diff(bs))


# --------------------------------------------------------------------------------------
# Neighbour links: hand-worked example, brute force, and noise-free chains.
# --------------------------------------------------------------------------------------
def test_links_hand_example():
    rx = np.array([0.0, 1.0, 2.0], np.float32)
    o = oracle.Oracle(rx, n_sectors=1)
    # row 0 (down): d0 (-1, 0), d1 (0.5, 0), d2 (-1, 0) duplicate of d0
    # row 1: h0 (0, 0); h1 (10, 0) sees u2 only above and d3 only below
    # row 2 (up):   u0 (1, 0), u1 (3.5, 0) outside the 3 cm window, u2 (10, 1.5),
    #               u3 (1, 0) duplicate of u0
    # row 0 also has d3 (10, -1.5)
    y0 = [-1.0, 0.5, -1.0, 10.0]; z0 = [0, 0, 0, -1.5]
    y1 = [0.0, 10.0]; z1 = [0, 0]
    y2 = [1.0, 3.5, 10.0, 1.0]; z2 = [0, 0, 1.5, 0]
    y = np.array(y0 + y1 + y2, np.float32)
    z = np.array(z0 + z1 + z2, np.float32)
    ro = np.array([0, 4, 6, 10], np.int64)
    up, dn = o.links_sector(y, z, ro)
    # h0: u0 or u3 with d0 or d2 gives D = (1 - 1)^2 = 0 (ties -> smaller u = u0, then
    #     smaller d = d0); any u with d1: D = (1 - (-0.5))^2 = 2.25 > 1.
    assert (up[4], dn[4]) == (0, 0)
    # h1: u2, d3: ty_u = 0, tz_u = 1.5, ty_d = 0, tz_d = 1.5 -> D = 0
    assert (up[5], dn[5]) == (2, 3)
    # rows 0 and 2 carry no links
    assert np.all(up[:4] == -1) and np.all(dn[:4] == -1) and np.all(up[6:] == -1)
    # kink above kink_max: move d3 to z = +1.5 -> tz_d = -1.5, D = 9 > 1 -> no pair
    z[3] = 1.5
    up, dn = o.links_sector(y, z, ro)
    assert (up[5], dn[5]) == (-1, -1)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_links_sorted_scan_equals_brute_force(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    rx = np.array([85 + i * 160 / 151 for i in range(12)], np.float32)
    o = oracle.Oracle(rx, n_sectors=1)
    counts = rng.integers(0, 25, 12)
    ro = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    n = int(ro[-1])
    # dense clusters plus exact duplicates to exercise the tie-breaks
    y = rng.uniform(-4, 4, n).astype(np.float32)
    z = rng.uniform(-4, 4, n).astype(np.float32)
    dup = rng.random(n) < 0.2
    y[dup] = np.round(y[dup])
    z[dup] = np.round(z[dup])
    a = o.links_sector(y, z, ro, brute=True)
    b = o.links_sector(y, z, ro, brute=False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert (a[0] >= 0).sum() > 10


def test_noise_free_chains_follow_truth(row_x):
    f = _noise_free_sector0(n_tracks=80, seed=5)
    o = _orc(row_x)
    d = o.track_frame(f.y, f.z, f.row_off, debug=True)["debug"]
    rows = np.repeat(np.arange(152), np.diff(f.row_off[:153]))
    ok = 0
    for h in range(f.n_clusters):
        if d["cup"][h] < 0:
            continue
        u = f.row_off[rows[h] + 1] + d["cup"][h]
        assert f.label[u] == f.label[h] and rows[u] == rows[h] + 1
        ok += 1
    assert ok > 1000


def test_link_graph_invariants(small_pbpb_frame, row_x):
    f = small_pbpb_frame
    o = _orc(row_x)
    d = o.track_frame(f.y, f.z, f.row_off, debug=True)["debug"]
    g_of = np.repeat(np.arange(36 * 152), np.diff(f.row_off))
    cup, cdn = d["cup"], d["cdn"]
    n_pred = np.zeros(f.n_clusters, np.int64)
    for h in np.flatnonzero(cup >= 0):
        u = f.row_off[g_of[h] + 1] + cup[h]
        assert g_of[u] == g_of[h] + 1                      # up goes to the next row
        assert cdn[u] == h - f.row_off[g_of[h]]            # and links back
        n_pred[u] += 1
    for h in np.flatnonzero(cdn >= 0):
        dd = f.row_off[g_of[h] - 1] + cdn[h]
        assert cup[dd] == h - f.row_off[g_of[h]]
    assert n_pred.max() <= 1                               # chains are vertex-disjoint
    # cleaned links are the reciprocal subset of the raw ones
    assert np.all((cup < 0) | (cup == d["up"])) and np.all((cdn < 0) | (cdn == d["dn"]))
    # starts are the chain bottoms; every linked cluster lies on exactly one start's chain
    starts = np.flatnonzero((cup >= 0) & (cdn < 0))
    assert np.array_equal(starts, np.flatnonzero(d["start"]))
    seen = np.zeros(f.n_clusters, np.int64)
    for s in starts:
        h = s
        while True:
            seen[h] += 1
            if cup[h] < 0:
                break
            h = f.row_off[g_of[h] + 1] + cup[h]
    linked = (cup >= 0) | (cdn >= 0)
    assert np.all(seen[linked] == 1) and np.all(seen[~linked] == 0)
    assert d["tl_start"].tolist() == starts.tolist()


def test_links_identical_in_both_builds(small_pbpb_frame, row_x):
    f = small_pbpb_frame
    a = _orc(row_x, "f64").track_frame(f.y, f.z, f.row_off, debug=True)["debug"]
    b = _orc(row_x, "f32").track_frame(f.y, f.z, f.row_off, debug=True)["debug"]
    for k in ("up", "dn", "cup", "cdn", "perm", "bin_start", "g_ny", "g_nz"):
        assert np.array_equal(a[k], b[k]), k


def test_grid_does_not_change_links_or_tracks(small_pbpb_frame, row_x):
    f = small_pbpb_frame
    ref = None
    for grid in (dict(bin_y=0.3, bin_z=0.3), dict(bin_y=2.0, bin_z=2.0), dict(bin_y=9.0, bin_z=40.0, cap_mul=1)):
        r = _orc(row_x, grid=dict(oracle.DEFAULT_GRID, **grid)).track_frame(f.y, f.z, f.row_off, debug=True)
        cur = (r["debug"]["up"], r["debug"]["dn"], r["hit_ids"], r["params"])
        if ref is None:
            ref = cur
        else:
            for a, b in zip(ref, cur):
                assert np.array_equal(a, b)


# --------------------------------------------------------------------------------------
# Selection: order independence and exclusivity.
# --------------------------------------------------------------------------------------
def test_selection_is_order_independent(small_pbpb_frame, row_x):
    f = small_pbpb_frame
    o = _orc(row_x)
    base = o.track_frame(f.y, f.z, f.row_off)
    for seed in (1, 99, 12345):
        r = o.track_frame(f.y, f.z, f.row_off, shuffle_seed=seed)
        for k in ("hit_off", "hit_ids", "params", "cov", "cluster_track"):
            assert np.array_equal(base[k], r[k]), k


def test_selection_invariants(small_pbpb_frame, row_x):
    f = small_pbpb_frame
    o = _orc(row_x)
    r = o.track_frame(f.y, f.z, f.row_off, debug=True)
    d = r["debug"]
    hits = r["hit_ids"]
    assert np.unique(hits).size == hits.size                      # a cluster is in <= 1 track
    ct = r["cluster_track"]
    for t in range(r["n_tracks"]):
        h = hits[r["hit_off"][t]:r["hit_off"][t + 1]]
        assert np.all(ct[h] == t) and h.size >= 20 and r["ndf"][t] == 2 * h.size - 5
    assert (ct >= 0).sum() == hits.size
    # every kept cluster carries the weight of its track's tracklet
    w_of = {}
    rank = {int(s): k for k, s in enumerate(d["tl_start"])}
    for k, s in enumerate(d["tl_start"]):
        n = d["tl_nhits"][k]
        w_of[int(s)] = (int(n) << 32) | (0xFFFFFFFF - k)
    assert len(rank) == len(w_of)
    Wmax = d["W"]
    for t in range(r["n_tracks"]):
        h = hits[r["hit_off"][t]:r["hit_off"][t + 1]]
        assert np.all(Wmax[h] == Wmax[h[0]])


# --------------------------------------------------------------------------------------
# Sanity of the whole method on the Pb-Pb event.
# --------------------------------------------------------------------------------------
def test_efficiency_on_pbpb_event(cfg2_frame, row_x):
    f = cfg2_frame
    r = _orc(row_x).track_frame(f.y, f.z, f.row_off)
    m = truthmatch.match(f.label, f.row_off, r["hit_off"], r["hit_ids"], r["sector"])
    assert m["efficiency"] > 0.97
    assert m["fake_rate"] < 0.01
    assert m["clone_rate"] < 0.01
