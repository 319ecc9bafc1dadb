// Kalman filter of the track model, shared by the tracking and the merging kernels.
#pragma once

#include "tpcsf_internal.h"

namespace tpcsf {

// ------------------------------------------------------------------------------------
// Kalman filter in binary64.  State (y, z, sin phi, tan lambda, q/pT) at plane x;
// curvature kappa = a * q/pT.  Covariance: 15-element lower triangle.
// ------------------------------------------------------------------------------------
struct Trk {
    double x;
    double p[5];
    double c[15];
};

// 1/x, 1/sqrt(x) and sqrt(x) of positive, normal binary64 values: the hardware estimate
// (relative error below 2^-22) refined by two Newton steps, within about an ulp.  The
// correctly rounded library forms take about twice the instructions; the filter needs
// neither their last ulp nor their handling of zero, infinity and denormals.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-h * y, y, 0.5);
    return fma(y, e, y);
}

__device__ __forceinline__ double sqrt_nr(double x)
{
    const double y = rsqrt_nr(x);
    const double s = x * y;
    return fma(fma(-s, s, x), 0.5 * y, s);
}

// asin out of line: the rare long steps need it, and inlined, its registers would count
// against every kernel that propagates
__device__ __attribute__((noinline)) double asin_outline(double h) { return asin(h); }

// asin(h)/h and its derivative; Taylor series near 0
__device__ __forceinline__ void arc_factor(double h, double& A, double& Ap)
{
    if (fabs(h) < 0.01) {
        const double h2 = h * h;
        A = 1.0 + h2 * (1.0 / 6.0 + h2 * (3.0 / 40.0 + h2 * (5.0 / 112.0)));
        Ap = h * (1.0 / 3.0 + h2 * (3.0 / 10.0 + h2 * (15.0 / 56.0 + h2 * (35.0 / 144.0))));
    } else {
        const double as = asin_outline(h);
        const double ih = 1.0 / h;
        A = as * ih;
        Ap = (h / sqrt((1.0 - h) * (1.0 + h)) - as) * ih * ih;
    }
}

// Exact helix step to the plane x1 with the analytic Jacobian.  sin(phi) is linear in x;
// y follows the chord at the mean angle; z follows the arc length chord*asin(h)/h with
// h = kappa*chord/2.  Fails (state unchanged) when |sin(phi)| would reach sinphi_max.
static __device__ bool trk_propagate(Trk& t, double x1, const DevParams& P)
{
    const double dx = x1 - t.x;
    const double s0 = t.p[2];
    const double tl = t.p[3];
    const double kap = P.a * t.p[4];
    const double s1 = s0 + kap * dx;
    if (!(fabs(s0) < P.sinphi_max) || !(fabs(s1) < P.sinphi_max)) return false;
    // cos(phi) at both ends and their reciprocals from one reciprocal square root each
    const double u0 = (1.0 - s0) * (1.0 + s0), u1 = (1.0 - s1) * (1.0 + s1);
    const double ic0 = rsqrt_nr(u0), ic1 = rsqrt_nr(u1);
    const double c0 = u0 * ic0, c1 = u1 * ic1;
    const double ics = rcp_nr(c0 + c1);
    const double tb = (s0 + s1) * ics;
    const double sec2 = 1.0 + tb * tb;
    const double sec = sqrt_nr(sec2);
    const double chord = dx * sec;
    const double h = 0.5 * kap * chord;
    if (!(fabs(h) < 1.0)) return false;
    double A, Ap;
    arc_factor(h, A, Ap);
    const double ds = chord * A;
    const double q = 0.5 * tb * dx * ic1;
    const double j02 = 0.5 * dx * sec2 * (ic0 + ic1);
    const double j04 = P.a * (0.5 * dx * dx * sec2 * ic1);
    const double j12 = tl * (dx * (s0 + s1) * ic0 * ic1 * ics);
    const double j13 = ds;
    const double j14 = tl * P.a * (chord * (q * A + Ap * (0.5 * chord) * (1.0 + kap * q)));
    const double j24 = P.a * dx;

    t.p[0] += dx * tb;
    t.p[1] += tl * ds;
    t.p[2] = s1;
    t.x = x1;

    // C <- J C J^T with J = identity + {j02, j04, j12, j13, j14, j24}, one column of the
    // result at a time: column j of C' (rows >= j) is J applied to v_j = C J_j^T, and v_j
    // needs only entries of C that the earlier columns did not overwrite.
    double* c = t.c;
    // column 0: v0 = C (e0 + j02 e2 + j04 e4)
    {
        const double v0 = c[0] + j02 * c[3] + j04 * c[10];
        const double v1 = c[1] + j02 * c[4] + j04 * c[11];
        const double v2 = c[3] + j02 * c[5] + j04 * c[12];
        const double v3 = c[6] + j02 * c[8] + j04 * c[13];
        const double v4 = c[10] + j02 * c[12] + j04 * c[14];
        c[0] = v0 + j02 * v2 + j04 * v4;
        c[1] = v1 + j12 * v2 + j13 * v3 + j14 * v4;
        c[3] = v2 + j24 * v4;
        c[6] = v3;
        c[10] = v4;
    }
    // column 1 (rows 1..4): v1 = C (e1 + j12 e2 + j13 e3 + j14 e4)
    {
        const double v1 = c[2] + j12 * c[4] + j13 * c[7] + j14 * c[11];
        const double v2 = c[4] + j12 * c[5] + j13 * c[8] + j14 * c[12];
        const double v3 = c[7] + j12 * c[8] + j13 * c[9] + j14 * c[13];
        const double v4 = c[11] + j12 * c[12] + j13 * c[13] + j14 * c[14];
        c[2] = v1 + j12 * v2 + j13 * v3 + j14 * v4;
        c[4] = v2 + j24 * v4;
        c[7] = v3;
        c[11] = v4;
    }
    // column 2 (rows 2..4): v2 = C (e2 + j24 e4); columns 3 and 4 are unchanged
    {
        const double v2 = c[5] + j24 * c[12];
        const double v3 = c[8] + j24 * c[13];
        const double v4 = c[12] + j24 * c[14];
        c[5] = v2 + j24 * v4;
        c[8] = v3;
        c[12] = v4;
    }
    return true;
}

// Position (y, z) of the helix of state p at plane x0 on the plane x1: the parameter part
// of trk_propagate, same arithmetic.  False where that step would fail.
__device__ __forceinline__ bool trk_predict(const double* p, double x0, double x1, const DevParams& P, double& y,
                                            double& z)
{
    const double dx = x1 - x0;
    const double s0 = p[2];
    const double kap = P.a * p[4];
    const double s1 = s0 + kap * dx;
    if (!(fabs(s0) < P.sinphi_max) || !(fabs(s1) < P.sinphi_max)) return false;
    const double u0 = (1.0 - s0) * (1.0 + s0), u1 = (1.0 - s1) * (1.0 + s1);
    const double ic0 = rsqrt_nr(u0), ic1 = rsqrt_nr(u1);
    const double c0 = u0 * ic0, c1 = u1 * ic1;
    const double ics = rcp_nr(c0 + c1);
    const double tb = (s0 + s1) * ics;
    const double sec2 = 1.0 + tb * tb;
    const double sec = sqrt_nr(sec2);
    const double chord = dx * sec;
    const double h = 0.5 * kap * chord;
    if (!(fabs(h) < 1.0)) return false;
    double A, Ap;
    arc_factor(h, A, Ap);
    y = p[0] + dx * tb;
    z = p[1] + p[3] * (chord * A);
    return true;
}

// Kalman update with the cluster (my, mz), R = diag(sy2, sz2); returns the cluster's chi2
// r^T S^-1 r before the update.  The gain rows K_i = (C_i0, C_i1) S^-1 and the covariance
// rows C_ij -= K_i (C_j0, C_j1)^T are taken from the last row to the first: row i reads
// columns 0 and 1 of rows j <= i only, which the rows after it have not changed yet.
static __device__ double trk_update(Trk& t, double my, double mz, const DevParams& P)
{
    const double r0 = my - t.p[0], r1 = mz - t.p[1];
    double* c = t.c;
    const double s00 = c[0] + P.sy2, s01 = c[1], s11 = c[2] + P.sz2;
    const double idet = rcp_nr(s00 * s11 - s01 * s01);
    const double i00 = s11 * idet, i01 = -s01 * idet, i11 = s00 * idet;
    const double chi2 = r0 * (r0 * i00 + r1 * i01) + r1 * (r0 * i01 + r1 * i11);
#pragma unroll
    for (int i = 4; i >= 0; --i) {
        const int ri = i * (i + 1) / 2;
        // C_i0, C_i1; row 1 has already replaced the shared entry C_10 = C_01 when row 0
        // comes, so row 0 takes it from s01
        const double a0 = c[ri], a1 = i == 0 ? s01 : c[ri + 1];
        const double k0 = a0 * i00 + a1 * i01;
        const double k1 = a0 * i01 + a1 * i11;
        t.p[i] += k0 * r0 + k1 * r1;
#pragma unroll
        for (int j = i; j >= 0; --j) {
            const double b0 = j == i ? a0 : c[j * (j + 1) / 2];
            const double b1 = j == i ? a1 : c[j == 0 ? 1 : j * (j + 1) / 2 + 1];
            c[ri + j] -= k0 * b0 + k1 * b1;
        }
    }
    return chi2;
}

__device__ __forceinline__ void trk_reset_cov(Trk& t, const DevParams& P)
{
#pragma unroll
    for (int i = 0; i < 15; ++i) t.c[i] = 0.0;
    t.c[0] = P.c0[0]; t.c[2] = P.c0[1]; t.c[5] = P.c0[2]; t.c[9] = P.c0[3]; t.c[14] = P.c0[4];
}

// Circle through three (x, y) points, traversed in order: curvature and sin(phi) at the
// first; tan(lambda) from the z change over the arc to the last.
static __device__ bool trk_seed(Trk& t, const double* x, const double* y, const double* z, const DevParams& P)
{
    const double ax = x[1] - x[0], ay = y[1] - y[0];
    const double bx = x[2] - x[1], by = y[2] - y[1];
    const double ex = x[2] - x[0], ey = y[2] - y[0];
    const double la = sqrt(ax * ax + ay * ay), lb = sqrt(bx * bx + by * by), lc = sqrt(ex * ex + ey * ey);
    const double den = la * lb * lc;
    if (!(den > 0.0)) return false;
    const double kap = 2.0 * (ax * by - ay * bx) / den;
    const double h = 0.5 * kap * lc;
    if (!(fabs(h) < 1.0)) return false;
    double A, Ap;
    arc_factor(h, A, Ap);
    const double il = 1.0 / lc;
    t.x = x[0];
    t.p[0] = y[0];
    t.p[1] = z[0];
    t.p[2] = ey * il * sqrt((1.0 - h) * (1.0 + h)) - ex * il * h;
    t.p[3] = (z[2] - z[0]) / (lc * A);
    t.p[4] = (P.a != 0.0) ? kap / P.a : 0.0;
    return true;
}

// z at the beam line: the helix of state p at plane x0 followed to its point of closest
// approach to the beam axis (the origin of the sector frame) in the transverse plane,
// along the shorter arc; z there.  For a primary from a vertex at the origin this is the
// most likely z of the track's origin (its drift offset in a time frame).
static __device__ double trk_beamline_z(const DevParams& P, double x0, const double* p)
{
    const double y0 = p[0], z0 = p[1], s0 = p[2], tl = p[3];
    const double c0 = sqrt((1.0 - s0) * (1.0 + s0));
    const double kap = P.a * p[4];
    double s;
    if (kap == 0.0) {
        s = -(x0 * c0 + y0 * s0);
    } else {
        const double xc = x0 - s0 / kap, yc = y0 + c0 / kap;   // circle centre
        const double d = sqrt(xc * xc + yc * yc);
        if (!(d > 0.0)) return z0;
        const double sg = kap > 0.0 ? 1.0 : -1.0;
        const double sd = -sg * xc / d, cd = sg * yc / d;       // direction at the closest point
        s = atan2(sd * c0 - cd * s0, cd * c0 + sd * s0) / kap;
    }
    return z0 + tl * s;
}

// State into the frame of a sector whose azimuth is larger by delta (c = cos delta,
// sn = sin delta): the point (x, y) and the direction are rotated and the state is given
// at the plane x' through the rotated point.  cos(phi') must stay positive (the track
// moves outward) and |sin(phi')| below sinphi_max, else the state is left unchanged and
// the call fails.  Covariance: a change dy moves the point by (sn dy, c dy) and the state
// at the fixed plane x' follows the helix back by sn dy, so that
//   dy'/dy = c - sn tan(phi'),  dz'/dy = -sn tan(lambda) / cos(phi'),
//   d sin(phi')/dy = -kappa sn,  d sin(phi')/d sin(phi) = cos(phi') / cos(phi).
static __device__ bool trk_rotate(Trk& t, double c, double sn, const DevParams& P)
{
    const double s0 = t.p[2];
    if (!(fabs(s0) < 1.0)) return false;
    const double c0 = sqrt(1.0 - s0 * s0);
    const double s1 = s0 * c - c0 * sn;
    const double c1 = c0 * c + s0 * sn;
    if (!(c1 > 0.0) || !(fabs(s1) < P.sinphi_max)) return false;
    const double j00 = c - sn * s1 / c1;
    const double j10 = -sn * t.p[3] / c1;
    const double j20 = -P.a * t.p[4] * sn;
    const double j22 = c1 / c0;
    const double x1 = t.x * c + t.p[0] * sn;
    const double y1 = -t.x * sn + t.p[0] * c;
    t.x = x1;
    t.p[0] = y1;
    t.p[2] = s1;
    // C <- J C J^T with J = identity except J00, J10, J20, J22
    double* q = t.c;
    const double c00 = q[0], c10 = q[1], c11 = q[2], c20 = q[3], c21 = q[4], c22 = q[5];
    const double c30 = q[6], c31 = q[7], c32 = q[8];
    const double c40 = q[10], c41 = q[11], c42 = q[12];
    // A = J C (the entries of rows 0..2 that C' needs); rows 3, 4 of A are those of C
    const double a00 = j00 * c00;
    const double a10 = j10 * c00 + c10, a11 = j10 * c10 + c11;
    const double a20 = j20 * c00 + j22 * c20, a21 = j20 * c10 + j22 * c21, a22 = j20 * c20 + j22 * c22;
    // C' = A J^T (lower triangle): column j of J^T is row j of J
    q[0] = a00 * j00;
    q[1] = a10 * j00;
    q[2] = a10 * j10 + a11;
    q[3] = a20 * j00;
    q[4] = a20 * j10 + a21;
    q[5] = a20 * j20 + a22 * j22;
    q[6] = j00 * c30;
    q[7] = j10 * c30 + c31;
    q[8] = j20 * c30 + j22 * c32;
    q[10] = j00 * c40;
    q[11] = j10 * c40 + c41;
    q[12] = j20 * c40 + j22 * c42;
    return true;
}

}  // namespace tpcsf
