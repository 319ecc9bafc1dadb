/*
 * Reference oracle for TPC sector track finding (test infrastructure only; see orc.h).
 *
 * The paper (arXiv:2009.07515, Sec. 6) states that TPC tracking runs standalone, without
 * position-dependent corrections, in continuous-readout time frames whose z coordinate is
 * shifted by the unknown collision time, and that the algorithm derives from the Run 2 HLT
 * cellular-automaton tracker.  Sec. 7.1 adds that a whole time frame is processed at once.
 * Nothing more of the method is printed.  The steps below are this project's definition of
 * that method, written as plainly as possible: sequential loops, no blocking, no fusion.
 *
 *   1. grid        per-row y/z bins and a stable counting sort (binary32)
 *   2. links       best (up, down) neighbour pair by slope change (binary32)
 *   3. cleaning    keep only reciprocal links
 *   4. starts      chain bottoms, ranked in (sector, row, in-row index) order
 *   5. tracklets   seed, Kalman fit along the chain, follow outward, refit and follow inward
 *   6. selection   per-cluster max-weight claim, accept tracklets that keep enough clusters
 *   7. final fit   two-pass Kalman refit of each accepted track's kept clusters
 *   8. merging     links of sector tracks across azimuthal sector edges, refit of the
 *                  merged tracks across sector frames (orc_merge_frame)
 *   9. hit removal keep only the clusters near good tracks, compression strategy B
 *                  (orc_reject_frame)
 *  10. residuals   track-model compression of the attached clusters (orc_compress_frame)
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORC_FP32
typedef float orc_real;
#define R_SQRT sqrtf
#define R_ASIN asinf
#define R_FABS fabsf
#define ARC_SERIES 0.1f
#else
typedef double orc_real;
#define R_SQRT sqrt
#define R_ASIN asin
#define R_FABS fabs
#define ARC_SERIES 0.01
#endif

/* kappa [1/cm] = -C_B * B [T] * q/pT [c/GeV] */
#define C_B 0.00299792458
#define ORC_PI 3.14159265358979323846

/* ---------------------------------------------------------------------------------- */
/* Step 1: per-row search grid (binary32).                                             */
/* Extents are the exact minima and maxima of the row.  ny = 1 + trunc((yhi-ylo)/by),  */
/* nz likewise; while ny*nz exceeds cap_mul*n + cap_add the z bin (or, once nz == 1,   */
/* the y bin) doubles.  A cluster's bin is iz*ny + iy with iy = min(ny-1,               */
/* trunc((y-ylo)/by)).  Clusters are ordered by bin, ties by in-row index.              */
/* ---------------------------------------------------------------------------------- */
int orc_grid_row(const orc_cfg* cfg, int64_t n, const float* y, const float* z,
                 float* ylo, float* zlo, float* by, float* bz, int32_t* ny, int32_t* nz,
                 uint32_t* bin_start, int64_t cap, uint32_t* perm)
{
    float lo_y = 0.0f, hi_y = 0.0f, lo_z = 0.0f, hi_z = 0.0f;
    float b_y = cfg->bin_y, b_z = cfg->bin_z;
    int32_t n_y = 1, n_z = 1;
    if (n > 0) {
        lo_y = hi_y = y[0];
        lo_z = hi_z = z[0];
        for (int64_t i = 1; i < n; ++i) {
            if (y[i] < lo_y) lo_y = y[i];
            if (y[i] > hi_y) hi_y = y[i];
            if (z[i] < lo_z) lo_z = z[i];
            if (z[i] > hi_z) hi_z = z[i];
        }
        n_y = 1 + (int32_t)((hi_y - lo_y) / b_y);
        n_z = 1 + (int32_t)((hi_z - lo_z) / b_z);
        int64_t max_bins = (int64_t)cfg->cap_mul * n + cfg->cap_add;
        while ((int64_t)n_y * n_z > max_bins) {
            if (n_z > 1) {
                b_z = b_z * 2.0f;
                n_z = 1 + (int32_t)((hi_z - lo_z) / b_z);
            } else {
                b_y = b_y * 2.0f;
                n_y = 1 + (int32_t)((hi_y - lo_y) / b_y);
            }
        }
    }
    int64_t nb = (int64_t)n_y * n_z;
    *ylo = lo_y; *zlo = lo_z; *by = b_y; *bz = b_z; *ny = n_y; *nz = n_z;
    if (nb + 1 > cap) return -3;

    int32_t* bin = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int32_t iy = (int32_t)((y[i] - lo_y) / b_y);
        int32_t iz = (int32_t)((z[i] - lo_z) / b_z);
        if (iy > n_y - 1) iy = n_y - 1;
        if (iz > n_z - 1) iz = n_z - 1;
        bin[i] = iz * n_y + iy;
    }
    /* counting sort: histogram, exclusive prefix sum, stable placement */
    for (int64_t b = 0; b <= nb; ++b) bin_start[b] = 0;
    for (int64_t i = 0; i < n; ++i) bin_start[bin[i] + 1] += 1;
    for (int64_t b = 0; b < nb; ++b) bin_start[b + 1] += bin_start[b];
    uint32_t* cursor = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)nb);
    for (int64_t b = 0; b < nb; ++b) cursor[b] = bin_start[b];
    for (int64_t i = 0; i < n; ++i) perm[cursor[bin[i]]++] = (uint32_t)i;
    free(cursor);
    free(bin);
    return 0;
}

/* ---------------------------------------------------------------------------------- */
/* Step 2: neighbour links (binary32).                                                 */
/* For a cluster h in row r (1 <= r <= n_rows-2), a cluster c of row r+1 or r-1 is a   */
/* candidate when |y_c - y_h| <= win_y and |z_c - z_h| <= win_z.  Over all candidate   */
/* pairs (u in r+1, d in r-1) the slope change                                          */
/*   D = (ty_u - ty_d)^2 + (tz_u - tz_d)^2,  ty_u = (y_u - y_h)/(X_{r+1} - X_r),        */
/*   ty_d = (y_h - y_d)/(X_r - X_{r-1})  (z alike)                                      */
/* is minimal; the pair wins if D <= kink_max.  Equal D: smaller u, then smaller d.     */
/* Rows 0 and n_rows-1 get no links.                                                    */
/* ---------------------------------------------------------------------------------- */
static int pair_better(float D, int32_t u, int32_t d, float bD, int32_t bu, int32_t bd)
{
    if (bu < 0) return 1;
    if (D < bD) return 1;
    if (D > bD) return 0;
    if (u != bu) return u < bu;
    return d < bd;
}

static float kink(float yh, float zh, float yu, float zu, float yd, float zd, float dxu, float dxd)
{
    float tuy = (yu - yh) / dxu;
    float tuz = (zu - zh) / dxu;
    float tdy = (yh - yd) / dxd;
    float tdz = (zh - zd) / dxd;
    float ay = tuy - tdy;
    float az = tuz - tdz;
    float sy = ay * ay;
    float sz = az * az;
    return sy + sz;
}

static int in_window(float yc, float zc, float yh, float zh, float wy, float wz)
{
    return fabsf(yc - yh) <= wy && fabsf(zc - zh) <= wz;
}

/* y-sorted order of a row's clusters (ties by in-row index), for window scans */
static __thread const float* g_sort_y;   /* per thread: callers may track sectors in parallel */
static int cmp_y(const void* a, const void* b)
{
    int32_t i = *(const int32_t*)a, j = *(const int32_t*)b;
    if (g_sort_y[i] < g_sort_y[j]) return -1;
    if (g_sort_y[i] > g_sort_y[j]) return 1;
    return (i > j) - (i < j);
}

static void sort_row_by_y(const float* y, int64_t n, int32_t* idx)
{
    for (int64_t i = 0; i < n; ++i) idx[i] = (int32_t)i;
    g_sort_y = y;
    qsort(idx, (size_t)n, sizeof(int32_t), cmp_y);
}

/* first position k in a y-sorted row with (y[idx[k]] - yh) >= -w, in binary32 */
static int64_t lower_f32(const float* y, const int32_t* idx, int64_t n, float yh, float w)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (y[idx[mid]] - yh >= -w) hi = mid; else lo = mid + 1;
    }
    return lo;
}

int orc_links_sector(const orc_cfg* cfg, const float* y, const float* z,
                     const int64_t* row_off, int brute, int32_t* up, int32_t* dn)
{
    const int nr = cfg->n_rows;
    const int64_t base = row_off[0];
    const int64_t nsec = row_off[nr] - base;
    for (int64_t i = 0; i < nsec; ++i) { up[i] = -1; dn[i] = -1; }
    int32_t* sidx = NULL;
    if (!brute) sidx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nsec > 0 ? nsec : 1));
    if (!brute)
        for (int r = 0; r < nr; ++r)
            sort_row_by_y(y + row_off[r], row_off[r + 1] - row_off[r], sidx + (row_off[r] - base));

    for (int r = 1; r + 1 < nr; ++r) {
        const float dxu = cfg->row_x[r + 1] - cfg->row_x[r];
        const float dxd = cfg->row_x[r] - cfg->row_x[r - 1];
        const int64_t oh = row_off[r], ou = row_off[r + 1], od = row_off[r - 1];
        const int64_t nh = row_off[r + 1] - oh, nu = row_off[r + 2] - ou, nd = row_off[r] - od;
        for (int64_t h = 0; h < nh; ++h) {
            const float yh = y[oh + h], zh = z[oh + h];
            float bD = 0.0f;
            int32_t bu = -1, bd = -1;
            if (brute) {
                for (int64_t u = 0; u < nu; ++u) {
                    if (!in_window(y[ou + u], z[ou + u], yh, zh, cfg->win_y, cfg->win_z)) continue;
                    for (int64_t d = 0; d < nd; ++d) {
                        if (!in_window(y[od + d], z[od + d], yh, zh, cfg->win_y, cfg->win_z)) continue;
                        float D = kink(yh, zh, y[ou + u], z[ou + u], y[od + d], z[od + d], dxu, dxd);
                        if (D <= cfg->kink_max && pair_better(D, (int32_t)u, (int32_t)d, bD, bu, bd)) {
                            bD = D; bu = (int32_t)u; bd = (int32_t)d;
                        }
                    }
                }
            } else {
                const int32_t* su = sidx + (ou - base);
                const int32_t* sd = sidx + (od - base);
                const float* yu_ = y + ou; const float* zu_ = z + ou;
                const float* yd_ = y + od; const float* zd_ = z + od;
                int64_t ku0 = lower_f32(yu_, su, nu, yh, cfg->win_y);
                int64_t kd0 = lower_f32(yd_, sd, nd, yh, cfg->win_y);
                for (int64_t ku = ku0; ku < nu && yu_[su[ku]] - yh <= cfg->win_y; ++ku) {
                    int32_t u = su[ku];
                    if (!in_window(yu_[u], zu_[u], yh, zh, cfg->win_y, cfg->win_z)) continue;
                    for (int64_t kd = kd0; kd < nd && yd_[sd[kd]] - yh <= cfg->win_y; ++kd) {
                        int32_t d = sd[kd];
                        if (!in_window(yd_[d], zd_[d], yh, zh, cfg->win_y, cfg->win_z)) continue;
                        float D = kink(yh, zh, yu_[u], zu_[u], yd_[d], zd_[d], dxu, dxd);
                        if (D <= cfg->kink_max && pair_better(D, u, d, bD, bu, bd)) {
                            bD = D; bu = u; bd = d;
                        }
                    }
                }
            }
            up[oh - base + h] = bu;
            dn[oh - base + h] = bd;
        }
    }
    free(sidx);
    return 0;
}

/* ---------------------------------------------------------------------------------- */
/* Kalman filter on the state p = (y, z, sin phi, tan lambda, q/pT) at a row plane x.  */
/* The field bends the track with curvature kappa = -C_B * Bz * q/pT; sin(phi) then    */
/* changes linearly in x, y follows the chord of the mean angle and z the arc length.  */
/* The covariance C is the 15-element lower triangle.                                  */
/* ---------------------------------------------------------------------------------- */
typedef struct { orc_real x; orc_real p[5]; orc_real C[15]; } kstate;

static int li(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

/* A(h) = asin(h)/h and its derivative A'(h); Taylor series near h = 0 */
static void arc_factor(orc_real h, orc_real* A, orc_real* Ap)
{
    if (R_FABS(h) < ARC_SERIES) {
        orc_real h2 = h * h;
        *A = 1 + h2 * ((orc_real)1 / 6 + h2 * ((orc_real)3 / 40 + h2 * ((orc_real)5 / 112)));
        *Ap = h * ((orc_real)1 / 3 + h2 * ((orc_real)3 / 10 + h2 * ((orc_real)15 / 56 + h2 * ((orc_real)35 / 144))));
    } else {
        orc_real as = R_ASIN(h);
        *A = as / h;
        *Ap = (h / R_SQRT(1 - h * h) - as) / (h * h);
    }
}

static int kprop(const orc_cfg* cfg, kstate* st, orc_real x1, orc_real* Jout)
{
    const orc_real a = -(orc_real)C_B * (orc_real)cfg->bz;
    const orc_real smax = (orc_real)cfg->sinphi_max;
    orc_real dx = x1 - st->x;
    orc_real s0 = st->p[2];
    orc_real tl = st->p[3];
    orc_real kap = a * st->p[4];
    orc_real s1 = s0 + kap * dx;
    if (!(R_FABS(s0) < smax) || !(R_FABS(s1) < smax)) return -1;
    orc_real c0 = R_SQRT(1 - s0 * s0);
    orc_real c1 = R_SQRT(1 - s1 * s1);
    orc_real tb = (s0 + s1) / (c0 + c1);          /* tan of the mean angle        */
    orc_real sec2 = 1 + tb * tb;
    orc_real sec = R_SQRT(sec2);
    orc_real chord = dx * sec;                    /* signed chord length          */
    orc_real h = kap * chord / 2;                 /* sin of half the turning angle */
    if (!(R_FABS(h) < 1)) return -1;
    orc_real A, Ap;
    arc_factor(h, &A, &Ap);
    orc_real ds = chord * A;                      /* signed transverse arc length */

    orc_real J[25];
    for (int i = 0; i < 25; ++i) J[i] = 0;
    for (int i = 0; i < 5; ++i) J[i * 5 + i] = 1;
    orc_real dy_ds0 = dx * sec2 * (1 / c0 + 1 / c1) / 2;
    orc_real dy_dkap = dx * dx * sec2 / (2 * c1);
    orc_real dds_ds0 = dx * (s0 + s1) / (c0 * c1 * (c0 + c1));
    orc_real dsec_dkap = sec * tb * dx / (2 * c1);
    orc_real dh_dkap = (dx * sec / 2) * (1 + kap * tb * dx / (2 * c1));
    orc_real dds_dkap = dx * dsec_dkap * A + chord * Ap * dh_dkap;
    J[0 * 5 + 2] = dy_ds0;
    J[0 * 5 + 4] = a * dy_dkap;
    J[1 * 5 + 2] = tl * dds_ds0;
    J[1 * 5 + 3] = ds;
    J[1 * 5 + 4] = tl * a * dds_dkap;
    J[2 * 5 + 4] = a * dx;

    st->p[0] = st->p[0] + dx * tb;
    st->p[1] = st->p[1] + tl * ds;
    st->p[2] = s1;
    st->x = x1;

    /* C <- J C J^T, plain matrix products */
    orc_real Cf[25], T[25];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) Cf[i * 5 + j] = st->C[li(i, j)];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
            orc_real s = 0;
            for (int k = 0; k < 5; ++k) s += J[i * 5 + k] * Cf[k * 5 + j];
            T[i * 5 + j] = s;
        }
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j) {
            orc_real s = 0;
            for (int k = 0; k < 5; ++k) s += T[i * 5 + k] * J[j * 5 + k];
            st->C[li(i, j)] = s;
        }
    if (Jout)
        for (int i = 0; i < 25; ++i) Jout[i] = J[i];
    return 0;
}

/* chi2 of measurement (my, mz) against the state, without updating */
static orc_real kchi2(const orc_cfg* cfg, const kstate* st, orc_real my, orc_real mz)
{
    orc_real r0 = my - st->p[0], r1 = mz - st->p[1];
    orc_real S00 = st->C[0] + (orc_real)(cfg->sigma_y * cfg->sigma_y);
    orc_real S01 = st->C[1];
    orc_real S11 = st->C[2] + (orc_real)(cfg->sigma_z * cfg->sigma_z);
    orc_real det = S00 * S11 - S01 * S01;
    return (r0 * r0 * S11 - 2 * r0 * r1 * S01 + r1 * r1 * S00) / det;
}

/* Kalman update with R = diag(sigma_y^2, sigma_z^2); returns the chi2 increment */
static orc_real kupdate(const orc_cfg* cfg, kstate* st, orc_real my, orc_real mz)
{
    orc_real r0 = my - st->p[0], r1 = mz - st->p[1];
    orc_real S00 = st->C[0] + (orc_real)(cfg->sigma_y * cfg->sigma_y);
    orc_real S01 = st->C[1];
    orc_real S11 = st->C[2] + (orc_real)(cfg->sigma_z * cfg->sigma_z);
    orc_real det = S00 * S11 - S01 * S01;
    orc_real i00 = S11 / det, i01 = -S01 / det, i11 = S00 / det;
    orc_real chi2 = r0 * r0 * i00 + 2 * r0 * r1 * i01 + r1 * r1 * i11;
    orc_real K0[5], K1[5], H0[5], H1[5];
    for (int i = 0; i < 5; ++i) {
        H0[i] = st->C[li(0, i)];   /* row 0 of C */
        H1[i] = st->C[li(1, i)];   /* row 1 of C */
    }
    for (int i = 0; i < 5; ++i) {
        K0[i] = H0[i] * i00 + H1[i] * i01;
        K1[i] = H0[i] * i01 + H1[i] * i11;
    }
    for (int i = 0; i < 5; ++i) st->p[i] += K0[i] * r0 + K1[i] * r1;
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j)
            st->C[li(i, j)] -= K0[i] * H0[j] + K1[i] * H1[j];
    return chi2;
}

static void kreset(const orc_cfg* cfg, kstate* st)
{
    for (int i = 0; i < 15; ++i) st->C[i] = 0;
    for (int i = 0; i < 5; ++i) st->C[li(i, i)] = (orc_real)cfg->c0[i];
}

/* Three-point seed: the circle through the (x, y) of the first, middle and last
 * cluster gives the curvature and the direction at the first cluster; tan(lambda) is the
 * z change over the arc length between first and last cluster. */
static int kseed(const orc_cfg* cfg, const orc_real* x, const orc_real* y, const orc_real* z,
                 orc_real* p)
{
    orc_real ax = x[1] - x[0], ay = y[1] - y[0];
    orc_real bx = x[2] - x[1], by = y[2] - y[1];
    orc_real cx = x[2] - x[0], cy = y[2] - y[0];
    orc_real la = R_SQRT(ax * ax + ay * ay);
    orc_real lb = R_SQRT(bx * bx + by * by);
    orc_real lc = R_SQRT(cx * cx + cy * cy);
    orc_real den = la * lb * lc;
    if (!(den > 0)) return -1;
    orc_real kap = 2 * (ax * by - ay * bx) / den;
    orc_real hh = kap * lc / 2;
    if (!(R_FABS(hh) < 1)) return -1;
    orc_real A, Ap;
    arc_factor(hh, &A, &Ap);
    orc_real ds = lc * A;
    orc_real a = -(orc_real)C_B * (orc_real)cfg->bz;
    p[0] = y[0];
    p[1] = z[0];
    p[2] = (cy / lc) * R_SQRT(1 - hh * hh) - (cx / lc) * hh;
    p[3] = (z[2] - z[0]) / ds;
    p[4] = (a != 0) ? kap / a : 0;
    return 0;
}

int orc_propagate(const orc_cfg* cfg, double x0, double x1, double* p, double* C, double* J)
{
    kstate st;
    st.x = (orc_real)x0;
    for (int i = 0; i < 5; ++i) st.p[i] = (orc_real)p[i];
    for (int i = 0; i < 15; ++i) st.C[i] = (orc_real)C[i];
    orc_real Jr[25];
    if (kprop(cfg, &st, (orc_real)x1, Jr) != 0) return -1;
    for (int i = 0; i < 5; ++i) p[i] = st.p[i];
    for (int i = 0; i < 15; ++i) C[i] = st.C[i];
    if (J)
        for (int i = 0; i < 25; ++i) J[i] = Jr[i];
    return 0;
}

double orc_beamline_z(const orc_cfg* cfg, double x0, const double* p)
{
    const double y0 = p[0], z0 = p[1], s0 = p[2], tl = p[3];
    const double c0 = sqrt((1.0 - s0) * (1.0 + s0));   /* tracks move outward: cos phi > 0 */
    const double kap = -C_B * cfg->bz * p[4];
    double s;                                          /* signed arc length to the DCA */
    if (kap == 0.0) {
        /* straight line: the point where the position is orthogonal to the direction */
        s = -(x0 * c0 + y0 * s0);
    } else {
        /* circle centre; the closest point of the circle to the axis lies on the line
         * from the centre towards the axis, where the direction angle phi_d has
         * (sin, cos) = sign(kappa) * (-xc, yc) / |centre| */
        const double xc = x0 - s0 / kap, yc = y0 + c0 / kap;
        const double d = sqrt(xc * xc + yc * yc);
        if (!(d > 0.0)) return z0;
        const double sg = kap > 0.0 ? 1.0 : -1.0;
        const double sd = -sg * xc / d, cd = sg * yc / d;
        const double dphi = atan2(sd * c0 - cd * s0, cd * c0 + sd * s0);
        s = dphi / kap;
    }
    return z0 + tl * s;
}

int orc_seed(const orc_cfg* cfg, const double* x, const double* y, const double* z, double* p)
{
    orc_real xr[3], yr[3], zr[3], pr[5];
    for (int i = 0; i < 3; ++i) { xr[i] = (orc_real)x[i]; yr[i] = (orc_real)y[i]; zr[i] = (orc_real)z[i]; }
    if (kseed(cfg, xr, yr, zr, pr) != 0) return -1;
    for (int i = 0; i < 5; ++i) p[i] = pr[i];
    return 0;
}

double orc_update(const orc_cfg* cfg, double my, double mz, double* p, double* C)
{
    kstate st;
    st.x = 0;
    for (int i = 0; i < 5; ++i) st.p[i] = (orc_real)p[i];
    for (int i = 0; i < 15; ++i) st.C[i] = (orc_real)C[i];
    orc_real chi2 = kupdate(cfg, &st, (orc_real)my, (orc_real)mz);
    for (int i = 0; i < 5; ++i) p[i] = st.p[i];
    for (int i = 0; i < 15; ++i) C[i] = st.C[i];
    return chi2;
}

/* ---------------------------------------------------------------------------------- */
/* Sector frames.  Sector s lies on side s / S (S = n_sectors / 2 sectors per side) at   */
/* centre azimuth alpha = ((s mod S) + 1/2) * 2 pi / S; its frame has x along the centre */
/* direction and y towards larger azimuth.  A state moves into the frame of a sector     */
/* whose azimuth is larger by delta: the point (x, y) and the direction phi are rotated,  */
/* and the state is then given at the plane x' through the rotated point.                */
/* ---------------------------------------------------------------------------------- */
static int side_sectors(const orc_cfg* cfg) { return cfg->n_sectors / 2; }

/* azimuth step from the frame of sector s0 to that of s1 (same side), in (-pi, pi] */
static double frame_delta(const orc_cfg* cfg, int s0, int s1)
{
    const int S = side_sectors(cfg);
    int d = (s1 % S) - (s0 % S);
    if (2 * d > S) d -= S;
    if (2 * d <= -S) d += S;
    return d * (2.0 * ORC_PI / S);
}

/* Rotation of the state by delta.  With c = cos delta, s = sin delta:
 *   x' = x c + y s,  y' = -x s + y c,  sin phi' = sin phi c - cos phi s,
 *   cos phi' = cos phi c + sin phi s (must stay > 0: the track moves outward),
 *   z, tan lambda and q/pT are unchanged.
 * Covariance: a change dy of y moves the point by (s dy, c dy) in the new frame; the
 * state at the fixed plane x' follows the helix back by s dy, which gives
 *   dy'/dy = c - s tan phi',  dz'/dy = -s tan(lambda) / cos phi',
 *   d sin phi'/dy = -kappa s,  d sin phi'/d sin phi = cos phi' / cos phi. */
static int krotate(const orc_cfg* cfg, kstate* st, double delta, orc_real* Jout)
{
    if (delta == 0.0) {
        if (Jout) { for (int i = 0; i < 25; ++i) Jout[i] = 0; for (int i = 0; i < 5; ++i) Jout[i * 5 + i] = 1; }
        return 0;
    }
    const orc_real c = (orc_real)cos(delta), sn = (orc_real)sin(delta);
    const orc_real a = -(orc_real)C_B * (orc_real)cfg->bz;
    orc_real s0 = st->p[2];
    if (!(R_FABS(s0) < 1)) return -1;
    orc_real c0 = R_SQRT(1 - s0 * s0);
    orc_real s1 = s0 * c - c0 * sn;
    orc_real c1 = c0 * c + s0 * sn;
    if (!(c1 > 0) || !(R_FABS(s1) < (orc_real)cfg->sinphi_max)) return -1;
    orc_real x1 = st->x * c + st->p[0] * sn;
    orc_real y1 = -st->x * sn + st->p[0] * c;
    orc_real J[25];
    for (int i = 0; i < 25; ++i) J[i] = 0;
    for (int i = 0; i < 5; ++i) J[i * 5 + i] = 1;
    J[0 * 5 + 0] = c - sn * s1 / c1;
    J[1 * 5 + 0] = -sn * st->p[3] / c1;
    J[2 * 5 + 0] = -a * st->p[4] * sn;
    J[2 * 5 + 2] = c1 / c0;
    st->x = x1;
    st->p[0] = y1;
    st->p[2] = s1;
    orc_real Cf[25], T[25];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) Cf[i * 5 + j] = st->C[li(i, j)];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
            orc_real v = 0;
            for (int k = 0; k < 5; ++k) v += J[i * 5 + k] * Cf[k * 5 + j];
            T[i * 5 + j] = v;
        }
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j) {
            orc_real v = 0;
            for (int k = 0; k < 5; ++k) v += T[i * 5 + k] * J[j * 5 + k];
            st->C[li(i, j)] = v;
        }
    if (Jout)
        for (int i = 0; i < 25; ++i) Jout[i] = J[i];
    return 0;
}

/* Step 7: final fit of n ordered clusters.  Seed from first/middle/last, C = C0, update
 * at the first cluster and outward over the rest; then C = C0 keeping p, update at the
 * last cluster and inward to the first.  Result at the innermost cluster.
 * sec (NULL: one sector) gives each cluster's sector, for tracks merged across sectors:
 * the seed points are rotated into the first cluster's frame, and the state is rotated
 * into a cluster's frame before it is propagated to that cluster's row. */
/* Counts one step of kind k (see orc_debug.work); no effect on any result. */
static void count(int64_t* work, int k)
{
    if (work) ++work[k];
}

static int kfit(const orc_cfg* cfg, int32_t n, const orc_real* x, const orc_real* y,
                const orc_real* z, const int32_t* sec, kstate* st, orc_real* chi2,
                orc_real* p_outer, orc_real* C_outer, int64_t* work)
{
    if (n < 3) return -1;
    const int32_t ids[3] = {0, (n - 1) / 2, n - 1};
    orc_real sx[3], sy[3], sz[3];
    for (int k = 0; k < 3; ++k) {
        int32_t i = ids[k];
        sx[k] = x[i]; sy[k] = y[i]; sz[k] = z[i];
        if (sec && sec[i] != sec[0]) {
            /* point of sector sec[i] in the frame of sec[0] (rotation by -delta) */
            double d = frame_delta(cfg, sec[0], sec[i]);
            orc_real c = (orc_real)cos(d), sn = (orc_real)sin(d);
            sx[k] = x[i] * c - y[i] * sn;
            sy[k] = x[i] * sn + y[i] * c;
        }
    }
    if (kseed(cfg, sx, sy, sz, st->p) != 0) return -1;
    st->x = x[0];
    int32_t frame = sec ? sec[0] : 0;
    kreset(cfg, st);
    count(work, 4);
    kupdate(cfg, st, y[0], z[0]);
    for (int32_t i = 1; i < n; ++i) {
        if (sec && sec[i] != frame) {
            if (krotate(cfg, st, frame_delta(cfg, frame, sec[i]), NULL) != 0) return -1;
            frame = sec[i];
        }
        count(work, 3);
        if (kprop(cfg, st, x[i], NULL) != 0) return -1;
        count(work, 4);
        kupdate(cfg, st, y[i], z[i]);
    }
    if (p_outer)
        for (int i = 0; i < 5; ++i) p_outer[i] = st->p[i];
    if (C_outer)
        for (int i = 0; i < 15; ++i) C_outer[i] = st->C[i];
    kreset(cfg, st);
    count(work, 4);
    count(work, 5);
    orc_real c2 = kupdate(cfg, st, y[n - 1], z[n - 1]);
    for (int32_t i = n - 2; i >= 0; --i) {
        if (sec && sec[i] != frame) {
            if (krotate(cfg, st, frame_delta(cfg, frame, sec[i]), NULL) != 0) return -1;
            frame = sec[i];
        }
        count(work, 3);
        if (kprop(cfg, st, x[i], NULL) != 0) return -1;
        count(work, 4);
        count(work, 5);
        c2 += kupdate(cfg, st, y[i], z[i]);
    }
    *chi2 = c2;
    for (int i = 0; i < 5; ++i)
        if (!isfinite((double)st->p[i])) return -1;
    for (int i = 0; i < 15; ++i)
        if (!isfinite((double)st->C[i])) return -1;
    return 0;
}

int orc_fit_hits(const orc_cfg* cfg, int32_t n, const double* x, const double* y,
                 const double* z, double* p, double* C, double* chi2, double* p_outer)
{
    orc_real* xr = (orc_real*)malloc(sizeof(orc_real) * (size_t)(n > 0 ? n : 1) * 3);
    orc_real* yr = xr + n;
    orc_real* zr = yr + n;
    for (int32_t i = 0; i < n; ++i) { xr[i] = (orc_real)x[i]; yr[i] = (orc_real)y[i]; zr[i] = (orc_real)z[i]; }
    kstate st;
    orc_real c2 = 0, po[5];
    int rc = kfit(cfg, n, xr, yr, zr, NULL, &st, &c2, po, NULL, NULL);
    free(xr);
    if (rc != 0) return -1;
    for (int i = 0; i < 5; ++i) p[i] = st.p[i];
    for (int i = 0; i < 15; ++i) C[i] = st.C[i];
    *chi2 = c2;
    if (p_outer)
        for (int i = 0; i < 5; ++i) p_outer[i] = po[i];
    return 0;
}

/* ---------------------------------------------------------------------------------- */
/* Step 5: tracklet construction from a chain, with the follow rule: at each row the    */
/* state is propagated (a failure ends the pass), the cluster of minimal chi2 inside    */
/* |dy| <= min(win_y, nsig*sqrt(S_yy)), |dz| <= min(win_z, nsig*sqrt(S_zz)) is taken if */
/* chi2 <= chi2_max (equal chi2: smaller in-row index), and the pass ends after more   */
/* than max_miss consecutive rows without a cluster.                                   */
/* ---------------------------------------------------------------------------------- */
typedef struct {
    const orc_cfg* cfg;
    const float* y; const float* z;
    const int64_t* row_off;          /* [n_rows+1] of this sector (absolute)          */
    const int32_t* sidx;             /* per-row y-sorted in-row indices (sector-relative) */
    int64_t base;
    int64_t* work;                   /* step counters (orc_debug.work) or NULL        */
} sector_view;


static int32_t search_row(const sector_view* sv, int r, const kstate* st, orc_real* chi2_out)
{
    const orc_cfg* cfg = sv->cfg;
    const int64_t o = sv->row_off[r], n = sv->row_off[r + 1] - o;
    const int32_t* s = sv->sidx + (o - sv->base);
    orc_real Syy = st->C[0] + (orc_real)(cfg->sigma_y * cfg->sigma_y);
    orc_real Szz = st->C[2] + (orc_real)(cfg->sigma_z * cfg->sigma_z);
    orc_real wy = (orc_real)cfg->nsig * R_SQRT(Syy);
    orc_real wz = (orc_real)cfg->nsig * R_SQRT(Szz);
    if (wy > (orc_real)cfg->win_y) wy = (orc_real)cfg->win_y;
    if (wz > (orc_real)cfg->win_z) wz = (orc_real)cfg->win_z;
    const orc_real yp = st->p[0], zp = st->p[1];
    /* first y-sorted position with y - yp >= -wy */
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if ((orc_real)sv->y[o + s[mid]] - yp >= -wy) hi = mid; else lo = mid + 1;
    }
    int32_t best = -1;
    orc_real bchi = 0;
    for (int64_t k = lo; k < n; ++k) {
        int32_t c = s[k];
        orc_real yc = (orc_real)sv->y[o + c], zc = (orc_real)sv->z[o + c];
        if (yc - yp > wy) break;
        if (R_FABS(zc - zp) > wz) continue;
        count(sv->work, 2);
        orc_real c2 = kchi2(cfg, st, yc, zc);
        if (best < 0 || c2 < bchi || (c2 == bchi && c < best)) { best = c; bchi = c2; }
    }
    *chi2_out = bchi;
    return best;
}

static int follow(const sector_view* sv, kstate* st, int r_from, int r_to, int step, int32_t* hits)
{
    const orc_cfg* cfg = sv->cfg;
    int misses = 0;
    for (int r = r_from; r != r_to; r += step) {
        count(sv->work, 0);
        if (kprop(cfg, st, (orc_real)cfg->row_x[r], NULL) != 0) break;
        orc_real c2;
        int32_t c = search_row(sv, r, st, &c2);
        if (c >= 0 && c2 <= (orc_real)cfg->chi2_max) {
            count(sv->work, 1);
            kupdate(cfg, st, (orc_real)sv->y[sv->row_off[r] + c], (orc_real)sv->z[sv->row_off[r] + c]);
            hits[r] = c;
            misses = 0;
        } else if (++misses > cfg->max_miss) {
            break;
        }
    }
    return 0;
}

/* Returns the number of clusters of the tracklet grown from start hit (r0, i0), 0 if
 * there is none.  hits[n_rows] receives the in-row index per row. */
static int32_t build_tracklet(const sector_view* sv, const int32_t* cup, int r0, int32_t i0,
                              int32_t* hits)
{
    const orc_cfg* cfg = sv->cfg;
    const int nr = cfg->n_rows;
    for (int r = 0; r < nr; ++r) hits[r] = -1;
    /* chain along the cleaned up-links */
    int L = 0;
    int32_t c = i0;
    for (int r = r0; r < nr && c >= 0; ++r) {
        hits[r] = c;
        ++L;
        c = cup[sv->row_off[r] - sv->base + c];
    }
    if (L < cfg->min_chain) {
        for (int r = 0; r < nr; ++r) hits[r] = -1;
        return 0;
    }
    orc_real xs[3], ys[3], zs[3];
    int ri[3] = {r0, r0 + (L - 1) / 2, r0 + L - 1};
    for (int k = 0; k < 3; ++k) {
        int64_t g = sv->row_off[ri[k]] + hits[ri[k]];
        xs[k] = (orc_real)cfg->row_x[ri[k]];
        ys[k] = (orc_real)sv->y[g];
        zs[k] = (orc_real)sv->z[g];
    }
    kstate st;
    if (kseed(cfg, xs, ys, zs, st.p) != 0) goto fail;
    st.x = xs[0];
    kreset(cfg, &st);
    for (int r = r0; r < r0 + L; ++r) {
        int64_t g = sv->row_off[r] + hits[r];
        if (r > r0) {
            count(sv->work, 0);
            if (kprop(cfg, &st, (orc_real)cfg->row_x[r], NULL) != 0) goto fail;
        }
        count(sv->work, 1);
        kupdate(cfg, &st, (orc_real)sv->y[g], (orc_real)sv->z[g]);
    }
    /* follow outward */
    follow(sv, &st, r0 + L, nr, +1, hits);
    /* refit inward over all clusters so far, from C0 keeping p */
    kreset(cfg, &st);
    int bottom = r0;
    for (int r = nr - 1; r >= r0; --r) {
        if (hits[r] < 0) continue;
        int64_t g = sv->row_off[r] + hits[r];
        count(sv->work, 0);
        if (kprop(cfg, &st, (orc_real)cfg->row_x[r], NULL) != 0) goto fail;
        count(sv->work, 1);
        kupdate(cfg, &st, (orc_real)sv->y[g], (orc_real)sv->z[g]);
    }
    /* follow inward */
    follow(sv, &st, bottom - 1, -1, -1, hits);
    {
        int32_t n = 0;
        for (int r = 0; r < nr; ++r) n += hits[r] >= 0;
        return n;
    }
fail:
    for (int r = 0; r < nr; ++r) hits[r] = -1;
    return 0;
}

/* splitmix64, only to shuffle the visiting order in the selection self-check */
static uint64_t mix64(uint64_t* s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ---------------------------------------------------------------------------------- */
/* Step 6: selection.  A tracklet's weight is w = (n << 32) | (2^32 - 1 - rank): more     */
/* clusters win, and at equal size the smaller start rank.  Every cluster takes the      */
/* largest weight of the tracklets holding it; a tracklet keeps the clusters whose weight */
/* is its own.  One pass: clusters a losing tracklet gives up are not handed on.        */
/* Tracklets with fewer than min_track_hits clusters can neither be accepted nor outweigh */
/* a longer one, so they do not take part (weight 0, nothing kept).                      */
/* ---------------------------------------------------------------------------------- */
void orc_select(const orc_cfg* cfg, int64_t n_clusters, int64_t n_tl, const int32_t* tl_n,
                const int64_t* rank, const int32_t* hits, uint64_t shuffle_seed, uint64_t* W,
                uint64_t* wt, int32_t* kept)
{
    const int nr = cfg->n_rows;
    for (int64_t h = 0; h < n_clusters; ++h) W[h] = 0;
    for (int64_t t = 0; t < n_tl; ++t) {
        wt[t] = tl_n[t] < cfg->min_track_hits
                    ? 0
                    : ((uint64_t)tl_n[t] << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)rank[t]);
        kept[t] = 0;
    }
    /* visiting order: identity, or a shuffle that must not change the result */
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_tl > 0 ? n_tl : 1));
    for (int64_t t = 0; t < n_tl; ++t) order[t] = t;
    if (shuffle_seed) {
        uint64_t st = shuffle_seed;
        for (int64_t t = n_tl - 1; t > 0; --t) {
            int64_t j = (int64_t)(mix64(&st) % (uint64_t)(t + 1));
            int64_t tmp = order[t]; order[t] = order[j]; order[j] = tmp;
        }
    }
    for (int64_t q = 0; q < n_tl; ++q) {
        const int64_t t = order[q];
        if (wt[t] == 0) continue;
        for (int r = 0; r < nr; ++r) {
            const int32_t h = hits[t * nr + r];
            if (h >= 0 && wt[t] > W[h]) W[h] = wt[t];
        }
    }
    for (int64_t t = 0; t < n_tl; ++t) {
        if (wt[t] == 0) continue;
        for (int r = 0; r < nr; ++r) {
            const int32_t h = hits[t * nr + r];
            if (h >= 0 && W[h] == wt[t]) kept[t] += 1;
        }
    }
    free(order);
}

/* ---------------------------------------------------------------------------------- */
/* Driver: every sector independently, in frame order.                                */
/* ---------------------------------------------------------------------------------- */
int orc_track_frame(const orc_cfg* cfg, int64_t n, const float* y, const float* z,
                    const int64_t* row_off, orc_tracks* out, orc_debug* dbg,
                    uint64_t shuffle_seed)
{
    const int nr = cfg->n_rows, ns = cfg->n_sectors;
    if (nr < 3 || ns < 1 || row_off[0] != 0 || row_off[(int64_t)ns * nr] != n) return -1;
    for (int64_t g = 0; g < (int64_t)ns * nr; ++g)
        if (row_off[g + 1] < row_off[g]) return -1;
    int rc = 0;
    int64_t n_tracks = 0, n_hits = 0, n_tl = 0, bin_used = 0;
    if (dbg)
        for (int k = 0; k < 6; ++k) dbg->work[k] = 0;
    if (out->cluster_track)
        for (int64_t i = 0; i < n; ++i) out->cluster_track[i] = -1;
    if (out->hit_off && out->cap_tracks >= 0) out->hit_off[0] = 0;

    for (int s = 0; s < ns; ++s) {
        const int64_t* ro = row_off + (int64_t)s * nr;
        const int64_t base = ro[0], nsec = ro[nr] - base;
        const size_t nn = (size_t)(nsec > 0 ? nsec : 1);
        /* grid (only needed for the bit-exact comparison of the GPU grid tables) */
        if (dbg && dbg->perm && dbg->bin_start) {
            for (int r = 0; r < nr; ++r) {
                int64_t g = (int64_t)s * nr + r;
                float ylo, zlo, by, bz;
                int32_t ny, nz;
                int64_t cap = dbg->bin_start_cap - bin_used;
                if (orc_grid_row(cfg, ro[r + 1] - ro[r], y + ro[r], z + ro[r], &ylo, &zlo, &by, &bz,
                                 &ny, &nz, dbg->bin_start + bin_used, cap, dbg->perm + ro[r]) != 0)
                    return -3;
                if (dbg->g_ylo) { dbg->g_ylo[g] = ylo; dbg->g_zlo[g] = zlo; dbg->g_by[g] = by; dbg->g_bz[g] = bz;
                                  dbg->g_ny[g] = ny; dbg->g_nz[g] = nz; dbg->g_bin_base[g] = bin_used; }
                bin_used += (int64_t)ny * nz + 1;
            }
        }
        int32_t* up = (int32_t*)malloc(sizeof(int32_t) * nn);
        int32_t* dn = (int32_t*)malloc(sizeof(int32_t) * nn);
        int32_t* cup = (int32_t*)malloc(sizeof(int32_t) * nn);
        int32_t* cdn = (int32_t*)malloc(sizeof(int32_t) * nn);
        int32_t* sidx = (int32_t*)malloc(sizeof(int32_t) * nn);
        orc_links_sector(cfg, y, z, ro, 0, up, dn);
        /* Step 3: cleaning.  A link survives only if the linked cluster links back. */
        for (int r = 0; r < nr; ++r)
            for (int64_t i = ro[r]; i < ro[r + 1]; ++i) {
                int64_t h = i - base;
                int32_t u = up[h], d = dn[h];
                int32_t hi = (int32_t)(i - ro[r]);
                cup[h] = (u >= 0 && dn[ro[r + 1] - base + u] == hi) ? u : -1;
                cdn[h] = (d >= 0 && up[ro[r - 1] - base + d] == hi) ? d : -1;
            }
        if (dbg) {
            if (dbg->up) memcpy(dbg->up + base, up, sizeof(int32_t) * (size_t)nsec);
            if (dbg->dn) memcpy(dbg->dn + base, dn, sizeof(int32_t) * (size_t)nsec);
            if (dbg->cup) memcpy(dbg->cup + base, cup, sizeof(int32_t) * (size_t)nsec);
            if (dbg->cdn) memcpy(dbg->cdn + base, cdn, sizeof(int32_t) * (size_t)nsec);
        }
        for (int r = 0; r < nr; ++r)
            sort_row_by_y(y + ro[r], ro[r + 1] - ro[r], sidx + (ro[r] - base));
        sector_view sv = {cfg, y, z, ro, sidx, base, dbg ? dbg->work : NULL};

        /* Step 4/5: start hits in (row, in-row index) order, one tracklet each */
        int64_t n_start = 0;
        for (int64_t h = 0; h < nsec; ++h) n_start += (cup[h] >= 0 && cdn[h] < 0);
        int32_t* tl_hits = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_start > 0 ? n_start : 1) * (size_t)nr);
        int32_t* tl_n = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_start > 0 ? n_start : 1));
        int64_t k = 0;
        for (int r = 0; r < nr; ++r)
            for (int64_t i = ro[r]; i < ro[r + 1]; ++i) {
                int64_t h = i - base;
                int st = cup[h] >= 0 && cdn[h] < 0;
                if (dbg && dbg->start) dbg->start[i] = (uint8_t)st;
                if (!st) continue;
                tl_n[k] = build_tracklet(&sv, cup, r, (int32_t)(i - ro[r]), tl_hits + k * nr);
                if (dbg && dbg->tl_nhits) {
                    int64_t t = n_tl + k;
                    if (t < dbg->cap_tracklets) {
                        dbg->tl_start[t] = i;
                        dbg->tl_nhits[t] = tl_n[k];
                        if (dbg->tl_hits) memcpy(dbg->tl_hits + t * nr, tl_hits + k * nr, sizeof(int32_t) * (size_t)nr);
                    } else {
                        rc = -3;
                    }
                }
                ++k;
            }

        /* Step 6: selection (orc_select) over this sector's tracklets, ranked from n_tl */
        uint64_t* W = (uint64_t*)calloc(nn, sizeof(uint64_t));
        const size_t ns1 = (size_t)(n_start > 0 ? n_start : 1);
        int64_t* rank = (int64_t*)malloc(sizeof(int64_t) * ns1);
        uint64_t* wt = (uint64_t*)malloc(sizeof(uint64_t) * ns1);
        int32_t* kept = (int32_t*)malloc(sizeof(int32_t) * ns1);
        int32_t* sel_hits = (int32_t*)malloc(sizeof(int32_t) * ns1 * (size_t)nr);
        for (int64_t t = 0; t < n_start; ++t) {
            rank[t] = n_tl + t;
            for (int r = 0; r < nr; ++r) {
                int32_t c = tl_hits[t * nr + r];
                sel_hits[t * nr + r] = c < 0 ? -1 : (int32_t)(ro[r] - base + c);
            }
        }
        orc_select(cfg, nsec, n_start, tl_n, rank, sel_hits, shuffle_seed, W, wt, kept);
        free(sel_hits);
        if (dbg && dbg->W) memcpy(dbg->W + base, W, sizeof(uint64_t) * (size_t)nsec);

        /* Step 7: final fit of the accepted tracklets' kept clusters, in rank order */
        orc_real* fx = (orc_real*)malloc(sizeof(orc_real) * (size_t)nr * 3);
        orc_real* fy = fx + nr;
        orc_real* fz = fy + nr;
        int64_t* fid = (int64_t*)malloc(sizeof(int64_t) * (size_t)nr);
        for (int64_t t = 0; t < n_start; ++t) {
            if (kept[t] < cfg->min_track_hits) continue;
            const uint64_t w = wt[t];
            int32_t m = 0;
            for (int r = 0; r < nr; ++r) {
                int32_t c = tl_hits[t * nr + r];
                if (c < 0) continue;
                int64_t g = ro[r] + c;
                if (W[g - base] != w) continue;
                fx[m] = (orc_real)cfg->row_x[r];
                fy[m] = (orc_real)y[g];
                fz[m] = (orc_real)z[g];
                fid[m] = g;
                ++m;
            }
            if (m < cfg->min_track_hits) continue;
            kstate st;
            orc_real c2;
            orc_real po[5], Co[15];
            if (kfit(cfg, m, fx, fy, fz, NULL, &st, &c2, po, Co, dbg ? dbg->work : NULL) != 0) continue;
            if (n_tracks < out->cap_tracks && n_hits + m <= out->cap_hits) {
                for (int i = 0; i < 5; ++i) out->params[n_tracks * 5 + i] = st.p[i];
                for (int i = 0; i < 15; ++i) out->cov[n_tracks * 15 + i] = st.C[i];
                out->x_ref[n_tracks] = fx[0];
                if (out->z_beam) {
                    double pd[5];
                    for (int i = 0; i < 5; ++i) pd[i] = (double)st.p[i];
                    out->z_beam[n_tracks] = orc_beamline_z(cfg, (double)fx[0], pd);
                }
                if (out->params_outer)
                    for (int i = 0; i < 5; ++i) out->params_outer[n_tracks * 5 + i] = po[i];
                if (out->cov_outer)
                    for (int i = 0; i < 15; ++i) out->cov_outer[n_tracks * 15 + i] = Co[i];
                out->chi2[n_tracks] = c2;
                out->ndf[n_tracks] = 2 * m - 5;
                out->nhits[n_tracks] = m;
                out->sector[n_tracks] = s;
                for (int32_t i = 0; i < m; ++i) {
                    out->hit_ids[n_hits + i] = fid[i];
                    out->cluster_track[fid[i]] = (int32_t)n_tracks;
                }
                out->hit_off[n_tracks + 1] = n_hits + m;
            } else {
                rc = -3;
            }
            n_tracks += 1;
            n_hits += m;
        }
        n_tl += n_start;
        free(fx); free(fid); free(W); free(rank); free(wt); free(kept); free(tl_hits); free(tl_n);
        free(up); free(dn); free(cup); free(cdn); free(sidx);
    }
    out->n_tracks = n_tracks;
    out->n_hits = n_hits;
    if (dbg) dbg->n_tracklets = n_tl;
    return rc;
}

int orc_rotate(const orc_cfg* cfg, double delta, double* x, double* p, double* C, double* J)
{
    kstate st;
    st.x = (orc_real)*x;
    for (int i = 0; i < 5; ++i) st.p[i] = (orc_real)p[i];
    for (int i = 0; i < 15; ++i) st.C[i] = (orc_real)C[i];
    orc_real Jr[25];
    if (krotate(cfg, &st, delta, Jr) != 0) return -1;
    *x = st.x;
    for (int i = 0; i < 5; ++i) p[i] = st.p[i];
    for (int i = 0; i < 15; ++i) C[i] = st.C[i];
    if (J)
        for (int i = 0; i < 25; ++i) J[i] = Jr[i];
    return 0;
}

int orc_fit_hits_sectors(const orc_cfg* cfg, int32_t n, const double* x, const double* y,
                         const double* z, const int32_t* sec, double* p, double* C, double* chi2)
{
    orc_real* xr = (orc_real*)malloc(sizeof(orc_real) * (size_t)(n > 0 ? n : 1) * 3);
    orc_real* yr = xr + n;
    orc_real* zr = yr + n;
    for (int32_t i = 0; i < n; ++i) { xr[i] = (orc_real)x[i]; yr[i] = (orc_real)y[i]; zr[i] = (orc_real)z[i]; }
    kstate st;
    orc_real c2 = 0;
    int rc = kfit(cfg, n, xr, yr, zr, sec, &st, &c2, NULL, NULL, NULL);
    free(xr);
    if (rc != 0) return -1;
    for (int i = 0; i < 5; ++i) p[i] = st.p[i];
    for (int i = 0; i < 15; ++i) C[i] = st.C[i];
    *chi2 = c2;
    return 0;
}

/* ---------------------------------------------------------------------------------- */
/* Merging across sector boundaries (the track-fit stage after sector tracking, Sec. 7,  */
/* Table 1 "Track Fit").  The paper gives no procedure; this is the definition used:     */
/*                                                                                        */
/* A track leaving its sector through an azimuthal edge continues in the neighbouring    */
/* sector of the same side.  A link A -> B is a candidate when                             */
/*   - A's outermost cluster lies within merge_edge of an edge (|y| >= x tan(pi/S) -      */
/*     merge_edge), at a larger radius than A's innermost cluster;                         */
/*   - B lies in the sector beyond that edge (the one at larger azimuth if that y >= 0,   */
/*     else the one at smaller azimuth), and B's innermost cluster lies within merge_edge */
/*     of the shared edge (y < 0, resp. y >= 0, in B's frame) at a larger radius than A's  */
/*     outermost cluster (radii from the cluster coordinates);                             */
/*   - A's outer state (the outward pass's state at its outermost cluster), rotated into  */
/*     B's frame, predicts B's inner state linearly within merge_window in y and in z:    */
/*     |y' + dx tan phi' - y_B| and |z' + dx tan(lambda) / cos phi' - z_B| <= merge_window */
/*     with dx = x_B - x';                                                                */
/*   - the rotated state propagates to B's innermost row, and the chi2 of the difference  */
/*     of the two 5-parameter states with the sum of their covariances is at most          */
/*     merge_chi2.                                                                        */
/* Every A takes its candidate of least chi2 (ties: smaller B); every B keeps, of the A   */
/* that took it, the one of least chi2 (ties: smaller A); that pair is linked.  Radii     */
/* grow strictly along links, so links form simple chains.  A chain of several tracks    */
/* becomes one track with the clusters of its segments in chain order, refitted across    */
/* the sectors (kfit with sector frames); if that fit fails the chain is dissolved into  */
/* its segments.  Merged tracks are emitted in the order of their first input track; a  */
/* single segment keeps its sector fit.                                                   */
/* ---------------------------------------------------------------------------------- */

/* d^T S^-1 d for a symmetric 5x5 S (lower triangle) by Cholesky; -1 if S is not
 * positive definite */
static int chi2_5(const orc_real* S15, const orc_real* d, orc_real* out)
{
    orc_real L[5][5];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j) {
            orc_real v = S15[li(i, j)];
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(v > 0)) return -1;
                L[i][i] = R_SQRT(v);
            } else {
                L[i][j] = v / L[j][j];
            }
        }
    orc_real u[5], c2 = 0;
    for (int i = 0; i < 5; ++i) {
        orc_real v = d[i];
        for (int k = 0; k < i; ++k) v -= L[i][k] * u[k];
        u[i] = v / L[i][i];
        c2 += u[i] * u[i];
    }
    *out = c2;
    return 0;
}

int orc_merge_frame(const orc_cfg* cfg, int64_t n, const float* y, const float* z,
                    const int64_t* row_off, const orc_tracks* trk, orc_merged* out)
{
    const int nr = cfg->n_rows, ns = cfg->n_sectors;
    const int S = ns / 2;
    const int64_t T = trk->n_tracks;
    if (ns < 2 || ns % 2 || !trk->params_outer || !trk->cov_outer || T < 0) return -1;
    if (row_off[0] != 0 || row_off[(int64_t)ns * nr] != n) return -1;
    const size_t nT = (size_t)(T > 0 ? T : 1);

    int32_t* row = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t g = 0; g < (int64_t)ns * nr; ++g)
        for (int64_t i = row_off[g]; i < row_off[g + 1]; ++i) row[i] = (int32_t)(g % nr);

    /* cluster coordinates of each track's innermost and outermost cluster */
    double* xi = (double*)malloc(sizeof(double) * nT * 4);
    double* yi = xi + nT;
    double* xo = yi + nT;
    double* yo = xo + nT;
    for (int64_t t = 0; t < T; ++t) {
        int64_t hi = trk->hit_ids[trk->hit_off[t]], ho = trk->hit_ids[trk->hit_off[t + 1] - 1];
        xi[t] = (double)cfg->row_x[row[hi]]; yi[t] = (double)y[hi];
        xo[t] = (double)cfg->row_x[row[ho]]; yo[t] = (double)y[ho];
    }
    const double te = tan(ORC_PI / S), m = cfg->merge_edge, W = cfg->merge_window;
    /* the tracks of each sector, in index order */
    int64_t* sec_start = (int64_t*)calloc((size_t)ns + 1, sizeof(int64_t));
    int64_t* sec_list = (int64_t*)malloc(sizeof(int64_t) * nT);
    for (int64_t t = 0; t < T; ++t) {
        if (trk->sector[t] < 0 || trk->sector[t] >= ns) { free(row); free(xi); free(sec_start); free(sec_list); return -1; }
        sec_start[trk->sector[t] + 1] += 1;
    }
    for (int s = 0; s < ns; ++s) sec_start[s + 1] += sec_start[s];
    {
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)ns);
        for (int s = 0; s < ns; ++s) fill[s] = sec_start[s];
        for (int64_t t = 0; t < T; ++t) sec_list[fill[trk->sector[t]]++] = t;
        free(fill);
    }

    /* candidates: each A's best B */
    int64_t* bestB = (int64_t*)malloc(sizeof(int64_t) * nT);
    orc_real* bestC = (orc_real*)malloc(sizeof(orc_real) * nT);
    for (int64_t a = 0; a < T; ++a) {
        bestB[a] = -1;
        bestC[a] = 0;
        const double ro2 = xo[a] * xo[a] + yo[a] * yo[a];
        if (!(fabs(yo[a]) >= xo[a] * te - m)) continue;
        if (!(ro2 > xi[a] * xi[a] + yi[a] * yi[a])) continue;
        const int sa = trk->sector[a], up = yo[a] >= 0;
        const int sb = (sa / S) * S + ((sa % S) + (up ? 1 : S - 1)) % S;
        kstate A0;
        A0.x = (orc_real)xo[a];
        for (int i = 0; i < 5; ++i) A0.p[i] = (orc_real)trk->params_outer[a * 5 + i];
        for (int i = 0; i < 15; ++i) A0.C[i] = (orc_real)trk->cov_outer[a * 15 + i];
        if (krotate(cfg, &A0, frame_delta(cfg, sa, sb), NULL) != 0) continue;
        const orc_real c1 = R_SQRT(1 - A0.p[2] * A0.p[2]);
        for (int64_t j = sec_start[sb]; j < sec_start[sb + 1]; ++j) {
            const int64_t b = sec_list[j];
            if (up ? !(yi[b] < 0) : !(yi[b] >= 0)) continue;
            if (!(fabs(yi[b]) >= xi[b] * te - m)) continue;
            if (!(xi[b] * xi[b] + yi[b] * yi[b] > ro2)) continue;
            const double* pb = trk->params + b * 5;
            const orc_real dx = (orc_real)xi[b] - A0.x;
            /* linear prediction at B's row: y' + dx tan phi', z' + dx tan(lambda) / cos phi' */
            const orc_real ylin = A0.p[0] + dx * A0.p[2] / c1;
            const orc_real zlin = A0.p[1] + dx * A0.p[3] / c1;
            if (!(R_FABS(ylin - (orc_real)pb[0]) <= (orc_real)W && R_FABS(zlin - (orc_real)pb[1]) <= (orc_real)W))
                continue;
            kstate A1 = A0;
            if (kprop(cfg, &A1, (orc_real)xi[b], NULL) != 0) continue;
            orc_real d[5], Ssum[15], c2;
            for (int i = 0; i < 5; ++i) d[i] = A1.p[i] - (orc_real)pb[i];
            for (int i = 0; i < 15; ++i) Ssum[i] = A1.C[i] + (orc_real)trk->cov[b * 15 + i];
            if (chi2_5(Ssum, d, &c2) != 0) continue;
            if (!(c2 <= (orc_real)cfg->merge_chi2)) continue;
            if (bestB[a] < 0 || c2 < bestC[a]) { bestB[a] = b; bestC[a] = c2; }
        }
    }
    /* each B keeps the best A that took it; links */
    int64_t* keepA = (int64_t*)malloc(sizeof(int64_t) * nT);
    int64_t* next = (int64_t*)malloc(sizeof(int64_t) * nT);
    int64_t* prev = (int64_t*)malloc(sizeof(int64_t) * nT);
    for (int64_t t = 0; t < T; ++t) { keepA[t] = -1; next[t] = -1; prev[t] = -1; }
    for (int64_t a = 0; a < T; ++a) {
        int64_t b = bestB[a];
        if (b < 0) continue;
        if (keepA[b] < 0 || bestC[a] < bestC[keepA[b]]) keepA[b] = a;
    }
    for (int64_t b = 0; b < T; ++b)
        if (keepA[b] >= 0) { next[keepA[b]] = b; prev[b] = keepA[b]; }
    if (out->next)
        for (int64_t t = 0; t < T; ++t) out->next[t] = (int32_t)next[t];
    if (out->link_chi2)
        for (int64_t t = 0; t < T; ++t) out->link_chi2[t] = next[t] >= 0 ? (double)bestC[t] : 0.0;

    /* chains: refit those of several segments; a failed fit dissolves the chain */
    int8_t* dissolved = (int8_t*)calloc(nT, 1);
    int8_t* fitted = (int8_t*)calloc(nT, 1);
    kstate* fit = (kstate*)malloc(sizeof(kstate) * nT);
    orc_real* fit_c2 = (orc_real*)malloc(sizeof(orc_real) * nT);
    int32_t* chain_hits = (int32_t*)calloc(nT, sizeof(int32_t));
    int32_t* chain_seg = (int32_t*)calloc(nT, sizeof(int32_t));
    int64_t max_h = 0;
    for (int64_t t = 0; t < T; ++t) {
        if (prev[t] >= 0) continue;
        int32_t nh = 0, nseg = 0;
        for (int64_t u = t; u >= 0; u = next[u]) { nh += (int32_t)(trk->hit_off[u + 1] - trk->hit_off[u]); ++nseg; }
        chain_hits[t] = nh;
        chain_seg[t] = nseg;
        if (nh > max_h) max_h = nh;
    }
    orc_real* fx = (orc_real*)malloc(sizeof(orc_real) * (size_t)(max_h > 0 ? max_h : 1) * 3);
    orc_real* fy = fx + (max_h > 0 ? max_h : 1);
    orc_real* fz = fy + (max_h > 0 ? max_h : 1);
    int32_t* fs = (int32_t*)malloc(sizeof(int32_t) * (size_t)(max_h > 0 ? max_h : 1));
    for (int64_t t = 0; t < T; ++t) {
        if (prev[t] >= 0 || chain_seg[t] < 2) continue;
        int32_t k = 0;
        for (int64_t u = t; u >= 0; u = next[u])
            for (int64_t j = trk->hit_off[u]; j < trk->hit_off[u + 1]; ++j) {
                int64_t h = trk->hit_ids[j];
                fx[k] = (orc_real)cfg->row_x[row[h]];
                fy[k] = (orc_real)y[h];
                fz[k] = (orc_real)z[h];
                fs[k] = trk->sector[u];
                ++k;
            }
        if (kfit(cfg, k, fx, fy, fz, fs, &fit[t], &fit_c2[t], NULL, NULL, NULL) == 0) {
            fitted[t] = 1;
        } else {
            for (int64_t u = t; u >= 0; u = next[u]) dissolved[u] = 1;
        }
    }

    /* emit in the order of the first input track */
    int rc = 0;
    int64_t M = 0, H = 0;
    if (out->hit_off && out->cap_merged >= 0) out->hit_off[0] = 0;
    for (int64_t t = 0; t < T; ++t) {
        const int whole = prev[t] < 0 && fitted[t];
        const int single = !whole && (prev[t] < 0 || dissolved[t]);
        if (!whole && !single) continue;
        const int32_t nh = whole ? chain_hits[t] : (int32_t)(trk->hit_off[t + 1] - trk->hit_off[t]);
        if (M < out->cap_merged && H + nh <= out->cap_hits) {
            double pd[5];
            if (whole) {
                for (int i = 0; i < 5; ++i) pd[i] = out->params[M * 5 + i] = fit[t].p[i];
                for (int i = 0; i < 15; ++i) out->cov[M * 15 + i] = fit[t].C[i];
                out->chi2[M] = fit_c2[t];
                out->n_segments[M] = chain_seg[t];
            } else {
                for (int i = 0; i < 5; ++i) pd[i] = out->params[M * 5 + i] = trk->params[t * 5 + i];
                for (int i = 0; i < 15; ++i) out->cov[M * 15 + i] = trk->cov[t * 15 + i];
                out->chi2[M] = trk->chi2[t];
                out->n_segments[M] = 1;
            }
            out->x_ref[M] = trk->x_ref[t];
            if (out->z_beam) out->z_beam[M] = orc_beamline_z(cfg, trk->x_ref[t], pd);
            out->ndf[M] = 2 * nh - 5;
            out->nhits[M] = nh;
            out->sector[M] = trk->sector[t];
            int64_t k = H;
            for (int64_t u = t; u >= 0; u = whole ? next[u] : -1) {
                out->track_merged[u] = (int32_t)M;
                for (int64_t j = trk->hit_off[u]; j < trk->hit_off[u + 1]; ++j) out->hit_ids[k++] = trk->hit_ids[j];
            }
            out->hit_off[M + 1] = H + nh;
        } else {
            rc = -3;
        }
        ++M;
        H += nh;
    }
    out->n_merged = M;
    out->n_hits = H;
    free(row); free(xi); free(sec_start); free(sec_list); free(bestB); free(bestC); free(keepA); free(next); free(prev);
    free(dissolved); free(fitted); free(fit); free(fit_c2); free(chain_hits); free(chain_seg);
    free(fx); free(fs);
    return rc;
}

/* ---------------------------------------------------------------------------------- */
/* Step 9: hit removal for data compression, strategy B (Sec. 4): the clusters that are  */
/* not in the vicinity of a good track are removed.  See orc.h for the definition.       */
/* ---------------------------------------------------------------------------------- */
int64_t orc_reject_frame(const orc_cfg* cfg, int64_t n, const float* y, const float* z,
                         const int64_t* row_off, const orc_tracks* trk, int brute, uint8_t* keep)
{
    const int nr = cfg->n_rows, ns = cfg->n_sectors;
    if (row_off[0] != 0 || row_off[(int64_t)ns * nr] != n) return -1;
    const double w = cfg->reject_window, pmin = cfg->reject_pt_min;
    int32_t* row = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t g = 0; g < (int64_t)ns * nr; ++g)
        for (int64_t i = row_off[g]; i < row_off[g + 1]; ++i) row[i] = (int32_t)(g % nr);
    /* each row's clusters ordered by y (ties: in-row index) for the window scan */
    int32_t* sidx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!brute)
        for (int64_t g = 0; g < (int64_t)ns * nr; ++g)
            sort_row_by_y(y + row_off[g], row_off[g + 1] - row_off[g], sidx + row_off[g]);
    for (int64_t i = 0; i < n; ++i) keep[i] = 0;
    for (int64_t t = 0; t < trk->n_tracks; ++t) {
        const double* p = trk->params + t * 5;
        if (!(fabs(p[4]) * pmin <= 1.0)) continue;
        const int s = trk->sector[t];
        const int64_t hb = trk->hit_off[t], he = trk->hit_off[t + 1];
        if (s < 0 || s >= ns || he <= hb) { free(row); free(sidx); return -1; }
        for (int64_t j = hb; j < he; ++j) keep[trk->hit_ids[j]] = 1;
        const int r0 = row[trk->hit_ids[hb]], r1 = row[trk->hit_ids[he - 1]];
        for (int r = r0; r <= r1; ++r) {
            kstate st;
            st.x = (orc_real)trk->x_ref[t];
            for (int i = 0; i < 5; ++i) st.p[i] = (orc_real)p[i];
            for (int i = 0; i < 15; ++i) st.C[i] = 0;
            if (kprop(cfg, &st, (orc_real)cfg->row_x[r], NULL) != 0) continue;
            const double yp = (double)st.p[0], zp = (double)st.p[1];
            const int64_t g = (int64_t)s * nr + r, b = row_off[g], m = row_off[g + 1] - b;
            if (brute) {
                for (int64_t i = b; i < b + m; ++i)
                    if (fabs((double)y[i] - yp) <= w && fabs((double)z[i] - zp) <= w) keep[i] = 1;
            } else {
                /* first cluster with y >= yp - w (generous by 1e-6 cm; the test decides) */
                int64_t lo = 0, hi = m;
                while (lo < hi) {
                    int64_t mid = (lo + hi) / 2;
                    if ((double)y[b + sidx[b + mid]] < yp - w - 1e-6) lo = mid + 1; else hi = mid;
                }
                for (int64_t k = lo; k < m; ++k) {
                    const int64_t i = b + sidx[b + k];
                    if ((double)y[i] > yp + w + 1e-6) break;
                    if (fabs((double)y[i] - yp) <= w && fabs((double)z[i] - zp) <= w) keep[i] = 1;
                }
            }
        }
    }
    int64_t kept = 0;
    for (int64_t i = 0; i < n; ++i) kept += keep[i];
    free(row);
    free(sidx);
    return kept;
}

/* ---------------------------------------------------------------------------------- */
/* Step 10: track-model compression (Sec. 4): residuals of the attached clusters to the  */
/* track's helix, quantised.  See orc.h for the definition.                               */
/* ---------------------------------------------------------------------------------- */
int orc_compress_frame(const orc_cfg* cfg, int64_t n, const float* y, const float* z,
                       const int64_t* row_off, const orc_tracks* trk, int32_t* codes, double* resid,
                       double* pred)
{
    const int nr = cfg->n_rows, ns = cfg->n_sectors;
    if (row_off[0] != 0 || row_off[(int64_t)ns * nr] != n || !(cfg->resid_step > 0)) return -1;
    const double step = cfg->resid_step, lim = 1073741824.0;   /* 2^30 */
    for (int64_t t = 0; t < trk->n_tracks; ++t) {
        const int s = trk->sector[t];
        if (s < 0 || s >= ns) return -1;
        for (int64_t j = trk->hit_off[t]; j < trk->hit_off[t + 1]; ++j) {
            const int64_t h = trk->hit_ids[j];
            if (h < row_off[(int64_t)s * nr] || h >= row_off[(int64_t)(s + 1) * nr]) return -1;
            int r = 0;
            while (row_off[(int64_t)s * nr + r + 1] <= h) ++r;
            kstate st;
            st.x = (orc_real)trk->x_ref[t];
            for (int i = 0; i < 5; ++i) st.p[i] = (orc_real)trk->params[t * 5 + i];
            for (int i = 0; i < 15; ++i) st.C[i] = 0;
            double yp = (double)st.p[0], zp = (double)st.p[1];
            if (kprop(cfg, &st, (orc_real)cfg->row_x[r], NULL) == 0) {
                yp = (double)st.p[0];
                zp = (double)st.p[1];
            }
            const double ry = ((double)y[h] - yp) / step, rz = ((double)z[h] - zp) / step;
            double qy = floor(ry + 0.5), qz = floor(rz + 0.5);
            if (qy > lim) qy = lim;
            if (qy < -lim) qy = -lim;
            if (qz > lim) qz = lim;
            if (qz < -lim) qz = -lim;
            codes[2 * j] = (int32_t)qy;
            codes[2 * j + 1] = (int32_t)qz;
            if (resid) { resid[2 * j] = ry; resid[2 * j + 1] = rz; }
            if (pred) { pred[2 * j] = yp; pred[2 * j + 1] = zp; }
        }
    }
    return 0;
}
