/*
 * Reference oracle for TPC sector track finding (test infrastructure only).
 *
 * A plain, sequential CPU implementation of the sector tracking method that the paper
 * (arXiv:2009.07515, Sec. 6 "Track reconstruction with continuous data") runs standalone
 * on the GPU: per-row search grids, neighbour links between adjacent pad rows, a cellular
 * automaton that turns reciprocal links into chains, and a 5-parameter Kalman filter that
 * fits and follows helix candidates in the solenoid field.  The paper only names the
 * method (derived from the Run 2 HLT tracker); every internal rule implemented here is a
 * reading of that description and is stated where it is implemented.
 *
 * Only the test suite, the smoke check and the CPU baseline of the benchmark use this
 * code.  It shares no source with the GPU library.
 *
 * Precision: the grid and the neighbour links are defined in IEEE binary32 (round to
 * nearest even, no contraction, correctly rounded division) in every build.  The Kalman
 * part runs in `orc_real`, which is double in liborc_f64.so and float in liborc_f32.so.
 * The API always exchanges doubles.
 */
#ifndef TPC_ORACLE_H
#define TPC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_sectors;        /* sectors per frame (36)                          */
    int32_t n_rows;           /* pad rows per sector (152)                       */
    const float* row_x;       /* [n_rows] row plane positions (cm)               */
    double bz;                /* solenoid field along z (T)                      */
    /* neighbour links (binary32 by definition) */
    float win_y, win_z;       /* rectangular window half-widths (cm)             */
    float kink_max;           /* largest accepted slope change D                 */
    /* Kalman filter and follow */
    double sigma_y, sigma_z;  /* cluster errors (cm)                             */
    double chi2_max;          /* largest accepted 2D chi2 of a followed cluster  */
    double sinphi_max;        /* propagation stops at |sin(phi)| >= this         */
    double nsig;              /* follow window in units of the predicted error   */
    double c0[5];             /* initial covariance diagonal                     */
    int32_t min_chain;        /* shortest chain that becomes a tracklet          */
    int32_t min_track_hits;   /* fewest kept clusters of an accepted track       */
    int32_t max_miss;         /* follow stops after more consecutive misses      */
    /* grid (tuning: changes the grid tables only, never links or tracks) */
    float bin_y, bin_z;
    int32_t cap_mul, cap_add; /* a row of n clusters has at most cap_mul*n+cap_add bins */
    /* merging across sector boundaries (orc_merge_frame) */
    double merge_edge;        /* a track end within this distance of a sector edge (cm) */
    double merge_window;      /* linear-prediction gate on y and z (cm)              */
    double merge_chi2;        /* largest accepted 5-parameter chi2 of a match        */
    /* hit removal, strategy B (orc_reject_frame) */
    double reject_pt_min;     /* good tracks have pT >= this (GeV/c)                 */
    double reject_window;     /* half-width in y and z of a good track's vicinity (cm) */
    /* track-model compression (orc_compress_frame) */
    double resid_step;        /* quantisation step of the residuals (cm)             */
} orc_cfg;

typedef struct {
    int64_t cap_tracks, cap_hits;
    int64_t n_tracks, n_hits;  /* written: the sizes the frame needs             */
    double* params;            /* [cap_tracks][5] (y, z, sin phi, tan lambda, q/pT) */
    double* cov;               /* [cap_tracks][15] lower triangle, row-major     */
    double* x_ref;             /* [cap_tracks] x of the innermost cluster        */
    double* chi2;              /* [cap_tracks]                                   */
    int32_t* ndf;              /* [cap_tracks] 2*nhits - 5                       */
    int32_t* nhits;            /* [cap_tracks]                                   */
    int32_t* sector;           /* [cap_tracks]                                   */
    int64_t* hit_off;          /* [cap_tracks+1]                                 */
    int64_t* hit_ids;          /* [cap_hits] frame cluster index, inner to outer */
    int32_t* cluster_track;    /* [N] track index or -1                          */
    double* z_beam;            /* [cap_tracks] z at the beam line, or NULL        */
    double* params_outer;      /* [cap_tracks][5] outward-pass state at the outermost
                                  cluster's row, or NULL                           */
    double* cov_outer;         /* [cap_tracks][15] its covariance, or NULL        */
} orc_tracks;

typedef struct {               /* optional intermediate results; NULL = skip     */
    /* grid, per frame row g = sector * n_rows + row */
    float* g_ylo; float* g_zlo; float* g_by; float* g_bz;
    int32_t* g_ny; int32_t* g_nz;
    int64_t* g_bin_base;       /* offset of row g's table inside bin_start       */
    uint32_t* bin_start;       /* concatenated, ny*nz+1 entries per row          */
    int64_t bin_start_cap;
    uint32_t* perm;            /* [N] in-row index of the k-th sorted cluster    */
    int32_t* up; int32_t* dn;  /* [N] raw links (in-row index, -1 none)          */
    int32_t* cup; int32_t* cdn;/* [N] cleaned links                              */
    uint8_t* start;            /* [N] start-hit flags                            */
    /* tracklets, one per start hit in frame cluster order */
    int64_t cap_tracklets;
    int64_t n_tracklets;       /* written                                        */
    int64_t* tl_start;         /* [cap] frame index of the start hit             */
    int32_t* tl_nhits;         /* [cap] 0 = no tracklet                          */
    int32_t* tl_hits;          /* [cap][n_rows] in-row index per row, -1 none    */
    uint64_t* W;               /* [N] selection weight per cluster               */
    /* step counts (written): tracklet propagations (attempts), tracklet updates,
     * clusters inside the follow windows, final-fit propagations, final-fit updates,
     * final-fit chi2 evaluations.  Counting changes no result. */
    int64_t work[6];
} orc_debug;

/* Track one frame.  y, z: [n] binary32 local coordinates grouped by (sector, row);
 * row_off: [n_sectors*n_rows+1].  shuffle_seed != 0 visits tracklets in a pseudo-random
 * order during selection (the result must not change).  Returns 0, or -1 on invalid
 * input, -3 if an output or debug capacity is too small (sizes are still written). */
int orc_track_frame(const orc_cfg* cfg, int64_t n, const float* y, const float* z,
                    const int64_t* row_off, orc_tracks* out, orc_debug* dbg,
                    uint64_t shuffle_seed);

/* Selection among the tracklets of one sector.  hits[t*n_rows + r] is the cluster of
 * tracklet t at row r as an index into the sector's n_clusters clusters (-1: none);
 * tl_n[t] its cluster count, rank[t] the frame rank of its start.  Tracklets with
 * tl_n >= min_track_hits take part with the weight w = (n << 32) | (2^32 - 1 - rank)
 * (wt[t], 0 for the others); W[h] receives the largest weight of the tracklets holding
 * cluster h (0: none), kept[t] the clusters of t whose W equals its own weight.  A
 * tracklet is accepted when kept >= min_track_hits.  shuffle_seed != 0 visits the
 * tracklets in a pseudo-random order (the result must not change). */
void orc_select(const orc_cfg* cfg, int64_t n_clusters, int64_t n_tl, const int32_t* tl_n,
                const int64_t* rank, const int32_t* hits, uint64_t shuffle_seed, uint64_t* W,
                uint64_t* wt, int32_t* kept);

/* Grid of one row (binary32).  bin_start has room for cap entries.  Returns 0 or -3. */
int orc_grid_row(const orc_cfg* cfg, int64_t n, const float* y, const float* z,
                 float* ylo, float* zlo, float* by, float* bz, int32_t* ny, int32_t* nz,
                 uint32_t* bin_start, int64_t cap, uint32_t* perm);

/* Raw neighbour links of one sector.  row_off: [n_rows+1] absolute offsets into y, z;
 * up/dn are indexed from row_off[0].  brute != 0 uses the all-pairs definition, else a
 * y-sorted window scan (same result). */
int orc_links_sector(const orc_cfg* cfg, const float* y, const float* z,
                     const int64_t* row_off, int brute, int32_t* up, int32_t* dn);

/* Helix propagation of (p, C) from x0 to x1; J receives the 5x5 Jacobian (row-major)
 * if not NULL.  Returns 0, or -1 if |sin phi| would reach sinphi_max. */
int orc_propagate(const orc_cfg* cfg, double x0, double x1, double* p, double* C, double* J);

/* Three-point seed from clusters (x_i, y_i, z_i), i = 0, 1, 2, ordered by x. */
int orc_seed(const orc_cfg* cfg, const double* x, const double* y, const double* z, double* p);

/* Kalman update with measurement (my, mz); returns the chi2 increment. */
double orc_update(const orc_cfg* cfg, double my, double mz, double* p, double* C);

/* Final fit of an ordered cluster list (inner to outer): seed, outward pass from C0,
 * inward pass from C0 keeping the parameters.  p, C at x[0]; p_outer receives the
 * outward-pass state at x[n-1] if not NULL.  Returns 0 or -1 (propagation failure). */
int orc_fit_hits(const orc_cfg* cfg, int32_t n, const double* x, const double* y,
                 const double* z, double* p, double* C, double* chi2, double* p_outer);

/* z at the beam line (Sec. 6, "Track
 * reconstruction with continuous data"): the helix of the state p at plane x0 of a sector
 * frame is followed to its point of closest approach to the beam axis in the transverse
 * plane (the axis is the origin of every sector frame), and z there is returned.  Under
 * the assumption that the track is a primary from a vertex at the origin, this is the
 * most likely z of the track's origin, i.e. its drift offset in the frame's z.  The arc
 * between the two points is the shorter one (|phi change| <= pi). */
double orc_beamline_z(const orc_cfg* cfg, double x0, const double* p);

/* Rotation of the state (x, p, C) into the frame of a sector whose azimuth is larger by
 * delta; J receives the 5x5 Jacobian if not NULL.  Returns -1 if the rotated track
 * would not move outward or |sin phi'| >= sinphi_max. */
int orc_rotate(const orc_cfg* cfg, double delta, double* x, double* p, double* C, double* J);

/* Final fit across sectors: as orc_fit_hits, with sec[i] the sector of cluster i (its
 * x, y in that sector's frame); the result is in the frame of sec[0]. */
int orc_fit_hits_sectors(const orc_cfg* cfg, int32_t n, const double* x, const double* y,
                         const double* z, const int32_t* sec, double* p, double* C, double* chi2);

/* Tracks merged across sector boundaries.  Every input track belongs to exactly one
 * merged track; merged tracks come in the order of their first input track. */
typedef struct {
    int64_t cap_merged, cap_hits;
    int64_t n_merged, n_hits;  /* written                                         */
    double* params;            /* [cap_merged][5] at the innermost cluster, in the
                                  frame of its sector                              */
    double* cov;               /* [cap_merged][15]                                 */
    double* x_ref;             /* [cap_merged]                                     */
    double* chi2;              /* [cap_merged]                                     */
    double* z_beam;            /* [cap_merged] or NULL                             */
    int32_t* ndf;              /* [cap_merged] 2*nhits - 5                         */
    int32_t* nhits;            /* [cap_merged]                                     */
    int32_t* sector;           /* [cap_merged] sector of the innermost cluster     */
    int32_t* n_segments;       /* [cap_merged] input tracks joined                 */
    int64_t* hit_off;          /* [cap_merged+1]                                   */
    int64_t* hit_ids;          /* [cap_hits] frame cluster index, segment by segment */
    int32_t* track_merged;     /* [n_tracks] merged track of each input track       */
    int32_t* next;             /* [n_tracks] accepted link to the next segment or -1;
                                  NULL to skip                                     */
    double* link_chi2;         /* [n_tracks] chi2 of that link; NULL to skip       */
} orc_merged;

/* Merge one frame's sector tracks (orc_track_frame output with params_outer and
 * cov_outer) across the azimuthal sector boundaries of each side, and refit each merged
 * track over all its clusters.  Returns 0, -1 on invalid input, -3 if an output is too
 * small (sizes are still written). */
int orc_merge_frame(const orc_cfg* cfg, int64_t n, const float* y, const float* z,
                    const int64_t* row_off, const orc_tracks* trk, orc_merged* out);

/* Hit removal for data compression, strategy B (Sec. 4): keep only the clusters in the
 * vicinity of good tracks.  A good track has pT >= reject_pt_min (|q/pT| * pT_min <= 1).
 * Its own clusters are kept, and at every row from its innermost to its outermost
 * cluster's row its state at x_ref, propagated in one helix step to the row plane,
 * keeps the clusters of its sector's row with |y - y_p| <= reject_window and
 * |z - z_p| <= reject_window (a row where the step fails keeps none by this rule).
 * keep: [n] 1 = kept.  brute != 0 compares every cluster of the row, else a y-sorted
 * window scan (same result).  Returns the number of kept clusters, or -1 on invalid
 * input. */
int64_t orc_reject_frame(const orc_cfg* cfg, int64_t n, const float* y, const float* z,
                         const int64_t* row_off, const orc_tracks* trk, int brute, uint8_t* keep);

/* Track-model compression (Sec. 4, entropy reduction): every cluster attached to a track
 * is stored as its residual to the track's position on the cluster's row plane, the
 * position being the track's state at x_ref (which the compressed stream keeps with the
 * track) propagated in one helix step to the row (or the state at x_ref itself where that
 * step fails).  Codes: q = floor(r / resid_step + 1/2) for r = y - y_p and r = z - z_p,
 * clamped to [-2^30, 2^30].  codes: [n_hits][2] in hit-list order; resid (or NULL):
 * [n_hits][2] the unrounded r / resid_step.  Decoding: y = y_p + q_y * resid_step.
 * pred (or NULL): [n_hits][2] the positions y_p, z_p.  Returns 0 or -1. */
int orc_compress_frame(const orc_cfg* cfg, int64_t n, const float* y, const float* z,
                       const int64_t* row_off, const orc_tracks* trk, int32_t* codes, double* resid,
                       double* pred);

#ifdef __cplusplus
}
#endif
#endif
