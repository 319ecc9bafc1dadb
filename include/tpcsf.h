/*
 * tpcsf — TPC sector track finding on AMD Instinct MI355X (gfx950).
 *
 * The operation is the standalone TPC track finding of arXiv:2009.07515, Sec. 6: in each
 * of the 36 sectors, clusters on the 152 pad rows are sorted into per-row search grids,
 * linked to their best neighbours in the adjacent rows, chained by a cellular automaton,
 * and fitted and followed as helices with a 5-parameter Kalman filter in the solenoid
 * field.  A whole continuous-readout time frame (or a batch of them) is processed at once
 * (Sec. 7.1).  The paper names the method (derived from the Run 2 HLT tracker) but prints
 * none of its rules; the rules this library implements are stated at the parameter
 * structures below and in the kernels.
 *
 * Conventions shared by every call:
 *   - Device pointers (marked [device]) must point to memory of the device that was
 *     current when the context was created; host pointers are marked [host].
 *   - Clusters are structure-of-arrays float32 in local sector coordinates (cm), grouped by
 *     (time frame, sector, pad row): the clusters of global row
 *     g = (tf * n_sectors + sector) * n_rows + row are [row_offsets[g], row_offsets[g+1]).
 *     z is the drift coordinate, which in continuous readout carries the unknown
 *     collision-time offset (Sec. 2); no z range is assumed.
 *   - A track state is p = (y, z, sin(phi), tan(lambda), q/pT [c/GeV]) at the row plane
 *     x = x_ref; the curvature is kappa = -0.00299792458 * bz * q/pT [1/cm].  Covariances
 *     are the 15-element lower triangle, row-major: C00, C10, C11, C20, C21, C22, ...
 *   - Calls are stream-ordered and asynchronous.  The returned status covers argument
 *     validation and launch errors; errors found on the device (non-finite or out-of-range
 *     coordinates, output capacity) are reported by tpcsf_sync().
 *   - The caller owns every input and output buffer; the library owns only its scratch
 *     arena (limited by the HBM budget given at creation).
 *   - No function falls back to the CPU.
 */
#ifndef TPCSF_H
#define TPCSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TPCSF_OK = 0,
    TPCSF_E_INVALID = -1,   /* bad argument or malformed input                          */
    TPCSF_E_NOMEM = -2,     /* scratch would exceed the HBM budget, or hipMalloc failed  */
    TPCSF_E_CAPACITY = -3,  /* an output buffer is too small; required sizes are written */
    TPCSF_E_HIP = -4,       /* HIP runtime error                                         */
    TPCSF_E_BUSY = -5,      /* server: no free slot or budget right now                  */
    TPCSF_E_TIMEOUT = -6    /* server: wait timed out                                    */
} tpcsf_status;

typedef struct tpcsf_ctx tpcsf_ctx;

/* Detector geometry (inputs).  Sector s < n_sectors/2 is the A side.  Row r is the plane
 * x = row_x[r] of the sector frame; rows must be strictly increasing in x. */
typedef struct {
    int32_t n_sectors;        /* sectors per time frame (36)                      */
    int32_t n_rows;           /* pad rows per sector (152); 3 <= n_rows <= 255     */
    const float* row_x;       /* [host] [n_rows] row plane positions (cm)           */
    double bz;                /* solenoid field along z (T)                         */
} tpcsf_geometry;

/* Method constants: they define the result.
 *   Neighbour links (binary32): a cluster c of row r+-1 is a candidate for cluster h of row
 *   r when |y_c - y_h| <= win_y and |z_c - z_h| <= win_z; the pair (u in r+1, d in r-1)
 *   with the least slope change D = (ty_u - ty_d)^2 + (tz_u - tz_d)^2 wins if
 *   D <= kink_max (ties: smaller in-row index of u, then of d).  Links that are not
 *   reciprocal are dropped; chains of >= min_chain clusters seed tracklets.
 *   Kalman filter (binary64): cluster errors sigma_y/z, initial covariance diagonal c0,
 *   propagation fails at |sin(phi)| >= sinphi_max; the follow step takes the least-chi2
 *   cluster inside min(win, nsig * predicted error) if chi2 <= chi2_max and stops after
 *   more than max_miss consecutive empty rows.  Tracks keep >= min_track_hits clusters. */
typedef struct {
    float win_y, win_z, kink_max;
    double sigma_y, sigma_z, chi2_max, sinphi_max, nsig;
    double c0[5];
    int32_t min_chain, min_track_hits, max_miss;
    double merge_edge, merge_window, merge_chi2;   /* tpcsf_merge, see there */
    double reject_pt_min, reject_window;           /* tpcsf_reject, see there */
    double resid_step;                             /* tpcsf_compress, see there */
} tpcsf_params;

/* Tuning: changes speed and the grid tables, never links or tracks.
 *   bin_y, bin_z: grid bin size (cm); a row of n clusters gets at most cap_mul*n+cap_add
 *   bins (the z bin, then the y bin, doubles until it fits).
 *   block: threads per block of the row kernels (64..1024, multiple of 64).
 *   tl_block: threads per block of the tracklet kernel (64..256, multiple of 64).
 *   chunk: work-queue chunk of the persistent tracklet kernel: a wave takes 64 * chunk
 *   tracklets per queue atomic and sweeps them 64 at a time (1..64). */
typedef struct {
    float bin_y, bin_z;
    int32_t cap_mul, cap_add;
    int32_t block, tl_block, chunk;
} tpcsf_tuning;

/* One batch of n_tf time frames in device memory. */
typedef struct {
    int32_t n_tf;                       /* time frames in the batch (>= 1)                */
    int64_t n_clusters;                 /* total clusters (< 2^31)                       */
    const float* y;                     /* [device] [n_clusters]                          */
    const float* z;                     /* [device] [n_clusters]                          */
    const int64_t* row_offsets;         /* [device] [n_tf*n_sectors*n_rows+1], [0] = 0    */
    const int64_t* row_offsets_host;    /* [host] same values, used for validation and
                                           planning; no row may hold 65535 clusters or more */
} tpcsf_frame;

/* Output buffers (caller-allocated device memory).  Tracks are ordered by (time frame,
 * sector, rank of the chain's bottom cluster in frame order); each track's clusters are
 * listed from the innermost row outward.  If the batch needs more than cap_tracks tracks
 * or cap_hits clusters, only what fits is written, *n_tracks / *n_hits hold the required
 * sizes and tpcsf_sync() returns TPCSF_E_CAPACITY. */
typedef struct {
    int64_t cap_tracks, cap_hits;
    int64_t* n_tracks;                  /* [device] scalar                                 */
    int64_t* n_hits;                    /* [device] scalar                                 */
    double* params;                     /* [device] [cap_tracks][5] at x_ref               */
    double* cov;                        /* [device] [cap_tracks][15]                       */
    double* x_ref;                      /* [device] [cap_tracks] innermost cluster's row x */
    double* chi2;                       /* [device] [cap_tracks]                           */
    int32_t* ndf;                       /* [device] [cap_tracks] 2*nhits - 5               */
    int32_t* nhits;                     /* [device] [cap_tracks]                           */
    int32_t* sector;                    /* [device] [cap_tracks]                           */
    int32_t* tf;                        /* [device] [cap_tracks] time frame in the batch   */
    int64_t* hit_off;                   /* [device] [cap_tracks+1]                         */
    int32_t* hit_ids;                   /* [device] [cap_hits] batch cluster index         */
    int32_t* cluster_track;             /* [device] [n_clusters] track index or -1         */
    double* z_beam;                     /* [device] [cap_tracks] z at the beam line, or
                                           NULL: the track's helix followed inward to its
                                           closest approach to the beam axis; under the
                                           assumption of a primary from a vertex at the
                                           origin, the most likely z of its origin (the
                                           continuous-readout z estimate of Sec. 6)        */
    double* params_outer;               /* [device] [cap_tracks][5] or NULL: the final
                                           fit's outward-pass state at the outermost
                                           cluster's row (input of tpcsf_merge)            */
    double* cov_outer;                  /* [device] [cap_tracks][15] or NULL: its
                                           covariance                                      */
    float* hit_rec;                     /* [device] [cap_hits][4] or NULL: per hit, in
                                           hit_ids order, the cluster's y, z, its row
                                           plane x and its batch index (int32 bits); read
                                           by tpcsf_merge and tpcsf_compress when given    */
} tpcsf_tracks;

/* Defaults of the method constants and of the tuning. */
void tpcsf_default_params(tpcsf_params* p);
void tpcsf_default_tuning(tpcsf_tuning* t);

/* Create a context on the current device.  hbm_budget_bytes bounds the scratch arena
 * (0 = no bound).  The geometry's row_x is copied. */
tpcsf_status tpcsf_create(const tpcsf_geometry* geo, const tpcsf_params* params,
                          const tpcsf_tuning* tuning, size_t hbm_budget_bytes, tpcsf_ctx** out);
tpcsf_status tpcsf_destroy(tpcsf_ctx* ctx);

/* Change the tuning of an existing context (result-invariant). */
tpcsf_status tpcsf_set_tuning(tpcsf_ctx* ctx, const tpcsf_tuning* tuning);

/* Scratch bytes a batch of n_clusters clusters in n_tf time frames needs. */
size_t tpcsf_arena_bytes(const tpcsf_ctx* ctx, int64_t n_clusters, int32_t n_tf);

/* Fix the scratch layout to a capacity of max_clusters clusters in max_tf time frames and
 * allocate it now (TPCSF_E_NOMEM beyond the budget).  Smaller batches then reuse the same
 * layout, so one captured graph serves every batch up to that capacity with the same
 * buffers.  max_clusters = 0 releases the reservation (the arena is kept). */
tpcsf_status tpcsf_reserve(tpcsf_ctx* ctx, int64_t max_clusters, int32_t max_tf);

/* Plain form: every stage launched separately for every (time frame, sector). */
tpcsf_status tpcsf_track_plain(tpcsf_ctx* ctx, const tpcsf_frame* frame, tpcsf_tracks* out,
                               void* stream);

/* Batched form: each stage is one launch over all (time frame, sector) of the batch, the
 * variable-length tracklet work runs from a persistent work queue, and the sequence is
 * captured once in a HIP graph and replayed while the batch shape and pointers repeat. */
tpcsf_status tpcsf_track_batch(tpcsf_ctx* ctx, const tpcsf_frame* frame, tpcsf_tracks* out,
                               void* stream);

/* Autotuner: run the batched form at each of n_points tuning points (reps timed calls
 * each, after one untimed call), check that every point gives exactly the first point's
 * result (digest of all outputs), and keep the fastest point as the context's tuning.
 * ms_out[i] (optional) receives the mean time per call of point i, *best its index.
 * Returns TPCSF_E_INVALID, with the context's tuning unchanged, if a point is out of
 * range or changes the result.  Synchronises the stream. */
tpcsf_status tpcsf_autotune(tpcsf_ctx* ctx, const tpcsf_frame* frame, tpcsf_tracks* out,
                            const tpcsf_tuning* points, int32_t n_points, int32_t reps, float* ms_out,
                            int32_t* best, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): tpcsf_track_batch with the scratch in a
 * fixed device array of TPCSF_NOALLOC_SCRATCH_BYTES per GPU instead of the context's arena.
 * The call allocates nothing (no hipMalloc, hipFree or graph instantiation): it validates
 * on the host and launches the stage sequence eagerly on `stream`; the outputs are the
 * same as tpcsf_track_batch's.  The caller still provides every input and output buffer.
 * A batch whose scratch (tpcsf_arena_bytes without a reservation, about 320 bytes per
 * cluster, so up to roughly 800k clusters) exceeds the array is refused with
 * TPCSF_E_NOMEM before anything is launched.  The array exists once per GPU and is shared
 * by every context and thread on it, is not counted against the HBM budget, is held until
 * the process ends and keeps the last call's contents: calls that overlap on one GPU race,
 * so the caller must order them (one stream, or events).  tpcsf_debug and tpcsf_reject
 * after this call read that array. */
#define TPCSF_NOALLOC_SCRATCH_BYTES (256ull << 20)
tpcsf_status tpcsf_track_batch_noalloc(tpcsf_ctx* ctx, const tpcsf_frame* frame, tpcsf_tracks* out, void* stream);

/* Wait for the stream and report errors the device found since the last sync:
 * TPCSF_E_INVALID (non-finite or |coordinate| > 1e5 cm), TPCSF_E_CAPACITY, or TPCSF_OK. */
tpcsf_status tpcsf_sync(tpcsf_ctx* ctx, void* stream);

/* Intermediate results of the last call, for verification (device pointers into the
 * arena, valid until the next call on the context).  The call synchronises the device
 * and converts the working arrays (kept in sorted bin order) to input order.  Layout:
 *   row_lo[2*g], row_lo[2*g+1]   y_lo, z_lo of global row g        (float)
 *   row_bin[2*g], row_bin[2*g+1] bin sizes b_y, b_z actually used     (float)
 *   row_nb[2*g], row_nb[2*g+1]   ny, nz                               (int32)
 *   bin_start + bin_base(g)      ny*nz+1 entries, bin_base(g) = cap_mul*row_offsets[g] +
 *                                (cap_add+1)*g                        (uint32)
 *   perm[row_offsets[g] + k]     in-row index of the k-th sorted cluster  (uint32)
 *   up, dn, cup, cdn             raw and cleaned links, in-row index or -1 (int32)
 *   n_starts                     number of chain bottoms (device scalar, int64)
 *   start_row, start_idx         global row and in-row index of each start, rank order
 *   tl_nhits                     clusters of the tracklet of each start (0 = none) (int32)
 *   work[6]                      algorithmic work of the call (int64): tracklet Kalman
 *                                propagations (attempts), updates, clusters inside the
 *                                follow windows; final-fit propagations, updates, chi2
 *                                evaluations */
typedef struct {
    const float* row_lo; const float* row_bin; const int32_t* row_nb;
    const uint32_t* bin_start; const uint32_t* perm;
    const int32_t* up; const int32_t* dn; const int32_t* cup; const int32_t* cdn;
    const int64_t* n_starts; const int32_t* start_row; const int32_t* start_idx;
    const int32_t* tl_nhits;
    const int64_t* work;
} tpcsf_debug_view;
tpcsf_status tpcsf_debug(tpcsf_ctx* ctx, tpcsf_debug_view* view);

/* Stage timing (tracing).  When on, tpcsf_track_batch() enqueues the same launch sequence
 * as its graph, but eagerly on the caller's stream with a HIP event before each stage and
 * after the last one.  After tpcsf_sync(), tpcsf_stage_times() writes the duration (ms) of
 * each stage of the last batched call into ms[0 .. min(n, tpcsf_stage_count())).
 * Stage names come from tpcsf_stage_name(i) (static strings). */
tpcsf_status tpcsf_set_stage_timing(tpcsf_ctx* ctx, int32_t on);
int32_t tpcsf_stage_count(void);
const char* tpcsf_stage_name(int32_t stage);
tpcsf_status tpcsf_stage_times(tpcsf_ctx* ctx, float* ms, int32_t n);

/* ---------------------------------------------------------------------------------------
 * Merging across sector boundaries and refit across sector frames: the track-fit stage
 * that follows sector tracking (Sec. 7, Table 1 "Track Fit"; the paper names the stage
 * and gives no procedure, so the rule below is this library's definition).
 *
 * Sector s lies on side s / S (S = n_sectors / 2) at azimuth ((s mod S) + 1/2) 2 pi / S;
 * its frame has x along that direction and y towards larger azimuth, so its edges are
 * |y| = x tan(pi / S).  A track is matched from its outer end A to the inner end B of a
 * track of the neighbouring sector of the same side when
 *   - A's outermost cluster is within merge_edge (cm) of an edge, at a larger radius
 *     than A's innermost cluster; B lies in the sector beyond that edge (larger azimuth
 *     if A's outermost y >= 0, else smaller) and its innermost cluster is within
 *     merge_edge of the shared edge, at a larger radius than A's outermost cluster (radii
 *     from the cluster coordinates; edge and radius tests without contraction);
 *   - A's outer state (params_outer, cov_outer), rotated into B's frame, predicts B's
 *     inner y and z linearly (y' + dx tan phi', z' + dx tan lambda / cos phi', dx the
 *     distance to B's innermost row) within merge_window (cm);
 *   - the rotated state propagates to B's innermost row, and the chi2 of the difference
 *     of the two 5-parameter states with the sum of their covariances is <= merge_chi2.
 * Each A takes its least-chi2 candidate (ties: smaller B); each B keeps, of the A that
 * took it, the least-chi2 one (ties: smaller A); those pairs are linked.  Radii grow
 * strictly along links, so links form simple chains.  A chain of several tracks is
 * refitted over all its clusters in chain order with the final fit (seed from the first,
 * middle and last cluster in the first cluster's frame; outward pass from C0; inward pass
 * from C0 keeping the parameters), the state being rotated into a cluster's sector frame
 * before the step to its row; if that fit fails, the chain is dissolved into its tracks.
 * A single track keeps its sector fit.  Merged tracks come in the order of their first
 * (innermost) track.  Rotation: with c = cos(delta), s = sin(delta) for a frame at an
 * azimuth larger by delta, x' = x c + y s, y' = -x s + y c, sin phi' = sin phi c -
 * cos phi s (cos phi' must stay > 0), the state given at the plane x' through the rotated
 * point; its covariance follows the first-order change of that state.
 * ------------------------------------------------------------------------------------- */
typedef struct {
    int64_t cap_merged, cap_hits;
    int64_t* n_merged;                  /* [device] scalar: merged tracks of the batch      */
    int64_t* n_hits;                    /* [device] scalar: their clusters                 */
    double* params;                     /* [device] [cap_merged][5] at x_ref, in the frame
                                           of the first track's sector                     */
    double* cov;                        /* [device] [cap_merged][15]                       */
    double* x_ref;                      /* [device] [cap_merged] innermost cluster's row x */
    double* chi2;                       /* [device] [cap_merged]                           */
    double* z_beam;                     /* [device] [cap_merged] or NULL: z at the beam
                                           line, as in tpcsf_tracks                        */
    int32_t* ndf;                       /* [device] [cap_merged] 2*nhits - 5               */
    int32_t* nhits;                     /* [device] [cap_merged]                           */
    int32_t* sector;                    /* [device] [cap_merged] first track's sector      */
    int32_t* tf;                        /* [device] [cap_merged]                           */
    int32_t* n_segments;                /* [device] [cap_merged] tracks joined             */
    int64_t* hit_off;                   /* [device] [cap_merged+1]                         */
    int32_t* hit_ids;                   /* [device] [cap_hits] batch cluster index, track
                                           by track in chain order, each inner to outer    */
    int32_t* track_merged;              /* [device] [input cap_tracks] merged track of each
                                           input track                                     */
    int32_t* next;                      /* [device] [input cap_tracks] or NULL: the input
                                           track linked after this one, or -1 (links of a
                                           dissolved chain included)                       */
    double* link_chi2;                  /* [device] [input cap_tracks] or NULL: chi2 of
                                           that link (0 without one)                       */
} tpcsf_merged;

/* Merge a batch's sector tracks (the output of tpcsf_track_batch or tpcsf_track_plain on
 * the same frame, with params_outer and cov_outer requested) and refit the merged tracks.
 * All device pointers; asynchronous on `stream`; the tracks stay owned by the caller.
 * Host validation: TPCSF_E_INVALID for missing arrays or an odd sector count; device
 * validation (reported by tpcsf_sync): TPCSF_E_INVALID if the tracks are not in (time
 * frame, sector) order or hold clusters outside their own sector (nothing is then
 * merged), TPCSF_E_CAPACITY if the merged output is too small (*n_merged and *n_hits
 * hold the required sizes).  Scratch: about 350 bytes per input track capacity, kept by
 * the context, within its HBM budget (TPCSF_E_NOMEM beyond). */
tpcsf_status tpcsf_merge(tpcsf_ctx* ctx, const tpcsf_frame* frame, const tpcsf_tracks* tracks,
                         tpcsf_merged* out, void* stream);

/* Work of the last merge call, after a sync: candidate pairs through the gate, their
 * propagations, chi2 evaluations; refit rotations, propagations, updates. */
tpcsf_status tpcsf_merge_work(tpcsf_ctx* ctx, int64_t* work6);

/* Hit removal for data compression, strategy B (Sec. 4): only the clusters in the
 * vicinity of good tracks are kept (the tracks' own clusters are found through their
 * cluster_track map, which must be the one of these tracks).  Definition: a good track has pT >= reject_pt_min
 * (|q/pT| * reject_pt_min <= 1); it keeps its own clusters, and at every row from the row
 * of its first cluster to the row of its last (none if the first lies further out) its
 * state at x_ref, propagated in one helix
 * step to the row plane (no contribution where that step fails, see tpcsf_params), keeps
 * the clusters of its sector's row with |y - y_p| <= reject_window and
 * |z - z_p| <= reject_window (binary64).  Defaults: 0.05 GeV/c (the paper's 50 MeV/c
 * limit for tracks used in physics) and 1 cm.
 *   frame, tracks: the frame and the sector tracks of this context's LAST tracking call
 *     (its search grids are reused; TPCSF_E_INVALID if the frame is another one).
 *   keep:   [device] [n_clusters] written: 1 = kept, 0 = removed, batch input order.
 *   n_kept: [device] scalar written.
 * Asynchronous on `stream`; tracks whose clusters lie outside their sector are skipped
 * and reported by tpcsf_sync as TPCSF_E_INVALID.  Scratch: the (track, row) pairs of the
 * windows, bucketed by row, 4 * cap_tracks * n_rows bytes plus small per-row arrays, held
 * by the context from the first call (counted against hbm_budget_bytes; TPCSF_E_NOMEM). */
tpcsf_status tpcsf_reject(tpcsf_ctx* ctx, const tpcsf_frame* frame, const tpcsf_tracks* tracks,
                          uint8_t* keep, int64_t* n_kept, void* stream);

/* Track-model compression of the attached clusters (Sec. 4, entropy reduction): each
 * cluster of a track is stored as its row and its residual to the track's position on
 * that row plane.  Definition: the position (y_p, z_p) is the track's state at x_ref
 * propagated in one helix step to the row plane (the state at x_ref itself where that
 * step fails); the codes are q = floor(r / resid_step + 1/2) for r = y - y_p and
 * r = z - z_p (binary64), clamped to [-2^30, 2^30].  The state at x_ref (params, x_ref,
 * sector) travels with the codes; tpcsf_decompress rebuilds y_p + q_y * resid_step and
 * z_p + q_z * resid_step, within half a step of the clusters.  Default step 0.01 cm.
 *   tracks: [device] any tracks of the batch (e.g. tpcsf_track_* output): n_tracks,
 *           params, x_ref, sector, tf, hit_off, hit_ids.
 *   codes:  [device] [cap_hits][2] written, in hit-list order (y, z).
 *   rows:   [device] [cap_hits] written: row of each cluster in its sector.
 * Clusters outside their track's sector get code 0 and row 0.  Asynchronous. */
tpcsf_status tpcsf_compress(tpcsf_ctx* ctx, const tpcsf_frame* frame, const tpcsf_tracks* tracks,
                            int32_t* codes, uint8_t* rows, void* stream);

/* Decoding of tpcsf_compress: yz [device] [cap_hits][2] (binary64) from the tracks'
 * n_tracks, params, x_ref and hit_off, the codes and the rows.  Asynchronous. */
tpcsf_status tpcsf_decompress(tpcsf_ctx* ctx, const tpcsf_tracks* tracks, const int32_t* codes,
                              const uint8_t* rows, double* yz, void* stream);

/* Message of the last error on this context (static storage of the context). */
const char* tpcsf_last_error(const tpcsf_ctx* ctx);

/* ---------------------------------------------------------------------------------------
 * Serving: continuous batching of time frames that arrive over time (the online setting
 * of Sec. 3 and 7.1: every frame is processed whole and independently).
 *
 * A server owns n_slots slots.  A slot is a tracking context with its own stream and its
 * own device and pinned host buffers, sized on first use and grown on demand; the device
 * bytes of all slots stay within hbm_budget_bytes (0 = no bound).  tpcsf_server_submit()
 * admits a frame into a free slot at once, or returns TPCSF_E_BUSY (an admission stall)
 * when no free slot can hold it within the budget.  Upload, tracking and the download of
 * the frame's track and hit counts run asynchronously on the slot's stream, so admitted
 * frames overlap on the device; the first tpcsf_server_poll()/tpcsf_server_wait() of the
 * frame after its counts arrived enqueues the download of exactly that many tracks and
 * hits (so a frame's completion needs its ticket to be polled or waited on).  Each
 * frame's result is the same as tpcsf_track_batch() on that frame alone.  All server
 * calls are thread-safe.
 * ------------------------------------------------------------------------------------- */
typedef struct tpcsf_server tpcsf_server;

/* Host copy of one frame's tracks (caller-allocated host buffers, layout as tpcsf_tracks;
 * cluster_track holds the frame's n_clusters entries). */
typedef struct {
    int64_t cap_tracks, cap_hits;
    int64_t n_tracks, n_hits;           /* written */
    double* params; double* cov; double* x_ref; double* chi2;
    int32_t* ndf; int32_t* nhits; int32_t* sector;
    int64_t* hit_off; int32_t* hit_ids; int32_t* cluster_track;
    double* z_beam;                     /* [cap_tracks] or NULL */
} tpcsf_host_tracks;

tpcsf_status tpcsf_server_create(const tpcsf_geometry* geo, const tpcsf_params* params,
                                 const tpcsf_tuning* tuning, int32_t n_slots, size_t hbm_budget_bytes,
                                 tpcsf_server** out);
tpcsf_status tpcsf_server_destroy(tpcsf_server* server);

/* Admit one time frame: y, z [host] [n_clusters], row_offsets [host] [n_sectors*n_rows+1].
 * The host arrays must stay valid until the ticket completes; pinned (hipHostMalloc)
 * memory makes the upload asynchronous.  *ticket identifies the frame. */
tpcsf_status tpcsf_server_submit(tpcsf_server* server, const float* y, const float* z,
                                 const int64_t* row_offsets, int64_t n_clusters, uint64_t* ticket);
/* *done = 1 once the frame's tracks are on the host. */
tpcsf_status tpcsf_server_poll(tpcsf_server* server, uint64_t ticket, int32_t* done);
/* Wait up to timeout_us (< 0: forever); TPCSF_E_TIMEOUT if the frame is not done. */
tpcsf_status tpcsf_server_wait(tpcsf_server* server, uint64_t ticket, int64_t timeout_us);
/* Copy a completed frame's tracks into `out` and release its slot (TPCSF_E_BUSY if not
 * done yet; TPCSF_E_CAPACITY, slot released, if out is too small).  out = NULL releases
 * the slot without copying (the frame's status is still returned). */
tpcsf_status tpcsf_server_result(tpcsf_server* server, uint64_t ticket, tpcsf_host_tracks* out);
/* Device bytes the slots hold now. */
size_t tpcsf_server_bytes_used(const tpcsf_server* server);
const char* tpcsf_server_last_error(const tpcsf_server* server);

#ifdef __cplusplus
}
#endif
#endif
