// Internal declarations shared by the kernels and the host runtime of libtpcsf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpcsf {

constexpr int kMaxRows = 256;      // row tables are sized for this many rows
constexpr int kMaxRowsGeo = 255;   // rows a geometry may have: a tracklet's cluster count
                                   // fills the 8 high bits of its selection weight
constexpr uint16_t kNoHit = 0xFFFF;
constexpr int kScanBlocks = 256;     // blocks of the device-wide scan
constexpr int kScanThreads = 256;

// error bits accumulated on the device
constexpr int32_t kErrInvalid = 1;
constexpr int32_t kErrOutCap = 2;
constexpr int32_t kErrTrackletCap = 4;

// Method constants and tuning as the kernels see them.
struct DevParams {
    float win_y, win_z, kink_max;
    float bin_y, bin_z;
    int32_t cap_mul, cap_add;
    double sy2, sz2, chi2_max, sinphi_max, nsig;
    double c0[5];
    double a;                       // -C_B * bz: kappa = a * q/pT
    int32_t min_chain, min_track_hits, max_miss;
    int32_t n_rows, n_sectors;
    const float* rx;                // [device] row plane positions
};

// Running counters of one call (device memory).
struct Counters {
    int64_t start_base;             // starts ranked so far (row scan base)
    int64_t rank_lo, rank_hi;       // rank range of the starts of the current launch set
    int64_t track_base;             // tracks emitted so far
    int64_t hit_base;               // hits emitted so far
    int64_t n_order;                // tracklets to build (chains of >= min_chain)
    int64_t n_fit;                  // track candidates (>= min_track_hits kept)
    int64_t n_fit_long;             // candidates of >= kFitLong kept clusters
    int32_t queue[8];               // tracklet work queue: head of each XCD's segment
    int32_t fit_queue[8];           // fit work queue: head of each XCD's segment
    int32_t err;                    // error bits
    unsigned long long hash;        // output digest (autotuner's result-invariance check)
    // algorithmic work of the call: tracklet propagations, updates, window candidates;
    // final-fit propagations, updates, chi2 evaluations
    int64_t work[6];
};

// Device pointers of one batch: inputs, arena and outputs.
//
// Working space.  After the grid stage every per-cluster array is indexed by the
// cluster's position in its row's sorted (bin) order, at row_first + k; `perm` maps a
// sorted position to the in-row index of the input, `iperm` the other way.  The method's
// tie-breaks and ranks are still taken on in-row indices.  Starts are processed in
// (row, sorted position) order ("p" below) for locality; each carries its rank.
struct Batch {
    // inputs
    const float* y;
    const float* z;
    const int64_t* off;             // [R+1]
    int64_t n;                      // clusters
    int32_t n_rows_total;           // R = n_tf * n_sectors * n_rows
    int32_t n_rows;                 // rows per sector
    // grid
    float2* row_lo;                 // [R] y_lo, z_lo
    float2* row_bin;                // [R] b_y, b_z
    int2* row_nb;                   // [R] ny, nz
    float4* row_f;                  // [R] y_lo, z_lo, 1/b_y, 1/b_z (search records)
    int4* row_i;                    // [R] first cluster, count, ny, nz
    uint32_t* bin_start;            // [cap_mul*N + (cap_add+1)*R]
    float2* yz;                     // [N] sorted (y, z)
    uint32_t* perm;                 // [N] sorted position -> in-row index
    uint32_t* iperm;                // [N] in-row index -> sorted position
    // links, sorted positions
    int32_t* upk; int32_t* dnk;     // [N] raw
    int32_t* cupk; int32_t* cdnk;   // [N] cleaned
    int64_t* row_nstart;            // [R] starts per row
    int64_t* row_sbase;             // [R] exclusive prefix (rank of the row's first start)
    int32_t* rank_at;               // [N] scratch: rank of the start at a sorted position
    // starts in processing order p
    int32_t* st_row;                // [cap_starts] global row
    int32_t* st_k;                  // [cap_starts] sorted position
    int32_t* st_rank;               // [cap_starts] rank
    int64_t cap_starts;
    // tracklets (p indexed)
    int32_t* tl_len;                // chain length
    int32_t* order;                 // [cap_starts] p of every tracklet to build, in p order
    int32_t* tl_n;                  // clusters, 0 = none
    int16_t* tl_rlo;                // first row holding a cluster
    int16_t* tl_rhi;                // last row holding a cluster
    uint32_t* tl_w;                 // selection weight, 0 = takes no part
    uint16_t* tl_hits;              // sorted position per row, kNoHit if none; tiles of
                                    //     64 starts x n_rows rows
    // keep and final fit: candidates listed densely
    int32_t* keep_n;                // [cap_starts] (p indexed) kept clusters, 0 = not a candidate
    int64_t* fit_pos;               // [cap_starts] (p indexed) candidate slot (scan of keep_n)
    int64_t* fit_pos_long;          // [cap_starts] (p indexed) scan of the long candidates
    int64_t* cand_off;              // [cap_starts] (p indexed) first entry of the kept list
    float4* kept_list;              // [N] kept clusters of the candidates, slot order, inner to
                                    //     outer: y, z, row plane x, input index (as bits)
    uint64_t* keep_mask;            // [cap_starts][4] (p indexed) kept rows
    int32_t* fit_list;              // [cap_fit] p of every candidate, in p order
    double* f_par;                  // [cap_fit][5]
    double* f_cov;                  // [cap_fit][15]
    double* f_chi2;                 // [cap_fit]
    double* f_xref;                 // [cap_fit]
    double* f_pout;                 // [cap_fit][5] outward-pass state at the outermost
                                    //     cluster, or null when not requested
    double* f_cout;                 // [cap_fit][15] its covariance
    int32_t cap_fit;
    // rank indexed
    int32_t* trk_flag;              // 1 = accepted and fitted
    int32_t* hit_cnt;               // kept clusters of accepted tracks
    int64_t* trk_idx;               // output track index
    int64_t* hit_pos;               // output hit offset
    int32_t* trk_out;               // output track written for this rank, -1 if none
    // selection (sorted positions)
    uint32_t* W;                    // [N]
    // scan scratch
    int64_t* scan_part;             // [4 * kScanBlocks + 2]
    Counters* ctr;
    // outputs
    int64_t cap_tracks, cap_hits;
    int64_t* o_ntracks; int64_t* o_nhits;
    double* o_par; double* o_cov; double* o_xref; double* o_chi2;
    int32_t* o_ndf; int32_t* o_nhits_trk; int32_t* o_sector; int32_t* o_tf;
    int64_t* o_hit_off; int32_t* o_hit_ids; int32_t* o_cluster_track;
    double* o_zbeam;                // may be null
    double* o_par_out;              // may be null
    double* o_cov_out;              // may be null
    float4* o_hit_rec;              // may be null
    // verification views in input order (filled only by launch_debug_views)
    int32_t* d_up; int32_t* d_dn; int32_t* d_cup; int32_t* d_cdn;   // [N]
    int32_t* d_start_row; int32_t* d_start_idx; int32_t* d_tl_n;     // [cap_starts] by rank
};

// Device-wide exclusive scan of up to two channels over [lo, hi) (bounds read from
// device memory where the pointers are given).
struct ScanJob {
    const int64_t* a64;       // channel A input (int64) or null
    const int32_t* a32;       // channel A input (int32) if a64 is null
    const int32_t* b32;       // channel B input (int32) or null
    int32_t a_min;            // > 0: channel A counts a32[i] >= a_min as 1, else 0
    int64_t* outA;
    int64_t* outB;
    int64_t lo, hi;           // range if lo_ptr is null
    const int64_t* lo_ptr;
    const int64_t* hi_ptr;
    int64_t* baseA;           // running base, advanced by the total
    int64_t* baseB;
    int64_t* totA;            // receives base + total (optional)
    int64_t* totB;
    int64_t* rangeA_lo;       // receives [base, base + total) (optional)
    int64_t* rangeA_hi;
    int64_t* part;            // [4 * kScanBlocks]
};

struct LaunchCfg {
    int block;      // row kernels
    int tl_block;   // tracklet kernels
    int chunk;      // groups of 64 tracklets a wave takes per work-queue atomic
    int n_cu;       // compute units
    int grid_lds;   // dynamic LDS bytes of the grid kernel
};

// Merging across sector boundaries (tpcsf_merge).
constexpr int kMergeMaxSide = 64;    // sectors per side the merge supports
constexpr int kMergeMaxChain = 64;   // walk bound of a chain (links raise the radius
                                     // strictly, so chains never revisit a track)
constexpr int32_t kErrMergeChain = 8;

struct MergeParams {
    double edge, window, chi2;      // merge_edge, merge_window, merge_chi2
    double te;                      // tan(pi / S): |y| = x te at a sector's edges
    int32_t S;                      // sectors per side
    // cos and sin of the azimuth step d * 2 pi / S between two sectors of one side, at
    // [d + S/2] for d in (-S/2, S/2]
    double rc[kMergeMaxSide + 1], rs[kMergeMaxSide + 1];
};

struct MergeCounters {
    int64_t T;                      // input tracks (min(n_tracks, cap_tracks))
    int32_t n_fit;                  // chains of several segments
    int32_t bad;                    // invalid input seen: nothing is merged
    unsigned long long fit_hits;    // clusters of those chains (gather offsets)
    int32_t n_outer;                // outer ends listed in a_idx
    // algorithmic work: candidate pairs through the gate, their propagations (attempts),
    // chi2 evaluations; merged-fit rotations, propagations, updates
    int64_t work[6];
};

// Device pointers of one merge call (T = cap_tracks of the input, K = n_tf * n_sectors).
struct MergeBatch {
    // inputs: the frame's clusters and the sector tracks with their outer states
    const float* y; const float* z; const int64_t* off;
    const int64_t* n_tracks; int64_t cap_tracks, cap_in_hits;
    const int64_t* hit_off; const int32_t* hit_ids;
    const double* par; const double* cov; const double* xref; const double* chi2;
    const int32_t* sector; const int32_t* tf;
    const double* par_out; const double* cov_out;
    const float4* hit_rec;          // per hit (y, z, row plane x, index), or null
    int32_t n_tf;
    // scratch
    float4* ends;                   // [T] innermost (x, y) and outermost (x, y) cluster
    int32_t* a_list;                // [T] list an outer end is matched against, or -1
    int32_t* a_idx;                 // [T] the tracks with an outer end, compactly (any order)
    int32_t* b_list;                // [T] list of an inner end, or -1
    int32_t* sec_first;             // [K] first track of each (time frame, sector)
    int32_t* cnt;                   // [2K] entries per list (list = key * 2 + edge)
    double4* brec;                  // [2T] entries: x_in, radius^2 of the inner cluster, y, z
    int32_t* bidx;                  // [2T] their tracks
    double4* brec_s;                // [2T] the same, each list ordered by z
    int32_t* bidx_s;                // [2T]
    float* zs;                      // [2T] z of the ordered entries (binary32)
    int32_t* lsorted;               // [2K] 1 if the list is ordered by z (short enough)
    double* mstate;                 // [T][21] rotated outer state (x, p, C); later the
                                    //     merged fit of a chain head (p, C, chi2)
    int32_t* bestB; double* bestChi;
    unsigned long long* keepChi;    // [T] least chi2 (bits) of the outer ends that chose B
    int32_t* keepA;                 // [T] smallest such end at that chi2
    int32_t* next; int32_t* prev;
    int32_t* nseg; int32_t* chain_hits; int32_t* fit_ok; int32_t* diss;
    int32_t* lead; int32_t* nh;     // scan inputs
    int32_t* fit_list;
    int32_t* seg_head;              // [T] head of the chain a track belongs to, or -1
    int32_t* seg_pre;               // [T] clusters of the chain before this track
    int64_t* fit_off;               // [T] first gathered record of a chain head
    float4* grec;                   // [input cap_hits] clusters of the chains to refit, in
                                    //     chain order: y, z, row plane x, sector (as bits)
    int64_t* m_idx; int64_t* m_hpos;
    int64_t* scan_part;
    MergeCounters* mc;
    Counters* ctr;                  // error bits
    // outputs
    int64_t cap_merged, cap_hits;
    int64_t* o_n; int64_t* o_nhits;
    double* o_par; double* o_cov; double* o_xref; double* o_chi2; double* o_zbeam;
    int32_t* o_ndf; int32_t* o_nhits_trk; int32_t* o_sector; int32_t* o_tf; int32_t* o_nseg;
    int64_t* o_hit_off; int32_t* o_hit_ids;
    int32_t* o_track_merged; int32_t* o_next; double* o_link_chi2;
};

void launch_merge(const MergeBatch& b, const DevParams& p, const MergeParams& m, int n_cu, hipStream_t s);

// Hit removal, strategy B (tpcsf_reject): the sector tracks of the context's last call and
// the keep flags to write.
struct RejectArgs {
    const int64_t* n_tracks; int64_t cap_tracks, cap_hits;
    const double* par; const double* xref;
    const int32_t* sector; const int32_t* tf;
    const int64_t* hit_off; const int32_t* hit_ids;
    const int32_t* cluster_track;   // [n_clusters] the tracks' cluster -> track map
    int32_t n_tf;
    double pt_min, window;
    uint8_t* keep;                  // [n_clusters]
    int64_t* n_kept;
    // the (track, row) pairs of the vicinities, bucketed by row
    int32_t* rspan;                 // [cap_tracks][2] rows of the first and last cluster, -1 none
    int32_t* rdiff;                 // [R+1] difference array of the row counts
    int32_t* rcnt;                  // [R] pairs per row
    int64_t* rtmp;                  // [R+1] scan scratch
    int64_t* roff;                  // [R+1] first pair of each row
    int32_t* rcur;                  // [R] fill cursors
    int32_t* ritems;                // [cap_items] tracks, row by row
    int64_t cap_items;
    int64_t* scan_part;             // [4 * kScanBlocks + 2]
    int32_t n_rows_total;
};
void launch_reject(const Batch& b, const DevParams& p, const RejectArgs& r, const LaunchCfg& c, hipStream_t s);

// Track-model compression (tpcsf_compress / tpcsf_decompress).
struct CompressArgs {
    const int64_t* n_tracks; int64_t cap_tracks, cap_hits;
    const double* par; const double* xref;
    const int32_t* sector; const int32_t* tf;
    const int64_t* hit_off; const int32_t* hit_ids;   // encode only
    const float* y; const float* z; const int64_t* off; // encode only
    const float4* hit_rec;          // encode: per hit (y, z, row plane x, index), or null
    int32_t n_tf;
    double step;
    int32_t* codes;                 // [cap_hits][2]: written by encode, read by decode
    uint8_t* rows;                  // [cap_hits]: written by encode, read by decode
    double* yz;                     // [cap_hits][2]: written by decode
};
void launch_compress(const CompressArgs& a, const DevParams& p, int n_cu, hipStream_t s);
void launch_decompress(const CompressArgs& a, const DevParams& p, int n_cu, hipStream_t s);

// Stage launchers (all asynchronous on `stream`).  Row ranges are [g0, g1).
// Allows the grid kernel the device's LDS per block; returns the dynamic LDS bytes to use.
int grid_lds_setup(int max_lds_per_block);
void launch_reset(const Batch& b, hipStream_t s);
void launch_grid(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s);
void launch_links(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s);
void launch_clean(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s);
void launch_row_scan(const Batch& b, int64_t g0, int64_t g1, hipStream_t s);
void launch_starts(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s);
void launch_walk(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_order(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_tracklets(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_claim(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s);
void launch_keep(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_fit_scan(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_fit(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_track_scan(const Batch& b, hipStream_t s);
void launch_emit(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_assign(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s);
void launch_debug_views(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_hash(const Batch& b, int64_t n_clusters, const LaunchCfg& c, hipStream_t s);
void launch_scan(const ScanJob& job, hipStream_t s);

}  // namespace tpcsf
