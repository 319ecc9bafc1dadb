// Internal declarations shared by the kernels and the host runtime of libtpcsf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpcsf {

constexpr int kMaxRows = 256;
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
    // tracklets (p indexed); hit table H[p * n_rows + r]
    int32_t* tl_len;                // chain length
    int32_t* order;                 // [cap_starts] p of every tracklet to build, in p order
    int32_t* tl_n;                  // clusters, 0 = none
    int16_t* tl_rlo;                // first row holding a cluster
    int16_t* tl_rhi;                // last row holding a cluster
    uint16_t* tl_hits;              // sorted position per row, kNoHit if none
    // keep and final fit: candidates listed densely
    int32_t* keep_n;                // [cap_starts] (p indexed) kept clusters, 0 = not a candidate
    int64_t* fit_pos;               // [cap_starts] (p indexed) candidate slot (scan of keep_n)
    int64_t* cand_off;              // [cap_starts] (p indexed) first entry of the kept list
    float4* kept_list;              // [N] kept clusters of the candidates, slot order, inner to
                                    //     outer: y, z, row plane x, input index (as bits)
    uint64_t* keep_mask;            // [cap_starts][4] (p indexed) kept rows
    int32_t* fit_list;              // [cap_fit] p of every candidate, in p order
    double* f_par;                  // [cap_fit][5]
    double* f_cov;                  // [cap_fit][15]
    double* f_chi2;                 // [cap_fit]
    double* f_xref;                 // [cap_fit]
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
    // verification views in input order (filled only by launch_debug_views)
    int32_t* d_up; int32_t* d_dn; int32_t* d_cup; int32_t* d_cdn;   // [N]
    int32_t* d_start_row; int32_t* d_start_idx; int32_t* d_tl_n;     // [cap_starts] by rank
};

struct LaunchCfg {
    int block;      // row kernels
    int tl_block;   // tracklet kernels
    int chunk;      // idle lanes that make a tracklet wave take new work
    int n_cu;       // compute units
    int grid_lds;   // dynamic LDS bytes of the grid kernel
};

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
void launch_keep(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_fit_scan(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_fit(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_track_scan(const Batch& b, hipStream_t s);
void launch_emit(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_assign(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s);
void launch_debug_views(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_hash(const Batch& b, int64_t n_clusters, const LaunchCfg& c, hipStream_t s);

}  // namespace tpcsf
