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
    int32_t tl_count;               // tracklet slots taken
    int32_t queue;                  // tracklet work-queue head
    int32_t err;                    // error bits
    int32_t pad;
};

// Device pointers of one batch: inputs, arena and outputs.
struct Batch {
    // inputs
    const float* y;
    const float* z;
    const int64_t* off;             // [R+1]
    int64_t n;                      // clusters
    int32_t n_rows_total;           // R = n_tf * n_sectors * n_rows
    // grid
    float2* row_lo;                 // [R] y_lo, z_lo
    float2* row_bin;                // [R] b_y, b_z
    int2* row_nb;                   // [R] ny, nz
    uint32_t* bin_start;            // [cap_mul*N + (cap_add+1)*R]
    uint32_t* bin_fill;             // same size
    float* ys;                      // [N] sorted y
    float* zs;                      // [N] sorted z
    uint32_t* perm;                 // [N] in-row index of sorted position
    // links
    int32_t* up; int32_t* dn;       // [N] raw
    int32_t* cup; int32_t* cdn;     // [N] cleaned
    int64_t* row_nstart;            // [R] starts per row
    int64_t* row_sbase;             // [R] exclusive prefix (rank of the row's first start)
    // starts and tracklets (rank indexed)
    int32_t* start_row;             // [cap_starts]
    int32_t* start_idx;             // [cap_starts]
    int32_t* tl_n;                  // [cap_starts] tracklet clusters, 0 = none
    int32_t* tl_slot;               // [cap_starts]
    int32_t* trk_flag;              // [cap_starts] 1 = accepted and fitted
    int32_t* hit_cnt;               // [cap_starts] kept clusters of accepted tracks
    int64_t* trk_idx;               // [cap_starts] output track index
    int64_t* hit_pos;               // [cap_starts] output hit offset
    int64_t cap_starts;
    // tracklet slots
    uint16_t* tl_hits;              // [cap_tl][n_rows] in-row index per row
    double* f_par;                  // [cap_tl][5]
    double* f_cov;                  // [cap_tl][15]
    double* f_chi2;                 // [cap_tl]
    double* f_xref;                 // [cap_tl]
    uint64_t* f_mask;               // [cap_tl][4] kept rows
    int32_t cap_tl;
    // selection
    unsigned long long* W;          // [N]
    // scan scratch
    int64_t* scan_part;             // [kScanBlocks * 2]
    Counters* ctr;
    // outputs
    int64_t cap_tracks, cap_hits;
    int64_t* o_ntracks; int64_t* o_nhits;
    double* o_par; double* o_cov; double* o_xref; double* o_chi2;
    int32_t* o_ndf; int32_t* o_nhits_trk; int32_t* o_sector; int32_t* o_tf;
    int64_t* o_hit_off; int32_t* o_hit_ids; int32_t* o_cluster_track;
};

struct LaunchCfg {
    int block;      // row kernels
    int tl_block;   // tracklet kernels
    int chunk;      // starts per lane taken from the queue
    int n_cu;       // compute units
};

// Stage launchers (all asynchronous on `stream`).  Row ranges are [g0, g1).
void launch_reset(const Batch& b, hipStream_t s);
void launch_grid(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s);
void launch_links(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s);
void launch_clean(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s);
void launch_row_scan(const Batch& b, int64_t g0, int64_t g1, hipStream_t s);
void launch_starts(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s);
void launch_tracklets(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_claim(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_keepfit(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);
void launch_track_scan(const Batch& b, hipStream_t s);
void launch_emit(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s);

}  // namespace tpcsf
