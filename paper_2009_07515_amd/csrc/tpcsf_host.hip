// Host runtime of libtpcsf: context, scratch arena under an HBM budget, input validation,
// the plain (per time frame and sector) and batched (whole batch per launch, HIP graph)
// execution plans, and the C ABI of include/tpcsf.h.
#include "tpcsf.h"
#include "tpcsf_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace tpcsf;

// Scratch of tpcsf_track_batch_noalloc: one fixed array per GPU, held from the loading of
// the library's code on that GPU until the process ends.  In host code `scratch` names
// only a host-side stand-in: its device address on each GPU comes from
// hipGetSymbolAddress (at context creation, with that GPU current) and is kept in
// g_scratch_ptr; that address, never the name, is what kernels receive.
static __device__ __align__(256) unsigned char scratch[TPCSF_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's fixed scratch array (looked up once per device).
hipError_t scratch_setup(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

namespace {

constexpr double kCB = 0.00299792458;   // cm^-1 T^-1 GeV

struct Layout {
    size_t total = 0;
    int64_t n = 0, R = 0, cap_starts = 0, cap_fit = 0, n_bins = 0;
    size_t row_lo, row_bin, row_nb, row_f, row_i, row_nstart, row_sbase;
    size_t bin_start, yz, perm, iperm, upk, dnk, cupk, cdnk, rank_at, W;
    size_t st_row, st_k, st_rank, tl_len, order, tl_n, tl_rlo, tl_rhi, tl_w, tl_hits;
    size_t keep_n, fit_pos, fit_pos_long, cand_off, kept_list, keep_mask, fit_list;
    size_t trk_flag, hit_cnt, trk_idx, hit_pos, trk_out;
    size_t f_par, f_cov, f_chi2, f_xref, f_pout, f_cout, scan_part;
    size_t d_up, d_dn, d_cup, d_cdn, d_start_row, d_start_idx, d_tl_n;
};

constexpr int kStages = 14;
const char* const kStageNames[kStages] = {"reset", "grid", "links", "clean",      "row_scan", "starts", "walk",
                                          "tracklets", "claim", "keep", "fit", "track_scan", "emit", "assign"};

struct GraphKey {
    const void* y = nullptr; const void* z = nullptr; const void* off = nullptr;
    int64_t n = -1; int64_t R = -1;
    const void* arena = nullptr;
    tpcsf_tracks out{};
    tpcsf_tuning tuning{};
    int32_t grid_lds = 0;
    bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof(GraphKey)) == 0; }
};

}  // namespace

struct tpcsf_ctx {
    int device = 0;
    int n_cu = 256;
    int grid_lds_max = 0;           // dynamic LDS bytes the grid kernel may use on the device
    int grid_lds_used = 0;          // dynamic LDS bytes it takes: the largest need seen so far
    int64_t frame_max_row = 0;      // largest row of the frame being tracked
    int32_t n_sectors = 36, n_rows = 152;
    std::vector<float> row_x;
    double bz = 0.5;
    tpcsf_params params{};
    tpcsf_tuning tuning{};
    size_t budget = 0;
    int64_t reserve_n = 0;          // layout capacity (clusters), see tpcsf_reserve
    int32_t reserve_tf = 0;
    float* d_rx = nullptr;
    Counters* d_ctr = nullptr;
    void* arena = nullptr;
    size_t arena_size = 0;
    void* fixed_scratch = nullptr;  // this device's fixed scratch array (tpcsf_track_batch_noalloc)
    void* marena = nullptr;         // scratch of tpcsf_merge
    size_t marena_size = 0;
    void* rarena = nullptr;         // scratch of tpcsf_reject
    size_t rarena_size = 0;
    MergeCounters* d_mc = nullptr;
    Layout lay{};
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    GraphKey gkey{};
    int32_t timing = 0;
    hipEvent_t ev[kStages + 1] = {};
    bool timed_last = false;
    Batch last{};
    DevParams last_P{};             // the method constants and tuning of that call
    bool have_last = false;
    std::string err;
};

namespace {

tpcsf_status fail(tpcsf_ctx* c, tpcsf_status st, const std::string& msg)
{
    if (c) c->err = msg;
    return st;
}

tpcsf_status hip_fail(tpcsf_ctx* c, hipError_t e, const char* what)
{
    return fail(c, TPCSF_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Scratch layout of a batch; `reserved` applies the capacity fixed by tpcsf_reserve.
Layout make_layout(const tpcsf_ctx* c, int64_t n, int32_t n_tf, bool reserved = true)
{
    if (reserved && n < c->reserve_n) n = c->reserve_n;
    if (reserved && n_tf < c->reserve_tf) n_tf = c->reserve_tf;
    Layout L;
    L.n = n;
    L.R = (int64_t)n_tf * c->n_sectors * c->n_rows;
    L.n_bins = (int64_t)c->tuning.cap_mul * n + (int64_t)(c->tuning.cap_add + 1) * L.R;
    // every start has a cleaned up-link and chains are vertex-disjoint: starts <= n/2;
    // kept cluster sets are disjoint: fitted candidates <= n / min_track_hits
    L.cap_starts = n / 2 + 1;
    L.cap_fit = n / (c->params.min_track_hits > 1 ? c->params.min_track_hits : 1) + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    const size_t N = (size_t)n, R = (size_t)L.R, S = (size_t)L.cap_starts, F = (size_t)L.cap_fit;
    L.row_lo = take(R * 8);
    L.row_bin = take(R * 8);
    L.row_nb = take(R * 8);
    L.row_f = take(R * 16);
    L.row_i = take(R * 16);
    L.row_nstart = take(R * 8);
    L.row_sbase = take(R * 8);
    L.bin_start = take((size_t)L.n_bins * 4);
    L.yz = take(N * 8);
    L.perm = take(N * 4);
    L.iperm = take(N * 4);
    L.upk = take(N * 4);
    L.dnk = take(N * 4);
    L.cupk = take(N * 4);
    L.cdnk = take(N * 4);
    L.rank_at = take(N * 4);
    L.W = take(N * 4);
    L.st_row = take(S * 4);
    L.st_k = take(S * 4);
    L.st_rank = take(S * 4);
    L.tl_len = take(S * 4);
    L.order = take(S * 4);
    L.tl_n = take(S * 4);
    L.tl_rlo = take(S * 2);
    L.tl_rhi = take(S * 2);
    L.tl_w = take(S * 4);
    L.tl_hits = take((S + 63) / 64 * 64 * (size_t)c->n_rows * 2);   // tiles of 64 starts
    L.keep_n = take(S * 4);
    L.fit_pos = take(S * 8);
    L.fit_pos_long = take(S * 8);
    L.cand_off = take(S * 8);
    L.kept_list = take(N * 16);
    L.keep_mask = take(S * 4 * 8);
    L.fit_list = take(F * 4);
    L.trk_flag = take(S * 4);
    L.hit_cnt = take(S * 4);
    L.trk_idx = take(S * 8);
    L.hit_pos = take(S * 8);
    L.trk_out = take(S * 4);
    L.f_par = take(F * 5 * 8);
    L.f_cov = take(F * 15 * 8);
    L.f_chi2 = take(F * 8);
    L.f_xref = take(F * 8);
    L.f_pout = take(F * 5 * 8);
    L.f_cout = take(F * 15 * 8);
    L.scan_part = take((4 * kScanBlocks + 2) * 8);
    L.d_up = take(N * 4);
    L.d_dn = take(N * 4);
    L.d_cup = take(N * 4);
    L.d_cdn = take(N * 4);
    L.d_start_row = take(S * 4);
    L.d_start_idx = take(S * 4);
    L.d_tl_n = take(S * 4);
    L.total = o;
    return L;
}

DevParams dev_params(const tpcsf_ctx* c)
{
    DevParams P;
    const tpcsf_params& p = c->params;
    P.win_y = p.win_y; P.win_z = p.win_z; P.kink_max = p.kink_max;
    P.bin_y = c->tuning.bin_y; P.bin_z = c->tuning.bin_z;
    P.cap_mul = c->tuning.cap_mul; P.cap_add = c->tuning.cap_add;
    P.sy2 = p.sigma_y * p.sigma_y; P.sz2 = p.sigma_z * p.sigma_z;
    P.chi2_max = p.chi2_max; P.sinphi_max = p.sinphi_max; P.nsig = p.nsig;
    for (int i = 0; i < 5; ++i) P.c0[i] = p.c0[i];
    P.a = -kCB * c->bz;
    P.min_chain = p.min_chain; P.min_track_hits = p.min_track_hits; P.max_miss = p.max_miss;
    P.n_rows = c->n_rows; P.n_sectors = c->n_sectors;
    P.rx = c->d_rx;
    return P;
}

LaunchCfg launch_cfg(const tpcsf_ctx* c)
{
    LaunchCfg L;
    L.block = c->tuning.block;
    L.tl_block = c->tuning.tl_block;
    L.chunk = c->tuning.chunk;
    L.n_cu = c->n_cu;
    L.grid_lds = c->grid_lds_used;
    return L;
}

bool tuning_ok(const tpcsf_tuning* t)
{
    return t && t->bin_y >= 1e-3f && t->bin_z >= 1e-3f && t->bin_y <= 1e5f && t->bin_z <= 1e5f &&
           t->cap_mul >= 1 && t->cap_mul <= 64 && t->cap_add >= 1 && t->cap_add <= 4096 &&
           t->block >= 64 && t->block <= 1024 && t->block % 64 == 0 && t->tl_block >= 64 &&
           t->tl_block <= 256 && t->tl_block % 64 == 0 && t->chunk >= 1 && t->chunk <= 64;
}

bool params_ok(const tpcsf_params* p)
{
    if (!p) return false;
    if (!(p->win_y > 0 && p->win_z > 0 && p->kink_max >= 0)) return false;
    if (!(p->sigma_y > 0 && p->sigma_z > 0 && p->chi2_max > 0 && p->nsig > 0)) return false;
    if (!(p->sinphi_max > 0 && p->sinphi_max < 1)) return false;
    for (int i = 0; i < 5; ++i)
        if (!(p->c0[i] > 0)) return false;
    if (!(p->merge_edge >= 0 && p->merge_window >= 0 && p->merge_chi2 >= 0)) return false;
    if (!(p->reject_pt_min >= 0 && p->reject_window >= 0 && p->reject_window < 1e4)) return false;
    if (!(p->resid_step > 1e-9 && p->resid_step < 1e4)) return false;
    return p->min_chain >= 3 && p->min_track_hits >= 3 && p->max_miss >= 0;
}

// Validate a frame against the context and its outputs (host-side offsets).
tpcsf_status check_frame(tpcsf_ctx* c, const tpcsf_frame* f, const tpcsf_tracks* o)
{
    if (!f || !o) return fail(c, TPCSF_E_INVALID, "null frame or output");
    if (f->n_tf < 1) return fail(c, TPCSF_E_INVALID, "n_tf < 1");
    if (f->n_clusters < 0 || f->n_clusters >= ((int64_t)1 << 31) - 1)
        return fail(c, TPCSF_E_INVALID, "n_clusters out of range [0, 2^31-1)");
    if (!f->row_offsets || !f->row_offsets_host) return fail(c, TPCSF_E_INVALID, "row offsets missing");
    if (f->n_clusters > 0 && (!f->y || !f->z)) return fail(c, TPCSF_E_INVALID, "cluster arrays missing");
    const int64_t R = (int64_t)f->n_tf * c->n_sectors * c->n_rows;
    const int64_t* off = f->row_offsets_host;
    if (off[0] != 0 || off[R] != f->n_clusters) return fail(c, TPCSF_E_INVALID, "row offsets do not span the clusters");
    int64_t max_row = 0;
    for (int64_t g = 0; g < R; ++g) {
        const int64_t d = off[g + 1] - off[g];
        if (d < 0) return fail(c, TPCSF_E_INVALID, "row offsets decrease");
        if (d >= 65535) return fail(c, TPCSF_E_INVALID, "a row holds 65535 clusters or more");
        if (d > max_row) max_row = d;
    }
    c->frame_max_row = max_row;
    // the grid kernel's LDS: bin counters (16-bit pairs) at the bin cap and the placement
    // of the largest row, rounded up to 4 KB; the less a block takes, the more row blocks
    // share a compute unit.  It only grows within a context (any size that holds the
    // largest row gives the same result), so that frames of different sizes keep one
    // launch configuration and one graph.  Rows beyond the device's limit take the
    // global-memory path.
    const int64_t need = 4 * ((c->tuning.cap_mul * max_row + c->tuning.cap_add + 2) / 2 + 1) + 2 * max_row + 256;
    int64_t fit = (need + 4095) / 4096 * 4096;
    if (fit > c->grid_lds_max) fit = c->grid_lds_max;
    if (fit > c->grid_lds_used) c->grid_lds_used = (int)fit;
    if (o->cap_tracks < 0 || o->cap_hits < 0 || !o->n_tracks || !o->n_hits || !o->hit_off)
        return fail(c, TPCSF_E_INVALID, "output descriptor incomplete");
    if (o->cap_tracks > 0 && (!o->params || !o->cov || !o->x_ref || !o->chi2 || !o->ndf || !o->nhits ||
                              !o->sector || !o->tf))
        return fail(c, TPCSF_E_INVALID, "track output arrays missing");
    if (o->cap_hits > 0 && !o->hit_ids) return fail(c, TPCSF_E_INVALID, "hit output array missing");
    if (f->n_clusters > 0 && !o->cluster_track) return fail(c, TPCSF_E_INVALID, "cluster_track missing");
    return TPCSF_OK;
}

tpcsf_status ensure_arena(tpcsf_ctx* c, const Layout& L)
{
    if (c->budget && L.total + c->marena_size + c->rarena_size > c->budget)
        return fail(c, TPCSF_E_NOMEM, "scratch of " + std::to_string(L.total) + " bytes exceeds the HBM budget");
    if (c->arena && c->arena_size >= L.total) return TPCSF_OK;
    hipError_t e;
    if (c->arena) {
        if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
        if ((e = hipFree(c->arena)) != hipSuccess) return hip_fail(c, e, "hipFree");
        c->arena = nullptr;
        c->arena_size = 0;
    }
    // reserved layouts are sized exactly; otherwise leave room for slightly larger batches
    const size_t want = c->reserve_n ? L.total : L.total + L.total / 8;
    const size_t sz = (c->budget && want + c->marena_size + c->rarena_size > c->budget) ? L.total : want;
    if ((e = hipMalloc(&c->arena, sz)) != hipSuccess) {
        c->arena = nullptr;
        return fail(c, TPCSF_E_NOMEM, std::string("hipMalloc of the arena: ") + hipGetErrorString(e));
    }
    c->arena_size = sz;
    return TPCSF_OK;
}

Batch make_batch(tpcsf_ctx* c, const Layout& L, const tpcsf_frame* f, const tpcsf_tracks* o, char* a)
{
    Batch B;
    B.y = f->y; B.z = f->z; B.off = f->row_offsets; B.n = L.n;
    B.n_rows_total = (int32_t)((int64_t)f->n_tf * c->n_sectors * c->n_rows);
    B.n_rows = c->n_rows;
    B.row_lo = (float2*)(a + L.row_lo);
    B.row_bin = (float2*)(a + L.row_bin);
    B.row_nb = (int2*)(a + L.row_nb);
    B.row_f = (float4*)(a + L.row_f);
    B.row_i = (int4*)(a + L.row_i);
    B.bin_start = (uint32_t*)(a + L.bin_start);
    B.yz = (float2*)(a + L.yz);
    B.perm = (uint32_t*)(a + L.perm);
    B.iperm = (uint32_t*)(a + L.iperm);
    B.upk = (int32_t*)(a + L.upk); B.dnk = (int32_t*)(a + L.dnk);
    B.cupk = (int32_t*)(a + L.cupk); B.cdnk = (int32_t*)(a + L.cdnk);
    B.row_nstart = (int64_t*)(a + L.row_nstart);
    B.row_sbase = (int64_t*)(a + L.row_sbase);
    B.rank_at = (int32_t*)(a + L.rank_at);
    B.st_row = (int32_t*)(a + L.st_row);
    B.st_k = (int32_t*)(a + L.st_k);
    B.st_rank = (int32_t*)(a + L.st_rank);
    B.cap_starts = L.cap_starts;
    B.tl_len = (int32_t*)(a + L.tl_len);
    B.order = (int32_t*)(a + L.order);
    B.tl_n = (int32_t*)(a + L.tl_n);
    B.tl_rlo = (int16_t*)(a + L.tl_rlo);
    B.tl_rhi = (int16_t*)(a + L.tl_rhi);
    B.tl_w = (uint32_t*)(a + L.tl_w);
    B.tl_hits = (uint16_t*)(a + L.tl_hits);
    B.keep_n = (int32_t*)(a + L.keep_n);
    B.fit_pos = (int64_t*)(a + L.fit_pos);
    B.fit_pos_long = (int64_t*)(a + L.fit_pos_long);
    B.cand_off = (int64_t*)(a + L.cand_off);
    B.kept_list = (float4*)(a + L.kept_list);
    B.keep_mask = (uint64_t*)(a + L.keep_mask);
    B.fit_list = (int32_t*)(a + L.fit_list);
    B.f_par = (double*)(a + L.f_par);
    B.f_cov = (double*)(a + L.f_cov);
    B.f_chi2 = (double*)(a + L.f_chi2);
    B.f_xref = (double*)(a + L.f_xref);
    const bool outer = o->params_outer && o->cov_outer;
    B.f_pout = outer ? (double*)(a + L.f_pout) : nullptr;
    B.f_cout = outer ? (double*)(a + L.f_cout) : nullptr;
    B.cap_fit = (int32_t)L.cap_fit;
    B.trk_flag = (int32_t*)(a + L.trk_flag);
    B.hit_cnt = (int32_t*)(a + L.hit_cnt);
    B.trk_idx = (int64_t*)(a + L.trk_idx);
    B.hit_pos = (int64_t*)(a + L.hit_pos);
    B.trk_out = (int32_t*)(a + L.trk_out);
    B.W = (uint32_t*)(a + L.W);
    B.scan_part = (int64_t*)(a + L.scan_part);
    B.ctr = c->d_ctr;
    B.cap_tracks = o->cap_tracks; B.cap_hits = o->cap_hits;
    B.o_ntracks = o->n_tracks; B.o_nhits = o->n_hits;
    B.o_par = o->params; B.o_cov = o->cov; B.o_xref = o->x_ref; B.o_chi2 = o->chi2;
    B.o_ndf = o->ndf; B.o_nhits_trk = o->nhits; B.o_sector = o->sector; B.o_tf = o->tf;
    B.o_hit_off = o->hit_off; B.o_hit_ids = o->hit_ids; B.o_cluster_track = o->cluster_track;
    B.o_zbeam = o->z_beam;
    B.o_par_out = outer ? o->params_outer : nullptr;
    B.o_cov_out = outer ? o->cov_outer : nullptr;
    B.o_hit_rec = (float4*)o->hit_rec;
    B.d_up = (int32_t*)(a + L.d_up); B.d_dn = (int32_t*)(a + L.d_dn);
    B.d_cup = (int32_t*)(a + L.d_cup); B.d_cdn = (int32_t*)(a + L.d_cdn);
    B.d_start_row = (int32_t*)(a + L.d_start_row);
    B.d_start_idx = (int32_t*)(a + L.d_start_idx);
    B.d_tl_n = (int32_t*)(a + L.d_tl_n);
    return B;
}

// The whole batch, one launch per stage; with `ev`, an event before each stage and after
// the last one (used only outside graph capture).
void enqueue_batch(const tpcsf_ctx* c, const Batch& B, hipStream_t s, hipEvent_t* ev)
{
    const DevParams P = dev_params(c);
    const LaunchCfg LC = launch_cfg(c);
    const int64_t R = B.n_rows_total;
    int k = 0;
    auto mark = [&]() {
        if (ev) (void)hipEventRecord(ev[k], s);
        ++k;
    };
    mark(); launch_reset(B, s);
    mark(); launch_grid(B, P, 0, R, LC, s);
    mark(); launch_links(B, P, 0, R, LC, s);
    mark(); launch_clean(B, P, 0, R, LC, s);
    mark(); launch_row_scan(B, 0, R, s);
    mark(); launch_starts(B, P, 0, R, LC, s);
    mark(); launch_walk(B, P, LC, s);
    launch_order(B, P, LC, s);
    mark(); launch_tracklets(B, P, LC, s);
    mark(); launch_claim(B, P, 0, R, LC, s);
    mark(); launch_keep(B, P, LC, s);
    launch_fit_scan(B, P, LC, s);
    mark(); launch_fit(B, P, LC, s);
    mark(); launch_track_scan(B, s);
    mark(); launch_emit(B, P, LC, s);
    mark(); launch_assign(B, P, 0, R, LC, s);
    mark();
}

// Scratch of one merge call: T = input track capacity, K = n_tf * n_sectors.
struct MergeLayout {
    size_t total = 0;
    size_t ends, a_list, a_idx, b_list, sec_first, cnt, brec, bidx, brec_s, bidx_s, zs, lsorted, mstate, bestB, bestChi,
        keepChi, keepA;
    size_t next, prev, nseg, chain_hits, fit_ok, diss, lead, nh, fit_list, seg_head, seg_pre, fit_off, grec, m_idx,
        m_hpos, scan_part;
};

MergeLayout make_merge_layout(int64_t T, int64_t K, int64_t H)
{
    MergeLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    const size_t t = (size_t)(T > 0 ? T : 1), k = (size_t)(K > 0 ? K : 1);
    L.ends = take(t * 16);
    L.a_list = take(t * 4);
    L.a_idx = take(t * 4);
    L.b_list = take(t * 4);
    L.sec_first = take(k * 4);
    L.cnt = take(2 * k * 4);
    L.brec = take(2 * t * 32);
    L.bidx = take(2 * t * 4);
    L.brec_s = take(2 * t * 32);
    L.bidx_s = take(2 * t * 4);
    L.zs = take(2 * t * 4);
    L.lsorted = take(2 * k * 4);
    L.mstate = take(t * 21 * 8);
    L.bestB = take(t * 4);
    L.bestChi = take(t * 8);
    L.keepChi = take(t * 8);
    L.keepA = take(t * 4);
    L.next = take(t * 4);
    L.prev = take(t * 4);
    L.nseg = take(t * 4);
    L.chain_hits = take(t * 4);
    L.fit_ok = take(t * 4);
    L.diss = take(t * 4);
    L.lead = take(t * 4);
    L.nh = take(t * 4);
    L.fit_list = take(t * 4);
    L.seg_head = take(t * 4);
    L.seg_pre = take(t * 4);
    L.fit_off = take(t * 8);
    L.grec = take((size_t)(H > 0 ? H : 1) * 16);
    L.m_idx = take(t * 8);
    L.m_hpos = take(t * 8);
    L.scan_part = take((4 * kScanBlocks + 2) * 8);
    L.total = o;
    return L;
}

}  // namespace

extern "C" tpcsf_status tpcsf_merge(tpcsf_ctx* c, const tpcsf_frame* f, const tpcsf_tracks* t, tpcsf_merged* o,
                                    void* stream)
{
    if (!c) return TPCSF_E_INVALID;
    if (!f || !t || !o) return fail(c, TPCSF_E_INVALID, "null frame, tracks or output");
    if (c->n_sectors < 2 || c->n_sectors % 2 || c->n_sectors / 2 > kMergeMaxSide)
        return fail(c, TPCSF_E_INVALID, "merging needs an even number of sectors, at most 128");
    if (f->n_tf < 1 || !f->row_offsets || !f->row_offsets_host || f->n_clusters < 0)
        return fail(c, TPCSF_E_INVALID, "frame incomplete");
    if (f->n_clusters > 0 && (!f->y || !f->z)) return fail(c, TPCSF_E_INVALID, "cluster arrays missing");
    const int64_t R = (int64_t)f->n_tf * c->n_sectors * c->n_rows;
    if (f->row_offsets_host[0] != 0 || f->row_offsets_host[R] != f->n_clusters)
        return fail(c, TPCSF_E_INVALID, "row offsets do not span the clusters");
    if (t->cap_tracks < 0 || !t->n_tracks || !t->hit_off)
        return fail(c, TPCSF_E_INVALID, "track input incomplete");
    if (t->cap_tracks > 0 && (!t->params || !t->cov || !t->x_ref || !t->chi2 || !t->sector || !t->tf ||
                              !t->hit_ids || !t->params_outer || !t->cov_outer))
        return fail(c, TPCSF_E_INVALID, "track input arrays missing (outer states are required)");
    if (t->cap_tracks >= ((int64_t)1 << 31) - 1) return fail(c, TPCSF_E_INVALID, "too many input tracks");
    if (o->cap_merged < 0 || o->cap_hits < 0 || !o->n_merged || !o->n_hits || !o->hit_off)
        return fail(c, TPCSF_E_INVALID, "merged output descriptor incomplete");
    if (o->cap_merged > 0 && (!o->params || !o->cov || !o->x_ref || !o->chi2 || !o->ndf || !o->nhits ||
                              !o->sector || !o->tf || !o->n_segments))
        return fail(c, TPCSF_E_INVALID, "merged output arrays missing");
    if (o->cap_hits > 0 && !o->hit_ids) return fail(c, TPCSF_E_INVALID, "merged hit array missing");
    if (t->cap_tracks > 0 && !o->track_merged) return fail(c, TPCSF_E_INVALID, "track_merged missing");
    const int64_t K = (int64_t)f->n_tf * c->n_sectors;
    const MergeLayout L = make_merge_layout(t->cap_tracks, K, t->cap_hits);
    hipError_t e;
    if (c->marena_size < L.total) {
        if (c->budget && c->arena_size + c->rarena_size + L.total > c->budget)
            return fail(c, TPCSF_E_NOMEM, "merge scratch of " + std::to_string(L.total) + " bytes exceeds the HBM budget");
        if (c->marena) {
            if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
            if ((e = hipFree(c->marena)) != hipSuccess) return hip_fail(c, e, "hipFree");
            c->marena = nullptr;
            c->marena_size = 0;
        }
        if ((e = hipMalloc(&c->marena, L.total)) != hipSuccess) {
            c->marena = nullptr;
            return fail(c, TPCSF_E_NOMEM, std::string("hipMalloc of the merge scratch: ") + hipGetErrorString(e));
        }
        c->marena_size = L.total;
    }
    if (!c->d_mc && (e = hipMalloc(&c->d_mc, sizeof(MergeCounters))) != hipSuccess) {
        c->d_mc = nullptr;
        return fail(c, TPCSF_E_NOMEM, "hipMalloc of the merge counters");
    }
    char* a = (char*)c->marena;
    MergeBatch M{};
    M.y = f->y; M.z = f->z; M.off = f->row_offsets;
    M.n_tracks = t->n_tracks; M.cap_tracks = t->cap_tracks; M.cap_in_hits = t->cap_hits;
    M.hit_off = t->hit_off; M.hit_ids = t->hit_ids;
    M.par = t->params; M.cov = t->cov; M.xref = t->x_ref; M.chi2 = t->chi2;
    M.sector = t->sector; M.tf = t->tf;
    M.par_out = t->params_outer; M.cov_out = t->cov_outer;
    M.hit_rec = (const float4*)t->hit_rec;
    M.n_tf = f->n_tf;
    M.ends = (float4*)(a + L.ends);
    M.a_list = (int32_t*)(a + L.a_list);
    M.a_idx = (int32_t*)(a + L.a_idx);
    M.b_list = (int32_t*)(a + L.b_list);
    M.sec_first = (int32_t*)(a + L.sec_first);
    M.cnt = (int32_t*)(a + L.cnt);
    M.brec = (double4*)(a + L.brec);
    M.bidx = (int32_t*)(a + L.bidx);
    M.brec_s = (double4*)(a + L.brec_s);
    M.bidx_s = (int32_t*)(a + L.bidx_s);
    M.zs = (float*)(a + L.zs);
    M.lsorted = (int32_t*)(a + L.lsorted);
    M.mstate = (double*)(a + L.mstate);
    M.bestB = (int32_t*)(a + L.bestB);
    M.bestChi = (double*)(a + L.bestChi);
    M.keepChi = (unsigned long long*)(a + L.keepChi);
    M.keepA = (int32_t*)(a + L.keepA);
    M.next = (int32_t*)(a + L.next);
    M.prev = (int32_t*)(a + L.prev);
    M.nseg = (int32_t*)(a + L.nseg);
    M.chain_hits = (int32_t*)(a + L.chain_hits);
    M.fit_ok = (int32_t*)(a + L.fit_ok);
    M.diss = (int32_t*)(a + L.diss);
    M.lead = (int32_t*)(a + L.lead);
    M.nh = (int32_t*)(a + L.nh);
    M.fit_list = (int32_t*)(a + L.fit_list);
    M.seg_head = (int32_t*)(a + L.seg_head);
    M.seg_pre = (int32_t*)(a + L.seg_pre);
    M.fit_off = (int64_t*)(a + L.fit_off);
    M.grec = (float4*)(a + L.grec);
    M.m_idx = (int64_t*)(a + L.m_idx);
    M.m_hpos = (int64_t*)(a + L.m_hpos);
    M.scan_part = (int64_t*)(a + L.scan_part);
    M.mc = c->d_mc;
    M.ctr = c->d_ctr;
    M.cap_merged = o->cap_merged; M.cap_hits = o->cap_hits;
    M.o_n = o->n_merged; M.o_nhits = o->n_hits;
    M.o_par = o->params; M.o_cov = o->cov; M.o_xref = o->x_ref; M.o_chi2 = o->chi2; M.o_zbeam = o->z_beam;
    M.o_ndf = o->ndf; M.o_nhits_trk = o->nhits; M.o_sector = o->sector; M.o_tf = o->tf;
    M.o_nseg = o->n_segments;
    M.o_hit_off = o->hit_off; M.o_hit_ids = o->hit_ids;
    M.o_track_merged = o->track_merged; M.o_next = o->next; M.o_link_chi2 = o->link_chi2;
    MergeParams Q{};
    const tpcsf_params& p = c->params;
    Q.edge = p.merge_edge; Q.window = p.merge_window; Q.chi2 = p.merge_chi2;
    Q.S = c->n_sectors / 2;
    const double pi = 3.14159265358979323846;
    Q.te = std::tan(pi / Q.S);
    for (int d = -(Q.S - 1) / 2; d <= Q.S / 2; ++d) {
        const double delta = d * (2.0 * pi / Q.S);
        Q.rc[d + Q.S / 2] = std::cos(delta);
        Q.rs[d + Q.S / 2] = std::sin(delta);
    }
    launch_merge(M, dev_params(c), Q, c->n_cu, (hipStream_t)stream);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "merge kernel launch");
    return TPCSF_OK;
}

namespace {

// Scratch of the hit removal: the (track, row) pairs of the vicinities bucketed by row.
// A track contributes at most one pair per row, so cap_tracks * n_rows bounds the pairs.
struct RejectLayout {
    size_t total = 0;
    int64_t cap_items = 0;
    size_t rspan, rdiff, rcnt, rtmp, roff, rcur, ritems, scan_part;
};

RejectLayout make_reject_layout(int64_t T, int64_t R, int n_rows)
{
    RejectLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    const size_t t = (size_t)(T > 0 ? T : 1), r = (size_t)(R > 0 ? R : 1);
    L.cap_items = (int64_t)t * n_rows;
    L.rspan = take(t * 8);
    L.rdiff = take((r + 1) * 4);
    L.rcnt = take(r * 4);
    L.rtmp = take((r + 1) * 8);
    L.roff = take((r + 1) * 8);
    L.rcur = take(r * 4);
    L.ritems = take((size_t)L.cap_items * 4);
    L.scan_part = take((4 * kScanBlocks + 2) * 8);
    L.total = o;
    return L;
}

}  // namespace

extern "C" tpcsf_status tpcsf_reject(tpcsf_ctx* c, const tpcsf_frame* f, const tpcsf_tracks* t, uint8_t* keep,
                                     int64_t* n_kept, void* stream)
{
    if (!c) return TPCSF_E_INVALID;
    if (!f || !t || !n_kept || (f->n_clusters > 0 && !keep)) return fail(c, TPCSF_E_INVALID, "null argument");
    const int64_t R = (int64_t)f->n_tf * c->n_sectors * c->n_rows;
    if (!c->have_last || c->last.y != f->y || c->last.z != f->z || c->last.off != f->row_offsets ||
        (int64_t)c->last.n_rows_total != R)
        return fail(c, TPCSF_E_INVALID, "tpcsf_reject needs the frame of the context's last tracking call");
    if (t->cap_tracks < 0 || !t->n_tracks || !t->hit_off) return fail(c, TPCSF_E_INVALID, "track input incomplete");
    if (t->cap_tracks > 0 && (!t->params || !t->x_ref || !t->sector || !t->tf || !t->hit_ids))
        return fail(c, TPCSF_E_INVALID, "track input arrays missing");
    if (f->n_clusters > 0 && !t->cluster_track) return fail(c, TPCSF_E_INVALID, "cluster_track missing");
    RejectArgs A{};
    A.n_tracks = t->n_tracks; A.cap_tracks = t->cap_tracks; A.cap_hits = t->cap_hits;
    A.par = t->params; A.xref = t->x_ref; A.sector = t->sector; A.tf = t->tf;
    A.hit_off = t->hit_off; A.hit_ids = t->hit_ids; A.cluster_track = t->cluster_track;
    A.n_tf = f->n_tf;
    A.pt_min = c->params.reject_pt_min;
    A.window = c->params.reject_window;
    A.keep = keep;
    A.n_kept = n_kept;
    const RejectLayout L = make_reject_layout(t->cap_tracks, R, c->n_rows);
    hipError_t e;
    if (c->rarena_size < L.total) {
        if (c->budget && c->arena_size + c->marena_size + L.total > c->budget)
            return fail(c, TPCSF_E_NOMEM, "reject scratch of " + std::to_string(L.total) + " bytes exceeds the HBM budget");
        if (c->rarena) {
            if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
            if ((e = hipFree(c->rarena)) != hipSuccess) return hip_fail(c, e, "hipFree");
            c->rarena = nullptr;
            c->rarena_size = 0;
        }
        if ((e = hipMalloc(&c->rarena, L.total)) != hipSuccess) {
            c->rarena = nullptr;
            return fail(c, TPCSF_E_NOMEM, std::string("hipMalloc of the reject scratch: ") + hipGetErrorString(e));
        }
        c->rarena_size = L.total;
    }
    char* ra = (char*)c->rarena;
    A.rspan = (int32_t*)(ra + L.rspan);
    A.rdiff = (int32_t*)(ra + L.rdiff);
    A.rcnt = (int32_t*)(ra + L.rcnt);
    A.rtmp = (int64_t*)(ra + L.rtmp);
    A.roff = (int64_t*)(ra + L.roff);
    A.rcur = (int32_t*)(ra + L.rcur);
    A.ritems = (int32_t*)(ra + L.ritems);
    A.cap_items = L.cap_items;
    A.scan_part = (int64_t*)(ra + L.scan_part);
    A.n_rows_total = (int32_t)R;
    Batch B = c->last;
    B.n = f->n_clusters;
    launch_reject(B, c->last_P, A, launch_cfg(c), (hipStream_t)stream);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "reject kernel launch");
    return TPCSF_OK;
}

extern "C" tpcsf_status tpcsf_compress(tpcsf_ctx* c, const tpcsf_frame* f, const tpcsf_tracks* t, int32_t* codes,
                                       uint8_t* rows, void* stream)
{
    if (!c) return TPCSF_E_INVALID;
    if (!f || !t) return fail(c, TPCSF_E_INVALID, "null frame or tracks");
    if (f->n_tf < 1 || !f->row_offsets || f->n_clusters < 0 || (f->n_clusters > 0 && (!f->y || !f->z)))
        return fail(c, TPCSF_E_INVALID, "frame incomplete");
    if (t->cap_tracks < 0 || t->cap_hits < 0 || !t->n_tracks || !t->hit_off)
        return fail(c, TPCSF_E_INVALID, "track input incomplete");
    if (t->cap_tracks > 0 && (!t->params || !t->x_ref || !t->sector || !t->tf || !t->hit_ids))
        return fail(c, TPCSF_E_INVALID, "track input arrays missing");
    if (t->cap_hits > 0 && (!codes || !rows)) return fail(c, TPCSF_E_INVALID, "code outputs missing");
    CompressArgs A{};
    A.n_tracks = t->n_tracks; A.cap_tracks = t->cap_tracks; A.cap_hits = t->cap_hits;
    A.par = t->params; A.xref = t->x_ref; A.sector = t->sector; A.tf = t->tf;
    A.hit_off = t->hit_off; A.hit_ids = t->hit_ids;
    A.y = f->y; A.z = f->z; A.off = f->row_offsets; A.n_tf = f->n_tf;
    A.hit_rec = (const float4*)t->hit_rec;
    A.step = c->params.resid_step;
    A.codes = codes; A.rows = rows;
    launch_compress(A, dev_params(c), c->n_cu, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "compress kernel launch");
    return TPCSF_OK;
}

extern "C" tpcsf_status tpcsf_decompress(tpcsf_ctx* c, const tpcsf_tracks* t, const int32_t* codes,
                                         const uint8_t* rows, double* yz, void* stream)
{
    if (!c) return TPCSF_E_INVALID;
    if (!t || t->cap_tracks < 0 || t->cap_hits < 0 || !t->n_tracks || !t->hit_off)
        return fail(c, TPCSF_E_INVALID, "track input incomplete");
    if (t->cap_tracks > 0 && (!t->params || !t->x_ref)) return fail(c, TPCSF_E_INVALID, "track input arrays missing");
    if (t->cap_hits > 0 && (!codes || !rows || !yz)) return fail(c, TPCSF_E_INVALID, "code arrays missing");
    CompressArgs A{};
    A.n_tracks = t->n_tracks; A.cap_tracks = t->cap_tracks; A.cap_hits = t->cap_hits;
    A.par = t->params; A.xref = t->x_ref; A.hit_off = t->hit_off;
    A.step = c->params.resid_step;
    A.codes = const_cast<int32_t*>(codes);
    A.rows = const_cast<uint8_t*>(rows);
    A.yz = yz;
    launch_decompress(A, dev_params(c), c->n_cu, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "decompress kernel launch");
    return TPCSF_OK;
}

extern "C" tpcsf_status tpcsf_merge_work(tpcsf_ctx* c, int64_t* work6)
{
    if (!c || !work6) return TPCSF_E_INVALID;
    if (!c->d_mc) return fail(c, TPCSF_E_INVALID, "no merge call yet");
    MergeCounters mc;
    hipError_t e = hipMemcpy(&mc, c->d_mc, sizeof mc, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "reading the merge counters");
    for (int k = 0; k < 6; ++k) work6[k] = mc.work[k];
    return TPCSF_OK;
}

extern "C" {

void tpcsf_default_params(tpcsf_params* p)
{
    if (!p) return;
    p->win_y = 3.0f;
    p->win_z = 3.0f;
    p->kink_max = 1.0f;
    p->sigma_y = 0.1;
    p->sigma_z = 0.1;
    p->chi2_max = 16.0;
    p->sinphi_max = 0.99;
    p->nsig = 5.0;
    p->c0[0] = 1.0; p->c0[1] = 1.0; p->c0[2] = 1.0; p->c0[3] = 1.0; p->c0[4] = 100.0;
    p->min_chain = 5;
    p->min_track_hits = 20;
    p->max_miss = 4;
    p->merge_edge = 6.0;
    p->merge_window = 5.0;
    p->merge_chi2 = 30.0;
    p->reject_pt_min = 0.05;
    p->reject_window = 1.0;
    p->resid_step = 0.01;
}

void tpcsf_default_tuning(tpcsf_tuning* t)
{
    if (!t) return;
    t->bin_y = 2.0f;
    t->bin_z = 2.0f;
    t->cap_mul = 2;
    t->cap_add = 64;
    t->block = 256;
    t->tl_block = 256;
    t->chunk = 1;
}

tpcsf_status tpcsf_create(const tpcsf_geometry* geo, const tpcsf_params* params, const tpcsf_tuning* tuning,
                          size_t hbm_budget_bytes, tpcsf_ctx** out)
{
    if (!out) return TPCSF_E_INVALID;
    *out = nullptr;
    if (!geo || !geo->row_x || geo->n_sectors < 1 || geo->n_rows < 3 || geo->n_rows > kMaxRowsGeo)
        return TPCSF_E_INVALID;
    for (int r = 0; r + 1 < geo->n_rows; ++r)
        if (!(geo->row_x[r + 1] > geo->row_x[r])) return TPCSF_E_INVALID;
    if (!(geo->bz == geo->bz) || geo->bz > 100.0 || geo->bz < -100.0) return TPCSF_E_INVALID;
    tpcsf_params p;
    tpcsf_tuning t;
    if (params) p = *params; else tpcsf_default_params(&p);
    if (tuning) t = *tuning; else tpcsf_default_tuning(&t);
    if (!params_ok(&p) || !tuning_ok(&t)) return TPCSF_E_INVALID;
    tpcsf_ctx* c = new tpcsf_ctx();
    c->n_sectors = geo->n_sectors;
    c->n_rows = geo->n_rows;
    c->row_x.assign(geo->row_x, geo->row_x + geo->n_rows);
    c->bz = geo->bz;
    c->params = p;
    c->tuning = t;
    c->budget = hbm_budget_bytes;
    hipError_t e;
    if ((e = hipGetDevice(&c->device)) != hipSuccess) { delete c; return TPCSF_E_HIP; }
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, c->device)) != hipSuccess) { delete c; return TPCSF_E_HIP; }
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    c->grid_lds_max = grid_lds_setup((int)prop.sharedMemPerBlock);
    if ((e = scratch_setup(c->device, &c->fixed_scratch)) != hipSuccess) { delete c; return TPCSF_E_HIP; }
    if ((e = hipMalloc(&c->d_rx, sizeof(float) * c->n_rows)) != hipSuccess) { delete c; return TPCSF_E_NOMEM; }
    if ((e = hipMalloc(&c->d_ctr, sizeof(Counters))) != hipSuccess) {
        (void)hipFree(c->d_rx);
        delete c;
        return TPCSF_E_NOMEM;
    }
    (void)hipMemcpy(c->d_rx, c->row_x.data(), sizeof(float) * c->n_rows, hipMemcpyHostToDevice);
    Counters zero{};
    (void)hipMemcpy(c->d_ctr, &zero, sizeof(Counters), hipMemcpyHostToDevice);
    if ((e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) != hipSuccess) {
        (void)hipFree(c->d_rx);
        (void)hipFree(c->d_ctr);
        delete c;
        return TPCSF_E_HIP;
    }
    *out = c;
    return TPCSF_OK;
}

tpcsf_status tpcsf_destroy(tpcsf_ctx* c)
{
    if (!c) return TPCSF_E_INVALID;
    (void)hipDeviceSynchronize();
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->arena) (void)hipFree(c->arena);
    if (c->marena) (void)hipFree(c->marena);
    if (c->rarena) (void)hipFree(c->rarena);
    if (c->d_mc) (void)hipFree(c->d_mc);
    for (int i = 0; i <= kStages; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    if (c->d_rx) (void)hipFree(c->d_rx);
    if (c->d_ctr) (void)hipFree(c->d_ctr);
    delete c;
    return TPCSF_OK;
}

tpcsf_status tpcsf_set_tuning(tpcsf_ctx* c, const tpcsf_tuning* t)
{
    if (!c) return TPCSF_E_INVALID;
    if (!tuning_ok(t)) return fail(c, TPCSF_E_INVALID, "tuning out of range");
    c->tuning = *t;
    c->grid_lds_used = 0;   // the grid's LDS need depends on the bin cap
    return TPCSF_OK;
}

size_t tpcsf_arena_bytes(const tpcsf_ctx* c, int64_t n_clusters, int32_t n_tf)
{
    if (!c || n_clusters < 0 || n_tf < 1) return 0;
    return make_layout(c, n_clusters, n_tf).total;
}

tpcsf_status tpcsf_track_plain(tpcsf_ctx* c, const tpcsf_frame* f, tpcsf_tracks* o, void* stream)
{
    if (!c) return TPCSF_E_INVALID;
    tpcsf_status st = check_frame(c, f, o);
    if (st != TPCSF_OK) return st;
    const Layout L = make_layout(c, f->n_clusters, f->n_tf);
    if ((st = ensure_arena(c, L)) != TPCSF_OK) return st;
    c->lay = L;
    const Batch B = make_batch(c, L, f, o, (char*)c->arena);
    const DevParams P = dev_params(c);
    const LaunchCfg LC = launch_cfg(c);
    hipStream_t s = (hipStream_t)stream;
    launch_reset(B, s);
    for (int32_t tf = 0; tf < f->n_tf; ++tf)
        for (int32_t sec = 0; sec < c->n_sectors; ++sec) {
            const int64_t g0 = ((int64_t)tf * c->n_sectors + sec) * c->n_rows;
            const int64_t g1 = g0 + c->n_rows;
            launch_grid(B, P, g0, g1, LC, s);
            launch_links(B, P, g0, g1, LC, s);
            launch_clean(B, P, g0, g1, LC, s);
            launch_row_scan(B, g0, g1, s);
            launch_starts(B, P, g0, g1, LC, s);
            launch_walk(B, P, LC, s);
            launch_order(B, P, LC, s);
            launch_tracklets(B, P, LC, s);
            launch_claim(B, P, g0, g1, LC, s);
            launch_keep(B, P, LC, s);
            launch_fit_scan(B, P, LC, s);
            launch_fit(B, P, LC, s);
            launch_track_scan(B, s);
            launch_emit(B, P, LC, s);
            launch_assign(B, P, g0, g1, LC, s);
        }
    c->last = B;
    c->last_P = dev_params(c);
    c->have_last = true;
    c->timed_last = false;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
    return TPCSF_OK;
}

tpcsf_status tpcsf_track_batch(tpcsf_ctx* c, const tpcsf_frame* f, tpcsf_tracks* o, void* stream)
{
    if (!c) return TPCSF_E_INVALID;
    tpcsf_status st = check_frame(c, f, o);
    if (st != TPCSF_OK) return st;
    const Layout L = make_layout(c, f->n_clusters, f->n_tf);
    if ((st = ensure_arena(c, L)) != TPCSF_OK) return st;
    c->lay = L;
    const Batch B = make_batch(c, L, f, o, (char*)c->arena);
    GraphKey k;
    std::memset(&k, 0, sizeof k);
    // the layout (not the cluster count) fixes every kernel argument
    k.y = f->y; k.z = f->z; k.off = f->row_offsets; k.n = L.n; k.R = B.n_rows_total;
    k.arena = c->arena;
    k.out = *o;
    k.tuning = c->tuning;
    k.grid_lds = launch_cfg(c).grid_lds;
    hipError_t e;
    if (c->timing) {
        // timed calls run the same launch sequence eagerly on the caller's stream, with an
        // event between stages (event timing is not available inside graphs here)
        enqueue_batch(c, B, (hipStream_t)stream, c->ev);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "kernel launch");
        c->timed_last = true;
        c->last = B;
        c->last_P = dev_params(c);
        c->have_last = true;
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "kernel launch");
        return TPCSF_OK;
    }
    if (!c->gexec || !(k == c->gkey)) {
        if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
        if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
        if ((e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(c, e, "hipStreamBeginCapture");
        enqueue_batch(c, B, c->cap_stream, nullptr);
        const hipError_t le = hipGetLastError();
        if ((e = hipStreamEndCapture(c->cap_stream, &c->graph)) != hipSuccess)
            return hip_fail(c, e, "hipStreamEndCapture");
        if (le != hipSuccess) {
            (void)hipGraphDestroy(c->graph);
            c->graph = nullptr;
            return hip_fail(c, le, "kernel launch during capture");
        }
        if ((e = hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0)) != hipSuccess) {
            (void)hipGraphDestroy(c->graph);
            c->graph = nullptr;
            c->gexec = nullptr;
            return hip_fail(c, e, "hipGraphInstantiate");
        }
        c->gkey = k;
    }
    if ((e = hipGraphLaunch(c->gexec, (hipStream_t)stream)) != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
    c->timed_last = false;
    c->last = B;
    c->last_P = dev_params(c);
    c->have_last = true;
    return TPCSF_OK;
}

tpcsf_status tpcsf_track_batch_noalloc(tpcsf_ctx* c, const tpcsf_frame* f, tpcsf_tracks* o, void* stream)
{
    if (!c) return TPCSF_E_INVALID;
    tpcsf_status st = check_frame(c, f, o);
    if (st != TPCSF_OK) return st;
    if (!c->fixed_scratch) return fail(c, TPCSF_E_HIP, "the fixed scratch array of this device is not set up");
    // the exact layout of this batch (no reservation), inside the fixed array
    const Layout L = make_layout(c, f->n_clusters, f->n_tf, false);
    if (L.total > (size_t)TPCSF_NOALLOC_SCRATCH_BYTES)
        return fail(c, TPCSF_E_NOMEM, "the batch needs " + std::to_string(L.total) +
                                          " bytes of scratch; the fixed array of tpcsf_track_batch_noalloc holds " +
                                          std::to_string((size_t)TPCSF_NOALLOC_SCRATCH_BYTES));
    const Batch B = make_batch(c, L, f, o, (char*)c->fixed_scratch);
    // eager launches: the same sequence as the batched form's graph, no allocation
    enqueue_batch(c, B, (hipStream_t)stream, nullptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
    c->timed_last = false;
    c->last = B;
    c->last_P = dev_params(c);
    c->have_last = true;
    return TPCSF_OK;
}

tpcsf_status tpcsf_sync(tpcsf_ctx* c, void* stream)
{
    if (!c) return TPCSF_E_INVALID;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    int32_t err = 0;
    if ((e = hipMemcpy(&err, &c->d_ctr->err, sizeof(err), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(c, e, "reading the error word");
    if (err) {
        const int32_t zero = 0;
        (void)hipMemcpy(&c->d_ctr->err, &zero, sizeof(zero), hipMemcpyHostToDevice);
    }
    if (err & kErrInvalid) return fail(c, TPCSF_E_INVALID, "non-finite or out-of-range cluster coordinates");
    if (err & kErrOutCap) return fail(c, TPCSF_E_CAPACITY, "output capacity too small");
    if (err & kErrTrackletCap) return fail(c, TPCSF_E_CAPACITY, "tracklet slots exhausted");
    if (err & kErrMergeChain) return fail(c, TPCSF_E_INVALID, "a merged chain exceeds the walk bound");
    return TPCSF_OK;
}

tpcsf_status tpcsf_debug(tpcsf_ctx* c, tpcsf_debug_view* v)
{
    if (!c || !v || !c->have_last) return TPCSF_E_INVALID;
    const Batch& B = c->last;
    // the working arrays are in sorted (bin) order; convert to input order on request
    hipError_t e;
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
    launch_debug_views(B, dev_params(c), launch_cfg(c), c->cap_stream);
    if ((e = hipStreamSynchronize(c->cap_stream)) != hipSuccess) return hip_fail(c, e, "debug views");
    v->row_lo = (const float*)B.row_lo;
    v->row_bin = (const float*)B.row_bin;
    v->row_nb = (const int32_t*)B.row_nb;
    v->bin_start = B.bin_start;
    v->perm = B.perm;
    v->up = B.d_up; v->dn = B.d_dn; v->cup = B.d_cup; v->cdn = B.d_cdn;
    v->n_starts = &c->d_ctr->start_base;
    v->start_row = B.d_start_row;
    v->start_idx = B.d_start_idx;
    v->tl_nhits = B.d_tl_n;
    v->work = c->d_ctr->work;
    return TPCSF_OK;
}

tpcsf_status tpcsf_reserve(tpcsf_ctx* c, int64_t max_clusters, int32_t max_tf)
{
    if (!c || max_clusters < 0 || max_clusters >= ((int64_t)1 << 31) - 1 || max_tf < 0) return TPCSF_E_INVALID;
    c->reserve_n = max_clusters;
    c->reserve_tf = max_tf;
    return ensure_arena(c, make_layout(c, max_clusters, max_tf > 0 ? max_tf : 1));
}

tpcsf_status tpcsf_autotune(tpcsf_ctx* c, const tpcsf_frame* f, tpcsf_tracks* o, const tpcsf_tuning* points,
                            int32_t n_points, int32_t reps, float* ms_out, int32_t* best, void* stream)
{
    if (!c || !points || n_points < 1 || reps < 1) return TPCSF_E_INVALID;
    for (int i = 0; i < n_points; ++i)
        if (!tuning_ok(&points[i])) return fail(c, TPCSF_E_INVALID, "tuning point " + std::to_string(i) + " out of range");
    const tpcsf_tuning saved = c->tuning;
    const int32_t timing = c->timing;
    c->timing = 0;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
        return hip_fail(c, e, "hipEventCreate");
    unsigned long long ref = 0;
    float best_ms = 0.0f;
    int32_t best_i = -1;
    tpcsf_status st = TPCSF_OK;
    for (int i = 0; i < n_points && st == TPCSF_OK; ++i) {
        c->tuning = points[i];
        c->grid_lds_used = 0;   // the grid's LDS need depends on the bin cap
        if ((st = tpcsf_track_batch(c, f, o, stream)) != TPCSF_OK) break;
        launch_hash(c->last, f->n_clusters, launch_cfg(c), s);
        if ((st = tpcsf_sync(c, stream)) != TPCSF_OK) break;
        unsigned long long h = 0;
        if ((e = hipMemcpy(&h, &c->d_ctr->hash, sizeof(h), hipMemcpyDeviceToHost)) != hipSuccess) {
            st = hip_fail(c, e, "reading the output digest");
            break;
        }
        if (i == 0) {
            ref = h;
        } else if (h != ref) {
            st = fail(c, TPCSF_E_INVALID, "tuning point " + std::to_string(i) + " changed the result");
            break;
        }
        (void)hipEventRecord(e0, s);
        for (int k = 0; k < reps && st == TPCSF_OK; ++k) st = tpcsf_track_batch(c, f, o, stream);
        (void)hipEventRecord(e1, s);
        if (st != TPCSF_OK) break;
        if ((st = tpcsf_sync(c, stream)) != TPCSF_OK) break;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)reps;
        if (ms_out) ms_out[i] = ms;
        if (best_i < 0 || ms < best_ms) { best_ms = ms; best_i = i; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->timing = timing;
    if (st != TPCSF_OK || best_i < 0) {
        c->tuning = saved;
        c->grid_lds_used = 0;   // the grid's LDS need depends on the bin cap
        return st != TPCSF_OK ? st : TPCSF_E_INVALID;
    }
    c->tuning = points[best_i];
    c->grid_lds_used = 0;   // the grid's LDS need depends on the bin cap
    if (best) *best = best_i;
    return TPCSF_OK;
}

tpcsf_status tpcsf_set_stage_timing(tpcsf_ctx* c, int32_t on)
{
    if (!c) return TPCSF_E_INVALID;
    if (on && !c->ev[0]) {
        for (int i = 0; i <= kStages; ++i) {
            hipError_t e = hipEventCreate(&c->ev[i]);
            if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
        }
    }
    c->timing = on ? 1 : 0;
    return TPCSF_OK;
}

int32_t tpcsf_stage_count(void) { return kStages; }

const char* tpcsf_stage_name(int32_t i) { return (i >= 0 && i < kStages) ? kStageNames[i] : ""; }

tpcsf_status tpcsf_stage_times(tpcsf_ctx* c, float* ms, int32_t n)
{
    if (!c || !ms) return TPCSF_E_INVALID;
    if (!c->timed_last) return fail(c, TPCSF_E_INVALID, "the last call was not a timed batched call");
    for (int i = 0; i < kStages && i < n; ++i) {
        hipError_t e = hipEventElapsedTime(&ms[i], c->ev[i], c->ev[i + 1]);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventElapsedTime");
    }
    return TPCSF_OK;
}

const char* tpcsf_last_error(const tpcsf_ctx* c)
{
    return c ? c->err.c_str() : "null context";
}

}  // extern "C"
