// Serving layer of libtpcsf: continuous batching of time frames that arrive over time.
//
// The paper processes every time frame independently and whole, reusing GPU memory
// across the steps of one frame (Sec. 7.1); frames are the unit of work of the online
// farm.  A server owns n_slots slots.  A slot is a tracking context with its own HIP
// stream, device input/output buffers and pinned host output buffers, all sized on first
// use and grown on demand, and a scratch layout reserved to that size so that one HIP
// graph serves every frame the slot takes.  A frame is admitted into any free slot whose
// growth stays inside the HBM budget; its upload, tracking and the download of its track
// and hit counts are enqueued on the slot's stream, so frames in different slots overlap
// on the device.  Once those counts are on the host, the next poll (or wait) of the frame
// enqueues the download of exactly that many tracks and hits.  Admission never waits:
// without a slot or budget it returns TPCSF_E_BUSY (an admission stall).
#include "tpcsf.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

enum SlotState { kFree = 0, kBusy = 1 };

struct Slot {
    tpcsf_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t tracked = nullptr;      // tracking done, counts on the host
    hipEvent_t done = nullptr;         // outputs on the host
    int64_t cap = 0;                   // clusters the buffers hold
    size_t bytes = 0;                  // device bytes held (buffers + scratch)
    // device inputs
    float* d_y = nullptr; float* d_z = nullptr; int64_t* d_off = nullptr;
    // device outputs
    int64_t* d_n = nullptr;            // [2] n_tracks, n_hits
    double* d_par = nullptr; double* d_cov = nullptr; double* d_x = nullptr; double* d_chi2 = nullptr;
    double* d_zb = nullptr;
    int32_t* d_ndf = nullptr; int32_t* d_nh = nullptr; int32_t* d_sec = nullptr; int32_t* d_tf = nullptr;
    int64_t* d_hoff = nullptr; int32_t* d_hid = nullptr; int32_t* d_ct = nullptr;
    // pinned host outputs
    int64_t* h_n = nullptr;
    double* h_par = nullptr; double* h_cov = nullptr; double* h_x = nullptr; double* h_chi2 = nullptr;
    double* h_zb = nullptr;
    int32_t* h_ndf = nullptr; int32_t* h_nh = nullptr; int32_t* h_sec = nullptr;
    int64_t* h_hoff = nullptr; int32_t* h_hid = nullptr; int32_t* h_ct = nullptr;
    std::vector<int64_t> h_off;        // host row offsets of the frame being tracked
    int state = kFree;
    uint64_t ticket = 0;
    int64_t n = 0;
    tpcsf_status status = TPCSF_OK;
    bool downloading = false;          // the output downloads are enqueued
    bool finished = false;
};

int64_t cap_tracks_for(int64_t n, int min_hits) { return n / (min_hits > 1 ? min_hits : 1) + 1; }

}  // namespace

struct tpcsf_server {
    tpcsf_geometry geo{};
    std::vector<float> row_x;
    tpcsf_params params{};
    tpcsf_tuning tuning{};
    size_t budget = 0;
    size_t used = 0;
    std::vector<Slot> slots;
    uint64_t next_ticket = 1;
    std::mutex mu;
    std::string err;
};

namespace {

tpcsf_status srv_fail(tpcsf_server* s, tpcsf_status st, const std::string& m)
{
    s->err = m;
    return st;
}

void free_slot_buffers(Slot& sl)
{
    void* dev[] = {sl.d_y, sl.d_z, sl.d_off, sl.d_n, sl.d_par, sl.d_cov, sl.d_x, sl.d_chi2, sl.d_zb, sl.d_ndf,
                   sl.d_nh, sl.d_sec, sl.d_tf, sl.d_hoff, sl.d_hid, sl.d_ct};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    void* host[] = {sl.h_n, sl.h_par, sl.h_cov, sl.h_x, sl.h_chi2, sl.h_zb, sl.h_ndf, sl.h_nh, sl.h_sec,
                    sl.h_hoff, sl.h_hid, sl.h_ct};
    for (void* p : host)
        if (p) (void)hipHostFree(p);
    sl.d_y = sl.d_z = nullptr; sl.d_off = nullptr; sl.d_n = nullptr;
    sl.d_par = sl.d_cov = sl.d_x = sl.d_chi2 = sl.d_zb = nullptr;
    sl.d_ndf = sl.d_nh = sl.d_sec = sl.d_tf = nullptr; sl.d_hoff = nullptr; sl.d_hid = sl.d_ct = nullptr;
    sl.h_n = nullptr; sl.h_par = sl.h_cov = sl.h_x = sl.h_chi2 = sl.h_zb = nullptr;
    sl.h_ndf = sl.h_nh = sl.h_sec = nullptr; sl.h_hoff = nullptr; sl.h_hid = sl.h_ct = nullptr;
}

// Device bytes a slot needs for a capacity of `cap` clusters in one time frame.
size_t slot_bytes(const tpcsf_server* s, int64_t cap)
{
    const int64_t R = (int64_t)s->geo.n_sectors * s->geo.n_rows;
    const int64_t T = cap_tracks_for(cap, s->params.min_track_hits);
    size_t io = (size_t)cap * (4 + 4) + (size_t)(R + 1) * 8 + 16;
    io += (size_t)T * (5 + 15 + 1 + 1 + 1) * 8 + (size_t)T * 4 * 4 + (size_t)(T + 1) * 8 + (size_t)cap * 8;
    return io;
}

template <typename T>
hipError_t dmalloc(T** p, size_t count) { return hipMalloc((void**)p, sizeof(T) * (count > 0 ? count : 1)); }
template <typename T>
hipError_t hmalloc(T** p, size_t count) { return hipHostMalloc((void**)p, sizeof(T) * (count > 0 ? count : 1), 0); }

// Grow a free slot to hold `n` clusters; TPCSF_E_BUSY (nothing changed) if the budget forbids.
tpcsf_status grow_slot(tpcsf_server* s, Slot& sl, int64_t n)
{
    if (sl.ctx && sl.cap >= n) return TPCSF_OK;
    int64_t cap = sl.cap > 0 ? sl.cap : 1;
    while (cap < n) cap *= 2;
    if (cap > ((int64_t)1 << 31) - 2) cap = ((int64_t)1 << 31) - 2;
    // the scratch of a fresh context for this capacity
    tpcsf_ctx* probe = sl.ctx;
    if (!probe) {
        tpcsf_status st = tpcsf_create(&s->geo, &s->params, &s->tuning, 0, &probe);
        if (st != TPCSF_OK) return srv_fail(s, st, "tpcsf_create failed");
    }
    const size_t need = tpcsf_arena_bytes(probe, cap, 1) + slot_bytes(s, cap);
    const size_t rel = sl.bytes;
    if (s->budget && s->used - rel + need > s->budget) {
        if (!sl.ctx) (void)tpcsf_destroy(probe);
        return TPCSF_E_BUSY;
    }
    sl.ctx = probe;
    (void)hipStreamSynchronize(sl.stream);
    free_slot_buffers(sl);
    const int64_t R = (int64_t)s->geo.n_sectors * s->geo.n_rows;
    const int64_t T = cap_tracks_for(cap, s->params.min_track_hits);
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(dmalloc(&sl.d_y, cap)); chk(dmalloc(&sl.d_z, cap)); chk(dmalloc(&sl.d_off, R + 1));
    chk(dmalloc(&sl.d_n, 2)); chk(dmalloc(&sl.d_par, T * 5)); chk(dmalloc(&sl.d_cov, T * 15));
    chk(dmalloc(&sl.d_x, T)); chk(dmalloc(&sl.d_chi2, T)); chk(dmalloc(&sl.d_zb, T)); chk(dmalloc(&sl.d_ndf, T)); chk(dmalloc(&sl.d_nh, T));
    chk(dmalloc(&sl.d_sec, T)); chk(dmalloc(&sl.d_tf, T)); chk(dmalloc(&sl.d_hoff, T + 1));
    chk(dmalloc(&sl.d_hid, cap)); chk(dmalloc(&sl.d_ct, cap));
    chk(hmalloc(&sl.h_n, 2)); chk(hmalloc(&sl.h_par, T * 5)); chk(hmalloc(&sl.h_cov, T * 15));
    chk(hmalloc(&sl.h_x, T)); chk(hmalloc(&sl.h_chi2, T)); chk(hmalloc(&sl.h_zb, T)); chk(hmalloc(&sl.h_ndf, T)); chk(hmalloc(&sl.h_nh, T));
    chk(hmalloc(&sl.h_sec, T)); chk(hmalloc(&sl.h_hoff, T + 1)); chk(hmalloc(&sl.h_hid, cap));
    chk(hmalloc(&sl.h_ct, cap));
    if (e != hipSuccess) {
        free_slot_buffers(sl);
        s->used -= rel;
        sl.bytes = 0;
        sl.cap = 0;
        return srv_fail(s, TPCSF_E_NOMEM, std::string("slot allocation: ") + hipGetErrorString(e));
    }
    tpcsf_status st = tpcsf_reserve(sl.ctx, cap, 1);
    if (st != TPCSF_OK) {
        free_slot_buffers(sl);
        s->used -= rel;
        sl.bytes = 0;
        sl.cap = 0;
        return srv_fail(s, st, std::string("slot scratch: ") + tpcsf_last_error(sl.ctx));
    }
    s->used = s->used - rel + need;
    sl.bytes = need;
    sl.cap = cap;
    return TPCSF_OK;
}

}  // namespace

extern "C" {

tpcsf_status tpcsf_server_create(const tpcsf_geometry* geo, const tpcsf_params* params, const tpcsf_tuning* tuning,
                                 int32_t n_slots, size_t hbm_budget_bytes, tpcsf_server** out)
{
    if (!out || !geo || !geo->row_x || n_slots < 1 || n_slots > 64) return TPCSF_E_INVALID;
    *out = nullptr;
    // validate the configuration once through a probe context
    tpcsf_ctx* probe = nullptr;
    tpcsf_status st = tpcsf_create(geo, params, tuning, 0, &probe);
    if (st != TPCSF_OK) return st;
    (void)tpcsf_destroy(probe);
    tpcsf_server* s = new tpcsf_server();
    s->row_x.assign(geo->row_x, geo->row_x + geo->n_rows);
    s->geo = *geo;
    s->geo.row_x = s->row_x.data();
    if (params) s->params = *params; else tpcsf_default_params(&s->params);
    if (tuning) s->tuning = *tuning; else tpcsf_default_tuning(&s->tuning);
    s->budget = hbm_budget_bytes;
    s->slots.resize(n_slots);
    for (Slot& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.tracked, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            (void)tpcsf_server_destroy(s);
            return TPCSF_E_HIP;
        }
    }
    *out = s;
    return TPCSF_OK;
}

tpcsf_status tpcsf_server_destroy(tpcsf_server* s)
{
    if (!s) return TPCSF_E_INVALID;
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        free_slot_buffers(sl);
        if (sl.ctx) (void)tpcsf_destroy(sl.ctx);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.tracked) (void)hipEventDestroy(sl.tracked);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete s;
    return TPCSF_OK;
}

tpcsf_status tpcsf_server_submit(tpcsf_server* s, const float* y, const float* z, const int64_t* row_offsets,
                                 int64_t n_clusters, uint64_t* ticket)
{
    if (!s || !ticket || !row_offsets || n_clusters < 0 || (n_clusters > 0 && (!y || !z))) return TPCSF_E_INVALID;
    std::lock_guard<std::mutex> lock(s->mu);
    const int64_t R = (int64_t)s->geo.n_sectors * s->geo.n_rows;
    if (row_offsets[0] != 0 || row_offsets[R] != n_clusters)
        return srv_fail(s, TPCSF_E_INVALID, "row offsets do not span the clusters");
    // prefer a free slot that already holds the frame; else grow the smallest free slot
    Slot* pick = nullptr;
    for (Slot& sl : s->slots)
        if (sl.state == kFree && sl.ctx && sl.cap >= n_clusters && (!pick || sl.cap < pick->cap)) pick = &sl;
    if (!pick) {
        tpcsf_status st = TPCSF_E_BUSY;
        for (Slot& sl : s->slots) {
            if (sl.state != kFree) continue;
            st = grow_slot(s, sl, n_clusters);
            if (st == TPCSF_OK) { pick = &sl; break; }
            if (st != TPCSF_E_BUSY) return st;
        }
        if (!pick) return TPCSF_E_BUSY;
    }
    Slot& sl = *pick;
    sl.h_off.assign(row_offsets, row_offsets + R + 1);
    tpcsf_frame f;
    f.n_tf = 1;
    f.n_clusters = n_clusters;
    f.y = sl.d_y;
    f.z = sl.d_z;
    f.row_offsets = sl.d_off;
    f.row_offsets_host = sl.h_off.data();
    const int64_t T = cap_tracks_for(sl.cap, s->params.min_track_hits);
    tpcsf_tracks o{};
    o.cap_tracks = T;
    o.cap_hits = sl.cap;
    o.n_tracks = sl.d_n; o.n_hits = sl.d_n + 1;
    o.params = sl.d_par; o.cov = sl.d_cov; o.x_ref = sl.d_x; o.chi2 = sl.d_chi2; o.z_beam = sl.d_zb;
    o.ndf = sl.d_ndf; o.nhits = sl.d_nh; o.sector = sl.d_sec; o.tf = sl.d_tf;
    o.hit_off = sl.d_hoff; o.hit_ids = sl.d_hid; o.cluster_track = sl.d_ct;
    hipStream_t st_ = sl.stream;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    if (n_clusters > 0) {
        chk(hipMemcpyAsync(sl.d_y, y, sizeof(float) * n_clusters, hipMemcpyHostToDevice, st_));
        chk(hipMemcpyAsync(sl.d_z, z, sizeof(float) * n_clusters, hipMemcpyHostToDevice, st_));
    }
    chk(hipMemcpyAsync(sl.d_off, sl.h_off.data(), sizeof(int64_t) * (R + 1), hipMemcpyHostToDevice, st_));
    if (e != hipSuccess) return srv_fail(s, TPCSF_E_HIP, std::string("upload: ") + hipGetErrorString(e));
    tpcsf_status ts = tpcsf_track_batch(sl.ctx, &f, &o, st_);
    if (ts != TPCSF_OK) return srv_fail(s, ts, tpcsf_last_error(sl.ctx));
    // the counts now; the outputs once the counts are known (advance)
    chk(hipMemcpyAsync(sl.h_n, sl.d_n, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st_));
    chk(hipEventRecord(sl.tracked, st_));
    if (e != hipSuccess) return srv_fail(s, TPCSF_E_HIP, std::string("download: ") + hipGetErrorString(e));
    sl.state = kBusy;
    sl.downloading = false;
    sl.finished = false;
    sl.status = TPCSF_OK;
    sl.n = n_clusters;
    sl.ticket = s->next_ticket++;
    *ticket = sl.ticket;
    return TPCSF_OK;
}

static Slot* find_ticket(tpcsf_server* s, uint64_t ticket)
{
    for (Slot& sl : s->slots)
        if (sl.state == kBusy && sl.ticket == ticket) return &sl;
    return nullptr;
}

// Moves a busy slot on (caller holds the lock): once the tracking and the counts are done,
// the download of exactly the frame's tracks and hits is enqueued; once that is done, the
// frame is finished.
static tpcsf_status advance(tpcsf_server* s, Slot& sl)
{
    if (sl.finished) return TPCSF_OK;
    if (!sl.downloading) {
        const hipError_t e = hipEventQuery(sl.tracked);
        if (e == hipErrorNotReady) return TPCSF_OK;
        if (e != hipSuccess) return srv_fail(s, TPCSF_E_HIP, hipGetErrorString(e));
        sl.status = tpcsf_sync(sl.ctx, sl.stream);
        const int64_t capT = cap_tracks_for(sl.cap, s->params.min_track_hits);
        const int64_t T = sl.h_n[0] < capT ? sl.h_n[0] : capT;
        const int64_t H = sl.h_n[1] < sl.cap ? sl.h_n[1] : sl.cap;
        hipStream_t st_ = sl.stream;
        hipError_t x = hipSuccess;
        auto chk = [&](hipError_t y) { if (x == hipSuccess) x = y; };
        if (sl.status == TPCSF_OK && T > 0) {
            chk(hipMemcpyAsync(sl.h_par, sl.d_par, sizeof(double) * 5 * T, hipMemcpyDeviceToHost, st_));
            chk(hipMemcpyAsync(sl.h_cov, sl.d_cov, sizeof(double) * 15 * T, hipMemcpyDeviceToHost, st_));
            chk(hipMemcpyAsync(sl.h_x, sl.d_x, sizeof(double) * T, hipMemcpyDeviceToHost, st_));
            chk(hipMemcpyAsync(sl.h_chi2, sl.d_chi2, sizeof(double) * T, hipMemcpyDeviceToHost, st_));
            chk(hipMemcpyAsync(sl.h_zb, sl.d_zb, sizeof(double) * T, hipMemcpyDeviceToHost, st_));
            chk(hipMemcpyAsync(sl.h_ndf, sl.d_ndf, sizeof(int32_t) * T, hipMemcpyDeviceToHost, st_));
            chk(hipMemcpyAsync(sl.h_nh, sl.d_nh, sizeof(int32_t) * T, hipMemcpyDeviceToHost, st_));
            chk(hipMemcpyAsync(sl.h_sec, sl.d_sec, sizeof(int32_t) * T, hipMemcpyDeviceToHost, st_));
        }
        if (sl.status == TPCSF_OK)
            chk(hipMemcpyAsync(sl.h_hoff, sl.d_hoff, sizeof(int64_t) * (T + 1), hipMemcpyDeviceToHost, st_));
        if (sl.status == TPCSF_OK && H > 0)
            chk(hipMemcpyAsync(sl.h_hid, sl.d_hid, sizeof(int32_t) * H, hipMemcpyDeviceToHost, st_));
        if (sl.status == TPCSF_OK && sl.n > 0)
            chk(hipMemcpyAsync(sl.h_ct, sl.d_ct, sizeof(int32_t) * sl.n, hipMemcpyDeviceToHost, st_));
        chk(hipEventRecord(sl.done, st_));
        if (x != hipSuccess) return srv_fail(s, TPCSF_E_HIP, std::string("download: ") + hipGetErrorString(x));
        sl.downloading = true;
    }
    const hipError_t e = hipEventQuery(sl.done);
    if (e == hipErrorNotReady) return TPCSF_OK;
    if (e != hipSuccess) return srv_fail(s, TPCSF_E_HIP, hipGetErrorString(e));
    sl.finished = true;
    return TPCSF_OK;
}

tpcsf_status tpcsf_server_poll(tpcsf_server* s, uint64_t ticket, int32_t* done)
{
    if (!s || !done) return TPCSF_E_INVALID;
    std::lock_guard<std::mutex> lock(s->mu);
    Slot* sl = find_ticket(s, ticket);
    if (!sl) return srv_fail(s, TPCSF_E_INVALID, "unknown ticket");
    const tpcsf_status st = advance(s, *sl);
    if (st != TPCSF_OK) return st;
    *done = sl->finished ? 1 : 0;
    return TPCSF_OK;
}

tpcsf_status tpcsf_server_wait(tpcsf_server* s, uint64_t ticket, int64_t timeout_us)
{
    if (!s) return TPCSF_E_INVALID;
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        int32_t done = 0;
        tpcsf_status st = tpcsf_server_poll(s, ticket, &done);
        if (st != TPCSF_OK) return st;
        if (done) return TPCSF_OK;
        const auto us = std::chrono::duration_cast<std::chrono::microseconds>(std::chrono::steady_clock::now() - t0).count();
        if (timeout_us >= 0 && us >= timeout_us) return TPCSF_E_TIMEOUT;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

tpcsf_status tpcsf_server_result(tpcsf_server* s, uint64_t ticket, tpcsf_host_tracks* out)
{
    if (!s) return TPCSF_E_INVALID;
    int32_t done = 0;
    tpcsf_status st = tpcsf_server_poll(s, ticket, &done);
    if (st != TPCSF_OK) return st;
    if (!done) return TPCSF_E_BUSY;
    std::lock_guard<std::mutex> lock(s->mu);
    Slot* sl = find_ticket(s, ticket);
    if (!sl) return srv_fail(s, TPCSF_E_INVALID, "unknown ticket");
    const int64_t T = sl->h_n[0], H = sl->h_n[1];
    st = sl->status;
    if (out) {
        out->n_tracks = T;
        out->n_hits = H;
    }
    if (out && st == TPCSF_OK && (T > out->cap_tracks || H > out->cap_hits)) st = TPCSF_E_CAPACITY;
    if (out && st == TPCSF_OK) {
        auto cp = [](void* d, const void* src, size_t b) { if (d && b) std::memcpy(d, src, b); };
        cp(out->params, sl->h_par, sizeof(double) * 5 * T);
        cp(out->cov, sl->h_cov, sizeof(double) * 15 * T);
        cp(out->x_ref, sl->h_x, sizeof(double) * T);
        cp(out->chi2, sl->h_chi2, sizeof(double) * T);
        cp(out->z_beam, sl->h_zb, sizeof(double) * T);
        cp(out->ndf, sl->h_ndf, sizeof(int32_t) * T);
        cp(out->nhits, sl->h_nh, sizeof(int32_t) * T);
        cp(out->sector, sl->h_sec, sizeof(int32_t) * T);
        cp(out->hit_off, sl->h_hoff, sizeof(int64_t) * (T + 1));
        cp(out->hit_ids, sl->h_hid, sizeof(int32_t) * H);
        cp(out->cluster_track, sl->h_ct, sizeof(int32_t) * sl->n);
    }
    sl->state = kFree;   // the slot's buffers are free for the next frame
    return st;
}

size_t tpcsf_server_bytes_used(const tpcsf_server* s)
{
    return s ? s->used : 0;
}

const char* tpcsf_server_last_error(const tpcsf_server* s)
{
    return s ? s->err.c_str() : "null server";
}

}  // extern "C"
