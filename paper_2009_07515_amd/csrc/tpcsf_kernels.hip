// Kernels of TPC sector track finding for CDNA4 (gfx950, wave64).
//
// The method is the standalone sector tracking of arXiv:2009.07515, Sec. 6 (HLT-derived
// cellular automaton plus Kalman filter); its internal rules are stated in include/tpcsf.h
// and at each stage below.  Precision: the grid and the neighbour links are IEEE binary32
// with no contraction and correctly rounded division (their result is defined bit for
// bit); the Kalman filter runs in binary64, which CDNA4 issues at the rate of unpacked
// binary32 and which keeps the covariance updates well conditioned after a reset to the
// (deliberately loose) initial covariance.
#include "tpcsf_internal.h"
#include "tpcsf_kalman.h"

#include <math.h>

namespace tpcsf {

// ------------------------------------------------------------------------------------
// wave64 helpers
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T o = __shfl_up(v, d, 64);
        if (l >= d) v += o;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Lanes (among `valid` ones) whose key equals this lane's key; keys < 2^nbits.
__device__ __forceinline__ uint64_t match_eq(uint32_t key, bool valid, int nbits)
{
    uint64_t m = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
        const bool bit = (key >> b) & 1u;
        const uint64_t on = __ballot(valid && bit);
        m &= bit ? on : ~on;
    }
    return valid ? m : 0ull;
}

// Relaxed agent-scope accesses: they bypass the non-coherent vector L1, so a wave sees
// what other lanes (and its own atomics) wrote earlier in the same kernel.
__device__ __forceinline__ uint32_t ld_rlx(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wave_mem_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Block-wide exclusive scan of one int per thread (blockDim multiple of 64, <= 1024).
__device__ int block_excl_scan(int v, int* total, int* lds /*[16]*/)
{
    const int lane = lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int inc = wave_incl_scan(v);
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    if (threadIdx.x < 64) {
        int s = (lane < nw) ? lds[lane] : 0;
        int si = wave_incl_scan(s);
        if (lane < nw) lds[lane] = si - s;
        if (lane == 63) lds[16] = si;
    }
    __syncthreads();
    const int r = lds[w] + inc - v;
    *total = lds[16];
    __syncthreads();
    return r;
}

__device__ __forceinline__ int64_t bin_base(const DevParams& P, int64_t row_first, int64_t g)
{
    return (int64_t)P.cap_mul * row_first + (int64_t)(P.cap_add + 1) * g;
}

// Bin of a coordinate: trunc((v - lo) / b) clamped to [0, nb-1] (binary32).
__device__ __forceinline__ int bin_of(float v, float lo, float b, int nb)
{
    const float f = (v - lo) / b;
    const int i = (f < (float)nb) ? (int)fmaxf(f, 0.0f) : nb - 1;
    return i;
}

// ------------------------------------------------------------------------------------
// XCD-aware work placement.  The workgroups of a launch are dispatched round-robin over
// the chip's 8 XCDs, each with its own L2.  Renumbering blocks so that the blocks of one
// XCD get consecutive numbers, and splitting index ranges into one contiguous segment
// per XCD, keeps neighbouring rows and the tracks of one sector in one L2.  Placement
// never changes a result.
// ------------------------------------------------------------------------------------
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_parts() { return (int)gridDim.x < kXcds ? (int)gridDim.x : kXcds; }

// Block number with the blocks of each XCD consecutive (a bijection on [0, gridDim.x)).
__device__ __forceinline__ int xcd_block()
{
    const int nb = (int)gridDim.x, b = (int)blockIdx.x, parts = xcd_parts();
    const int x = b % parts, j = b / parts, q = nb / parts, rem = nb % parts;
    return x * q + (x < rem ? x : rem) + j;
}

// Segment `x` of `parts` equal segments of [lo, hi).
__device__ __forceinline__ void segment(int64_t lo, int64_t hi, int x, int parts, int64_t& s0, int64_t& s1)
{
    s0 = lo + (hi - lo) * x / parts;
    s1 = lo + (hi - lo) * (x + 1) / parts;
}

// Per-thread loop bounds over [lo, hi): this block's XCD takes its segment, and the
// XCD's blocks stride over it.  Iterate i = first; i < end; i += stride.  Segment
// boundaries inside the range fall on multiples of 64, so that (with blocks of whole
// waves) every wave but a segment's first takes 64 indices of one 64-aligned group, the
// unit of the hit table's tiles.
__device__ __forceinline__ void xcd_span(int64_t lo, int64_t hi, int64_t& first, int64_t& end, int64_t& stride)
{
    const int parts = xcd_parts(), x = (int)blockIdx.x % parts, j = (int)blockIdx.x / parts;
    const int nbx = ((int)gridDim.x - x + parts - 1) / parts;
    int64_t s0, s1;
    segment(lo, hi, x, parts, s0, s1);
    if (x > 0) s0 = max(lo, s0 & ~(int64_t)63);
    if (x < parts - 1) s1 = max(lo, s1 & ~(int64_t)63);
    first = s0 + (int64_t)j * blockDim.x + threadIdx.x;
    end = s1;
    stride = (int64_t)nbx * blockDim.x;
}

// ------------------------------------------------------------------------------------
// k_reset: per-call counters.
// ------------------------------------------------------------------------------------
__global__ void k_reset(Batch B)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        Counters* c = B.ctr;
        c->start_base = 0;
        c->rank_lo = 0;
        c->rank_hi = 0;
        c->track_base = 0;
        c->hit_base = 0;
        c->n_fit = 0;
        c->n_fit_long = 0;
        c->n_order = 0;
        for (int w = 0; w < 6; ++w) c->work[w] = 0;
        for (int x = 0; x < kXcds; ++x) {
            c->queue[x] = 0;
            c->fit_queue[x] = 0;
        }
        *B.o_ntracks = 0;
        *B.o_nhits = 0;
        if (B.cap_tracks >= 0) B.o_hit_off[0] = 0;
    }
}

// ------------------------------------------------------------------------------------
// Stage 1, grid (binary32).  One block per row.  Extents are exact minima/maxima;
// ny = 1 + trunc((y_hi - y_lo)/b_y), nz alike; while ny*nz > cap_mul*n + cap_add the z bin
// (once nz == 1 the y bin) doubles.  Clusters are ordered by bin iz*ny + iy, ties by
// in-row index (a stable counting sort).
//
// The sort runs in LDS: bin counts (16-bit, two per word) by LDS atomics, an in-place
// block scan, placement by LDS atomics (arbitrary order inside a bin), then every bin is
// put in index order by an insertion sort (bins hold a few clusters).  All global writes are then row-contiguous:
// sorted (y, z), perm (sorted -> in-row index), the bin table, and the inverse
// permutation inside the row.  A row whose tables do not fit in LDS takes the same steps
// on the global bin table, ordered chunk by chunk by one wave (a ballot match on the bin
// key ranks equal keys inside a chunk).
// ------------------------------------------------------------------------------------
constexpr int kGridThreads = 512;
constexpr int kGridStaticLds = 1024;    // bytes reserved for the kernel's static LDS
constexpr int kGridMaxLdsBin = 64;      // largest bin ordered by the in-LDS insertion sort

__device__ __forceinline__ uint32_t grid_key(float y, float z, float ylo, float zlo, float by, float bz, int ny,
                                             int nz)
{
    return (uint32_t)(bin_of(z, zlo, bz, nz) * ny + bin_of(y, ylo, by, ny));
}

// 16-bit counter b of an array of counter pairs (two per 32-bit word, low half first).
__device__ __forceinline__ uint32_t half_get(const uint32_t* a2, int b) { return (a2[b >> 1] >> ((b & 1) << 4)) & 0xFFFFu; }
__device__ __forceinline__ uint32_t half_one(int b) { return (b & 1) ? 0x10000u : 1u; }

// In-place exclusive scan of m 16-bit counters packed in pairs (all sums < 2^16).
__device__ void block_excl_scan_lds16(uint32_t* a2, int m, int* tmp /*[17]*/)
{
    const int t = threadIdx.x, nt = blockDim.x;
    const int words = (m + 1) >> 1;
    const int seg = (words + nt - 1) / nt;
    const int w0 = min(words, t * seg), w1 = min(words, w0 + seg);
    uint32_t sum = 0;
    for (int w = w0; w < w1; ++w) sum += (a2[w] & 0xFFFFu) + (a2[w] >> 16);
    int total;
    uint32_t run = (uint32_t)block_excl_scan((int)sum, &total, tmp);
    for (int w = w0; w < w1; ++w) {
        const uint32_t v = a2[w];
        const uint32_t lo = run;
        run += v & 0xFFFFu;
        const uint32_t hi = run;
        run += v >> 16;
        a2[w] = lo | (hi << 16);
    }
    __syncthreads();
}

// In-place exclusive scan of a[0, m) in LDS by the whole block (sums < 2^31).
__device__ void block_excl_scan_lds(uint32_t* a, int m, int* tmp /*[17]*/)
{
    const int t = threadIdx.x, nt = blockDim.x;
    const int seg = (m + nt - 1) / nt;
    const int s0 = min(m, t * seg), s1 = min(m, s0 + seg);
    uint32_t sum = 0;
    for (int i = s0; i < s1; ++i) sum += a[i];
    int total;
    uint32_t run = (uint32_t)block_excl_scan((int)sum, &total, tmp);
    for (int i = s0; i < s1; ++i) {
        const uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kGridThreads) k_grid(Batch B, DevParams P, int64_t g0, int64_t g1, int lds_bytes)
{
#pragma clang fp contract(off)
    extern __shared__ uint32_t sm[];
    __shared__ float red[4][16];
    __shared__ int badw[16];
    __shared__ int tmp[17];
    __shared__ uint32_t maxbin;
    const int t = threadIdx.x, nt = blockDim.x, lane = lane_id(), w = t >> 6, nw = nt >> 6;
    for (int64_t g = g0 + xcd_block(); g < g1; g += gridDim.x) {
        const int64_t base = B.off[g];
        const int n = (int)(B.off[g + 1] - base);
        const float* yr = B.y + base;
        const float* zr = B.z + base;
        float ylo = INFINITY, yhi = -INFINITY, zlo = INFINITY, zhi = -INFINITY;
        bool bad = false;
        for (int i = t; i < n; i += nt) {
            const float y = yr[i], z = zr[i];
            bad |= !(fabsf(y) <= 1.0e5f) || !(fabsf(z) <= 1.0e5f);
            ylo = fminf(ylo, y); yhi = fmaxf(yhi, y);
            zlo = fminf(zlo, z); zhi = fmaxf(zhi, z);
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            ylo = fminf(ylo, __shfl_xor(ylo, d, 64));
            yhi = fmaxf(yhi, __shfl_xor(yhi, d, 64));
            zlo = fminf(zlo, __shfl_xor(zlo, d, 64));
            zhi = fmaxf(zhi, __shfl_xor(zhi, d, 64));
        }
        const bool wbad = __ballot(bad) != 0ull;
        if (lane == 0) {
            red[0][w] = ylo; red[1][w] = yhi; red[2][w] = zlo; red[3][w] = zhi;
            badw[w] = wbad ? 1 : 0;
        }
        __syncthreads();
        bad = false;
        for (int j = 0; j < nw; ++j) {
            ylo = fminf(ylo, red[0][j]); yhi = fmaxf(yhi, red[1][j]);
            zlo = fminf(zlo, red[2][j]); zhi = fmaxf(zhi, red[3][j]);
            bad |= badw[j] != 0;
        }
        if (bad) {
            if (t == 0) atomicOr(&B.ctr->err, kErrInvalid);
            ylo = yhi = zlo = zhi = 0.0f;   // keep every index in range; the call reports the error
        }
        if (n == 0) ylo = yhi = zlo = zhi = 0.0f;
        float by = P.bin_y, bz = P.bin_z;
        int ny = 1, nz = 1;
        if (n > 0) {
            ny = 1 + (int)((yhi - ylo) / by);
            nz = 1 + (int)((zhi - zlo) / bz);
            const int64_t cap = (int64_t)P.cap_mul * n + P.cap_add;
            while ((int64_t)ny * nz > cap) {
                if (nz > 1) {
                    bz = bz * 2.0f;
                    nz = 1 + (int)((zhi - zlo) / bz);
                } else {
                    by = by * 2.0f;
                    ny = 1 + (int)((yhi - ylo) / by);
                }
            }
        }
        if (t == 0) {
            B.row_lo[g] = make_float2(ylo, zlo);
            B.row_bin[g] = make_float2(by, bz);
            B.row_nb[g] = make_int2(ny, nz);
            B.row_f[g] = make_float4(ylo, zlo, 1.0f / by, 1.0f / bz);
            B.row_i[g] = make_int4((int)base, n, ny, nz);
        }
        const int nb = ny * nz;
        uint32_t* bs = B.bin_start + bin_base(P, base, g);
        // LDS: counts / cursors [nb + 1] (16-bit, two per word; a row holds < 65535
        // clusters, so no count or prefix carries into the next counter), then the
        // placement [n] (u16)
        const int words = (nb + 2) >> 1;
        bool in_lds = n <= 65535 && 4 * (int64_t)words + 2 * (int64_t)n <= (int64_t)lds_bytes;
        uint32_t* cnt = sm;
        uint16_t* pl = (uint16_t*)(sm + words);
        if (in_lds) {
            for (int w = t; w < words; w += nt) cnt[w] = 0u;
            if (t == 0) maxbin = 0;
            __syncthreads();
            uint32_t mx = 0;
            for (int i = t; i < n; i += nt) {
                const int b = (int)grid_key(yr[i], zr[i], ylo, zlo, by, bz, ny, nz);
                const uint32_t old = atomicAdd(&cnt[b >> 1], half_one(b));
                mx = max(mx, ((old >> ((b & 1) << 4)) & 0xFFFFu) + 1u);
            }
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, 64));
            if (lane == 0) atomicMax(&maxbin, mx);
            __syncthreads();
            // the in-bin insertion sort is quadratic: a crowded bin takes the global path
            in_lds = maxbin <= (uint32_t)kGridMaxLdsBin;
        }
        if (in_lds) {
            block_excl_scan_lds16(cnt, nb + 1, tmp);   // counter b = first slot of bin b, counter nb = n
            for (int b = t; b <= nb; b += nt) bs[b] = half_get(cnt, b);
            __syncthreads();
            for (int i = t; i < n; i += nt) {
                const int b = (int)grid_key(yr[i], zr[i], ylo, zlo, by, bz, ny, nz);
                const uint32_t old = atomicAdd(&cnt[b >> 1], half_one(b));
                pl[(old >> ((b & 1) << 4)) & 0xFFFFu] = (uint16_t)i;
            }
            __syncthreads();
            // counter b is now the end of bin b; order each bin by in-row index
            for (int b = t; b < nb; b += nt) {
                const int s0 = b ? (int)half_get(cnt, b - 1) : 0, e = (int)half_get(cnt, b);
                for (int a = s0 + 1; a < e; ++a) {
                    const uint16_t v = pl[a];
                    int c = a;
                    while (c > s0 && pl[c - 1] > v) {
                        pl[c] = pl[c - 1];
                        --c;
                    }
                    pl[c] = v;
                }
            }
            __syncthreads();
            for (int k = t; k < n; k += nt) {
                const uint32_t i = pl[k];
                B.yz[base + k] = make_float2(yr[i], zr[i]);
                B.perm[base + k] = i;
                B.iperm[base + i] = (uint32_t)k;
            }
        } else {
            __syncthreads();
            for (int b = t; b <= nb; b += nt) st_rlx(bs + b, 0u);
            __threadfence();
            __syncthreads();
            for (int i = t; i < n; i += nt) atomicAdd(bs + grid_key(yr[i], zr[i], ylo, zlo, by, bz, ny, nz), 1u);
            __threadfence();
            __syncthreads();
            if (w == 0) {
                uint32_t carry = 0;   // exclusive scan: bs[b] = first slot of bin b, bs[nb] = n
                for (int b0 = 0; b0 <= nb; b0 += 64) {
                    const int b = b0 + lane;
                    const uint32_t v = (b <= nb) ? ld_rlx(bs + b) : 0u;
                    const uint32_t inc = wave_incl_scan(v) + carry;
                    if (b <= nb) st_rlx(bs + b, inc - v);
                    carry = __shfl(inc, 63, 64);
                }
                wave_mem_fence();
                const int nbits = 32 - __clz(nb > 1 ? nb - 1 : 1);
                for (int i0 = 0; i0 < n; i0 += 64) {
                    const int i = i0 + lane;
                    const bool valid = i < n;
                    const float y = valid ? yr[i] : 0.0f;
                    const float z = valid ? zr[i] : 0.0f;
                    const uint32_t bin = valid ? grid_key(y, z, ylo, zlo, by, bz, ny, nz) : 0u;
                    const uint64_t eq = match_eq(bin, valid, nbits);
                    const int rank = __popcll(eq & lanemask_lt());
                    const int leader = valid ? (__ffsll((unsigned long long)eq) - 1) : 0;
                    uint32_t old = 0;
                    if (valid && lane == leader) old = atomicAdd(bs + bin, (uint32_t)__popcll(eq));
                    old = __shfl(old, leader, 64);
                    if (valid) {
                        const uint32_t pos = old + (uint32_t)rank;
                        B.yz[base + pos] = make_float2(y, z);
                        B.perm[base + pos] = (uint32_t)i;
                        B.iperm[base + i] = pos;
                    }
                }
                wave_mem_fence();
                // bs[b] is now the end of bin b: shift up by one bin to restore the starts,
                // descending so that every value is read before it is overwritten
                for (int hi = nb - 1; hi >= 1; hi -= 64) {
                    const int b = hi - lane;
                    const uint32_t v = (b >= 1) ? ld_rlx(bs + b - 1) : 0u;
                    if (b >= 1) st_rlx(bs + b, v);
                    wave_mem_fence();
                }
                if (lane == 0) st_rlx(bs, 0u);
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// Stage 2, neighbour links (binary32, no contraction, correctly rounded division).
// One block per row; each thread takes clusters in sorted (bin) order so that the lanes
// of a wave query neighbouring windows.  A candidate in row r+-1 must satisfy
// |y_c - y_h| <= win_y and |z_c - z_h| <= win_z; the grid bins visited cover the window
// widened by a few ulps, and every candidate is then tested exactly.  The pair with the
// least slope change D wins if D <= kink_max; ties go to the smaller u, then the
// smaller d (in-row indices).  Results are stored as sorted positions.
//
// The qualifying up-row candidates are gathered into registers (slopes computed once per
// candidate), kSlots at a time; the down row is then scanned and every qualifying
// down-row candidate is scored against all of them.
// ------------------------------------------------------------------------------------
struct RowView {
    int64_t first;            // first cluster of the row
    int n;                    // clusters in the row
    float ylo, zlo;
    float iby, ibz;           // reciprocal bin sizes, for conservative window bins only
    int ny, nz;
    const uint32_t* bs;       // bin_start of the row
};

__device__ __forceinline__ RowView row_view(const Batch& B, const DevParams& P, int64_t g)
{
    RowView v;
    const float4 f = B.row_f[g];
    const int4 i = B.row_i[g];
    v.first = i.x;
    v.n = i.y;
    v.ylo = f.x; v.zlo = f.y; v.iby = f.z; v.ibz = f.w; v.ny = i.z; v.nz = i.w;
    v.bs = B.bin_start + bin_base(P, v.first, g);
    return v;
}

// Bin index range of [q - w, q + w] (clamped).  Visiting a superset of the bins suffices:
// every candidate is tested exactly.  The window is widened by a relative margin that
// covers the rounding of |c - q|, of q -+ w and of the reciprocal bin size.
__device__ __forceinline__ void bin_span(float q, float w, float lo, float ib, int nb, int& i0, int& i1)
{
    const float e = (fabsf(q) + fabsf(lo) + w + 1.0f) * 8.0e-6f;
    const float f0 = (q - (w + e) - lo) * ib;
    const float f1 = (q + (w + e) - lo) * ib;
    i0 = (f0 < (float)nb) ? (int)fmaxf(f0, 0.0f) : nb - 1;
    i1 = (f1 < (float)nb) ? (int)fmaxf(f1, 0.0f) : nb - 1;
}

// First candidate range of a window: the y-span of z-bin iz0; when the y-span covers the
// whole row, the ranges of all z-bins of the window are adjacent and form one range.
// `iz` is the last z-bin the range covers.
__device__ __forceinline__ void first_range(const RowView& V, int iy0, int iy1, int iz0, int iz1, int& iz,
                                            uint32_t& q, uint32_t& qe)
{
    if (iy0 == 0 && iy1 == V.ny - 1) {
        q = V.bs[iz0 * V.ny];
        qe = V.bs[(iz1 + 1) * V.ny];
        iz = iz1;
    } else {
        q = V.bs[iz0 * V.ny + iy0];
        qe = V.bs[iz0 * V.ny + iy1 + 1];
        iz = iz0;
    }
}

constexpr int kSlots = 6;

constexpr int kLinkBatch = 3;   // candidates per load batch of the link search

struct LinkBest {
    float D;
    int ku, kd;      // sorted positions, -1 = none
};

// Pair (ku, kd) with slope change Dk against the best so far.  Equal D: the smaller u,
// then the smaller d, by in-row index (looked up only on an exact tie).
__device__ __forceinline__ void link_consider(LinkBest& b, float Dk, int ku, int kd, float kmax, const uint32_t* pu,
                                              const uint32_t* pd)
{
    if (!(Dk <= kmax)) return;
    bool better = b.ku < 0 || Dk < b.D;
    if (!better && Dk == b.D) {
        const uint32_t u_new = pu[ku], u_old = pu[b.ku];
        better = u_new < u_old || (u_new == u_old && pd[kd] < pd[b.kd]);
    }
    if (better) { b.D = Dk; b.ku = ku; b.kd = kd; }
}

// Qualifying candidates of one neighbour row for the cluster (yh, zh): skips the first
// `skip`, keeps up to kSlots (slopes, sorted position), returns how many qualify in all.
// The bins of the window are visited z-bin by z-bin (each z-bin's y-span is one
// contiguous range); bins and candidates form one flat loop, so lanes with different
// bin and candidate counts do not diverge on nested loop bounds.
__device__ __forceinline__ int gather_side(const RowView& V, const float2* yz, int iy0, int iy1, int iz0, int iz1,
                                           float yh, float zh, float wy, float wz, float dx, bool above, int skip,
                                           float (&ty)[kSlots], float (&tz)[kSlots], int (&kk)[kSlots])
{
#pragma clang fp contract(off)
    int cnt = 0;
    int iz;
    uint32_t q, qe;
    first_range(V, iy0, iy1, iz0, iz1, iz, q, qe);
    for (;;) {
        while (q >= qe && iz < iz1) {
            ++iz;
            q = V.bs[iz * V.ny + iy0];
            qe = V.bs[iz * V.ny + iy1 + 1];
        }
        if (q >= qe) break;
        float2 cb[kLinkBatch];
#pragma unroll
        for (int u = 0; u < kLinkBatch; ++u) cb[u] = yz[min(q + (uint32_t)u, qe - 1u)];
#pragma unroll
        for (int u = 0; u < kLinkBatch; ++u) {
            const float2 c = cb[u];
            if (q + u < qe && fabsf(c.x - yh) <= wy && fabsf(c.y - zh) <= wz) {
                const int slot = cnt - skip;
                if (slot >= 0 && slot < kSlots) {
                    const float sy = above ? (c.x - yh) / dx : (yh - c.x) / dx;
                    const float sz = above ? (c.y - zh) / dx : (zh - c.y) / dx;
#pragma unroll
                    for (int m = 0; m < kSlots; ++m)
                        if (m == slot) { ty[m] = sy; tz[m] = sz; kk[m] = (int)(q + u); }
                }
                ++cnt;
            }
        }
        q += kLinkBatch;
    }
    return cnt;
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_links(Batch B, DevParams P, int64_t g0, int64_t g1)
{
#pragma clang fp contract(off)
    const int nr = P.n_rows;
    for (int64_t g = g0 + xcd_block(); g < g1; g += gridDim.x) {
        const int r = (int)(g % nr);
        const int64_t base = B.off[g];
        const int n = (int)(B.off[g + 1] - base);
        if (r == 0 || r == nr - 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                B.upk[base + i] = -1;
                B.dnk[base + i] = -1;
            }
            continue;
        }
        const RowView U = row_view(B, P, g + 1);
        const RowView D = row_view(B, P, g - 1);
        const float2* yzu = B.yz + U.first;
        const float2* yzd = B.yz + D.first;
        const uint32_t* pu = B.perm + U.first;
        const uint32_t* pd = B.perm + D.first;
        const float dxu = P.rx[r + 1] - P.rx[r];
        const float dxd = P.rx[r] - P.rx[r - 1];
        const float wy = P.win_y, wz = P.win_z, kmax = P.kink_max;
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            const float2 h = B.yz[base + k];
            const float yh = h.x, zh = h.y;
            int uy0, uy1, uz0, uz1, dy0, dy1, dz0, dz1;
            bin_span(yh, wy, U.ylo, U.iby, U.ny, uy0, uy1);
            bin_span(zh, wz, U.zlo, U.ibz, U.nz, uz0, uz1);
            bin_span(yh, wy, D.ylo, D.iby, D.ny, dy0, dy1);
            bin_span(zh, wz, D.zlo, D.ibz, D.nz, dz0, dz1);
            float uty[kSlots], utz[kSlots];
            int uk[kSlots];
            LinkBest best = {0.0f, -1, -1};
            // the up-side candidates in registers, kSlots at a time; every down-side
            // candidate is scored against them as the down row is scanned
            for (int us = 0;; us += kSlots) {
                const int nu_all = U.n ? gather_side(U, yzu, uy0, uy1, uz0, uz1, yh, zh, wy, wz, dxu, true, us, uty,
                                                     utz, uk)
                                       : 0;
                const int nu = min(kSlots, nu_all - us);
                if (nu <= 0) break;
                if (D.n) {
                    int iz;
                    uint32_t q, qe;
                    first_range(D, dy0, dy1, dz0, dz1, iz, q, qe);
                    for (;;) {
                        while (q >= qe && iz < dz1) {
                            ++iz;
                            q = D.bs[iz * D.ny + dy0];
                            qe = D.bs[iz * D.ny + dy1 + 1];
                        }
                        if (q >= qe) break;
                        float2 cb[kLinkBatch];
#pragma unroll
                        for (int u = 0; u < kLinkBatch; ++u) cb[u] = yzd[min(q + (uint32_t)u, qe - 1u)];
                        for (int u = 0; u < kLinkBatch; ++u) {
                            const float2 c = cb[u];
                            if (q + u < qe && fabsf(c.x - yh) <= wy && fabsf(c.y - zh) <= wz) {
                                const float ty = (yh - c.x) / dxd;
                                const float tz = (zh - c.y) / dxd;
#pragma unroll
                                for (int i = 0; i < kSlots; ++i) {
                                    if (i < nu) {
                                        const float ay = uty[i] - ty;
                                        const float az = utz[i] - tz;
                                        const float sy = ay * ay;
                                        const float sz = az * az;
                                        link_consider(best, sy + sz, uk[i], (int)(q + u), kmax, pu, pd);
                                    }
                                }
                            }
                        }
                        q += kLinkBatch;
                    }
                }
                if (us + kSlots >= nu_all) break;
            }
            B.upk[base + k] = best.ku;
            B.dnk[base + k] = best.kd;
        }
    }
}

// ------------------------------------------------------------------------------------
// Stage 3, cleaning: a link survives only if the linked cluster links back.  The same
// pass counts the row's chain bottoms (cleaned up-link, no cleaned down-link).
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_clean(Batch B, DevParams P, int64_t g0, int64_t g1)
{
    __shared__ int lds[17];
    const int nr = P.n_rows;
    for (int64_t g = g0 + xcd_block(); g < g1; g += gridDim.x) {
        const int r = (int)(g % nr);
        const int64_t base = B.off[g];
        const int n = (int)(B.off[g + 1] - base);
        const int64_t fu = (r + 1 < nr) ? B.off[g + 1] : 0;
        const int64_t fd = (r > 0) ? B.off[g - 1] : 0;
        int cnt = 0;
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            const int u = B.upk[base + k], d = B.dnk[base + k];
            const int cu = (u >= 0 && B.dnk[fu + u] == k) ? u : -1;
            const int cd = (d >= 0 && B.upk[fd + d] == k) ? d : -1;
            B.cupk[base + k] = cu;
            B.cdnk[base + k] = cd;
            cnt += (cu >= 0 && cd < 0);
        }
        int total;
        block_excl_scan(cnt, &total, lds);
        if (threadIdx.x == 0) B.row_nstart[g] = total;
    }
}

// ------------------------------------------------------------------------------------
// Stage 4, starts.  A start's rank is its position among the chain bottoms in
// (row, in-row index) order, from the row's scanned base.  The starts are also listed in
// (row, sorted position) order, the order in which they are processed.  The start flags
// and the row-local ranks are kept in LDS by sorted position, so the links are read once,
// coalesced (rows beyond kStartsLdsRow clusters take the same steps in global memory).
// ------------------------------------------------------------------------------------
constexpr int kStartsLdsRow = 16384;   // rows up to this size rank their starts in LDS

__global__ void __launch_bounds__(1024) k_starts(Batch B, DevParams P, int64_t g0, int64_t g1)
{
    __shared__ int lds[17];
    __shared__ uint8_t flag[kStartsLdsRow];     // start flag by sorted position
    __shared__ uint16_t rnk[kStartsLdsRow];     // row-local rank by sorted position
    for (int64_t g = g0 + xcd_block(); g < g1; g += gridDim.x) {
        const int64_t base = B.off[g];
        const int n = (int)(B.off[g + 1] - base);
        const int64_t sb = B.row_sbase[g];
        const bool in_lds = n <= kStartsLdsRow;
        if (in_lds) {
            // flags in sorted order (coalesced), ranks in input order through iperm
            for (int k = threadIdx.x; k < n; k += blockDim.x)
                flag[k] = B.cupk[base + k] >= 0 && B.cdnk[base + k] < 0;
            __syncthreads();
            int run = 0;
            for (int h0 = 0; h0 < n; h0 += blockDim.x) {
                const int h = h0 + threadIdx.x;
                const int k = (h < n) ? (int)B.iperm[base + h] : 0;
                const int f = (h < n) && flag[k];
                int total;
                const int pos = block_excl_scan(f, &total, lds);
                if (f) rnk[k] = (uint16_t)(run + pos);
                run += total;
            }
            __syncthreads();
            int64_t out = sb;
            for (int k0 = 0; k0 < n; k0 += blockDim.x) {
                const int k = k0 + threadIdx.x;
                const int f = (k < n) && flag[k];
                int total;
                const int pos = block_excl_scan(f, &total, lds);
                if (f) {
                    const int64_t p = out + pos;
                    B.st_row[p] = (int32_t)g;
                    B.st_k[p] = k;
                    B.st_rank[p] = (int32_t)(sb + rnk[k]);
                }
                out += total;
            }
            __syncthreads();
            continue;
        }
        int64_t run = sb;
        for (int h0 = 0; h0 < n; h0 += blockDim.x) {
            const int h = h0 + threadIdx.x;
            const int k = (h < n) ? (int)B.iperm[base + h] : 0;
            const int f = (h < n) && B.cupk[base + k] >= 0 && B.cdnk[base + k] < 0;
            int total;
            const int pos = block_excl_scan(f, &total, lds);
            if (f) B.rank_at[base + k] = (int32_t)(run + pos);
            run += total;
        }
        __threadfence_block();
        __syncthreads();
        run = sb;
        for (int k0 = 0; k0 < n; k0 += blockDim.x) {
            const int k = k0 + threadIdx.x;
            const int f = (k < n) && B.cupk[base + k] >= 0 && B.cdnk[base + k] < 0;
            int total;
            const int pos = block_excl_scan(f, &total, lds);
            if (f) {
                const int64_t p = run + pos;
                B.st_row[p] = (int32_t)g;
                B.st_k[p] = k;
                B.st_rank[p] = B.rank_at[base + k];
            }
            run += total;
        }
    }
}

// ------------------------------------------------------------------------------------
// Device-wide exclusive scans (three kernels: per-block sums, a one-block scan of the
// sums that also advances the running bases, per-block scans).  Ranges may come from
// device memory, so one graph serves every batch of the same shape.
// ------------------------------------------------------------------------------------

__device__ __forceinline__ void scan_range(const ScanJob& J, int64_t& lo, int64_t& hi)
{
    lo = J.lo_ptr ? *J.lo_ptr : J.lo;
    hi = J.hi_ptr ? *J.hi_ptr : J.hi;
    if (hi < lo) hi = lo;
}

__device__ __forceinline__ void scan_seg(int64_t lo, int64_t hi, int b, int64_t& s0, int64_t& s1)
{
    const int64_t len = hi - lo;
    const int64_t per = (len + kScanBlocks - 1) / kScanBlocks;
    s0 = lo + (int64_t)b * per;
    s1 = s0 + per;
    if (s0 > hi) s0 = hi;
    if (s1 > hi) s1 = hi;
}

__device__ __forceinline__ int64_t scanA(const ScanJob& J, int64_t i)
{
    if (J.a64) return J.a64[i];
    if (J.a_min > 0) return J.a32[i] >= J.a_min ? 1 : 0;
    return (int64_t)J.a32[i];
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(ScanJob J)
{
    __shared__ int64_t red[2][kScanThreads / 64];
    int64_t lo, hi, s0, s1;
    scan_range(J, lo, hi);
    scan_seg(lo, hi, blockIdx.x, s0, s1);
    int64_t a = 0, b = 0;
    for (int64_t i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
        a += scanA(J, i);
        if (J.b32) b += J.b32[i];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane_id() == 0) { red[0][threadIdx.x >> 6] = a; red[1][threadIdx.x >> 6] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t sa = 0, sb = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { sa += red[0][w]; sb += red[1][w]; }
        J.part[blockIdx.x] = sa;
        J.part[kScanBlocks + blockIdx.x] = sb;
    }
}

__global__ void __launch_bounds__(kScanBlocks) k_scan_top(ScanJob J)
{
    __shared__ int64_t lds[2][kScanBlocks / 64];
    const int t = threadIdx.x, lane = lane_id(), w = t >> 6;
    const int64_t va = J.part[t], vb = J.part[kScanBlocks + t];
    const int64_t ia = wave_incl_scan(va), ib = wave_incl_scan(vb);
    if (lane == 63) { lds[0][w] = ia; lds[1][w] = ib; }
    __syncthreads();
    int64_t pa = 0, pb = 0;
    for (int k = 0; k < w; ++k) { pa += lds[0][k]; pb += lds[1][k]; }
    int64_t ta = 0, tb = 0;
    for (int k = 0; k < kScanBlocks / 64; ++k) { ta += lds[0][k]; tb += lds[1][k]; }
    const int64_t baseA = J.baseA ? *J.baseA : 0;
    const int64_t baseB = J.baseB ? *J.baseB : 0;
    J.part[2 * kScanBlocks + t] = baseA + pa + ia - va;
    J.part[3 * kScanBlocks + t] = baseB + pb + ib - vb;
    __syncthreads();
    if (t == 0) {
        if (J.totA) *J.totA = baseA + ta;
        if (J.totB) *J.totB = baseB + tb;
        if (J.rangeA_lo) *J.rangeA_lo = baseA;
        if (J.rangeA_hi) *J.rangeA_hi = baseA + ta;
        if (J.baseA) *J.baseA = baseA + ta;
        if (J.baseB) *J.baseB = baseB + tb;
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_down(ScanJob J)
{
    __shared__ int64_t lds[2][kScanThreads / 64 + 1];
    int64_t lo, hi, s0, s1;
    scan_range(J, lo, hi);
    scan_seg(lo, hi, blockIdx.x, s0, s1);
    int64_t ca = J.part[2 * kScanBlocks + blockIdx.x];
    int64_t cb = J.part[3 * kScanBlocks + blockIdx.x];
    const int lane = lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int64_t i0 = s0; i0 < s1; i0 += blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        const int64_t va = (i < s1) ? scanA(J, i) : 0;
        const int64_t vb = (i < s1 && J.b32) ? (int64_t)J.b32[i] : 0;
        const int64_t ia = wave_incl_scan(va), ib = wave_incl_scan(vb);
        if (lane == 63) { lds[0][w] = ia; lds[1][w] = ib; }
        __syncthreads();
        int64_t pa = 0, pb = 0, ta = 0, tb = 0;
        for (int k = 0; k < nw; ++k) {
            if (k < w) { pa += lds[0][k]; pb += lds[1][k]; }
            ta += lds[0][k]; tb += lds[1][k];
        }
        if (i < s1) {
            J.outA[i] = ca + pa + ia - va;
            if (J.outB) J.outB[i] = cb + pb + ib - vb;
        }
        ca += ta;
        cb += tb;
        __syncthreads();
    }
}

// Snapshot of a device-resident range, so that the three scan kernels agree on it even
// if a pointer it came from is rewritten by the scan itself.
__global__ void k_scan_range(ScanJob J)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t lo, hi;
        scan_range(J, lo, hi);
        J.part[4 * kScanBlocks] = lo;
        J.part[4 * kScanBlocks + 1] = hi;
    }
}

static void run_scan(ScanJob J, hipStream_t s)
{
    if (J.lo_ptr) {
        hipLaunchKernelGGL(k_scan_range, dim3(1), dim3(64), 0, s, J);
        // read the snapshot instead of the live pointers from here on
        J.lo_ptr = J.part + 4 * kScanBlocks;
        J.hi_ptr = J.part + 4 * kScanBlocks + 1;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3(kScanBlocks), dim3(kScanThreads), 0, s, J);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlocks), 0, s, J);
    hipLaunchKernelGGL(k_scan_down, dim3(kScanBlocks), dim3(kScanThreads), 0, s, J);
}

void launch_scan(const ScanJob& job, hipStream_t s)
{
    run_scan(job, s);
}

// Least-chi2 cluster of row g (row record rf, ri) inside the follow window: its sorted
// position (-1 if none) and coordinates.  Equal chi2: the smaller in-row index.  n_win
// counts the clusters inside the window.
__device__ int search_row(const Batch& B, const DevParams& P, const float4 rf, const int4 ri, int64_t g, const Trk& t,
                          double& best_chi2, float2& best_c, int& n_win)
{
    RowView v;
    v.first = ri.x;
    v.n = ri.y;
    v.ylo = rf.x; v.zlo = rf.y; v.iby = rf.z; v.ibz = rf.w; v.ny = ri.z; v.nz = ri.w;
    v.bs = B.bin_start + bin_base(P, v.first, g);
    best_chi2 = 0.0;
    if (v.n == 0) return -1;
    const double s00 = t.c[0] + P.sy2, s01 = t.c[1], s11 = t.c[2] + P.sz2;
    double wy = P.nsig * sqrt_nr(s00), wz = P.nsig * sqrt_nr(s11);
    if (wy > (double)P.win_y) wy = (double)P.win_y;
    if (wz > (double)P.win_z) wz = (double)P.win_z;
    const double yp = t.p[0], zp = t.p[1];
    if (!(fabs(yp) < 1.0e6) || !(fabs(zp) < 1.0e6)) return -1;
    int iy0, iy1, iz0, iz1;
    bin_span((float)yp, (float)wy, v.ylo, v.iby, v.ny, iy0, iy1);
    bin_span((float)zp, (float)wz, v.zlo, v.ibz, v.nz, iz0, iz1);
    const double idet = rcp_nr(s00 * s11 - s01 * s01);
    const float2* yz = B.yz + v.first;
    int best = -1;
    int iz;
    uint32_t q, qe;
    first_range(v, iy0, iy1, iz0, iz1, iz, q, qe);
    for (;;) {
        while (q >= qe && iz < iz1) {
            ++iz;
            q = v.bs[iz * v.ny + iy0];
            qe = v.bs[iz * v.ny + iy1 + 1];
        }
        if (q >= qe) break;
        float2 c2[2];
        c2[0] = yz[q];
        c2[1] = (q + 1 < qe) ? yz[q + 1] : make_float2(INFINITY, INFINITY);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const double dy = (double)c2[j].x - yp;
            const double dz = (double)c2[j].y - zp;
            if (!(fabs(dy) <= wy) || !(fabs(dz) <= wz)) continue;
            ++n_win;
            const int k = (int)(q + j);
            const double chi2 = (dy * dy * s11 - 2.0 * dy * dz * s01 + dz * dz * s00) * idet;
            bool take = best < 0 || chi2 < best_chi2;
            if (!take && chi2 == best_chi2) take = B.perm[v.first + k] < B.perm[v.first + best];
            if (take) {
                best = k;
                best_chi2 = chi2;
                best_c = c2[j];
            }
        }
        q += 2;
    }
    return best;
}

// ------------------------------------------------------------------------------------
// Stage 5a, chains: walk the cleaned up-links from every start (one lane each), record
// the chain in the tracklet's hit table and its length; chains of >= min_chain clusters
// become tracklets.
// ------------------------------------------------------------------------------------
// Hit table in tiles of 64 starts: tile p/64 holds rows 0..n_rows-1 of its 64 starts,
// row by row, so that neighbouring tracklets' entries for one row are adjacent (one
// 128-byte line for a wave of 64) and one tracklet's rows lie within one 19 KB tile.
__device__ __forceinline__ uint16_t* hit_slot(const Batch& B, int r, int64_t p)
{
    return B.tl_hits + (((p >> 6) * B.n_rows + r) << 6) + (p & 63);
}

__global__ void __launch_bounds__(256) k_walk(Batch B, DevParams P)
{
    const int nr = P.n_rows;
    if (blockIdx.x == 0 && threadIdx.x == 0)   // the fit queue of this launch set
        for (int x = 0; x < kXcds; ++x) B.ctr->fit_queue[x] = 0;
    int64_t first, end, stride;
    xcd_span(B.ctr->rank_lo, B.ctr->rank_hi, first, end, stride);
    for (int64_t p = first; p < end; p += stride) {
        const int64_t g = B.st_row[p];
        const int r0 = (int)(g % nr);
        const int64_t gs = g - r0;
        int L = 0;
        for (int r = r0, k = B.st_k[p]; r < nr && k >= 0; ++r) {
            *hit_slot(B, r, p) = (uint16_t)k;
            ++L;
            k = B.cupk[B.off[gs + r] + k];
        }
        B.tl_len[p] = L;
        B.tl_n[p] = 0;
        B.tl_w[p] = 0u;
    }
}

// The tracklets to build, listed in processing order: slot from a device scan of the
// chain lengths (fit_pos serves as the scan's output here; the fit stage rewrites it).
__global__ void __launch_bounds__(256) k_order(Batch B, DevParams P)
{
    int64_t first, end, stride;
    xcd_span(B.ctr->rank_lo, B.ctr->rank_hi, first, end, stride);
    for (int64_t p = first; p < end; p += stride)
        if (B.tl_len[p] >= P.min_chain) B.order[B.fit_pos[p]] = (int32_t)p;
}

// ------------------------------------------------------------------------------------
// Stage 6, selection.  A tracklet's weight orders tracklets by (clusters, then smaller
// rank); every cluster ends with the largest weight of the tracklets that contain it
// (a maximum, order independent; reduced row by row in k_claim from the weight each
// tracklet records when it is built).  Weights are only ever compared within a sector, so
// the rank counts from the sector's first start: w = (n << 24) | (2^24 - 1 - rank_s)
// (n <= n_rows <= 255, checked at context creation; rank_s < 2^24 since a sector of at
// most 255 rows of < 65535 clusters holds < 2^23 starts).  Tracklets shorter than
// min_track_hits can neither be accepted nor outweigh a longer one and do not take part.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t weight_of(const Batch& B, const DevParams& P, int n, int64_t rank, int64_t gs)
{
    const int64_t rs = rank - B.row_sbase[gs];
    return ((uint32_t)n << 24) | (0xFFFFFFu - (uint32_t)rs);
}

// ------------------------------------------------------------------------------------
// Stage 5b, tracklets.  Per chain: three-point seed (first, middle and last cluster),
// Kalman update over the chain, follow outward, reset C to C0 keeping p and refit inward
// over all clusters so far, follow inward.  A follow step propagates to the next row and
// takes the least-chi2 cluster inside the window if chi2 <= chi2_max; it stops after
// more than max_miss consecutive misses or when the propagation fails.  Clusters are
// recorded per row (sorted positions); rows [rlo, rhi] are all written.  A failed seed,
// fit or refit leaves a tracklet of size 0.  A tracklet of >= min_track_hits clusters
// records the weight with which it claims them (stage 6).
//
// Execution is row-synchronous: a wave takes 64 consecutive tracklets of the list, which
// is in processing order (one start row, neighbouring bins: the tracks lie close
// together), and sweeps the rows with all of them: upward for the chain fit and the outward follow, downward
// for the refit and the inward follow.  At every pass all
// lanes work on the same row, so row records, hit table entries (adjacent per row) and search
// windows are shared between the lanes of the wave.
// ------------------------------------------------------------------------------------
// Hands work items of [lo, hi) to the idle lanes of a wave, in lane order.  The range is
// split into one segment per XCD with a queue head each; a wave takes `grab` items of its
// own XCD's segment at a time (one atomic per grab, the queue chunk of the tuning) and
// moves on to the next segment once its own is used up.  Returns -1 once every segment
// is used up.  `next`, `end`, `seg` and `tried` are the wave's (uniform) queue state.
__device__ int64_t take_item(int32_t* heads, int64_t lo, int64_t hi, uint64_t idle, int grab, int64_t& next,
                             int64_t& end, int& seg, int& tried)
{
    const int parts = xcd_parts();
    const int want = __popcll(idle);
    const int rank = __popcll(idle & lanemask_lt());
    int64_t item = -1;
    int given = 0;
    while (given < want) {
        if (next >= end) {
            if (tried >= parts) break;
            int64_t s0, s1;
            segment(lo, hi, seg, parts, s0, s1);
            int h = 0;
            if (lane_id() == 0) h = atomicAdd(&heads[seg], grab);
            h = __shfl(h, 0, 64);
            if (s0 + h >= s1) {
                seg = (seg + 1) % parts;
                ++tried;
                continue;
            }
            next = s0 + h;
            end = (s0 + h + grab < s1) ? s0 + h + grab : s1;
        }
        const int64_t avail = end - next;
        const int take = (int64_t)(want - given) < avail ? want - given : (int)avail;
        if (rank >= given && rank < given + take) item = next + (rank - given);
        next += take;
        given += take;
    }
    return item;
}

__device__ __forceinline__ int wave_min_i(int v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d, 64));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
    return v;
}

// Adds a per-lane count, summed over the wave, to a device counter (one atomic per wave).
__device__ __forceinline__ void wave_count(int64_t* ctr, int v)
{
    const int t = wave_sum(v);
    if (lane_id() == 0 && t != 0) atomicAdd((unsigned long long*)ctr, (unsigned long long)t);
}

constexpr int kRowBatch = 8;   // rows per pass of the keep sweep

// What a tracklet sweep needs of a row before the state reaches it: the row's search
// records, its first cluster and the tracklet's hit-table entry (stale outside the rows
// the tracklet has written; used only inside them).
struct RowAhead {
    float4 f;
    int4 i;
    int64_t off;
    int k;
};

__device__ __forceinline__ RowAhead row_ahead(const Batch& B, int64_t p, int64_t gs, int r, bool on)
{
    RowAhead a;
    if (on) {
        a.f = B.row_f[gs + r];
        a.i = B.row_i[gs + r];
        a.off = B.off[gs + r];
        a.k = *hit_slot(B, r, p);
    } else {
        a.f = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        a.i = make_int4(0, 0, 0, 0);
        a.off = 0;
        a.k = kNoHit;
    }
    return a;
}

enum : int { kWait = 0, kFit = 1, kOut = 2, kUpDone = 3, kRefit = 4, kIn = 5, kDone = 6 };

__global__ void __launch_bounds__(256) k_tracklets(Batch B, DevParams P, int grab)
{
    const int nr = P.n_rows;
    int64_t q_next = 0, q_end = 0;
    int q_seg = (int)blockIdx.x % xcd_parts(), q_tried = 0;
    for (;;) {
        const int64_t j = take_item(B.ctr->queue, 0, B.ctr->n_order, ~0ull, grab, q_next, q_end, q_seg, q_tried);
        if (__ballot(j >= 0) == 0ull) break;
        const int64_t p = j >= 0 ? (int64_t)B.order[j] : -1;
        const int L = p >= 0 ? B.tl_len[p] : 0;
        const bool live = L >= P.min_chain;
        int r0 = 0, rend = 0, rlo = 0, rhi = 0, n = 0, misses = 0, phase = kDone;
        int nprop = 0, nupd = 0, nwin = 0;   // algorithmic work of this lane
        int64_t gs = 0;
        Trk tr;
        if (live) {
            const int64_t g = B.st_row[p];
            r0 = (int)(g % nr);
            gs = g - r0;
            rend = r0 + L;
            rlo = r0;
            rhi = r0 + L - 1;
            const int rs[3] = {r0, r0 + (L - 1) / 2, r0 + L - 1};
            double sx[3], sy[3], sz[3];
            for (int q = 0; q < 3; ++q) {
                const float2 c = B.yz[B.off[gs + rs[q]] + *hit_slot(B, rs[q], p)];
                sx[q] = (double)P.rx[rs[q]];
                sy[q] = (double)c.x;
                sz[q] = (double)c.y;
            }
            if (trk_seed(tr, sx, sy, sz, P)) {
                trk_reset_cov(tr, P);
                phase = kWait;
                n = L;
            }
        }

        // upward: chain fit from r0, then follow outward; each row's loads that do not
        // depend on the state are issued one row ahead
        int ru = wave_min_i(phase == kWait ? r0 : nr);
        RowAhead nx = row_ahead(B, p, gs, ru, live && ru < nr);
        for (int r = ru; r < nr && __ballot(phase <= kOut) != 0ull; ++r) {
            const RowAhead cur = nx;
            nx = row_ahead(B, p, gs, r + 1, live && r + 1 < nr);
            if (phase == kWait && r == r0) phase = kFit;
            const bool act = phase == kFit || phase == kOut;
            bool moved = true;
            if (act && !(phase == kFit && r == r0)) {
                moved = trk_propagate(tr, (double)P.rx[r], P);
                ++nprop;
            }
            int k = -1;
            float2 c = make_float2(0.0f, 0.0f);
            if (act && moved) {
                if (phase == kFit) {
                    k = cur.k;
                    c = B.yz[cur.off + k];
                } else {
                    double chi2;
                    k = search_row(B, P, cur.f, cur.i, gs + r, tr, chi2, c, nwin);
                    if (k >= 0 && !(chi2 <= P.chi2_max)) k = -1;
                }
            }
            if (k >= 0) {
                trk_update(tr, (double)c.x, (double)c.y, P);
                ++nupd;
            }
            if (phase == kFit) {
                if (!moved) {
                    phase = kDone;
                    n = 0;
                } else if (r == rend - 1) {
                    phase = kOut;
                    misses = 0;
                }
            } else if (phase == kOut) {
                if (!moved) {
                    phase = kUpDone;
                } else if (k >= 0) {
                    *hit_slot(B, r, p) = (uint16_t)k;
                    rhi = r;
                    misses = 0;
                    ++n;
                } else {
                    *hit_slot(B, r, p) = kNoHit;
                    if (++misses > P.max_miss) phase = kUpDone;
                }
            }
        }
        if (phase == kOut || phase == kUpDone) {
            trk_reset_cov(tr, P);
            phase = kRefit;
        }

        // downward: refit over the rows with a cluster from rhi to r0, then follow inward
        int rd = wave_max_i(phase == kRefit ? rhi : -1);
        nx = row_ahead(B, p, gs, rd, live && rd >= 0);
        for (int r = rd; r >= 0 && __ballot(phase == kRefit || phase == kIn) != 0ull; --r) {
            const RowAhead cur = nx;
            nx = row_ahead(B, p, gs, r - 1, live && r >= 1);
            bool act = false;
            int k = -1;
            if (phase == kRefit && r <= rhi) {
                k = cur.k;
                act = k != kNoHit;
            } else if (phase == kIn) {
                act = true;
            }
            bool moved = true;
            if (act) {
                moved = trk_propagate(tr, (double)P.rx[r], P);
                ++nprop;
            }
            float2 c = make_float2(0.0f, 0.0f);
            if (act && moved) {
                if (phase == kRefit) {
                    c = B.yz[cur.off + k];
                } else {
                    double chi2;
                    k = search_row(B, P, cur.f, cur.i, gs + r, tr, chi2, c, nwin);
                    if (k >= 0 && !(chi2 <= P.chi2_max)) k = -1;
                }
                if (k >= 0) {
                    trk_update(tr, (double)c.x, (double)c.y, P);
                    ++nupd;
                }
            }
            if (phase == kRefit && r <= rhi) {
                if (act && !moved) {
                    phase = kDone;
                    n = 0;
                } else if (r == r0) {
                    phase = r0 > 0 ? kIn : kDone;
                    misses = 0;
                }
            } else if (phase == kIn) {
                if (!moved) {
                    phase = kDone;
                } else {
                    if (k >= 0) {
                        *hit_slot(B, r, p) = (uint16_t)k;
                        rlo = r;
                        misses = 0;
                        ++n;
                    } else {
                        *hit_slot(B, r, p) = kNoHit;
                        if (++misses > P.max_miss) phase = kDone;
                    }
                    if (r == 0) phase = kDone;
                }
            }
        }

        if (live) {
            B.tl_n[p] = n;
            B.tl_rlo[p] = (int16_t)rlo;
            B.tl_rhi[p] = (int16_t)rhi;
            // the weight with which the tracklet claims its clusters (stage 6), 0 if it
            // takes no part
            B.tl_w[p] = n >= P.min_track_hits ? weight_of(B, P, n, B.st_rank[p], gs) : 0u;
        }
        wave_count(&B.ctr->work[0], nprop);
        wave_count(&B.ctr->work[1], nupd);
        wave_count(&B.ctr->work[2], nwin);
    }
}

// ------------------------------------------------------------------------------------
// Stage 6, selection, one block per row: every cluster of the row takes the largest
// weight of the tracklets that hold it, 0 if none does.  The tracklets of a sector are
// the starts [first start of its first row, end of the starts of its last row); the hit
// table keeps a row's entries of neighbouring tracklets adjacent, so the block reads
// them in coalesced runs, and reduces the weights by LDS atomics on the row's clusters
// (sorted positions); the row's weights are then written out contiguously.  A row of
// more than kClaimLds clusters takes the same steps with global atomics.
// ------------------------------------------------------------------------------------
constexpr int kClaimLds = 12288;   // clusters of a row reduced in LDS (48 KB)
constexpr int kClaimBatch = 4;     // starts per thread and pass

__global__ void __launch_bounds__(512) k_claim(Batch B, DevParams P, int64_t g0, int64_t g1)
{
    __shared__ uint32_t wl[kClaimLds];
    const int nr = P.n_rows;
    for (int64_t g = g0 + xcd_block(); g < g1; g += gridDim.x) {
        const int r = (int)(g % nr);
        const int64_t gs = g - r;
        const int64_t base = B.off[g];
        const int n = (int)(B.off[g + 1] - base);
        const int64_t p0 = B.row_sbase[gs];
        const int64_t p1 = B.row_sbase[gs + nr - 1] + B.row_nstart[gs + nr - 1];
        const bool in_lds = n <= kClaimLds;
        uint32_t* wr = in_lds ? wl : B.W + base;
        for (int k = threadIdx.x; k < n; k += blockDim.x) wr[k] = 0u;
        __threadfence_block();
        __syncthreads();
        // kClaimBatch starts per thread and pass, all their loads issued before any test
        // (hit-table entries outside a tracklet's rows are stale and are not used); the
        // waves start at a tile boundary
        for (int64_t pb = (p0 & ~(int64_t)63) + threadIdx.x; pb < p1; pb += kClaimBatch * (int64_t)blockDim.x) {
            uint32_t w[kClaimBatch];
            int lo[kClaimBatch], hi[kClaimBatch];
            uint16_t kk[kClaimBatch];
#pragma unroll
            for (int u = 0; u < kClaimBatch; ++u) {
                const int64_t p = pb + (int64_t)u * blockDim.x;
                const bool on = p >= p0 && p < p1;
                w[u] = on ? B.tl_w[p] : 0u;
                lo[u] = on ? B.tl_rlo[p] : 0;
                hi[u] = on ? B.tl_rhi[p] : -1;
                kk[u] = on ? *hit_slot(B, r, p) : kNoHit;
            }
#pragma unroll
            for (int u = 0; u < kClaimBatch; ++u)
                if (w[u] != 0u && r >= lo[u] && r <= hi[u] && kk[u] != kNoHit) atomicMax(&wr[kk[u]], w[u]);
        }
        __threadfence_block();
        __syncthreads();
        if (in_lds) {
            for (int k = threadIdx.x; k < n; k += blockDim.x) B.W[base + k] = wl[k];
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------------------------
// Stage 7a, keep: a tracklet keeps the clusters that carry its own weight and is a track
// candidate if it keeps >= min_track_hits.  A device scan over the candidate flags then
// gives every candidate its slot, in processing order.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_keep(Batch B, DevParams P)
{
    const int nr = P.n_rows;
    const int lane = lane_id();
    if (blockIdx.x == 0 && threadIdx.x == 0)   // the tracklet queue is done
        for (int x = 0; x < kXcds; ++x) B.ctr->queue[x] = 0;
    int64_t first, end, stride;
    xcd_span(B.ctr->rank_lo, B.ctr->rank_hi, first, end, stride);
    // wave-uniform loop over 64 consecutive tracklets, their rows swept together
    for (int64_t p0 = first - lane; p0 < end; p0 += stride) {
        const int64_t p = p0 + lane;
        const bool in = p < end;
        int n = 0, rlo = nr, rhi = -1;
        int64_t gs = 0;
        uint32_t w = 0u;
        if (in) {
            const int64_t rank = B.st_rank[p];
            B.trk_flag[rank] = 0;
            B.hit_cnt[rank] = 0;
            B.trk_out[rank] = -1;
            n = B.tl_n[p];
            if (n >= P.min_track_hits) {
                const int64_t g = B.st_row[p];
                gs = g - g % nr;
                w = B.tl_w[p];
                rlo = B.tl_rlo[p];
                rhi = B.tl_rhi[p];
            }
        }
        const bool sel = in && n >= P.min_track_hits;
        uint64_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
        int kept = 0;
        const int rb = wave_max_i(sel ? rhi : -1);
        for (int r = wave_min_i(sel ? rlo : nr); r <= rb; r += kRowBatch) {
            uint16_t kk[kRowBatch];
            int64_t ff[kRowBatch];
            uint32_t ww[kRowBatch];
#pragma unroll
            for (int u = 0; u < kRowBatch; ++u) {
                const int rr = r + u;
                const bool on = sel && rr >= rlo && rr <= rhi;
                kk[u] = on ? *hit_slot(B, rr, p) : kNoHit;
                ff[u] = on ? B.off[gs + rr] : 0;
            }
#pragma unroll
            for (int u = 0; u < kRowBatch; ++u) ww[u] = kk[u] != kNoHit ? B.W[ff[u] + kk[u]] : 0u;
#pragma unroll
            for (int u = 0; u < kRowBatch; ++u) {
                if (kk[u] == kNoHit || ww[u] != w) continue;
                const int rr = r + u;
                const uint64_t bit = 1ull << (rr & 63);
                const int wd = rr >> 6;
                m0 |= wd == 0 ? bit : 0ull;
                m1 |= wd == 1 ? bit : 0ull;
                m2 |= wd == 2 ? bit : 0ull;
                m3 |= wd == 3 ? bit : 0ull;
                ++kept;
            }
        }
        if (sel && kept >= P.min_track_hits) {
            B.keep_mask[p * 4 + 0] = m0; B.keep_mask[p * 4 + 1] = m1;
            B.keep_mask[p * 4 + 2] = m2; B.keep_mask[p * 4 + 3] = m3;
        } else {
            kept = 0;
        }
        if (in) B.keep_n[p] = kept;
    }
}

// ------------------------------------------------------------------------------------
// Stage 7b, final fit on the kept clusters (inner to outer): three-point seed (first,
// middle and last kept cluster), C = C0, update outward; C = C0 keeping p, update inward
// from the last kept cluster, summing the chi2 of each cluster before its update.
// Result at the innermost kept cluster; a failed fit drops the track.  Results are
// stored at the candidate's list slot.
//
// The kept clusters are first gathered into one contiguous list per candidate; the fit then
// streams each lane's own list, the candidates of a block ordered by kept count.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mask_word(uint64_t m0, uint64_t m1, uint64_t m2, uint64_t m3, int w)
{
    return w == 0 ? m0 : (w == 1 ? m1 : (w == 2 ? m2 : m3));
}

// Smallest set row >= r (-1 if none) and largest set row <= r (-1 if none).
__device__ __forceinline__ int row_at_or_above(uint64_t m0, uint64_t m1, uint64_t m2, uint64_t m3, int r)
{
    for (int w = r >> 6; w < 4; ++w) {
        uint64_t x = mask_word(m0, m1, m2, m3, w);
        if (w == (r >> 6)) x &= ~0ull << (r & 63);
        if (x) return (w << 6) + __ffsll((unsigned long long)x) - 1;
    }
    return -1;
}

__device__ __forceinline__ int row_at_or_below(uint64_t m0, uint64_t m1, uint64_t m2, uint64_t m3, int r)
{
    for (int w = r >> 6; w >= 0; --w) {
        uint64_t x = mask_word(m0, m1, m2, m3, w);
        if (w == (r >> 6) && (r & 63) != 63) x &= (1ull << ((r & 63) + 1)) - 1ull;
        if (x) return (w << 6) + 63 - __clzll((long long)x);
    }
    return -1;
}

// Position of the k-th (from 0) set bit of x; x has more than k set bits.
__device__ __forceinline__ int nth_set_bit(uint64_t x, int k)
{
    int pos = 0;
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) {
        const int c = __popcll(x & ((1ull << sh) - 1ull));
        if (k >= c) {
            k -= c;
            x >>= sh;
            pos += sh;
        }
    }
    return pos;
}

// Candidates listed by slot: those of at least kFitLong kept clusters first, then the
// others, each part in processing order (from two scans of the kept counts).  The fit's
// lanes outnumber the candidates less than twice, so the lanes that take a second
// candidate then take a short one.  A slot only says which lane fits the candidate; the
// tracks are emitted in rank order whatever the slot.
constexpr int kFitLong = 64;

__global__ void __launch_bounds__(256) k_fit_list(Batch B, DevParams P)
{
    int64_t first, end, stride;
    xcd_span(B.ctr->rank_lo, B.ctr->rank_hi, first, end, stride);
    const int64_t n_long = B.ctr->n_fit_long;
    for (int64_t p = first; p < end; p += stride) {
        const int kept = B.keep_n[p];
        if (kept <= 0) continue;
        const int64_t slot = kept >= kFitLong ? B.fit_pos_long[p] : n_long + B.fit_pos[p] - B.fit_pos_long[p];
        B.fit_list[slot] = (int32_t)p;
    }
}

__device__ __forceinline__ bool row_set(uint64_t m0, uint64_t m1, uint64_t m2, uint64_t m3, int r)
{
    return (mask_word(m0, m1, m2, m3, r >> 6) >> (r & 63)) & 1ull;
}

// The kept clusters of every candidate as one list per candidate in slot order (inner to
// outer), at offsets from the scan of the kept counts.  Work items are (32 consecutive
// candidates, kKeptRows consecutive rows): kKeptRows neighbouring lanes take one candidate,
// a row each, and place its kept cluster of that row (if any) at its position in the list
// (the kept rows below, from its mask).  A candidate's entries for these rows are
// consecutive, so the lanes of one candidate write one contiguous run and a store
// instruction covers whole runs of 64 / kKeptRows candidates.  Consecutive work items take
// neighbouring candidates in the same rows, whose clusters then stay in L2.
constexpr int kKeptRows = 8;   // divides 64: an item's rows lie in one word of a kept mask
constexpr int kKeptCands = 256 / kKeptRows;

__global__ void __launch_bounds__(256) k_kept(Batch B, DevParams P)
{
    const int nr = P.n_rows;
    const int groups = (nr + kKeptRows - 1) / kKeptRows;
    const int64_t nfit = B.ctr->n_fit;
    const int64_t n_chunks = (nfit + kKeptCands - 1) / kKeptCands;
    const int64_t n_items = n_chunks * groups;
    const int u = (int)threadIdx.x % kKeptRows;
    for (int64_t it = xcd_block(); it < n_items; it += gridDim.x) {
        const int r0 = (int)(it / n_chunks) * kKeptRows;
        const int r = r0 + u;
        const int64_t i = (it % n_chunks) * kKeptCands + (int)threadIdx.x / kKeptRows;
        if (i >= nfit || r >= nr) continue;
        const int64_t p = B.fit_list[i];
        const int rlo = B.tl_rlo[p], rhi = B.tl_rhi[p];
        if (r < rlo || r > rhi) continue;
        const int w0 = r0 >> 6;
        uint64_t mw[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) mw[w] = w <= w0 ? B.keep_mask[p * 4 + w] : 0ull;
        const uint64_t word = w0 == 0 ? mw[0] : (w0 == 1 ? mw[1] : (w0 == 2 ? mw[2] : mw[3]));
        if (!((word >> (r & 63)) & 1ull)) continue;
        // kept rows below r
        int below = __popcll(word & ((1ull << (r & 63)) - 1ull));
#pragma unroll
        for (int w = 0; w < 3; ++w) below += w < w0 ? __popcll(mw[w]) : 0;
        const int64_t g = B.st_row[p];
        const int64_t f = B.off[g - g % nr + r];
        const uint32_t k = *hit_slot(B, r, p);
        const int64_t j = B.cand_off[p] + below;
        const float2 c = B.yz[f + k];
        const uint32_t o = B.perm[f + k];
        B.kept_list[j] = make_float4(c.x, c.y, P.rx[r], __int_as_float((int)(f + o)));
    }
}

// Block-wide bitonic sort of 256 keys in LDS, descending.
__device__ void bitonic_desc_256(uint32_t* key)
{
    const int t = threadIdx.x;
    for (int k = 2; k <= 256; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int o = t ^ j;
            if (o > t) {
                const uint32_t a = key[t], b = key[o];
                const bool desc = (t & k) == 0;
                if (desc ? (a < b) : (a > b)) {
                    key[t] = b;
                    key[o] = a;
                }
            }
            __syncthreads();
        }
    }
}

// Each block takes 256 consecutive candidate slots and orders them by kept count, so that
// the lanes of a wave run passes of similar length over their own contiguous kept lists.
__global__ void __launch_bounds__(256) k_fit(Batch B, DevParams P)
{
    __shared__ uint32_t key[256];
    const int t = threadIdx.x;
    const int64_t nfit = B.ctr->n_fit;
    const int parts = xcd_parts(), x = (int)blockIdx.x % parts, bj = (int)blockIdx.x / parts;
    const int nbx = ((int)gridDim.x - x + parts - 1) / parts;
    // chunks of 256 candidates dealt round-robin to the XCDs, each XCD's blocks taking its
    // chunks in slot order: the long candidates first everywhere
    const int64_t n_ch = (nfit + 255) / 256;
    for (int64_t ch = x + (int64_t)parts * bj; ch < n_ch; ch += (int64_t)parts * nbx) {
        const int64_t i_own = ch * 256 + t;
        const int kept_own = i_own < nfit ? B.keep_n[B.fit_list[i_own]] : 0;
        key[t] = ((uint32_t)kept_own << 8) | (uint32_t)t;
        __syncthreads();
        bitonic_desc_256(key);
        const int64_t i = ch * 256 + (key[t] & 0xFFu);
        __syncthreads();
        const bool live = i < nfit;
        int64_t p = 0, base = 0;
        int kept = 0;
        bool ok = false;
        Trk tr;
        if (live) {
            p = B.fit_list[i];
            kept = B.keep_n[p];
            base = B.cand_off[p];
            const float4 e[3] = {B.kept_list[base], B.kept_list[base + (kept - 1) / 2],
                                 B.kept_list[base + kept - 1]};
            double sx[3], sy[3], sz[3];
            for (int q = 0; q < 3; ++q) {
                sx[q] = (double)e[q].z;
                sy[q] = (double)e[q].x;
                sz[q] = (double)e[q].y;
            }
            ok = trk_seed(tr, sx, sy, sz, P);
            if (ok) trk_reset_cov(tr, P);
        }
        int nprop = 0, nupd = 0, nchi = 0;   // algorithmic work of this lane
        const int kw = wave_max_i(ok ? kept : 0);
        // outward over the kept clusters
        for (int j = 0; j < kw; ++j) {
            if (!(ok && j < kept)) continue;
            const float4 e = B.kept_list[base + j];
            if (j > 0) {
                ++nprop;
                if (!trk_propagate(tr, (double)e.z, P)) {
                    ok = false;
                    continue;
                }
            }
            trk_update(tr, (double)e.x, (double)e.y, P);
            ++nupd;
        }
        if (ok && B.f_pout) {
            for (int q = 0; q < 5; ++q) B.f_pout[i * 5 + q] = tr.p[q];
            for (int q = 0; q < 15; ++q) B.f_cout[i * 15 + q] = tr.c[q];
        }
        if (ok) trk_reset_cov(tr, P);
        // inward from the last kept cluster, summing chi2 before each update
        double chi2 = 0.0;
        for (int j = kw - 1; j >= 0; --j) {
            if (!(ok && j < kept)) continue;
            const float4 e = B.kept_list[base + j];
            if (j < kept - 1) {
                ++nprop;
                if (!trk_propagate(tr, (double)e.z, P)) {
                    ok = false;
                    continue;
                }
            }
            chi2 += trk_update(tr, (double)e.x, (double)e.y, P);
            ++nupd;
            ++nchi;
        }
        wave_count(&B.ctr->work[3], nprop);
        wave_count(&B.ctr->work[4], nupd);
        wave_count(&B.ctr->work[5], nchi);
        if (ok) {
            for (int q = 0; q < 5; ++q) ok = ok && isfinite(tr.p[q]);
            for (int q = 0; q < 15; ++q) ok = ok && isfinite(tr.c[q]);
        }
        if (ok) {
            double* fp = B.f_par + i * 5;
            double* fc = B.f_cov + i * 15;
            for (int q = 0; q < 5; ++q) fp[q] = tr.p[q];
            for (int q = 0; q < 15; ++q) fc[q] = tr.c[q];
            B.f_chi2[i] = chi2;
            B.f_xref[i] = tr.x;
            const int64_t rank = B.st_rank[p];
            B.trk_flag[rank] = 1;
            B.hit_cnt[rank] = kept;
        }
    }
}

// ------------------------------------------------------------------------------------
// Stage 8, emit: tracks at their scanned positions (rank order), hits inner to outer as
// input cluster indices (from the kept list), each track's z at the beam line and, on
// request, its outer state.  Writes beyond the caller's capacity are dropped and flagged.
// ------------------------------------------------------------------------------------
constexpr int kEmitTracks = 4;   // hit lists copied per pass of the emit

__global__ void __launch_bounds__(256) k_emit(Batch B, DevParams P)
{
    const int nr = P.n_rows;
    const int lane = lane_id();
    int64_t first, end, stride;
    xcd_span(0, B.ctr->n_fit, first, end, stride);
    // wave-uniform loop over 64 candidates: records per lane, then each written track's
    // hit list copied by the whole wave (64 consecutive entries per pass)
    for (int64_t i0 = first - lane; i0 < end; i0 += stride) {
        const int64_t i = i0 + lane;
        bool on = i < end;
        int64_t hp = 0, src = 0;
        int nk = 0;
        if (on) {
            const int64_t p = B.fit_list[i];
            const int64_t rank = B.st_rank[p];
            on = B.trk_flag[rank] != 0;
            if (on) {
                const int64_t T = B.trk_idx[rank];
                hp = B.hit_pos[rank];
                nk = B.hit_cnt[rank];
                const int64_t g = B.st_row[p];
                if (T >= B.cap_tracks || hp + nk > B.cap_hits) {
                    atomicOr(&B.ctr->err, kErrOutCap);
                    on = false;
                } else {
                    for (int q = 0; q < 5; ++q) B.o_par[T * 5 + q] = B.f_par[i * 5 + q];
                    for (int q = 0; q < 15; ++q) B.o_cov[T * 15 + q] = B.f_cov[i * 15 + q];
                    B.o_xref[T] = B.f_xref[i];
                    B.o_chi2[T] = B.f_chi2[i];
                    B.o_ndf[T] = 2 * nk - 5;
                    B.o_nhits_trk[T] = nk;
                    B.o_sector[T] = (int32_t)((g / nr) % P.n_sectors);
                    B.o_tf[T] = (int32_t)(g / ((int64_t)nr * P.n_sectors));
                    B.o_hit_off[T + 1] = hp + nk;
                    B.trk_out[rank] = (int32_t)T;
                    if (B.o_zbeam) B.o_zbeam[T] = trk_beamline_z(P, B.f_xref[i], B.f_par + i * 5);
                    if (B.o_par_out) {
                        for (int q = 0; q < 5; ++q) B.o_par_out[T * 5 + q] = B.f_pout[i * 5 + q];
                        for (int q = 0; q < 15; ++q) B.o_cov_out[T * 15 + q] = B.f_cout[i * 15 + q];
                    }
                    src = B.cand_off[p];
                }
            }
        }
        // four tracks' hit lists per pass, the loads of all four issued before the stores
        uint64_t todo = __ballot(on);
        while (todo != 0ull) {
            int64_t d[kEmitTracks], sj[kEmitTracks];
            int m[kEmitTracks];
            int mm = 0;
#pragma unroll
            for (int u = 0; u < kEmitTracks; ++u) {
                const int l = todo != 0ull ? __ffsll((unsigned long long)todo) - 1 : 0;
                const bool has = todo != 0ull;
                todo &= todo - 1ull;
                d[u] = __shfl(hp, l, 64);
                sj[u] = __shfl(src, l, 64);
                m[u] = has ? __shfl(nk, l, 64) : 0;
                mm = max(mm, m[u]);
            }
            for (int q = lane; q < mm; q += 64) {
                float4 e[kEmitTracks];
#pragma unroll
                for (int u = 0; u < kEmitTracks; ++u)
                    e[u] = q < m[u] ? B.kept_list[sj[u] + q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
                for (int u = 0; u < kEmitTracks; ++u) {
                    if (q >= m[u]) continue;
                    B.o_hit_ids[d[u] + q] = __float_as_int(e[u].w);
                    if (B.o_hit_rec) B.o_hit_rec[d[u] + q] = e[u];
                }
            }
        }
    }
}

// ------------------------------------------------------------------------------------
// Stage 9, cluster -> track map, per cluster in input order.  A cluster belongs to the
// track whose weight it carries (the kept clusters of a track are exactly those), so the
// weight names the tracklet by its rank within the sector; the map is -1 where that
// tracklet was not accepted or its track was not written (emit records, per rank, the
// track it wrote).
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_assign(Batch B, DevParams P, int64_t g0, int64_t g1)
{
    const int nr = P.n_rows;
    for (int64_t g = g0 + xcd_block(); g < g1; g += gridDim.x) {
        const int64_t base = B.off[g];
        const int n = (int)(B.off[g + 1] - base);
        const int64_t sbase = B.row_sbase[g - g % nr];
        // four clusters per thread and pass: their loads are issued before they are used
        constexpr int kU = 4;
        for (int i0 = threadIdx.x; i0 < n; i0 += kU * blockDim.x) {
            uint32_t ip[kU], w[kU];
            int32_t T[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                ip[u] = i < n ? B.iperm[base + i] : 0u;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                w[u] = i < n ? B.W[base + ip[u]] : 0u;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u)
                T[u] = w[u] != 0u ? B.trk_out[sbase + (int64_t)(0xFFFFFFu - (w[u] & 0xFFFFFFu))] : -1;
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                if (i < n) B.o_cluster_track[base + i] = T[u];
            }
        }
    }
}

// ------------------------------------------------------------------------------------
// Verification views: links in input (in-row index) order, starts and tracklet sizes in
// rank order.  Not part of the tracking; run only on request.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_debug_links(Batch B, DevParams P, int64_t g0, int64_t g1)
{
    const int nr = P.n_rows;
    for (int64_t g = g0 + xcd_block(); g < g1; g += gridDim.x) {
        const int r = (int)(g % nr);
        const int64_t base = B.off[g];
        const int n = (int)(B.off[g + 1] - base);
        const int64_t fu = (r + 1 < nr) ? B.off[g + 1] : 0;
        const int64_t fd = (r > 0) ? B.off[g - 1] : 0;
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            const int64_t h = base + B.perm[base + k];
            const int u = B.upk[base + k], d = B.dnk[base + k];
            const int cu = B.cupk[base + k], cd = B.cdnk[base + k];
            B.d_up[h] = u >= 0 ? (int)B.perm[fu + u] : -1;
            B.d_dn[h] = d >= 0 ? (int)B.perm[fd + d] : -1;
            B.d_cup[h] = cu >= 0 ? (int)B.perm[fu + cu] : -1;
            B.d_cdn[h] = cd >= 0 ? (int)B.perm[fd + cd] : -1;
        }
    }
}

__global__ void __launch_bounds__(256) k_debug_starts(Batch B, DevParams P)
{
    const int64_t hi = B.ctr->start_base;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < hi; p += stride) {
        const int64_t rank = B.st_rank[p];
        const int64_t g = B.st_row[p];
        B.d_start_row[rank] = (int32_t)g;
        B.d_start_idx[rank] = (int32_t)B.perm[B.off[g] + B.st_k[p]];
        B.d_tl_n[rank] = B.tl_n[p];
    }
}

// ------------------------------------------------------------------------------------
// Output digest: XOR over every output element of a mix of (array, index, bits).  The
// XOR is independent of the order of the atomics, so equal outputs give equal digests.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long mix64(unsigned long long x)
{
    x ^= x >> 30; x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27; x *= 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__device__ __forceinline__ unsigned long long elem_hash(unsigned long long tag, int64_t i, unsigned long long v)
{
    return mix64(v + mix64(((unsigned long long)i << 4) ^ tag));
}

__global__ void __launch_bounds__(256) k_hash(Batch B, int64_t n_clusters)
{
    const int64_t T = min(*B.o_ntracks, B.cap_tracks);
    const int64_t H = min(*B.o_nhits, B.cap_hits);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long h = 0;
    if (t0 == 0) h ^= elem_hash(1, 0, (unsigned long long)T) ^ elem_hash(2, 0, (unsigned long long)H);
    for (int64_t i = t0; i < T; i += stride) {
        for (int q = 0; q < 5; ++q) h ^= elem_hash(3, i * 5 + q, __double_as_longlong(B.o_par[i * 5 + q]));
        for (int q = 0; q < 15; ++q) h ^= elem_hash(4, i * 15 + q, __double_as_longlong(B.o_cov[i * 15 + q]));
        h ^= elem_hash(5, i, (unsigned long long)B.o_hit_off[i + 1]);
        h ^= elem_hash(6, i, __double_as_longlong(B.o_chi2[i]));
        if (B.o_zbeam) h ^= elem_hash(9, i, __double_as_longlong(B.o_zbeam[i]));
    }
    for (int64_t i = t0; i < H; i += stride) h ^= elem_hash(7, i, (unsigned long long)(uint32_t)B.o_hit_ids[i]);
    for (int64_t i = t0; i < n_clusters; i += stride)
        h ^= elem_hash(8, i, (unsigned long long)(uint32_t)B.o_cluster_track[i]);
    for (int d = 32; d >= 1; d >>= 1) h ^= __shfl_xor(h, d, 64);
    if (lane_id() == 0 && h) atomicXor(&B.ctr->hash, h);
}

__global__ void k_hash_clear(Batch B)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) B.ctr->hash = 0ull;
}

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------
static inline unsigned grid_for(int64_t items, int64_t per_block, int64_t cap)
{
    int64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

void launch_reset(const Batch& b, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, b);
}

int grid_lds_setup(int max_lds_per_block)
{
    int dyn = max_lds_per_block - kGridStaticLds;
    if (dyn < 0) dyn = 0;
    if (hipFuncSetAttribute((const void*)k_grid, hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess) {
        (void)hipGetLastError();
        dyn = 65536 - kGridStaticLds;
    }
    return dyn;
}

void launch_grid(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_grid, dim3(grid_for(g1 - g0, 1, 1 << 16)), dim3(kGridThreads), (size_t)c.grid_lds, s, b, p,
                       g0, g1, c.grid_lds);
}

void launch_links(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s)
{
    // k_links is compiled for at most 256 threads per block (register budget)
    const int threads = c.block < 256 ? c.block : 256;
    hipLaunchKernelGGL(k_links, dim3(grid_for(g1 - g0, 1, 1 << 16)), dim3(threads), 0, s, b, p, g0, g1);
}

void launch_clean(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_clean, dim3(grid_for(g1 - g0, 1, 1 << 16)), dim3(c.block), 0, s, b, p, g0, g1);
}

void launch_row_scan(const Batch& b, int64_t g0, int64_t g1, hipStream_t s)
{
    ScanJob J = {};
    J.a64 = b.row_nstart;
    J.outA = b.row_sbase;
    J.lo = g0;
    J.hi = g1;
    J.baseA = &b.ctr->start_base;
    J.rangeA_lo = &b.ctr->rank_lo;
    J.rangeA_hi = &b.ctr->rank_hi;
    J.part = b.scan_part;
    run_scan(J, s);
}

void launch_starts(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_starts, dim3(grid_for(g1 - g0, 1, 1 << 16)), dim3(c.block), 0, s, b, p, g0, g1);
}

void launch_walk(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_walk, dim3(c.n_cu * 16), dim3(256), 0, s, b, p);
}

void launch_order(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s)
{
    ScanJob J = {};
    J.a32 = b.tl_len;
    J.a_min = p.min_chain > 0 ? p.min_chain : 1;
    J.outA = b.fit_pos;
    J.lo_ptr = &b.ctr->rank_lo;
    J.hi_ptr = &b.ctr->rank_hi;
    J.totA = &b.ctr->n_order;
    J.part = b.scan_part;
    run_scan(J, s);
    hipLaunchKernelGGL(k_order, dim3(c.n_cu * 4), dim3(256), 0, s, b, p);
}

void launch_tracklets(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s)
{
    const int wpb = c.tl_block / 64;
    const int blocks = c.n_cu * (16 / wpb > 0 ? 16 / wpb : 1);
    // a wave takes chunk groups of 64 tracklets per queue atomic and sweeps them one
    // group after the other
    hipLaunchKernelGGL(k_tracklets, dim3(blocks), dim3(c.tl_block), 0, s, b, p, 64 * c.chunk);
}

void launch_claim(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_claim, dim3(grid_for(g1 - g0, 1, 1 << 16)), dim3(512), 0, s, b, p, g0, g1);
}

void launch_keep(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_keep, dim3(c.n_cu * 5), dim3(256), 0, s, b, p);
}

void launch_fit_scan(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s)
{
    ScanJob J = {};
    J.a32 = b.keep_n;
    J.a_min = 1;
    J.outA = b.fit_pos;
    J.lo_ptr = &b.ctr->rank_lo;
    J.hi_ptr = &b.ctr->rank_hi;
    J.totA = &b.ctr->n_fit;
    J.b32 = b.keep_n;          // channel B: offsets of the candidates' kept lists
    J.outB = b.cand_off;
    J.part = b.scan_part;
    run_scan(J, s);
    ScanJob L = {};            // the long candidates
    L.a32 = b.keep_n;
    L.a_min = kFitLong;
    L.outA = b.fit_pos_long;
    L.lo_ptr = &b.ctr->rank_lo;
    L.hi_ptr = &b.ctr->rank_hi;
    L.totA = &b.ctr->n_fit_long;
    L.part = b.scan_part;
    run_scan(L, s);
    hipLaunchKernelGGL(k_fit_list, dim3(c.n_cu * 4), dim3(256), 0, s, b, p);
}

void launch_fit(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_kept, dim3(c.n_cu * 8), dim3(256), 0, s, b, p);
    hipLaunchKernelGGL(k_fit, dim3(c.n_cu * 4), dim3(256), 0, s, b, p);
}

void launch_track_scan(const Batch& b, hipStream_t s)
{
    ScanJob J = {};
    J.a32 = b.trk_flag;
    J.b32 = b.hit_cnt;
    J.outA = b.trk_idx;
    J.outB = b.hit_pos;
    J.lo_ptr = &b.ctr->rank_lo;
    J.hi_ptr = &b.ctr->rank_hi;
    J.baseA = &b.ctr->track_base;
    J.baseB = &b.ctr->hit_base;
    J.totA = b.o_ntracks;
    J.totB = b.o_nhits;
    J.part = b.scan_part;
    run_scan(J, s);
}

void launch_emit(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_emit, dim3(c.n_cu * 4), dim3(256), 0, s, b, p);
}

void launch_assign(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_assign, dim3(grid_for(g1 - g0, 1, 1 << 16)), dim3(256), 0, s, b, p, g0, g1);
}

// ------------------------------------------------------------------------------------
// Hit removal for data compression, strategy B (Sec. 4): keep only the clusters in the
// vicinity of good tracks (pT >= pt_min).  A good track keeps its own clusters and, at
// every row from its innermost to its outermost cluster's row, the clusters of its
// sector's row within `window` in y and z of its state at x_ref propagated in one helix
// step to the row.  The rows are searched with the grids of the same call.  Wave per
// track; the flags are bytes in input order (concurrent stores all write 1).
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_r_clear(RejectArgs A)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) *A.n_kept = 0;
    for (int64_t i = i0; i <= A.n_rows_total; i += stride) {
        A.rdiff[i] = 0;
        if (i < A.n_rows_total) A.rcur[i] = 0;
    }
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t wave_min_l(int64_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int64_t wave_max_l(int64_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Row span of every good track (the rows of its first and last cluster) after the input
// checks, and the +1 / -1 of that span in the difference array of the row counts.  A wave
// takes 64 neighbouring tracks, whose cluster lists are adjacent, and checks them in
// coalesced passes of 64 clusters; the few tracks a pass touches are visited in turn.
__global__ void __launch_bounds__(256) k_r_span(Batch B, DevParams P, RejectArgs A)
{
    const int nr = P.n_rows, ns = P.n_sectors;
    const int lane = lane_id();
    int64_t T = *A.n_tracks;
    if (T > A.cap_tracks) T = A.cap_tracks;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t w0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64; w0 < T; w0 += nw * 64) {
        const int64_t t = w0 + lane;
        bool on = false;
        int64_t g0 = 0, hb = 0, he = 0, lo = 0, hi = 0;
        if (t < T) {
            const int s = A.sector[t], f = A.tf[t];
            hb = A.hit_off[t];
            he = A.hit_off[t + 1];
            if (!(s >= 0 && s < ns && f >= 0 && f < A.n_tf && hb >= 0 && he > hb && he <= A.cap_hits)) {
                atomicOr(&B.ctr->err, kErrInvalid);
            } else if (fabs(A.par[t * 5 + 4]) * A.pt_min <= 1.0) {
                g0 = ((int64_t)f * ns + s) * nr;
                lo = B.off[g0];
                hi = B.off[g0 + nr];
                on = true;
            }
        }
        // every cluster inside the track's own sector
        const int64_t H0 = wave_min_l(on ? hb : INT64_MAX), H1 = wave_max_l(on ? he : INT64_MIN);
        bool bad = false;
        for (int64_t jb = H0; jb < H1; jb += 8 * 64) {
            int32_t hv[8];   // eight passes' loads issued together
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t j = jb + u * 64 + lane;
                hv[u] = (j < H1) ? A.hit_ids[j] : 0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t j0 = jb + u * 64, j = j0 + lane;
                const int64_t h = hv[u];
                uint64_t own = __ballot(on && hb < j0 + 64 && he > j0);
                int who = -1;
                while (own) {
                    const int o = __ffsll((unsigned long long)own) - 1;
                    own &= own - 1ull;
                    const int64_t ob = readlane64(hb, o), oe = readlane64(he, o);
                    const int64_t ol = readlane64(lo, o), oh = readlane64(hi, o);
                    if (j >= ob && j < oe && (h < ol || h >= oh)) who = o;
                }
                uint64_t bm = __ballot(who >= 0);
                while (bm) {
                    const int l = __ffsll((unsigned long long)bm) - 1;
                    bm &= bm - 1ull;
                    if (lane == __shfl(who, l, 64)) bad = true;
                }
            }
        }
        if (bad) {
            on = false;
            atomicOr(&B.ctr->err, kErrInvalid);
        }
        // rows of the first and the last cluster; the span is empty if the first is further out
        int r0 = -1, r1 = -1;
        if (on) {
            const int64_t hs[2] = {A.hit_ids[hb], A.hit_ids[he - 1]};
            int rr[2];
            for (int q = 0; q < 2; ++q) {
                int a = 0, b = nr - 1;
                while (a < b) {
                    const int mid = (a + b + 1) >> 1;
                    if (B.off[g0 + mid] <= hs[q]) a = mid; else b = mid - 1;
                }
                rr[q] = a;
            }
            if (rr[0] <= rr[1]) {
                r0 = rr[0];
                r1 = rr[1];
            }
        }
        if (t < T) {
            A.rspan[2 * t] = r0;
            A.rspan[2 * t + 1] = r1;
        }
        // most tracks of a sector start and end on the same few rows: one atomic per
        // distinct entry of the wave
        for (int e = 0; e < 2; ++e) {
            const int64_t key = (r0 >= 0) ? (e == 0 ? g0 + r0 : g0 + r1 + 1) : -1;
            uint64_t todo = __ballot(key >= 0);
            while (todo) {
                const int64_t kw = readlane64(key, __ffsll((unsigned long long)todo) - 1);
                const uint64_t same = __ballot(key == kw);
                todo &= ~same;
                if (lane == __ffsll((unsigned long long)same) - 1)
                    atomicAdd(&A.rdiff[kw], e == 0 ? (int)__popcll(same) : -(int)__popcll(same));
            }
        }
    }
}

// pairs per row: the inclusive prefix of the difference array
__global__ void __launch_bounds__(256) k_r_count(RejectArgs A)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < A.n_rows_total; g += stride)
        A.rcnt[g] = (int32_t)(A.rtmp[g] + A.rdiff[g]);
}

// The pairs into their rows' buckets.  A wave takes 64 neighbouring tracks and serves the
// sectors among them in turn (usually one): it counts the sector's tracks on each row with
// ballots, takes every row's positions with one atomic, the atomics of 64 rows issued
// together, and then writes the pairs.
__global__ void __launch_bounds__(256) k_r_fill(Batch B, DevParams P, RejectArgs A)
{
    const int nr = P.n_rows, ns = P.n_sectors;
    const int lane = lane_id();
    int64_t T = *A.n_tracks;
    if (T > A.cap_tracks) T = A.cap_tracks;
    if (A.roff[A.n_rows_total] > A.cap_items) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&B.ctr->err, kErrOutCap);
        return;
    }
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t w0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64; w0 < T; w0 += nw * 64) {
        const int64_t t = w0 + lane;
        int r0 = -1, r1 = -1;
        int64_t g0 = -1;
        if (t < T) {
            r0 = A.rspan[2 * t];
            r1 = A.rspan[2 * t + 1];
            if (r0 >= 0) g0 = ((int64_t)A.tf[t] * ns + A.sector[t]) * nr;
        }
        uint64_t todo = __ballot(r0 >= 0);
        while (todo) {
            const int64_t gw = readlane64(g0, __ffsll((unsigned long long)todo) - 1);
            const bool on = r0 >= 0 && g0 == gw;
            todo &= ~__ballot(on);
            const int rlo = wave_min_i(on ? r0 : nr), rhi = wave_max_i(on ? r1 : -1);
            for (int c0 = rlo; c0 <= rhi; c0 += 64) {
                // lane L owns row c0 + L: count, then one atomic per row
                const int cn = min(64, rhi - c0 + 1);
                int cnt = 0;
                for (int q = 0; q < cn; ++q) {
                    const int r = c0 + q;
                    const int m = __popcll(__ballot(on && r >= r0 && r <= r1));
                    if (lane == q) cnt = m;
                }
                int64_t at = 0;
                if (lane < cn && cnt > 0) at = A.roff[gw + c0 + lane] + atomicAdd(&A.rcur[gw + c0 + lane], cnt);
                for (int q = 0; q < cn; ++q) {
                    const int r = c0 + q;
                    const bool act = on && r >= r0 && r <= r1;
                    const uint64_t m = __ballot(act);
                    const int64_t b = readlane64(at, q);
                    if (act) A.ritems[b + __popcll(m & lanemask_lt())] = (int32_t)t;
                }
            }
        }
    }
}

// Vicinity flags and keep flags, a block per row: a thread takes a pair, predicts its
// track's position on the row and tests the candidates of the window's bins.  The flags
// live in LDS; rows with more clusters than it holds take several passes, each flagging
// one slice of the row.  The keep flags are then written in input order: in the vicinity
// of a good track, or a cluster of one.
constexpr int kRowFlags = 16384;

__global__ void __launch_bounds__(256) k_r_rows(Batch B, DevParams P, RejectArgs A)
{
    __shared__ uint8_t lf[kRowFlags];
    const int nr = P.n_rows;
    const int lane = lane_id();
    int64_t T = *A.n_tracks;
    if (T > A.cap_tracks) T = A.cap_tracks;
    const bool have = A.roff[A.n_rows_total] <= A.cap_items;
    const double w = A.window;
    int64_t kept = 0;
    for (int64_t g = xcd_block(); g < A.n_rows_total; g += gridDim.x) {
        const int64_t base = B.off[g];
        const int n = (int)(B.off[g + 1] - base);
        if (n == 0) continue;
        const int64_t i0 = have ? A.roff[g] : 0, i1 = have ? A.roff[g + 1] : 0;
        const RowView v = row_view(B, P, g);
        const double x1 = (double)P.rx[g % nr];
        const float2* yz = B.yz + v.first;
        for (int c0 = 0; c0 < n; c0 += kRowFlags) {
            const int c1 = min(n, c0 + kRowFlags);
            for (int k = threadIdx.x; k < c1 - c0; k += blockDim.x) lf[k] = 0;
            __syncthreads();
            // pairs of this thread: i0 + threadIdx.x + m * blockDim.x; the next pair's track
            // and state are loaded while the current one is searched
            int64_t i = i0 + threadIdx.x;
            const int64_t tc = (i < i1) ? A.ritems[i] : -1;
            double p[5], x0 = 0.0;
            if (tc >= 0) {
                for (int q = 0; q < 5; ++q) p[q] = A.par[tc * 5 + q];
                x0 = A.xref[tc];
            }
            for (; i < i1; i += blockDim.x) {
                const int64_t tn = (i + blockDim.x < i1) ? A.ritems[i + blockDim.x] : -1;
                double yp = 0.0, zp = 0.0;
                int iy0 = 0, iy1 = 0, iz0 = 0, iz1 = -1;
                const bool ok = trk_predict(p, x0, x1, P, yp, zp) && fabs(yp) < 1.0e6 && fabs(zp) < 1.0e6;
                if (ok) {
                    bin_span((float)yp, (float)w, v.ylo, v.iby, v.ny, iy0, iy1);
                    bin_span((float)zp, (float)w, v.zlo, v.ibz, v.nz, iz0, iz1);
                }
                uint32_t a0 = 0, a1 = 0;
                if (ok) {
                    a0 = v.bs[iz0 * v.ny + iy0];
                    a1 = v.bs[iz0 * v.ny + iy1 + 1];
                }
                if (tn >= 0) {
                    for (int q = 0; q < 5; ++q) p[q] = A.par[tn * 5 + q];
                    x0 = A.xref[tn];
                }
                if (ok) {
                    // the window's bin rows; the next one's bounds are loaded ahead, and the
                    // candidates are read eight at a time
                    for (int iz = iz0; iz <= iz1; ++iz) {
                        uint32_t n0 = 0, n1 = 0;
                        if (iz < iz1) {
                            n0 = v.bs[(iz + 1) * v.ny + iy0];
                            n1 = v.bs[(iz + 1) * v.ny + iy1 + 1];
                        }
                        for (uint32_t k = a0; k < a1; k += 8) {
                            float2 cc[8];
#pragma unroll
                            for (int q = 0; q < 8; ++q) cc[q] = yz[min(k + (uint32_t)q, a1 - 1u)];
#pragma unroll
                            for (int q = 0; q < 8; ++q) {
                                const int kk = (int)k + q;
                                if ((uint32_t)kk < a1 && fabs((double)cc[q].x - yp) <= w &&
                                    fabs((double)cc[q].y - zp) <= w && kk >= c0 && kk < c1)
                                    lf[kk - c0] = 1;
                            }
                        }
                        a0 = n0;
                        a1 = n1;
                    }
                }
            }
            __syncthreads();
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int k = (int)B.iperm[base + i];
                if (k < c0 || k >= c1) continue;
                bool kp = lf[k - c0] != 0;
                if (!kp) {
                    const int32_t t = A.cluster_track[base + i];
                    if (t >= 0 && t < T) kp = fabs(A.par[(int64_t)t * 5 + 4]) * A.pt_min <= 1.0;
                }
                A.keep[base + i] = kp ? 1 : 0;
                kept += kp;
            }
            __syncthreads();
        }
    }
    kept = wave_sum(kept);
    if (lane == 0 && kept) atomicAdd((unsigned long long*)A.n_kept, (unsigned long long)kept);
}

void launch_reject(const Batch& b, const DevParams& p, const RejectArgs& r, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_r_clear, dim3(grid_for(r.n_rows_total + 1, 256, 1 << 16)), dim3(256), 0, s, r);
    hipLaunchKernelGGL(k_r_span, dim3(c.n_cu * 4), dim3(256), 0, s, b, p, r);
    ScanJob J1{};   // exclusive prefix of the difference array
    J1.a32 = r.rdiff;
    J1.outA = r.rtmp;
    J1.lo = 0;
    J1.hi = r.n_rows_total;
    J1.part = r.scan_part;
    launch_scan(J1, s);
    hipLaunchKernelGGL(k_r_count, dim3(grid_for(r.n_rows_total, 256, 1 << 16)), dim3(256), 0, s, r);
    ScanJob J2{};   // first pair of each row; roff[R] = all pairs
    J2.a32 = r.rcnt;
    J2.outA = r.roff;
    J2.lo = 0;
    J2.hi = r.n_rows_total;
    J2.totA = r.roff + r.n_rows_total;
    J2.part = r.scan_part;
    launch_scan(J2, s);
    hipLaunchKernelGGL(k_r_fill, dim3(c.n_cu * 8), dim3(256), 0, s, b, p, r);
    hipLaunchKernelGGL(k_r_rows, dim3(grid_for(r.n_rows_total, 1, 1 << 16)), dim3(256), 0, s, b, p, r);
}

void launch_hash(const Batch& b, int64_t n_clusters, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_hash_clear, dim3(1), dim3(64), 0, s, b);
    hipLaunchKernelGGL(k_hash, dim3(c.n_cu * 4), dim3(256), 0, s, b, n_clusters);
}

void launch_debug_views(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_links, dim3(grid_for(b.n_rows_total, 1, 1 << 16)), dim3(256), 0, s, b, p,
                       (int64_t)0, (int64_t)b.n_rows_total);
    hipLaunchKernelGGL(k_debug_starts, dim3(c.n_cu * 4), dim3(256), 0, s, b, p);
}

}  // namespace tpcsf
