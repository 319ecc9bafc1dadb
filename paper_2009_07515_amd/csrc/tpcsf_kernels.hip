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
        c->tl_count = 0;
        c->queue = 0;
        *B.o_ntracks = 0;
        *B.o_nhits = 0;
        if (B.cap_tracks >= 0) B.o_hit_off[0] = 0;
    }
}

// ------------------------------------------------------------------------------------
// Stage 1, grid (binary32).  One wave per row.  Extents are exact minima/maxima;
// ny = 1 + trunc((y_hi - y_lo)/b_y), nz alike; while ny*nz > cap_mul*n + cap_add the z bin
// (once nz == 1 the y bin) doubles.  Clusters are ordered by bin iz*ny + iy, ties by
// in-row index (stable counting sort: histogram, scan, then placement chunk by chunk in
// index order, each chunk ranked inside the wave by a ballot match on the bin key).
// The same pass clears the selection weights and the cluster->track map of the row.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_grid(Batch B, DevParams P, int64_t g0, int64_t g1)
{
#pragma clang fp contract(off)
    const int lane = lane_id();
    const int wpb = blockDim.x >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * wpb;
    for (int64_t g = g0 + (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); g < g1; g += nwaves) {
        const int64_t base = B.off[g];
        const int n = (int)(B.off[g + 1] - base);
        float ylo = INFINITY, yhi = -INFINITY, zlo = INFINITY, zhi = -INFINITY;
        bool bad = false;
        for (int i = lane; i < n; i += 64) {
            const float y = B.y[base + i], z = B.z[base + i];
            bad |= !(fabsf(y) <= 1.0e5f) || !(fabsf(z) <= 1.0e5f);
            ylo = fminf(ylo, y); yhi = fmaxf(yhi, y);
            zlo = fminf(zlo, z); zhi = fmaxf(zhi, z);
            B.W[base + i] = 0ull;
            B.o_cluster_track[base + i] = -1;
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            ylo = fminf(ylo, __shfl_xor(ylo, d, 64));
            yhi = fmaxf(yhi, __shfl_xor(yhi, d, 64));
            zlo = fminf(zlo, __shfl_xor(zlo, d, 64));
            zhi = fmaxf(zhi, __shfl_xor(zhi, d, 64));
        }
        if (__ballot(bad) != 0ull) {
            if (lane == 0) atomicOr(&B.ctr->err, kErrInvalid);
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
        if (lane == 0) {
            B.row_lo[g] = make_float2(ylo, zlo);
            B.row_bin[g] = make_float2(by, bz);
            B.row_nb[g] = make_int2(ny, nz);
        }
        const int nb = ny * nz;
        uint32_t* bs = B.bin_start + bin_base(P, base, g);
        uint32_t* bf = B.bin_fill + bin_base(P, base, g);
        for (int b = lane; b <= nb; b += 64) {
            st_rlx(bs + b, 0u);
            st_rlx(bf + b, 0u);
        }
        wave_mem_fence();
        for (int i = lane; i < n; i += 64) {
            const int bin = bin_of(B.z[base + i], zlo, bz, nz) * ny + bin_of(B.y[base + i], ylo, by, ny);
            atomicAdd(bs + bin + 1, 1u);
        }
        wave_mem_fence();
        uint32_t carry = 0;
        for (int b0 = 0; b0 < nb; b0 += 64) {
            const int b = b0 + lane;
            const uint32_t v = (b < nb) ? ld_rlx(bs + 1 + b) : 0u;
            const uint32_t inc = wave_incl_scan(v) + carry;
            if (b < nb) st_rlx(bs + 1 + b, inc);
            carry = __shfl(inc, 63, 64);
        }
        wave_mem_fence();
        const int nbits = 32 - __clz(nb > 1 ? nb - 1 : 1);
        for (int i0 = 0; i0 < n; i0 += 64) {
            const int i = i0 + lane;
            const bool valid = i < n;
            const float y = valid ? B.y[base + i] : 0.0f;
            const float z = valid ? B.z[base + i] : 0.0f;
            const uint32_t bin = valid ? (uint32_t)(bin_of(z, zlo, bz, nz) * ny + bin_of(y, ylo, by, ny)) : 0u;
            const uint64_t eq = match_eq(bin, valid, nbits);
            const int rank = __popcll(eq & lanemask_lt());
            const int leader = valid ? (__ffsll((unsigned long long)eq) - 1) : 0;
            uint32_t old = 0;
            if (valid && lane == leader) old = atomicAdd(bf + bin, (uint32_t)__popcll(eq));
            old = __shfl(old, leader, 64);
            if (valid) {
                const uint32_t pos = ld_rlx(bs + bin) + old + (uint32_t)rank;
                B.ys[base + pos] = y;
                B.zs[base + pos] = z;
                B.perm[base + pos] = (uint32_t)i;
            }
        }
    }
}

// ------------------------------------------------------------------------------------
// Stage 2, neighbour links (binary32, no contraction, correctly rounded division).
// One block per row; each thread takes clusters in sorted (bin) order so that the lanes
// of a wave query neighbouring windows.  A candidate in row r+-1 must satisfy
// |y_c - y_h| <= win_y and |z_c - z_h| <= win_z; the grid bins visited cover the window
// widened by a few ulps, and every candidate is then tested exactly.  The pair with the
// least slope change D wins if D <= kink_max; ties go to the smaller u, then the
// smaller d (in-row indices).
// ------------------------------------------------------------------------------------
struct RowView {
    int64_t first;            // first cluster of the row
    float ylo, zlo, by, bz;
    int ny, nz;
    const uint32_t* bs;       // bin_start of the row
};

__device__ __forceinline__ RowView row_view(const Batch& B, const DevParams& P, int64_t g)
{
    RowView v;
    v.first = B.off[g];
    const float2 lo = B.row_lo[g], bn = B.row_bin[g];
    const int2 nb = B.row_nb[g];
    v.ylo = lo.x; v.zlo = lo.y; v.by = bn.x; v.bz = bn.y; v.ny = nb.x; v.nz = nb.y;
    v.bs = B.bin_start + bin_base(P, v.first, g);
    return v;
}

__device__ __forceinline__ void window_bins(const RowView& v, float yq, float zq, float wy, float wz,
                                            int& iy0, int& iy1, int& iz0, int& iz1)
{
    // widen by a relative margin that exceeds the rounding of |c - q| and of q -+ w
    const float ey = (fabsf(yq) + wy + 1.0f) * 4.0e-6f;
    const float ez = (fabsf(zq) + wz + 1.0f) * 4.0e-6f;
    iy0 = bin_of(yq - (wy + ey), v.ylo, v.by, v.ny);
    iy1 = bin_of(yq + (wy + ey), v.ylo, v.by, v.ny);
    iz0 = bin_of(zq - (wz + ez), v.zlo, v.bz, v.nz);
    iz1 = bin_of(zq + (wz + ez), v.zlo, v.bz, v.nz);
}

__global__ void __launch_bounds__(1024) k_links(Batch B, DevParams P, int64_t g0, int64_t g1)
{
#pragma clang fp contract(off)
    const int nr = P.n_rows;
    for (int64_t g = g0 + blockIdx.x; g < g1; g += gridDim.x) {
        const int r = (int)(g % nr);
        const int64_t base = B.off[g];
        const int n = (int)(B.off[g + 1] - base);
        if (r == 0 || r == nr - 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                B.up[base + i] = -1;
                B.dn[base + i] = -1;
            }
            continue;
        }
        const RowView U = row_view(B, P, g + 1);
        const RowView D = row_view(B, P, g - 1);
        const float dxu = P.rx[r + 1] - P.rx[r];
        const float dxd = P.rx[r] - P.rx[r - 1];
        const float wy = P.win_y, wz = P.win_z, kmax = P.kink_max;
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            const float yh = B.ys[base + k], zh = B.zs[base + k];
            const int h = (int)B.perm[base + k];
            int uy0, uy1, uz0, uz1, dy0, dy1, dz0, dz1;
            window_bins(U, yh, zh, wy, wz, uy0, uy1, uz0, uz1);
            window_bins(D, yh, zh, wy, wz, dy0, dy1, dz0, dz1);
            float bD = 0.0f;
            int bu = -1, bd = -1;
            for (int iz = uz0; iz <= uz1; ++iz) {
                const uint32_t ka = U.bs[iz * U.ny + uy0], kb = U.bs[iz * U.ny + uy1 + 1];
                for (uint32_t ku = ka; ku < kb; ++ku) {
                    const float yu = B.ys[U.first + ku], zu = B.zs[U.first + ku];
                    if (!(fabsf(yu - yh) <= wy && fabsf(zu - zh) <= wz)) continue;
                    const int u = (int)B.perm[U.first + ku];
                    const float tuy = (yu - yh) / dxu;
                    const float tuz = (zu - zh) / dxu;
                    for (int jz = dz0; jz <= dz1; ++jz) {
                        const uint32_t ma = D.bs[jz * D.ny + dy0], mb = D.bs[jz * D.ny + dy1 + 1];
                        for (uint32_t kd = ma; kd < mb; ++kd) {
                            const float yd = B.ys[D.first + kd], zd = B.zs[D.first + kd];
                            if (!(fabsf(yd - yh) <= wy && fabsf(zd - zh) <= wz)) continue;
                            const int d = (int)B.perm[D.first + kd];
                            const float tdy = (yh - yd) / dxd;
                            const float tdz = (zh - zd) / dxd;
                            const float ay = tuy - tdy;
                            const float az = tuz - tdz;
                            const float sy = ay * ay;
                            const float sz = az * az;
                            const float Dk = sy + sz;
                            if (!(Dk <= kmax)) continue;
                            const bool better = bu < 0 || Dk < bD ||
                                                (Dk == bD && (u < bu || (u == bu && d < bd)));
                            if (better) { bD = Dk; bu = u; bd = d; }
                        }
                    }
                }
            }
            B.up[base + h] = bu;
            B.dn[base + h] = bd;
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
    for (int64_t g = g0 + blockIdx.x; g < g1; g += gridDim.x) {
        const int r = (int)(g % nr);
        const int64_t base = B.off[g];
        const int n = (int)(B.off[g + 1] - base);
        const int64_t fu = (r + 1 < nr) ? B.off[g + 1] : 0;
        const int64_t fd = (r > 0) ? B.off[g - 1] : 0;
        int cnt = 0;
        for (int h = threadIdx.x; h < n; h += blockDim.x) {
            const int u = B.up[base + h], d = B.dn[base + h];
            const int cu = (u >= 0 && B.dn[fu + u] == h) ? u : -1;
            const int cd = (d >= 0 && B.up[fd + d] == h) ? d : -1;
            B.cup[base + h] = cu;
            B.cdn[base + h] = cd;
            cnt += (cu >= 0 && cd < 0);
        }
        int total;
        block_excl_scan(cnt, &total, lds);
        if (threadIdx.x == 0) B.row_nstart[g] = total;
    }
}

// ------------------------------------------------------------------------------------
// Stage 4, starts: compaction of the chain bottoms in (row, in-row index) order at the
// row's scanned base; the position in this list is the start's rank.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_starts(Batch B, DevParams P, int64_t g0, int64_t g1)
{
    __shared__ int lds[17];
    for (int64_t g = g0 + blockIdx.x; g < g1; g += gridDim.x) {
        const int64_t base = B.off[g];
        const int n = (int)(B.off[g + 1] - base);
        int64_t sb = B.row_sbase[g];
        for (int h0 = 0; h0 < n; h0 += blockDim.x) {
            const int h = h0 + threadIdx.x;
            const int f = (h < n) && B.cup[base + h] >= 0 && B.cdn[base + h] < 0;
            int total;
            const int pos = block_excl_scan(f, &total, lds);
            if (f) {
                B.start_row[sb + pos] = (int32_t)g;
                B.start_idx[sb + pos] = h;
            }
            sb += total;
        }
    }
}

// ------------------------------------------------------------------------------------
// Device-wide exclusive scans (three kernels: per-block sums, a one-block scan of the
// sums that also advances the running bases, per-block scans).  Ranges may come from
// device memory, so one graph serves every batch of the same shape.
// ------------------------------------------------------------------------------------
struct ScanJob {
    const int64_t* a64;       // channel A input (int64) or null
    const int32_t* a32;       // channel A input (int32) if a64 is null
    const int32_t* b32;       // channel B input (int32) or null
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

__device__ __forceinline__ int64_t scanA(const ScanJob& J, int64_t i) { return J.a64 ? J.a64[i] : (int64_t)J.a32[i]; }

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

// ------------------------------------------------------------------------------------
// Kalman filter in binary64.  State (y, z, sin phi, tan lambda, q/pT) at plane x;
// curvature kappa = a * q/pT.  Covariance: 15-element lower triangle.
// ------------------------------------------------------------------------------------
struct Trk {
    double x;
    double p[5];
    double c[15];
};

// asin(h)/h and its derivative; Taylor series near 0
__device__ __forceinline__ void arc_factor(double h, double& A, double& Ap)
{
    if (fabs(h) < 0.01) {
        const double h2 = h * h;
        A = 1.0 + h2 * (1.0 / 6.0 + h2 * (3.0 / 40.0 + h2 * (5.0 / 112.0)));
        Ap = h * (1.0 / 3.0 + h2 * (3.0 / 10.0 + h2 * (15.0 / 56.0 + h2 * (35.0 / 144.0))));
    } else {
        const double as = asin(h);
        const double ih = 1.0 / h;
        A = as * ih;
        Ap = (h / sqrt((1.0 - h) * (1.0 + h)) - as) * ih * ih;
    }
}

// Exact helix step to the plane x1 with the analytic Jacobian.  sin(phi) is linear in x;
// y follows the chord at the mean angle; z follows the arc length chord*asin(h)/h with
// h = kappa*chord/2.  Fails (state unchanged) when |sin(phi)| would reach sinphi_max.
__device__ bool trk_propagate(Trk& t, double x1, const DevParams& P)
{
    const double dx = x1 - t.x;
    const double s0 = t.p[2];
    const double tl = t.p[3];
    const double kap = P.a * t.p[4];
    const double s1 = s0 + kap * dx;
    if (!(fabs(s0) < P.sinphi_max) || !(fabs(s1) < P.sinphi_max)) return false;
    const double c0 = sqrt((1.0 - s0) * (1.0 + s0));
    const double c1 = sqrt((1.0 - s1) * (1.0 + s1));
    const double cs = c0 + c1;
    const double tb = (s0 + s1) / cs;
    const double sec2 = 1.0 + tb * tb;
    const double sec = sqrt(sec2);
    const double chord = dx * sec;
    const double h = 0.5 * kap * chord;
    if (!(fabs(h) < 1.0)) return false;
    double A, Ap;
    arc_factor(h, A, Ap);
    const double ds = chord * A;
    const double ic0 = 1.0 / c0, ic1 = 1.0 / c1;
    const double q = 0.5 * tb * dx * ic1;
    const double j02 = 0.5 * dx * sec2 * (ic0 + ic1);
    const double j04 = P.a * (0.5 * dx * dx * sec2 * ic1);
    const double j12 = tl * (dx * (s0 + s1) * ic0 * ic1 / cs);
    const double j13 = ds;
    const double j14 = tl * P.a * (chord * (q * A + Ap * (0.5 * chord) * (1.0 + kap * q)));
    const double j24 = P.a * dx;

    t.p[0] += dx * tb;
    t.p[1] += tl * ds;
    t.p[2] = s1;
    t.x = x1;

    // C <- J C J^T with J = identity + {j02, j04, j12, j13, j14, j24}
    double* c = t.c;
    const double c00 = c[0], c10 = c[1], c11 = c[2], c20 = c[3], c21 = c[4], c22 = c[5];
    const double c30 = c[6], c31 = c[7], c32 = c[8], c33 = c[9];
    const double c40 = c[10], c41 = c[11], c42 = c[12], c43 = c[13], c44 = c[14];
    // rows of A = J C (A_ij for all i, j)
    const double a00 = c00 + j02 * c20 + j04 * c40, a01 = c10 + j02 * c21 + j04 * c41;
    const double a02 = c20 + j02 * c22 + j04 * c42, a03 = c30 + j02 * c32 + j04 * c43;
    const double a04 = c40 + j02 * c42 + j04 * c44;
    const double a10 = c10 + j12 * c20 + j13 * c30 + j14 * c40;
    const double a11 = c11 + j12 * c21 + j13 * c31 + j14 * c41;
    const double a12 = c21 + j12 * c22 + j13 * c32 + j14 * c42;
    const double a13 = c31 + j12 * c32 + j13 * c33 + j14 * c43;
    const double a14 = c41 + j12 * c42 + j13 * c43 + j14 * c44;
    const double a20 = c20 + j24 * c40, a21 = c21 + j24 * c41, a22 = c22 + j24 * c42;
    const double a23 = c32 + j24 * c43, a24 = c42 + j24 * c44;
    // C' = A J^T (lower triangle); rows 3 and 4 of A equal those of C
    c[0] = a00 + j02 * a02 + j04 * a04;
    c[1] = a10 + j02 * a12 + j04 * a14;
    c[2] = a11 + j12 * a12 + j13 * a13 + j14 * a14;
    c[3] = a20 + j02 * a22 + j04 * a24;
    c[4] = a21 + j12 * a22 + j13 * a23 + j14 * a24;
    c[5] = a22 + j24 * a24;
    c[6] = c30 + j02 * c32 + j04 * c43;
    c[7] = c31 + j12 * c32 + j13 * c33 + j14 * c43;
    c[8] = c32 + j24 * c43;
    c[9] = c33;
    c[10] = c40 + j02 * c42 + j04 * c44;
    c[11] = c41 + j12 * c42 + j13 * c43 + j14 * c44;
    c[12] = c42 + j24 * c44;
    c[13] = c43;
    c[14] = c44;
    return true;
}

__device__ __forceinline__ double trk_chi2(const Trk& t, double my, double mz, const DevParams& P)
{
    const double r0 = my - t.p[0], r1 = mz - t.p[1];
    const double s00 = t.c[0] + P.sy2, s01 = t.c[1], s11 = t.c[2] + P.sz2;
    return (r0 * r0 * s11 - 2.0 * r0 * r1 * s01 + r1 * r1 * s00) / (s00 * s11 - s01 * s01);
}

// Kalman update with the cluster (my, mz), R = diag(sy2, sz2).
__device__ void trk_update(Trk& t, double my, double mz, const DevParams& P)
{
    const double r0 = my - t.p[0], r1 = mz - t.p[1];
    double* c = t.c;
    const double s00 = c[0] + P.sy2, s01 = c[1], s11 = c[2] + P.sz2;
    const double idet = 1.0 / (s00 * s11 - s01 * s01);
    const double i00 = s11 * idet, i01 = -s01 * idet, i11 = s00 * idet;
    const double h0[5] = {c[0], c[1], c[3], c[6], c[10]};
    const double h1[5] = {c[1], c[2], c[4], c[7], c[11]};
    double k0[5], k1[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        k0[i] = h0[i] * i00 + h1[i] * i01;
        k1[i] = h0[i] * i01 + h1[i] * i11;
        t.p[i] += k0[i] * r0 + k1[i] * r1;
    }
    int k = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j, ++k) c[k] -= k0[i] * h0[j] + k1[i] * h1[j];
}

__device__ __forceinline__ void trk_reset_cov(Trk& t, const DevParams& P)
{
#pragma unroll
    for (int i = 0; i < 15; ++i) t.c[i] = 0.0;
    t.c[0] = P.c0[0]; t.c[2] = P.c0[1]; t.c[5] = P.c0[2]; t.c[9] = P.c0[3]; t.c[14] = P.c0[4];
}

// Circle through three (x, y) points, traversed in order: curvature and sin(phi) at the
// first; tan(lambda) from the z change over the arc to the last.
__device__ bool trk_seed(Trk& t, const double* x, const double* y, const double* z, const DevParams& P)
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

// Least-chi2 cluster of row g inside the follow window; -1 if none.
__device__ int search_row(const Batch& B, const DevParams& P, int64_t g, const Trk& t, double& best_chi2)
{
    const int64_t first = B.off[g];
    const int n = (int)(B.off[g + 1] - first);
    best_chi2 = 0.0;
    if (n == 0) return -1;
    const RowView v = row_view(B, P, g);
    const double s00 = t.c[0] + P.sy2, s01 = t.c[1], s11 = t.c[2] + P.sz2;
    double wy = P.nsig * sqrt(s00), wz = P.nsig * sqrt(s11);
    if (wy > (double)P.win_y) wy = (double)P.win_y;
    if (wz > (double)P.win_z) wz = (double)P.win_z;
    const double yp = t.p[0], zp = t.p[1];
    if (!(fabs(yp) < 1.0e6) || !(fabs(zp) < 1.0e6)) return -1;
    const double my = (fabs(yp) + wy + 1.0) * 1.0e-5, mz = (fabs(zp) + wz + 1.0) * 1.0e-5;
    const int iy0 = bin_of((float)(yp - wy - my), v.ylo, v.by, v.ny);
    const int iy1 = bin_of((float)(yp + wy + my), v.ylo, v.by, v.ny);
    const int iz0 = bin_of((float)(zp - wz - mz), v.zlo, v.bz, v.nz);
    const int iz1 = bin_of((float)(zp + wz + mz), v.zlo, v.bz, v.nz);
    const double idet = 1.0 / (s00 * s11 - s01 * s01);
    int best = -1;
    for (int iz = iz0; iz <= iz1; ++iz) {
        const uint32_t ka = v.bs[iz * v.ny + iy0], kb = v.bs[iz * v.ny + iy1 + 1];
        for (uint32_t k = ka; k < kb; ++k) {
            const double dy = (double)B.ys[first + k] - yp;
            const double dz = (double)B.zs[first + k] - zp;
            if (!(fabs(dy) <= wy) || !(fabs(dz) <= wz)) continue;
            const double chi2 = (dy * dy * s11 - 2.0 * dy * dz * s01 + dz * dz * s00) * idet;
            const int c = (int)B.perm[first + k];
            if (best < 0 || chi2 < best_chi2 || (chi2 == best_chi2 && c < best)) {
                best = c;
                best_chi2 = chi2;
            }
        }
    }
    return best;
}

__device__ int follow(const Batch& B, const DevParams& P, Trk& t, int64_t gs, int r_from, int r_to, int step,
                      uint16_t* H)
{
    int misses = 0, added = 0;
    for (int r = r_from; r != r_to; r += step) {
        if (!trk_propagate(t, (double)P.rx[r], P)) break;
        double chi2;
        const int c = search_row(B, P, gs + r, t, chi2);
        if (c >= 0 && chi2 <= P.chi2_max) {
            const int64_t gi = B.off[gs + r] + c;
            trk_update(t, (double)B.y[gi], (double)B.z[gi], P);
            H[r] = (uint16_t)c;
            misses = 0;
            ++added;
        } else if (++misses > P.max_miss) {
            break;
        }
    }
    return added;
}

// ------------------------------------------------------------------------------------
// Stage 5, tracklets: one lane per chain bottom, pulled from a persistent work queue.
// Chain along the cleaned up-links (>= min_chain clusters), three-point seed, Kalman
// update over the chain, follow outward, reset C to C0 keeping p and refit inward over
// all clusters so far, follow inward.  The clusters are recorded per row in a slot.
// ------------------------------------------------------------------------------------
__device__ void build_tracklet(const Batch& B, const DevParams& P, int64_t t)
{
    const int nr = P.n_rows;
    const int64_t g = B.start_row[t];
    const int i0 = B.start_idx[t];
    const int r0 = (int)(g % nr);
    const int64_t gs = g - r0;
    int L = 0;
    for (int r = r0, c = i0; r < nr && c >= 0; ++r) {
        ++L;
        c = B.cup[B.off[gs + r] + c];
    }
    if (L < P.min_chain) {
        B.tl_n[t] = 0;
        return;
    }
    const int slot = atomicAdd(&B.ctr->tl_count, 1);
    if (slot >= B.cap_tl) {
        atomicOr(&B.ctr->err, kErrTrackletCap);
        B.tl_n[t] = 0;
        return;
    }
    B.tl_slot[t] = slot;
    uint16_t* H = B.tl_hits + (int64_t)slot * nr;
    for (int r = 0; r < nr; ++r) H[r] = kNoHit;
    // seed clusters: first, middle and last of the chain (distinct rows for L >= 3)
    const int rs[3] = {r0, r0 + (L - 1) / 2, r0 + L - 1};
    double sx[3], sy[3], sz[3];
    for (int r = r0, c = i0; r < r0 + L; ++r) {
        H[r] = (uint16_t)c;
        const int64_t gi = B.off[gs + r] + c;
        for (int q = 0; q < 3; ++q)
            if (r == rs[q]) {
                sx[q] = (double)P.rx[r];
                sy[q] = (double)B.y[gi];
                sz[q] = (double)B.z[gi];
            }
        c = B.cup[gi];
    }
    Trk tr;
    int n = 0;
    bool ok = trk_seed(tr, sx, sy, sz, P);
    if (ok) {
        trk_reset_cov(tr, P);
        for (int r = r0; r < r0 + L; ++r) {
            if (r > r0 && !trk_propagate(tr, (double)P.rx[r], P)) { ok = false; break; }
            const int64_t gi = B.off[gs + r] + H[r];
            trk_update(tr, (double)B.y[gi], (double)B.z[gi], P);
        }
    }
    if (ok) {
        n = L + follow(B, P, tr, gs, r0 + L, nr, +1, H);
        trk_reset_cov(tr, P);
        for (int r = nr - 1; r >= r0; --r) {
            if (H[r] == kNoHit) continue;
            if (!trk_propagate(tr, (double)P.rx[r], P)) { ok = false; break; }
            const int64_t gi = B.off[gs + r] + H[r];
            trk_update(tr, (double)B.y[gi], (double)B.z[gi], P);
        }
    }
    if (ok) {
        n += follow(B, P, tr, gs, r0 - 1, -1, -1, H);
    } else {
        for (int r = 0; r < nr; ++r) H[r] = kNoHit;
        n = 0;
    }
    B.tl_n[t] = n;
}

__global__ void __launch_bounds__(256) k_tracklets(Batch B, DevParams P, int chunk)
{
    const int64_t lo = B.ctr->rank_lo, hi = B.ctr->rank_hi;
    const int lane = lane_id();
    const int per_wave = 64 * chunk;
    for (;;) {
        int take = 0;
        if (lane == 0) take = atomicAdd(&B.ctr->queue, per_wave);
        take = __shfl(take, 0, 64);
        const int64_t t0 = lo + take;
        if (t0 >= hi) break;
        for (int k = 0; k < chunk; ++k) {
            const int64_t t = t0 + (int64_t)k * 64 + lane;
            if (t < hi) build_tracklet(B, P, t);
        }
    }
}

// ------------------------------------------------------------------------------------
// Stage 6, selection.  w = (n << 32) | (2^32 - 1 - rank); every cluster ends with the
// largest w of the tracklets that contain it (64-bit atomic max, order independent).
// Tracklets shorter than min_track_hits can neither be accepted nor outweigh a longer
// one, so they do not take part.  The same launch rewinds the tracklet work queue.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long weight_of(int n, int64_t t)
{
    return ((unsigned long long)(uint32_t)n << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)t);
}

__global__ void __launch_bounds__(256) k_claim(Batch B, DevParams P)
{
    const int64_t lo = B.ctr->rank_lo, hi = B.ctr->rank_hi;
    const int nr = P.n_rows;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < hi; t += stride) {
        const int n = B.tl_n[t];
        if (n < P.min_track_hits) continue;
        const unsigned long long w = weight_of(n, t);
        const int64_t g = B.start_row[t];
        const int64_t gs = g - g % nr;
        const uint16_t* H = B.tl_hits + (int64_t)B.tl_slot[t] * nr;
        for (int r = 0; r < nr; ++r) {
            const uint16_t c = H[r];
            if (c != kNoHit) atomicMax(&B.W[B.off[gs + r] + c], w);
        }
    }
}

// ------------------------------------------------------------------------------------
// Stage 7, keep + final fit.  A tracklet keeps the clusters that carry its own weight and
// is a track if it keeps >= min_track_hits.  Final fit on the kept clusters (inner to
// outer): three-point seed, C = C0, update outward; C = C0 keeping p, update inward.
// Result at the innermost kept cluster; a failed fit drops the track.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_keepfit(Batch B, DevParams P)
{
    const int64_t lo = B.ctr->rank_lo, hi = B.ctr->rank_hi;
    const int nr = P.n_rows;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) B.ctr->queue = 0;   // tracklet queue is done
    for (int64_t t = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < hi; t += stride) {
        B.trk_flag[t] = 0;
        B.hit_cnt[t] = 0;
        const int n = B.tl_n[t];
        if (n < P.min_track_hits) continue;
        const unsigned long long w = weight_of(n, t);
        const int64_t g = B.start_row[t];
        const int64_t gs = g - g % nr;
        const int slot = B.tl_slot[t];
        const uint16_t* H = B.tl_hits + (int64_t)slot * nr;
        uint64_t m[4] = {0, 0, 0, 0};
        int kept = 0;
        for (int r = 0; r < nr; ++r) {
            const uint16_t c = H[r];
            if (c == kNoHit) continue;
            if (B.W[B.off[gs + r] + c] == w) {
                m[r >> 6] |= 1ull << (r & 63);
                ++kept;
            }
        }
        if (kept < P.min_track_hits) continue;
        // seed rows: first, middle and last kept cluster
        const int want[3] = {0, (kept - 1) / 2, kept - 1};
        int rsel[3] = {0, 0, 0};
        for (int r = 0, idx = 0; r < nr; ++r) {
            if (!((m[r >> 6] >> (r & 63)) & 1ull)) continue;
            for (int q = 0; q < 3; ++q)
                if (want[q] == idx) rsel[q] = r;
            ++idx;
        }
        double sx[3], sy[3], sz[3];
        for (int q = 0; q < 3; ++q) {
            const int64_t gi = B.off[gs + rsel[q]] + H[rsel[q]];
            sx[q] = (double)P.rx[rsel[q]];
            sy[q] = (double)B.y[gi];
            sz[q] = (double)B.z[gi];
        }
        Trk tr;
        bool ok = trk_seed(tr, sx, sy, sz, P);
        if (ok) {
            trk_reset_cov(tr, P);
            for (int r = rsel[0]; r <= rsel[2]; ++r) {
                if (!((m[r >> 6] >> (r & 63)) & 1ull)) continue;
                if (r > rsel[0] && !trk_propagate(tr, (double)P.rx[r], P)) { ok = false; break; }
                const int64_t gi = B.off[gs + r] + H[r];
                trk_update(tr, (double)B.y[gi], (double)B.z[gi], P);
            }
        }
        double chi2 = 0.0;
        if (ok) {
            trk_reset_cov(tr, P);
            for (int r = rsel[2]; r >= rsel[0]; --r) {
                if (!((m[r >> 6] >> (r & 63)) & 1ull)) continue;
                if (r < rsel[2] && !trk_propagate(tr, (double)P.rx[r], P)) { ok = false; break; }
                const int64_t gi = B.off[gs + r] + H[r];
                const double my = (double)B.y[gi], mz = (double)B.z[gi];
                chi2 += trk_chi2(tr, my, mz, P);
                trk_update(tr, my, mz, P);
            }
        }
        if (ok) {
            for (int i = 0; i < 5; ++i) ok = ok && isfinite(tr.p[i]);
            for (int i = 0; i < 15; ++i) ok = ok && isfinite(tr.c[i]);
        }
        if (!ok) continue;
        double* fp = B.f_par + (int64_t)slot * 5;
        double* fc = B.f_cov + (int64_t)slot * 15;
        for (int i = 0; i < 5; ++i) fp[i] = tr.p[i];
        for (int i = 0; i < 15; ++i) fc[i] = tr.c[i];
        B.f_chi2[slot] = chi2;
        B.f_xref[slot] = tr.x;
        for (int i = 0; i < 4; ++i) B.f_mask[(int64_t)slot * 4 + i] = m[i];
        B.trk_flag[t] = 1;
        B.hit_cnt[t] = kept;
    }
}

// ------------------------------------------------------------------------------------
// Stage 8, emit: tracks in rank order at their scanned positions, hits inner to outer,
// cluster -> track map.  Writes beyond the caller's capacity are dropped and flagged.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_emit(Batch B, DevParams P)
{
    const int64_t lo = B.ctr->rank_lo, hi = B.ctr->rank_hi;
    const int nr = P.n_rows;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < hi; t += stride) {
        if (!B.trk_flag[t]) continue;
        const int64_t T = B.trk_idx[t];
        const int64_t hp = B.hit_pos[t];
        const int nk = B.hit_cnt[t];
        const int slot = B.tl_slot[t];
        const int64_t g = B.start_row[t];
        const int64_t gs = g - g % nr;
        if (T >= B.cap_tracks || hp + nk > B.cap_hits) {
            atomicOr(&B.ctr->err, kErrOutCap);
            continue;
        }
        for (int i = 0; i < 5; ++i) B.o_par[T * 5 + i] = B.f_par[(int64_t)slot * 5 + i];
        for (int i = 0; i < 15; ++i) B.o_cov[T * 15 + i] = B.f_cov[(int64_t)slot * 15 + i];
        B.o_xref[T] = B.f_xref[slot];
        B.o_chi2[T] = B.f_chi2[slot];
        B.o_ndf[T] = 2 * nk - 5;
        B.o_nhits_trk[T] = nk;
        B.o_sector[T] = (int32_t)((g / nr) % P.n_sectors);
        B.o_tf[T] = (int32_t)(g / ((int64_t)nr * P.n_sectors));
        B.o_hit_off[T + 1] = hp + nk;
        const uint64_t* m = B.f_mask + (int64_t)slot * 4;
        const uint16_t* H = B.tl_hits + (int64_t)slot * nr;
        int64_t j = hp;
        for (int w = 0; w < 4; ++w) {
            uint64_t bits = m[w];
            while (bits) {
                const int r = w * 64 + __ffsll((unsigned long long)bits) - 1;
                bits &= bits - 1;
                const int64_t gi = B.off[gs + r] + H[r];
                B.o_hit_ids[j++] = (int32_t)gi;
                B.o_cluster_track[gi] = (int32_t)T;
            }
        }
    }
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

void launch_grid(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s)
{
    const int wpb = c.block / 64;
    hipLaunchKernelGGL(k_grid, dim3(grid_for(g1 - g0, wpb, 1 << 16)), dim3(c.block), 0, s, b, p, g0, g1);
}

void launch_links(const Batch& b, const DevParams& p, int64_t g0, int64_t g1, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_links, dim3(grid_for(g1 - g0, 1, 1 << 16)), dim3(c.block), 0, s, b, p, g0, g1);
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

void launch_tracklets(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s)
{
    const int wpb = c.tl_block / 64;
    const int blocks = c.n_cu * (16 / wpb > 0 ? 16 / wpb : 1);
    hipLaunchKernelGGL(k_tracklets, dim3(blocks), dim3(c.tl_block), 0, s, b, p, c.chunk);
}

void launch_claim(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_claim, dim3(c.n_cu * 4), dim3(256), 0, s, b, p);
}

void launch_keepfit(const Batch& b, const DevParams& p, const LaunchCfg& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_keepfit, dim3(c.n_cu * 4), dim3(256), 0, s, b, p);
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

}  // namespace tpcsf
