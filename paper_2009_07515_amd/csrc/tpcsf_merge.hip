// Merging of sector tracks across the azimuthal sector edges, and the refit of the merged
// tracks across sector frames: the track-fit stage that follows sector tracking
// (arXiv:2009.07515, Sec. 7, Table 1 "Track Fit"; the paper gives no procedure).
//
// Definition (stated in full at tpcsf_merge in include/tpcsf.h): a track whose outermost
// cluster lies near an edge, at a larger radius than its innermost one, is an "outer end"
// A; it is matched against the "inner ends" B of the neighbouring sector beyond that edge
// (innermost cluster near the shared edge, at a larger radius than A's outermost).  A's
// outer state is rotated into B's frame, gated by a linear prediction of B's y and z, and
// propagated to B's innermost row; the pair's chi2 of the 5-parameter difference with the
// summed covariances must not exceed merge_chi2.  Each A takes its least-chi2 B (ties:
// smaller B), each B keeps the least-chi2 A among those (ties: smaller A): a link.  Chains
// of links become merged tracks, refitted across the sectors; a failed refit dissolves
// the chain.  Merged tracks come in the order of their first segment.
//
// Layout: a lane per track for the per-track steps and per outer end for the match (8
// lanes per outer end, splitting its window, measured slower), a wave per input track for
// the cluster gathers and copies, 256 chains per block for the refit; the inner ends of
// each (time frame, sector, edge) are listed densely in a region starting at that sector's
// first track and ordered by z, so that an outer end scans only the part of its candidate
// list its gate can accept.  Decisions that the oracle takes on cluster coordinates and on the
// linear gate are evaluated without contraction, as there.
#include "tpcsf_internal.h"
#include "tpcsf_kalman.h"

#include <math.h>

namespace tpcsf {

namespace {

constexpr int kMergeThreads = 256;
constexpr int kCopyTracks = 4;   // hit lists copied per pass by the gather and copy kernels

__device__ __forceinline__ int64_t wave_sum64(int64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// adds each lane's v to *ctr (all lanes of the wave must call it)
__device__ __forceinline__ void wave_add(int64_t* ctr, int64_t v)
{
    const int64_t t = wave_sum64(v);
    if ((threadIdx.x & 63) == 0 && t != 0) atomicAdd((unsigned long long*)ctr, (unsigned long long)t);
}

// row of cluster h inside the sector whose rows start at global row g0: the last r with
// off[g0 + r] <= h
__device__ __forceinline__ int row_of(const int64_t* off, int64_t g0, int nr, int64_t h)
{
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[g0 + mid] <= h) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// orders the LDS accesses of the lanes of one wave (no block barrier)
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// azimuth step index between two sectors of one side, d in (-S/2, S/2], as a table index
__device__ __forceinline__ int step_index(int s0, int s1, int S)
{
    int d = (s1 % S) - (s0 % S);
    if (2 * d > S) d -= S;
    if (2 * d <= -S) d += S;
    return d + S / 2;
}

// d^T S^-1 d for a symmetric 5x5 S (lower triangle) by Cholesky; false if S is not
// positive definite
__device__ bool chi2_5(const double* S15, const double* d, double& out)
{
    double L[15];
    int k = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j, ++k) {
            double v = S15[k];
#pragma unroll
            for (int m = 0; m < j; ++m) v -= L[i * (i + 1) / 2 + m] * L[j * (j + 1) / 2 + m];
            if (i == j) {
                if (!(v > 0.0)) return false;
                L[k] = sqrt(v);
            } else {
                L[k] = v / L[j * (j + 1) / 2 + j];
            }
        }
    double u[5], c2 = 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        double v = d[i];
#pragma unroll
        for (int m = 0; m < i; ++m) v -= L[i * (i + 1) / 2 + m] * u[m];
        u[i] = v / L[i * (i + 1) / 2 + i];
        c2 += u[i] * u[i];
    }
    out = c2;
    return true;
}

// ------------------------------------------------------------------------------------
// 0: clear the per-track and per-list state; the effective track count
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kMergeThreads) k_m_init(MergeBatch M, int64_t n_lists)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) {
        int64_t T = *M.n_tracks;
        if (T > M.cap_tracks) T = M.cap_tracks;
        if (T < 0) T = 0;
        M.mc->T = T;
        M.mc->n_fit = 0;
        M.mc->bad = 0;
        M.mc->fit_hits = 0;
        M.mc->n_outer = 0;
        for (int k = 0; k < 6; ++k) M.mc->work[k] = 0;
    }
    for (int64_t i = i0; i < M.cap_tracks; i += stride) {
        M.a_list[i] = -1;
        M.b_list[i] = -1;
        M.bestB[i] = -1;
        M.keepChi[i] = ~0ull;
        M.keepA[i] = 0x7FFFFFFF;
        M.next[i] = -1;
        M.prev[i] = -1;
        M.diss[i] = 0;
        M.fit_ok[i] = 0;
        M.nseg[i] = 0;
        M.seg_head[i] = -1;
    }
    for (int64_t i = i0; i < n_lists; i += stride) M.cnt[i] = 0;
}

// ------------------------------------------------------------------------------------
// 1: input checks, track ends (cluster coordinates), first track of each sector, outer
// ends rotated into the neighbouring sector's frame, list membership.  The input must be
// tracks of this batch in (time frame, sector) order, each with >= 3 clusters of its own
// sector; otherwise nothing is merged (invalid input).  A wave checks its 64 tracks' hit
// lists together, 64 clusters per pass.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kMergeThreads) k_m_ends(MergeBatch M, DevParams P, MergeParams Q)
{
#pragma clang fp contract(off)
    const int64_t T = M.mc->T;
    const int nr = P.n_rows, ns = P.n_sectors, S = Q.S;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); t0 < T; t0 += stride) {
        const int64_t t = t0 + lane;
        bool valid = t < T;
        int s = 0, f = 0;
        int64_t key = 0, hb = 0, he = 0, lo = 0, hi = 0;
        if (valid) {
            s = M.sector[t];
            f = M.tf[t];
            valid = s >= 0 && s < ns && f >= 0 && f < M.n_tf;
            key = (int64_t)f * ns + s;
            if (valid && t > 0 && (int64_t)M.tf[t - 1] * ns + M.sector[t - 1] > key) valid = false;
            hb = M.hit_off[t];
            he = M.hit_off[t + 1];
            if (!(hb >= 0 && he - hb >= 3 && he <= M.cap_in_hits)) valid = false;
            if (valid) {
                lo = M.off[key * nr];
                hi = M.off[key * nr + nr];
            }
        }
        // every cluster inside the track's own sector
        uint64_t todo = __ballot(valid);
        while (todo) {
            const int l = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1ull;
            const int64_t b0 = __shfl(hb, l, 64), b1 = __shfl(he, l, 64);
            const int64_t c0 = __shfl(lo, l, 64), c1 = __shfl(hi, l, 64);
            bool out = false;
            for (int64_t j = b0 + lane; j < b1; j += 64) {
                const int64_t h = M.hit_ids[j];
                out = out || h < c0 || h >= c1;
            }
            if (__ballot(out) != 0ull && lane == l) valid = false;
        }
        if (t < T && !valid) {
            atomicOr(&M.mc->bad, 1);
            atomicOr(&M.ctr->err, kErrInvalid);
        }
        if (!valid) continue;
        if (t == 0 || (int64_t)M.tf[t - 1] * ns + M.sector[t - 1] != key) M.sec_first[key] = (int32_t)t;
        const int64_t g0 = key * nr;
        const int64_t hi_ = M.hit_ids[hb], ho = M.hit_ids[he - 1];
        const float xi = P.rx[row_of(M.off, g0, nr, hi_)], yi = M.y[hi_];
        const float xo = P.rx[row_of(M.off, g0, nr, ho)], yo = M.y[ho];
        M.ends[t] = make_float4(xi, yi, xo, yo);
        const double dxi = xi, dyi = yi, dxo = xo, dyo = yo;
        if (fabs(dyi) >= dxi * Q.te - Q.edge) M.b_list[t] = (int32_t)(key * 2 + (dyi >= 0.0 ? 1 : 0));
        const double ro2 = dxo * dxo + dyo * dyo, ri2 = dxi * dxi + dyi * dyi;
        if (!(fabs(dyo) >= dxo * Q.te - Q.edge) || !(ro2 > ri2)) continue;
        const bool up = dyo >= 0.0;
        const int sb = (s / S) * S + ((s % S) + (up ? 1 : S - 1)) % S;
        Trk a;
        a.x = dxo;
        for (int q = 0; q < 5; ++q) a.p[q] = M.par_out[t * 5 + q];
        for (int q = 0; q < 15; ++q) a.c[q] = M.cov_out[t * 15 + q];
        const int di = step_index(s, sb, S);
        if (!trk_rotate(a, Q.rc[di], Q.rs[di], P)) continue;
        double* ms = M.mstate + t * 21;
        ms[0] = a.x;
        for (int q = 0; q < 5; ++q) ms[1 + q] = a.p[q];
        for (int q = 0; q < 15; ++q) ms[6 + q] = a.c[q];
        M.a_list[t] = (int32_t)(((int64_t)f * ns + sb) * 2 + (up ? 0 : 1));
    }
}

// ------------------------------------------------------------------------------------
// 2: inner ends into their lists (order inside a list is free: every decision below
// breaks ties on track indices).  Neighbouring tracks share lists, so a wave takes the
// positions of each of its lists with one atomic.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kMergeThreads) k_m_lists(MergeBatch M)
{
    if (M.mc->bad) return;
    const int64_t T = M.mc->T;
    __shared__ int32_t wcnt[kMergeThreads / 64];
    __shared__ int32_t bbase;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < T; b0 += stride) {   // block-uniform
        const int64_t t = b0 + threadIdx.x;
        // the outer ends, listed compactly for the match (one atomic per block)
        const bool oe = t < T && M.a_list[t] >= 0;
        const uint64_t om = __ballot(oe);
        if (lane == 0) wcnt[wv] = (int32_t)__popcll(om);
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t tot = 0;
            for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
                const int32_t c = wcnt[k];
                wcnt[k] = tot;
                tot += c;
            }
            bbase = tot > 0 ? atomicAdd(&M.mc->n_outer, tot) : 0;
        }
        __syncthreads();
        if (oe) M.a_idx[bbase + wcnt[wv] + (int32_t)__popcll(om & ((1ull << lane) - 1ull))] = (int32_t)t;
        __syncthreads();   // wcnt and bbase are reused by the next pass
        const int32_t L = t < T ? M.b_list[t] : -1;
        uint64_t todo = __ballot(L >= 0);
        int32_t pos = 0;
        while (todo) {
            const int l = __ffsll((unsigned long long)todo) - 1;
            const int32_t L0 = __shfl(L, l, 64);
            const uint64_t same = __ballot(L == L0);
            int32_t base = 0;
            if (lane == l) base = atomicAdd(&M.cnt[L0], (int32_t)__popcll(same));
            base = __shfl(base, l, 64);
            if (L == L0) pos = base + (int32_t)__popcll(same & ((1ull << lane) - 1ull));
            todo &= ~same;
        }
        if (L < 0) continue;
        const int64_t at = (int64_t)(L & 1) * M.cap_tracks + M.sec_first[L >> 1] + pos;
        const float4 e = M.ends[t];
        const double xi = e.x, yi = e.y;
        M.brec[at] = make_double4(xi, xi * xi + yi * yi, M.par[t * 5 + 0], M.par[t * 5 + 1]);
        M.bidx[at] = (int32_t)t;
    }
}

// ------------------------------------------------------------------------------------
// 2b: each list ordered by z (binary32 keys), so that an outer end scans only the entries
// its gate can accept; lists longer than kSortMax keep their order and are scanned whole
// ------------------------------------------------------------------------------------
constexpr int kSortMax = 8192;
constexpr int kSortThreads = 1024;

__device__ __forceinline__ uint32_t float_order_key(float v)
{
    const uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ void __launch_bounds__(kSortThreads) k_m_sort(MergeBatch M, int64_t n_lists)
{
    __shared__ unsigned long long keys[kSortMax];
    if (M.mc->bad) return;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int64_t L = blockIdx.x; L < n_lists; L += gridDim.x) {
        const int32_t n = M.cnt[L];
        if (n == 0) continue;
        const int64_t base = (L & 1) * M.cap_tracks + M.sec_first[L >> 1];
        if (n > kSortMax) {
            for (int32_t j = t; j < n; j += nt) {
                M.brec_s[base + j] = M.brec[base + j];
                M.bidx_s[base + j] = M.bidx[base + j];
                M.zs[base + j] = (float)M.brec[base + j].w;
            }
            if (t == 0) M.lsorted[L] = 0;
            continue;
        }
        int np = 2;
        while (np < n) np <<= 1;
        for (int j = t; j < np; j += nt)
            keys[j] = j < n ? ((unsigned long long)float_order_key((float)M.brec[base + j].w) << 32) | (uint32_t)j
                            : ~0ull;
        __syncthreads();
        for (int k = 2; k <= np; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = t; i < np; i += nt) {
                    const int o = i ^ j;
                    if (o > i) {
                        const unsigned long long a = keys[i], b = keys[o];
                        if (((i & k) == 0) ? a > b : a < b) {
                            keys[i] = b;
                            keys[o] = a;
                        }
                    }
                }
                __syncthreads();
            }
        for (int32_t j = t; j < n; j += nt) {
            const int32_t src = (int32_t)(keys[j] & 0xFFFFFFFFull);
            const double4 r = M.brec[base + src];
            M.brec_s[base + j] = r;
            M.bidx_s[base + j] = M.bidx[base + src];
            M.zs[base + j] = (float)r.w;
        }
        if (t == 0) M.lsorted[L] = 1;
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// 3: each outer end's least-chi2 inner end; the least chi2 per inner end (a lane per
// listed outer end)
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kMergeThreads) k_m_match(MergeBatch M, DevParams P, MergeParams Q)
{
    if (M.mc->bad) return;
    const int64_t n_outer = M.mc->n_outer;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t n_gate = 0, n_prop = 0, n_chi2 = 0;
    // over the listed outer ends, so that every lane has one
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_outer; i += stride) {
        const int64_t t = M.a_idx[i];
        const int32_t L = M.a_list[t];
        const int32_t n = M.cnt[L];
        if (n == 0) continue;
        const int64_t base = (int64_t)(L & 1) * M.cap_tracks + M.sec_first[L >> 1];
        Trk a;
        const double* ms = M.mstate + t * 21;
        a.x = ms[0];
        for (int q = 0; q < 5; ++q) a.p[q] = ms[1 + q];
        for (int q = 0; q < 15; ++q) a.c[q] = ms[6 + q];
        const float4 e = M.ends[t];
        double ro2, ty, tz;
        {
#pragma clang fp contract(off)
            const double xo = e.z, yo = e.w;
            ro2 = xo * xo + yo * yo;
            const double c1 = sqrt(1.0 - a.p[2] * a.p[2]);
            ty = a.p[2] / c1;
            tz = a.p[3] / c1;
        }
        int32_t j0 = 0, j1 = n;
        if (M.lsorted[L]) {
            // entries the gate can accept have z within W of z' + dx tz for some dx between
            // the first and the last row; the binary32 keys get a margin of their rounding
            const double za = a.p[1] + ((double)P.rx[0] - a.x) * tz;
            const double zb = a.p[1] + ((double)P.rx[P.n_rows - 1] - a.x) * tz;
            const double zlo = fmin(za, zb) - Q.window, zhi = fmax(za, zb) + Q.window;
            const double marg = 1.0e-3 + 1.0e-6 * fmax(fabs(zlo), fabs(zhi));
            const double qlo = zlo - marg, qhi = zhi + marg;
            int32_t lo = 0, hi = n;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if ((double)M.zs[base + mid] < qlo) lo = mid + 1; else hi = mid;
            }
            j0 = lo;
            hi = n;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if ((double)M.zs[base + mid] <= qhi) lo = mid + 1; else hi = mid;
            }
            j1 = lo;
        }
        int32_t best = -1;
        double bestc = 0.0;
        // the window's entries four at a time, their loads issued together; the few that
        // pass the gate are propagated and scored
        for (int32_t jb = j0; jb < j1; jb += 4) {
            double4 rr[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) rr[u] = M.brec_s[base + min(jb + u, j1 - 1)];
            uint32_t passm = 0u;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma clang fp contract(off)
                const double4 r = rr[u];
                const double dx = r.x - a.x;
                const double ylin = a.p[0] + dx * ty;
                const double zlin = a.p[1] + dx * tz;
                if (jb + u < j1 && r.y > ro2 && fabs(ylin - r.z) <= Q.window && fabs(zlin - r.w) <= Q.window)
                    passm |= 1u << u;
            }
            while (passm) {
                const int u = __ffs(passm) - 1;
                passm &= passm - 1u;
                const int32_t j = jb + u;
                const double4 r = M.brec_s[base + j];
                ++n_gate;
                const int32_t b = M.bidx_s[base + j];
                Trk a1 = a;
                ++n_prop;
                if (!trk_propagate(a1, r.x, P)) continue;
                double d[5], Ss[15], c2;
                for (int q = 0; q < 5; ++q) d[q] = a1.p[q] - M.par[(int64_t)b * 5 + q];
                for (int q = 0; q < 15; ++q) Ss[q] = a1.c[q] + M.cov[(int64_t)b * 15 + q];
                ++n_chi2;
                if (!chi2_5(Ss, d, c2) || !(c2 <= Q.chi2)) continue;
                if (best < 0 || c2 < bestc || (c2 == bestc && b < best)) {
                    best = b;
                    bestc = c2;
                }
            }
        }
        M.bestB[t] = best;
        M.bestChi[t] = bestc;
        if (best >= 0) atomicMin(&M.keepChi[best], (unsigned long long)__double_as_longlong(bestc));
    }
    wave_add(&M.mc->work[0], n_gate);
    wave_add(&M.mc->work[1], n_prop);
    wave_add(&M.mc->work[2], n_chi2);
}

// 4: among the outer ends at an inner end's least chi2, the smallest index
__global__ void __launch_bounds__(kMergeThreads) k_m_tie(MergeBatch M)
{
    if (M.mc->bad) return;
    const int64_t T = M.mc->T;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += stride) {
        const int32_t b = M.bestB[t];
        if (b >= 0 && (unsigned long long)__double_as_longlong(M.bestChi[t]) == M.keepChi[b])
            atomicMin(&M.keepA[b], (int32_t)t);
    }
}

// 5: links
__global__ void __launch_bounds__(kMergeThreads) k_m_link(MergeBatch M)
{
    if (M.mc->bad) return;
    const int64_t T = M.mc->T;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += stride) {
        const int32_t b = M.bestB[t];
        if (b >= 0 && M.keepA[b] == (int32_t)t) {
            M.next[t] = b;
            M.prev[b] = (int32_t)t;
        }
    }
}

// 6: chains from their heads: segments and clusters; heads of several segments listed
__global__ void __launch_bounds__(kMergeThreads) k_m_chain(MergeBatch M)
{
    if (M.mc->bad) return;
    const int64_t T = M.mc->T;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += stride) {
        if (M.prev[t] >= 0) continue;
        int32_t ns = 0, nh = 0, u = (int32_t)t;
        while (u >= 0 && ns < kMergeMaxChain) {
            nh += (int32_t)(M.hit_off[u + 1] - M.hit_off[u]);
            ++ns;
            u = M.next[u];
        }
        if (u >= 0) atomicOr(&M.ctr->err, kErrMergeChain);
        M.nseg[t] = ns;
        M.chain_hits[t] = nh;
        if (ns >= 2) {
            M.fit_list[atomicAdd(&M.mc->n_fit, 1)] = (int32_t)t;
            M.fit_off[t] = (int64_t)atomicAdd(&M.mc->fit_hits, (unsigned long long)nh);
        }
        // every segment's chain head and the clusters before it in the chain
        int32_t pre = 0;
        u = (int32_t)t;
        for (int k = 0; k < ns; ++k, u = M.next[u]) {
            M.seg_head[u] = (int32_t)t;
            M.seg_pre[u] = pre;
            pre += (int32_t)(M.hit_off[u + 1] - M.hit_off[u]);
        }
    }
}

// ------------------------------------------------------------------------------------
// 7a: the clusters of every chain to refit, in chain order, as records (y, z, row plane x,
// sector); one wave per track of such a chain, 64 clusters per pass, the rows found in
// the sector's row offsets staged in the wave's LDS
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kMergeThreads) k_m_gather(MergeBatch M, DevParams P)
{
    __shared__ int64_t offs[kMergeThreads / 64][kMaxRows + 1];
    if (M.mc->bad) return;
    const int nr = P.n_rows, ns = P.n_sectors;
    const int64_t T = M.mc->T;
    const int lane = threadIdx.x & 63;
    int64_t* o = offs[threadIdx.x >> 6];
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    if (M.hit_rec) {
        // the tracking call's own records of these clusters, contiguous: a wave takes 64
        // input tracks, each lane finds its track's place, and the wave copies
        // kCopyTracks lists per pass with the loads of all of them issued together
        for (int64_t u0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64; u0 < T; u0 += nw * 64) {
            const int64_t u = u0 + lane;
            bool on = false;
            int64_t k = 0, hb = 0, n = 0;
            int su = 0;
            if (u < T) {
                const int32_t head = M.seg_head[u];
                if (head >= 0 && M.nseg[head] >= 2) {
                    on = true;
                    su = M.sector[u];
                    k = M.fit_off[head] + M.seg_pre[u];
                    hb = M.hit_off[u];
                    n = M.hit_off[u + 1] - hb;
                }
            }
            uint64_t todo = __ballot(on);
            while (todo != 0ull) {
                int64_t d[kCopyTracks], sb[kCopyTracks], c[kCopyTracks];
                float sf[kCopyTracks];
                int64_t mm = 0;
#pragma unroll
                for (int q = 0; q < kCopyTracks; ++q) {
                    const bool has = todo != 0ull;
                    const int l = has ? __ffsll((unsigned long long)todo) - 1 : 0;
                    todo &= todo - 1ull;
                    d[q] = __shfl(k, l, 64);
                    sb[q] = __shfl(hb, l, 64);
                    c[q] = has ? __shfl(n, l, 64) : 0;
                    sf[q] = __int_as_float(__shfl(su, l, 64));
                    mm = c[q] > mm ? c[q] : mm;
                }
                for (int64_t j = lane; j < mm; j += 64) {
                    float4 e[kCopyTracks];
#pragma unroll
                    for (int q = 0; q < kCopyTracks; ++q)
                        e[q] = j < c[q] ? M.hit_rec[sb[q] + j] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
                    for (int q = 0; q < kCopyTracks; ++q)
                        if (j < c[q]) M.grec[d[q] + j] = make_float4(e[q].x, e[q].y, e[q].z, sf[q]);
                }
            }
        }
        return;
    }
    for (int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; u < T; u += nw) {
        const int32_t head = M.seg_head[u];
        if (head < 0 || M.nseg[head] < 2) continue;
        const int su = M.sector[u];
        const int64_t k = M.fit_off[head] + M.seg_pre[u];
        const int64_t hb = M.hit_off[u], n = M.hit_off[u + 1] - hb;
        const int64_t g0 = ((int64_t)M.tf[u] * ns + su) * nr;
        wave_lds_sync();
        for (int r = lane; r <= nr; r += 64) o[r] = M.off[g0 + r];
        wave_lds_sync();
        for (int64_t j = lane; j < n; j += 64) {
            const int64_t h = M.hit_ids[hb + j];
            M.grec[k + j] = make_float4(M.y[h], M.z[h], P.rx[row_of(o, 0, nr, h)], __int_as_float(su));
        }
    }
}

// descending bitonic sort of 256 keys in LDS (all threads of the block call it)
__device__ void sort_desc_256(uint32_t* key)
{
    const int t = threadIdx.x;
    for (int k = 2; k <= 256; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int o = t ^ j;
            if (o > t) {
                const uint32_t a = key[t], b = key[o];
                const bool desc = (t & k) == 0;
                if (desc ? a < b : a > b) {
                    key[t] = b;
                    key[o] = a;
                }
            }
            __syncthreads();
        }
}

// ------------------------------------------------------------------------------------
// 7b: refit of each chain over all its clusters, across the sector frames: the final fit
// (seed from the first, middle and last cluster in the first cluster's frame; outward
// pass from C0; inward pass from C0 keeping the parameters), with the state rotated into
// a cluster's frame before the step to its row.  A failure dissolves the chain.  Blocks
// take 256 chains and order them by length, so that a wave's lanes run similar lengths.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kMergeThreads) k_m_fit(MergeBatch M, DevParams P, MergeParams Q)
{
    __shared__ uint32_t key[kMergeThreads];
    if (M.mc->bad) return;
    const int S = Q.S;
    const int64_t nf = M.mc->n_fit;
    int64_t n_rot = 0, n_prop = 0, n_upd = 0;
    for (int64_t ch = blockIdx.x; ch * kMergeThreads < nf; ch += gridDim.x) {
        const int64_t i_own = ch * kMergeThreads + threadIdx.x;
        const uint32_t n_own = i_own < nf ? (uint32_t)M.chain_hits[M.fit_list[i_own]] : 0u;
        key[threadIdx.x] = ((n_own < 0xFFFFFFu ? n_own : 0xFFFFFFu) << 8) | (uint32_t)threadIdx.x;
        __syncthreads();
        sort_desc_256(key);
        const int64_t i = ch * kMergeThreads + (key[threadIdx.x] & 0xFFu);
        __syncthreads();
        if (i >= nf) continue;
        const int32_t t = M.fit_list[i];
        const int32_t n = M.chain_hits[t];
        const int64_t base = M.fit_off[t];
        const int s0 = M.sector[t];
        // seed points in the frame of the first cluster's sector
        double sx[3], sy[3], sz[3];
        const int32_t ids[3] = {0, (n - 1) / 2, n - 1};
        for (int q = 0; q < 3; ++q) {
            const float4 e = M.grec[base + ids[q]];
            const int su = __float_as_int(e.w);
            const double x = e.z, y = e.x;
            sz[q] = e.y;
            if (su == s0) {
                sx[q] = x;
                sy[q] = y;
            } else {
                // rotation by -delta, delta the step from s0 to su
                const int di = step_index(s0, su, S);
                sx[q] = x * Q.rc[di] - y * Q.rs[di];
                sy[q] = x * Q.rs[di] + y * Q.rc[di];
            }
        }
        Trk tr;
        bool ok = trk_seed(tr, sx, sy, sz, P);
        double chi2 = 0.0;
        if (ok) {
            trk_reset_cov(tr, P);
            int frame = s0;
            for (int32_t k = 0; k < n; ++k) {
                const float4 e = M.grec[base + k];
                const int su = __float_as_int(e.w);
                if (su != frame) {
                    const int di = step_index(frame, su, S);
                    ++n_rot;
                    if (!trk_rotate(tr, Q.rc[di], Q.rs[di], P)) { ok = false; break; }
                    frame = su;
                }
                if (k > 0) {
                    ++n_prop;
                    if (!trk_propagate(tr, (double)e.z, P)) { ok = false; break; }
                }
                trk_update(tr, (double)e.x, (double)e.y, P);
                ++n_upd;
            }
            if (ok) {
                trk_reset_cov(tr, P);
                for (int32_t k = n - 1; k >= 0; --k) {
                    const float4 e = M.grec[base + k];
                    const int su = __float_as_int(e.w);
                    if (su != frame) {
                        const int di = step_index(frame, su, S);
                        ++n_rot;
                        if (!trk_rotate(tr, Q.rc[di], Q.rs[di], P)) { ok = false; break; }
                        frame = su;
                    }
                    if (k < n - 1) {
                        ++n_prop;
                        if (!trk_propagate(tr, (double)e.z, P)) { ok = false; break; }
                    }
                    chi2 += trk_update(tr, (double)e.x, (double)e.y, P);
                    ++n_upd;
                }
            }
        }
        if (ok) {
            for (int q = 0; q < 5; ++q) ok = ok && isfinite(tr.p[q]);
            for (int q = 0; q < 15; ++q) ok = ok && isfinite(tr.c[q]);
        }
        if (ok) {
            double* ms = M.mstate + (int64_t)t * 21;
            for (int q = 0; q < 5; ++q) ms[q] = tr.p[q];
            for (int q = 0; q < 15; ++q) ms[5 + q] = tr.c[q];
            ms[20] = chi2;
            M.fit_ok[t] = 1;
        } else {
            int32_t u = t;
            for (int seg = 0; u >= 0 && seg < M.nseg[t]; ++seg, u = M.next[u]) M.diss[u] = 1;
        }
    }
    wave_add(&M.mc->work[3], n_rot);
    wave_add(&M.mc->work[4], n_prop);
    wave_add(&M.mc->work[5], n_upd);
}

// 8: which tracks start a merged track, and its cluster count
__global__ void __launch_bounds__(kMergeThreads) k_m_lead(MergeBatch M)
{
    if (M.mc->bad) return;
    const int64_t T = M.mc->T;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += stride) {
        const bool head = M.prev[t] < 0;
        const bool lead = head || M.diss[t];
        const bool whole = head && M.nseg[t] >= 2 && M.fit_ok[t];
        M.lead[t] = lead ? 1 : 0;
        M.nh[t] = lead ? (whole ? M.chain_hits[t] : (int32_t)(M.hit_off[t + 1] - M.hit_off[t])) : 0;
    }
}

// 9: merged tracks at their scanned positions (lane per merged track)
__global__ void __launch_bounds__(kMergeThreads) k_m_emit(MergeBatch M, DevParams P)
{
    if (M.mc->bad) return;
    const int64_t T = M.mc->T;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (blockIdx.x == 0 && threadIdx.x == 0 && M.cap_merged >= 0) M.o_hit_off[0] = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += stride) {
        if (M.o_next) {
            M.o_next[t] = M.next[t];
            if (M.o_link_chi2) M.o_link_chi2[t] = M.next[t] >= 0 ? M.bestChi[t] : 0.0;
        }
        if (!M.lead[t]) continue;
        const int64_t m = M.m_idx[t], hp = M.m_hpos[t];
        const int32_t nh = M.nh[t];
        if (m >= M.cap_merged || hp + nh > M.cap_hits) {
            atomicOr(&M.ctr->err, kErrOutCap);
            continue;
        }
        const bool whole = M.prev[t] < 0 && M.nseg[t] >= 2 && M.fit_ok[t];
        const double* src_p;
        if (whole) {
            const double* ms = M.mstate + t * 21;
            for (int q = 0; q < 5; ++q) M.o_par[m * 5 + q] = ms[q];
            for (int q = 0; q < 15; ++q) M.o_cov[m * 15 + q] = ms[5 + q];
            M.o_chi2[m] = ms[20];
            src_p = ms;
        } else {
            for (int q = 0; q < 5; ++q) M.o_par[m * 5 + q] = M.par[t * 5 + q];
            for (int q = 0; q < 15; ++q) M.o_cov[m * 15 + q] = M.cov[t * 15 + q];
            M.o_chi2[m] = M.chi2[t];
            src_p = M.par + t * 5;
        }
        M.o_nseg[m] = whole ? M.nseg[t] : 1;
        M.o_xref[m] = M.xref[t];
        if (M.o_zbeam) M.o_zbeam[m] = trk_beamline_z(P, M.xref[t], src_p);
        M.o_ndf[m] = 2 * nh - 5;
        M.o_nhits_trk[m] = nh;
        M.o_sector[m] = M.sector[t];
        M.o_tf[m] = M.tf[t];
        M.o_hit_off[m + 1] = hp + nh;
    }
}

// 10: every input track's clusters into its merged track's hit list, and its entry in the
// input-to-merged map; a wave takes 64 input tracks
__global__ void __launch_bounds__(kMergeThreads) k_m_copy(MergeBatch M)
{
    if (M.mc->bad) return;
    const int64_t T = M.mc->T;
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t u0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64; u0 < T; u0 += nw * 64) {
        // each lane finds its track's place, then the wave copies the hit lists
        const int64_t u = u0 + lane;
        bool on = false;
        int64_t dst = 0, hb = 0, n = 0;
        if (u < T) {
            const int32_t head = M.seg_head[u];
            if (head >= 0) {
                const bool whole = M.prev[head] < 0 && M.nseg[head] >= 2 && M.fit_ok[head];
                int64_t m = -1;
                if (whole) {
                    m = M.m_idx[head];
                    dst = M.m_hpos[head] + M.seg_pre[u];
                } else if (M.lead[u]) {
                    m = M.m_idx[u];
                    dst = M.m_hpos[u];
                }
                hb = M.hit_off[u];
                n = M.hit_off[u + 1] - hb;
                on = m >= 0 && m < M.cap_merged && dst + n <= M.cap_hits;
                if (on) M.o_track_merged[u] = (int32_t)m;
            }
        }
        // kCopyTracks lists per pass, the loads of all of them issued before the stores
        uint64_t todo = __ballot(on);
        while (todo != 0ull) {
            int64_t d[kCopyTracks], sb[kCopyTracks], c[kCopyTracks];
            int64_t mm = 0;
#pragma unroll
            for (int k = 0; k < kCopyTracks; ++k) {
                const bool has = todo != 0ull;
                const int l = has ? __ffsll((unsigned long long)todo) - 1 : 0;
                todo &= todo - 1ull;
                d[k] = __shfl(dst, l, 64);
                sb[k] = __shfl(hb, l, 64);
                c[k] = has ? __shfl(n, l, 64) : 0;
                mm = c[k] > mm ? c[k] : mm;
            }
            for (int64_t j = lane; j < mm; j += 64) {
                int32_t h[kCopyTracks];
#pragma unroll
                for (int k = 0; k < kCopyTracks; ++k) h[k] = j < c[k] ? M.hit_ids[sb[k] + j] : 0;
#pragma unroll
                for (int k = 0; k < kCopyTracks; ++k)
                    if (j < c[k]) M.o_hit_ids[d[k] + j] = h[k];
            }
        }
    }
}

}  // namespace

void launch_merge(const MergeBatch& M, const DevParams& P, const MergeParams& Q, int n_cu, hipStream_t s)
{
    const int64_t n_lists = (int64_t)M.n_tf * P.n_sectors * 2;
    int64_t need = (M.cap_tracks > n_lists ? M.cap_tracks : n_lists);
    int64_t blocks = (need + kMergeThreads - 1) / kMergeThreads;
    const int64_t max_blocks = (int64_t)n_cu * 16;
    if (blocks > max_blocks) blocks = max_blocks;
    if (blocks < 1) blocks = 1;
    const dim3 g((unsigned)blocks), b(kMergeThreads);
    hipLaunchKernelGGL(k_m_init, g, b, 0, s, M, n_lists);
    hipLaunchKernelGGL(k_m_ends, g, b, 0, s, M, P, Q);
    hipLaunchKernelGGL(k_m_lists, g, b, 0, s, M);
    {
        int64_t sb = n_lists < (int64_t)n_cu * 2 ? n_lists : (int64_t)n_cu * 2;
        hipLaunchKernelGGL(k_m_sort, dim3((unsigned)(sb > 0 ? sb : 1)), dim3(kSortThreads), 0, s, M, n_lists);
    }
    hipLaunchKernelGGL(k_m_match, g, b, 0, s, M, P, Q);
    hipLaunchKernelGGL(k_m_tie, g, b, 0, s, M);
    hipLaunchKernelGGL(k_m_link, g, b, 0, s, M);
    hipLaunchKernelGGL(k_m_chain, g, b, 0, s, M);
    hipLaunchKernelGGL(k_m_gather, dim3((unsigned)(n_cu * 16)), b, 0, s, M, P);
    hipLaunchKernelGGL(k_m_fit, g, b, 0, s, M, P, Q);
    hipLaunchKernelGGL(k_m_lead, g, b, 0, s, M);
    ScanJob J{};
    J.a32 = M.lead;
    J.a_min = 1;
    J.b32 = M.nh;
    J.outA = M.m_idx;
    J.outB = M.m_hpos;
    J.lo = 0;
    J.hi_ptr = &M.mc->T;
    J.totA = M.o_n;
    J.totB = M.o_nhits;
    J.part = M.scan_part;
    launch_scan(J, s);
    hipLaunchKernelGGL(k_m_emit, g, b, 0, s, M, P);
    hipLaunchKernelGGL(k_m_copy, dim3((unsigned)(n_cu * 16)), b, 0, s, M);
}

}  // namespace tpcsf
