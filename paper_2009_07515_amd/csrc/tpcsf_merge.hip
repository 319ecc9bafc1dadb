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
// Layout: one lane per track in every kernel (the track counts are small next to the
// tracking stages); the inner ends of each (time frame, sector, edge) are listed densely
// in a region starting at that sector's first track, so that an outer end scans exactly
// its candidate list.  Decisions that the oracle takes on cluster coordinates and on the
// linear gate are evaluated without contraction, as there.
#include "tpcsf_internal.h"
#include "tpcsf_kalman.h"

#include <math.h>

namespace tpcsf {

namespace {

constexpr int kMergeThreads = 256;

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
    }
    for (int64_t i = i0; i < n_lists; i += stride) M.cnt[i] = 0;
}

// ------------------------------------------------------------------------------------
// 1: track ends (cluster coordinates), first track of each sector, outer ends rotated
// into the neighbouring sector's frame, list membership
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kMergeThreads) k_m_ends(MergeBatch M, DevParams P, MergeParams Q)
{
#pragma clang fp contract(off)
    const int64_t T = M.mc->T;
    const int nr = P.n_rows, ns = P.n_sectors, S = Q.S;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += stride) {
        const int s = M.sector[t], f = M.tf[t];
        // the input must be tracks of this batch in (time frame, sector) order, each with
        // >= 3 clusters of its own sector: otherwise nothing is merged (invalid input)
        bool valid = s >= 0 && s < ns && f >= 0 && f < M.n_tf;
        const int64_t key = (int64_t)f * ns + s;
        if (valid && t > 0 && (int64_t)M.tf[t - 1] * ns + M.sector[t - 1] > key) valid = false;
        const int64_t g0 = key * nr;
        const int64_t hb = M.hit_off[t], he = M.hit_off[t + 1];
        if (!(hb >= 0 && he - hb >= 3 && he <= M.cap_in_hits)) valid = false;
        for (int64_t j = hb; valid && j < he; ++j) {
            const int64_t h = M.hit_ids[j];
            valid = h >= M.off[g0] && h < M.off[g0 + nr];
        }
        if (!valid) {
            atomicOr(&M.mc->bad, 1);
            atomicOr(&M.ctr->err, kErrInvalid);
            continue;
        }
        if (t == 0 || (int64_t)M.tf[t - 1] * ns + M.sector[t - 1] != key) M.sec_first[key] = (int32_t)t;
        const int64_t hi_ = M.hit_ids[M.hit_off[t]], ho = M.hit_ids[M.hit_off[t + 1] - 1];
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
// breaks ties on track indices)
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kMergeThreads) k_m_lists(MergeBatch M)
{
    if (M.mc->bad) return;
    const int64_t T = M.mc->T;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += stride) {
        const int32_t L = M.b_list[t];
        if (L < 0) continue;
        const int32_t pos = atomicAdd(&M.cnt[L], 1);
        const int64_t at = (int64_t)(L & 1) * M.cap_tracks + M.sec_first[L >> 1] + pos;
        const float4 e = M.ends[t];
        const double xi = e.x, yi = e.y;
        M.brec[at] = make_double4(xi, xi * xi + yi * yi, M.par[t * 5 + 0], M.par[t * 5 + 1]);
        M.bidx[at] = (int32_t)t;
    }
}

// ------------------------------------------------------------------------------------
// 3: each outer end's least-chi2 inner end; the least chi2 per inner end
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kMergeThreads) k_m_match(MergeBatch M, DevParams P, MergeParams Q)
{
    if (M.mc->bad) return;
    const int64_t T = M.mc->T;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t n_gate = 0, n_prop = 0, n_chi2 = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += stride) {
        const int32_t L = M.a_list[t];
        if (L < 0) continue;
        const int32_t n = M.cnt[L];
        if (n == 0) continue;
        const int64_t base = (int64_t)(L & 1) * M.cap_tracks + M.sec_first[L >> 1];
        Trk a;
        const double* ms = M.mstate + t * 21;
        a.x = ms[0];
        for (int q = 0; q < 5; ++q) a.p[q] = ms[1 + q];
        for (int q = 0; q < 15; ++q) a.c[q] = ms[6 + q];
        const float4 e = M.ends[t];
        double ro2, c1;
        {
#pragma clang fp contract(off)
            const double xo = e.z, yo = e.w;
            ro2 = xo * xo + yo * yo;
            c1 = sqrt(1.0 - a.p[2] * a.p[2]);
        }
        int32_t best = -1;
        double bestc = 0.0;
        for (int32_t j = 0; j < n; ++j) {
            const double4 r = M.brec[base + j];
            bool pass;
            {
#pragma clang fp contract(off)
                const double dx = r.x - a.x;
                const double ylin = a.p[0] + dx * a.p[2] / c1;
                const double zlin = a.p[1] + dx * a.p[3] / c1;
                pass = r.y > ro2 && fabs(ylin - r.z) <= Q.window && fabs(zlin - r.w) <= Q.window;
            }
            if (!pass) continue;
            ++n_gate;
            const int32_t b = M.bidx[base + j];
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
        if (ns >= 2) M.fit_list[atomicAdd(&M.mc->n_fit, 1)] = (int32_t)t;
    }
}

// k-th cluster of the chain from head t (k < its cluster count): index and segment
__device__ __forceinline__ int64_t chain_hit(const MergeBatch& M, int32_t t, int32_t k, int32_t& seg)
{
    int32_t u = t;
    for (;;) {
        const int32_t n = (int32_t)(M.hit_off[u + 1] - M.hit_off[u]);
        if (k < n) break;
        k -= n;
        u = M.next[u];
    }
    seg = u;
    return M.hit_ids[M.hit_off[u] + k];
}

// ------------------------------------------------------------------------------------
// 7: refit of each chain over all its clusters, across the sector frames: the final fit
// (seed from the first, middle and last cluster in the first cluster's frame; outward
// pass from C0; inward pass from C0 keeping the parameters), with the state rotated into
// a cluster's frame before the step to its row.  A failure dissolves the chain.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kMergeThreads) k_m_fit(MergeBatch M, DevParams P, MergeParams Q)
{
    if (M.mc->bad) return;
    const int nr = P.n_rows, ns = P.n_sectors, S = Q.S;
    const int64_t nf = M.mc->n_fit;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t n_rot = 0, n_prop = 0, n_upd = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += stride) {
        const int32_t t = M.fit_list[i];
        const int32_t n = M.chain_hits[t];
        const int s0 = M.sector[t];
        const int64_t tfb = (int64_t)M.tf[t] * ns;
        // seed points in the frame of the first cluster's sector
        double sx[3], sy[3], sz[3];
        const int32_t ids[3] = {0, (n - 1) / 2, n - 1};
        for (int q = 0; q < 3; ++q) {
            int32_t u;
            const int64_t h = chain_hit(M, t, ids[q], u);
            const int su = M.sector[u];
            const double x = P.rx[row_of(M.off, (tfb + su) * nr, nr, h)], y = M.y[h];
            sz[q] = M.z[h];
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
        int32_t last = t;
        if (ok) {
            trk_reset_cov(tr, P);
            int frame = s0;
            int32_t u = t;
            bool first = true;
            for (int seg = 0; ok && u >= 0 && seg < M.nseg[t]; ++seg) {
                const int su = M.sector[u];
                const int64_t g0 = (tfb + su) * nr;
                if (su != frame) {
                    const int di = step_index(frame, su, S);
                    ++n_rot;
                    ok = trk_rotate(tr, Q.rc[di], Q.rs[di], P);
                    frame = su;
                }
                for (int64_t j = M.hit_off[u]; ok && j < M.hit_off[u + 1]; ++j) {
                    const int64_t h = M.hit_ids[j];
                    if (!first) {
                        ++n_prop;
                        ok = trk_propagate(tr, (double)P.rx[row_of(M.off, g0, nr, h)], P);
                        if (!ok) break;
                    }
                    first = false;
                    trk_update(tr, (double)M.y[h], (double)M.z[h], P);
                    ++n_upd;
                }
                last = u;
                u = M.next[u];
            }
            if (ok) {
                trk_reset_cov(tr, P);
                u = last;
                bool lastc = true;
                for (int seg = 0; ok && u >= 0 && seg < M.nseg[t]; ++seg) {
                    const int su = M.sector[u];
                    const int64_t g0 = (tfb + su) * nr;
                    if (su != frame) {
                        const int di = step_index(frame, su, S);
                        ++n_rot;
                        ok = trk_rotate(tr, Q.rc[di], Q.rs[di], P);
                        frame = su;
                    }
                    for (int64_t j = M.hit_off[u + 1] - 1; ok && j >= M.hit_off[u]; --j) {
                        const int64_t h = M.hit_ids[j];
                        if (!lastc) {
                            ++n_prop;
                            ok = trk_propagate(tr, (double)P.rx[row_of(M.off, g0, nr, h)], P);
                            if (!ok) break;
                        }
                        lastc = false;
                        const double my = M.y[h], mz = M.z[h];
                        chi2 += trk_chi2(tr, my, mz, P);
                        trk_update(tr, my, mz, P);
                        ++n_upd;
                    }
                    u = (u == t) ? -1 : M.prev[u];
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

// 9: merged tracks at their scanned positions
__global__ void __launch_bounds__(kMergeThreads) k_m_emit(MergeBatch M, DevParams P)
{
    if (M.mc->bad) return;
    const int64_t T = M.mc->T;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 == 0 && M.cap_merged >= 0) M.o_hit_off[0] = 0;
    for (int64_t t = t0; t < T; t += stride) {
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
            M.o_nseg[m] = M.nseg[t];
            src_p = ms;
        } else {
            for (int q = 0; q < 5; ++q) M.o_par[m * 5 + q] = M.par[t * 5 + q];
            for (int q = 0; q < 15; ++q) M.o_cov[m * 15 + q] = M.cov[t * 15 + q];
            M.o_chi2[m] = M.chi2[t];
            M.o_nseg[m] = 1;
            src_p = M.par + t * 5;
        }
        M.o_xref[m] = M.xref[t];
        if (M.o_zbeam) M.o_zbeam[m] = trk_beamline_z(P, M.xref[t], src_p);
        M.o_ndf[m] = 2 * nh - 5;
        M.o_nhits_trk[m] = nh;
        M.o_sector[m] = M.sector[t];
        M.o_tf[m] = M.tf[t];
        M.o_hit_off[m + 1] = hp + nh;
        int64_t k = hp;
        const int32_t nseg = whole ? M.nseg[t] : 1;
        int32_t u = (int32_t)t;
        for (int seg = 0; u >= 0 && seg < nseg; ++seg, u = M.next[u]) {
            M.o_track_merged[u] = (int32_t)m;
            for (int64_t j = M.hit_off[u]; j < M.hit_off[u + 1]; ++j) M.o_hit_ids[k++] = M.hit_ids[j];
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
    hipLaunchKernelGGL(k_m_match, g, b, 0, s, M, P, Q);
    hipLaunchKernelGGL(k_m_tie, g, b, 0, s, M);
    hipLaunchKernelGGL(k_m_link, g, b, 0, s, M);
    hipLaunchKernelGGL(k_m_chain, g, b, 0, s, M);
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
}

}  // namespace tpcsf
