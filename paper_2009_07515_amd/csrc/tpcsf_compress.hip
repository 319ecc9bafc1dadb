// Track-model compression of the attached clusters (arXiv:2009.07515, Sec. 4, entropy
// reduction step): each cluster attached to a track is stored as its row and its residual
// to the track's position on that row plane, quantised; the track's state at x_ref is
// kept with the track.  The position is the state propagated in one helix step to the row
// (the state at x_ref itself where that step fails), so that every cluster decodes
// independently: y = y_p + q_y * step, z = z_p + q_z * step, within half a step.
//
// Layout: with the tracking call's per-hit records (contiguous y, z, row plane x), and for
// the decoder, a wave takes 64 tracks and spreads their clusters over its lanes; from the
// clusters themselves, a wave takes one track and finds each cluster's row in the sector's
// row offsets, staged in the wave's LDS.
#include "tpcsf_internal.h"
#include "tpcsf_kalman.h"

#include <math.h>

namespace tpcsf {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// position of the track on the row plane x1
__device__ __forceinline__ void predict(const double* p, double x0, double x1, const DevParams& P, double& y,
                                        double& z)
{
    if (!trk_predict(p, x0, x1, P, y, z)) {
        y = p[0];
        z = p[1];
    }
}

__device__ __forceinline__ int32_t quantise(double r)
{
    double q = floor(r + 0.5);
    if (q > 1073741824.0) q = 1073741824.0;
    if (q < -1073741824.0) q = -1073741824.0;
    return (int32_t)q;
}

__global__ void __launch_bounds__(kThreads) k_c_encode(CompressArgs A, DevParams P)
{
    __shared__ int64_t offs[kThreads / 64][kMaxRows + 1];
    const int nr = P.n_rows, ns = P.n_sectors;
    const int lane = threadIdx.x & 63;
    int64_t* o = offs[threadIdx.x >> 6];
    int64_t T = *A.n_tracks;
    if (T > A.cap_tracks) T = A.cap_tracks;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; t < T; t += nw) {
        const int s = A.sector[t], f = A.tf[t];
        const int64_t hb = A.hit_off[t], he = A.hit_off[t + 1];
        if (!(s >= 0 && s < ns && f >= 0 && f < A.n_tf && hb >= 0 && he >= hb && he <= A.cap_hits)) continue;
        const int64_t g0 = ((int64_t)f * ns + s) * nr;
        double p[5];
        for (int q = 0; q < 5; ++q) p[q] = A.par[t * 5 + q];
        const double x0 = A.xref[t];
        wave_lds_sync();
        for (int r = lane; r <= nr; r += 64) o[r] = A.off[g0 + r];
        wave_lds_sync();
        for (int64_t j = hb + lane; j < he; j += 64) {
            const int64_t h = A.hit_ids[j];
            if (h < o[0] || h >= o[nr]) {
                A.codes[2 * j] = 0;
                A.codes[2 * j + 1] = 0;
                A.rows[j] = 0;
                continue;
            }
            int a = 0, b = nr - 1;
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if (o[mid] <= h) a = mid; else b = mid - 1;
            }
            double yp, zp;
            predict(p, x0, (double)P.rx[a], P, yp, zp);
            A.codes[2 * j] = quantise(((double)A.y[h] - yp) / A.step);
            A.codes[2 * j + 1] = quantise(((double)A.z[h] - zp) / A.step);
            A.rows[j] = (uint8_t)a;
        }
    }
}

// A wave takes kGroup consecutive tracks (a lane per track: state, x_ref, hit range),
// whose clusters are consecutive in hit-list order, and spreads those clusters over its
// lanes, 64 per pass; a lane finds its cluster's track among the wave's by the prefix of
// the cluster counts.  Small groups keep many waves in flight (each pass waits on loads).
constexpr int kGroup = 8;
struct WaveTracks {
    double p[5], x0;
    int64_t hb;
    int cnt, incl;
};

__device__ __forceinline__ void wave_tracks_load(const CompressArgs& A, int64_t t, int64_t T, WaveTracks& w)
{
    w.cnt = 0;
    w.hb = 0;
    w.x0 = 0.0;
    for (int q = 0; q < 5; ++q) w.p[q] = 0.0;
    if ((threadIdx.x & 63) < kGroup && t < T) {
        const int64_t hb = A.hit_off[t], he = A.hit_off[t + 1];
        if (hb >= 0 && he >= hb && he <= A.cap_hits) {
            w.hb = hb;
            w.cnt = (int)(he - hb);
            for (int q = 0; q < 5; ++q) w.p[q] = A.par[t * 5 + q];
            w.x0 = A.xref[t];
        }
    }
    int v = w.cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o, 64);
        if ((threadIdx.x & 63) >= o) v += u;
    }
    w.incl = v;
}

// the wave lane whose clusters hold the wave's q-th one, and that cluster's hit index
__device__ __forceinline__ int wave_tracks_find(const WaveTracks& w, int q, int64_t& j)
{
    int l = 0;
    for (int step = kGroup / 2; step > 0; step >>= 1) {
        const int v = __shfl(w.incl, l + step - 1, 64);
        if (v <= q) l += step;
    }
    const int lincl = __shfl(w.incl, l, 64), lcnt = __shfl(w.cnt, l, 64);
    j = __shfl(w.hb, l, 64) + (q - (lincl - lcnt));
    return l;
}

__global__ void __launch_bounds__(kThreads) k_c_encode_rec(CompressArgs A, DevParams P)
{
    __shared__ float rx[kMaxRows];
    const int nr = P.n_rows;
    for (int r = threadIdx.x; r < nr; r += blockDim.x) rx[r] = P.rx[r];
    __syncthreads();
    int64_t T = *A.n_tracks;
    if (T > A.cap_tracks) T = A.cap_tracks;
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t t0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * kGroup; t0 < T; t0 += nw * kGroup) {
        WaveTracks w;
        wave_tracks_load(A, t0 + lane, T, w);
        const int total = __shfl(w.incl, kGroup - 1, 64);
        for (int q0 = 0; q0 < total; q0 += 64) {
            const int q = q0 + lane;
            int64_t j;
            const int l = wave_tracks_find(w, q, j);
            double p[5];
            for (int k = 0; k < 5; ++k) p[k] = __shfl(w.p[k], l, 64);
            const double x0 = __shfl(w.x0, l, 64);
            if (q >= total) continue;
            // the record's row plane: the row whose x it holds
            const float4 e = A.hit_rec[j];
            int a = 0, b = nr - 1;
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if (rx[mid] <= e.z) a = mid; else b = mid - 1;
            }
            double yp, zp;
            predict(p, x0, (double)rx[a], P, yp, zp);
            A.codes[2 * j] = quantise(((double)e.x - yp) / A.step);
            A.codes[2 * j + 1] = quantise(((double)e.y - zp) / A.step);
            A.rows[j] = (uint8_t)a;
        }
    }
}

__global__ void __launch_bounds__(kThreads) k_c_decode(CompressArgs A, DevParams P)
{
    int64_t T = *A.n_tracks;
    if (T > A.cap_tracks) T = A.cap_tracks;
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t t0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * kGroup; t0 < T; t0 += nw * kGroup) {
        WaveTracks w;
        wave_tracks_load(A, t0 + lane, T, w);
        const int total = __shfl(w.incl, kGroup - 1, 64);
        for (int q0 = 0; q0 < total; q0 += 64) {
            const int q = q0 + lane;
            int64_t j;
            const int l = wave_tracks_find(w, q, j);
            double p[5];
            for (int k = 0; k < 5; ++k) p[k] = __shfl(w.p[k], l, 64);
            const double x0 = __shfl(w.x0, l, 64);
            if (q >= total) continue;
            const int r = A.rows[j] < P.n_rows ? A.rows[j] : P.n_rows - 1;
            double yp, zp;
            predict(p, x0, (double)P.rx[r], P, yp, zp);
            A.yz[2 * j] = yp + (double)A.codes[2 * j] * A.step;
            A.yz[2 * j + 1] = zp + (double)A.codes[2 * j + 1] * A.step;
        }
    }
}

}  // namespace

void launch_compress(const CompressArgs& a, const DevParams& p, int n_cu, hipStream_t s)
{
    if (a.hit_rec)
        hipLaunchKernelGGL(k_c_encode_rec, dim3(n_cu * 16), dim3(kThreads), 0, s, a, p);
    else
        hipLaunchKernelGGL(k_c_encode, dim3(n_cu * 8), dim3(kThreads), 0, s, a, p);
}

void launch_decompress(const CompressArgs& a, const DevParams& p, int n_cu, hipStream_t s)
{
    hipLaunchKernelGGL(k_c_decode, dim3(n_cu * 16), dim3(kThreads), 0, s, a, p);
}

}  // namespace tpcsf
