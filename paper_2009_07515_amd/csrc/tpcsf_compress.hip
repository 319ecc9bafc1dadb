// Track-model compression of the attached clusters (arXiv:2009.07515, Sec. 4, entropy
// reduction step): each cluster attached to a track is stored as its row and its residual
// to the track's position on that row plane, quantised; the track's state at x_ref is
// kept with the track.  The position is the state propagated in one helix step to the row
// (the state at x_ref itself where that step fails), so that every cluster decodes
// independently: y = y_p + q_y * step, z = z_p + q_z * step, within half a step.
//
// Layout: one wave per track, its lanes over the track's clusters (64 per pass); the
// encoder finds each cluster's row in the sector's row offsets, staged in the wave's LDS.
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
        wave_lds_sync();
        for (int r = lane; r <= nr; r += 64) o[r] = A.off[g0 + r];
        wave_lds_sync();
        double p[5];
        for (int q = 0; q < 5; ++q) p[q] = A.par[t * 5 + q];
        const double x0 = A.xref[t];
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

__global__ void __launch_bounds__(kThreads) k_c_decode(CompressArgs A, DevParams P)
{
    int64_t T = *A.n_tracks;
    if (T > A.cap_tracks) T = A.cap_tracks;
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; t < T; t += nw) {
        const int64_t hb = A.hit_off[t], he = A.hit_off[t + 1];
        if (!(hb >= 0 && he >= hb && he <= A.cap_hits)) continue;
        double p[5];
        for (int q = 0; q < 5; ++q) p[q] = A.par[t * 5 + q];
        const double x0 = A.xref[t];
        for (int64_t j = hb + lane; j < he; j += 64) {
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
    hipLaunchKernelGGL(k_c_encode, dim3(n_cu * 8), dim3(kThreads), 0, s, a, p);
}

void launch_decompress(const CompressArgs& a, const DevParams& p, int n_cu, hipStream_t s)
{
    hipLaunchKernelGGL(k_c_decode, dim3(n_cu * 8), dim3(kThreads), 0, s, a, p);
}

}  // namespace tpcsf
