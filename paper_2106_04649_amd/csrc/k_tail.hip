// Series-tail application: the recorded first k iterates of each trace ->
// an estimate of the remaining odd-pass sum, added to f1+ inside the mute
// window.  One wave per trace.  The even-pass sum would feed f1-, but the
// restart that judges every tail rebuilds f1- from f1+ alone
// (f1- := theta S f1+), so it is not applied.
//
// Window convention: recorded sample u of a trace holds time t = u - T/2
// (periodic index t mod nt).  T_odd feeds f1+ += T_odd (odd passes), as in
// the series itself.
#include "mk_internal.h"

namespace {

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// x[tr][c][u] = hist[tr][c][u] / s_tr with s_tr the RMS of the first iterate
// over the window (0 for a silent trace, which the network then skips); with
// x NULL only s_tr is written (the fused network scales as it stages).
__global__ __launch_bounds__(256) void k_tail_prep(const float* __restrict__ hist, int ntr, int k, int T,
                                                   float* __restrict__ x, float* __restrict__ scale, Ext3 ext) {
    const int lane = threadIdx.x & 63;
    const int tr = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tr >= ntr) return;
    // checked build: this trace's recorded iterates, and its scaled copy
    MK_DCHECK((int64_t)(tr + 1) * k * T * 4 <= ext.r);
    if (x) MK_DCHECK((int64_t)(tr + 1) * k * T * 4 <= ext.x);
    const float* h = hist + (size_t)tr * k * T;
    float ss = 0.f;
    for (int u = lane; u < T; u += 64) ss += h[u] * h[u];
    ss = wave_sum_f(ss);
    const float s = sqrtf(ss / (float)T);
    const float inv = s > 1e-30f ? 1.f / s : 0.f;
    if (x) {
        float* xo = x + (size_t)tr * k * T;
        for (int i = lane; i < k * T; i += 64) xo[i] = h[i] * inv;
    }
    if (lane == 0) scale[tr] = inv > 0.f ? s : 0.f;
}

// mode 0: the odd tail from the network output y[tr][2][T] (channel 1)
// mode 1: geometric extrapolation of the last two odd iterates
__global__ __launch_bounds__(256) void k_tail_apply(const float* __restrict__ hist, const float* __restrict__ y,
                                                    const float* __restrict__ scale, const int32_t* __restrict__ itd,
                                                    int shift, int ntr, int k, int T, int nt, int mode,
                                                    float* __restrict__ f1p, Ext3 ext) {
    const int lane = threadIdx.x & 63;
    const int tr = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tr >= ntr) return;
    // checked build: this trace's recorded iterates, network output and f1+
    MK_DCHECK((int64_t)(tr + 1) * k * T * 4 <= ext.r);
    if (mode == 0) MK_DCHECK((int64_t)(tr + 1) * 2 * T * 4 <= ext.x);
    MK_DCHECK((int64_t)(tr + 1) * nt * 4 <= ext.y);
    const float* h = hist + (size_t)tr * k * T;
    const int L = itd[tr] - shift;
    const int hT = T >> 1;
    float g = 0.f;
    constexpr int U = 8;                       // samples per lane whose loads are in flight together
    if (mode == 1) {
        // ratio of the norms of the last two odd iterates (k even: channels k-3, k-1)
        float n[2] = {0.f, 0.f};
        for (int u0 = 0; u0 < T; u0 += 64 * U) {
            float v[U][2];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int u = min(u0 + lane + 64 * j, T - 1);
                v[j][0] = h[(size_t)(k - 3) * T + u];
                v[j][1] = h[(size_t)(k - 1) * T + u];
            }
#pragma unroll
            for (int j = 0; j < U; ++j)
                if (u0 + lane + 64 * j < T) {
                    n[0] += v[j][0] * v[j][0];
                    n[1] += v[j][1] * v[j][1];
                }
        }
        n[0] = sqrtf(wave_sum_f(n[0]));
        n[1] = sqrtf(wave_sum_f(n[1]));
        const float qo = n[0] > 0.f ? fminf(n[1] / n[0], 0.9f) : 0.f;
        g = qo / (1.f - qo);
    } else {
        g = scale[tr];
    }
    float* fp = f1p + (size_t)tr * nt;
    // window samples t = u - T/2 with |t| < L (t = +-nt/2 excluded); every
    // read of a group is issued before the first update (addresses of samples
    // outside the window are clamped to the trace's first sample and unused)
    for (int u0 = 0; u0 < T; u0 += 64 * U) {
        float to[U], pv[U];
        int ip[U];
        bool in[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int u = u0 + lane + 64 * j;
            const int t = u - hT;
            in[j] = (u < T) & (t < L) & (-t < L) & (t != nt / 2) & (-t != nt / 2);
            const int uc = min(u, T - 1);
            to[j] = mode == 1 ? h[(size_t)(k - 1) * T + uc] : y[((size_t)tr * 2 + 1) * T + uc];
            ip[j] = in[j] ? ((t % nt) + nt) % nt : 0;
            pv[j] = fp[ip[j]];
        }
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (in[j]) fp[ip[j]] = pv[j] + g * to[j];      // odd passes feed f1+
    }
}

}  // namespace

MK_CHECK_TAKE(check_take_tail)


hipError_t launch_tail_prep(const float* hist, int ntr, int k, int T, float* x, float* scale, hipStream_t s) {
    if (ntr <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tail_prep, dim3((ntr + 3) / 4), dim3(256), 0, s, hist, ntr, k, T, x, scale,
                       Ext3{device_extent(hist), device_extent(x), kExtentUnknown});
    return hipGetLastError();
}

hipError_t launch_tail_apply(const float* hist, const float* y, const float* scale, const int32_t* itd, int shift,
                             int ntr, int k, int T, int nt, int mode, float* f1p, hipStream_t s) {
    if (ntr <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tail_apply, dim3((ntr + 3) / 4), dim3(256), 0, s, hist, y, scale, itd, shift, ntr, k, T,
                       nt, mode, f1p, Ext3{device_extent(hist), device_extent(y), device_extent(f1p)});
    return hipGetLastError();
}
