// Kernels of the series-tail network: a 3-layer dilated 1D convolution over
// the first k Neumann iterates of a trace, trained and run on the GPU.
//
//   conv(k -> H, 5 taps, dilation 1), ReLU,
//   conv(H -> H, 5 taps, dilation 4), ReLU,
//   conv(H -> 2, 5 taps, dilation 16)
//
// with H hidden channels (64 for the reference architecture).
//
// y[n][o][t] = b[o] + sum_c sum_j W[o][c][j] x[n][c][t + d (j - 2)], zero
// outside [0, T).  Activations are [N][C][T] float32.  The forward pass uses
// BF16-rounded weights (the stored form of the trained network); training
// keeps FP32 master weights and Adam moments.  All reductions run in a fixed
// order, so every kernel is deterministic.
#include "mk_internal.h"

namespace {

constexpr int kTaps = 5;
constexpr int kHalf = kTaps / 2;

// y = conv(x, W, b) (+ ReLU); 64 samples x (4 * OPT) outputs per block.
// x is staged in LDS with its dilated halo; the weights of one output group
// are uniform across a wave, so they come through the scalar cache.
template <int OPT>
__global__ __launch_bounds__(256) void k_conv_fwd(const float* __restrict__ x, const float* __restrict__ W,
                                                  const float* __restrict__ b, float* __restrict__ y,
                                                  int C, int O, int T, int d, int relu) {
    extern __shared__ float xs[];                  // [C][64 + 2 halo]
    const int n = blockIdx.x;
    const int t0 = blockIdx.y * 64;
    // the output group is uniform over a wave: say so, so that the weights
    // come through the scalar cache and the bounds checks do not diverge
    const int og = __builtin_amdgcn_readfirstlane(blockIdx.z * 4 + (threadIdx.x >> 6));
    const int tl = threadIdx.x & 63;
    const int halo = d * kHalf;
    const int W64 = 64 + 2 * halo;
    const float* xn = x + (size_t)n * C * T;
    for (int i = threadIdx.x; i < C * W64; i += 256) {
        const int c = i / W64, u = i - c * W64;
        const int t = t0 - halo + u;
        xs[i] = (t >= 0 && t < T) ? xn[(size_t)c * T + t] : 0.f;
    }
    __syncthreads();
    const int o0 = og * OPT;
    if (o0 >= O) return;
    float acc[OPT];
#pragma unroll
    for (int i = 0; i < OPT; ++i) acc[i] = (o0 + i < O && b) ? b[o0 + i] : 0.f;
    // channel by channel: the five taps of one (output, channel) pair are
    // contiguous, so they come in one scalar load of five words; the sum over
    // taps and channels keeps the order c, then j
    const int nout = min(OPT, O - o0);            // uniform
    for (int c = 0; c < C; ++c) {
        const float* xr = xs + c * W64 + tl;
        float xv[kTaps];
#pragma unroll
        for (int j = 0; j < kTaps; ++j) xv[j] = xr[j * d];
        if (nout == OPT) {
#pragma unroll
            for (int i = 0; i < OPT; ++i) {
                const float* w5 = W + ((size_t)(o0 + i) * C + c) * kTaps;
#pragma unroll
                for (int j = 0; j < kTaps; ++j) acc[i] = fmaf(w5[j], xv[j], acc[i]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < OPT; ++i) {
                if (i < nout) {
                    const float* w5 = W + ((size_t)(o0 + i) * C + c) * kTaps;
#pragma unroll
                    for (int j = 0; j < kTaps; ++j) acc[i] = fmaf(w5[j], xv[j], acc[i]);
                }
            }
        }
    }
    const int t = t0 + tl;
    if (t < T) {
#pragma unroll
        for (int i = 0; i < OPT; ++i)
            if (o0 + i < O) {
                float v = acc[i];
                if (relu) v = fmaxf(v, 0.f);
                y[((size_t)n * O + o0 + i) * T + t] = v;
            }
    }
}

// Wt[c][o][j'] = W[o][c][K-1-j']: the input gradient is a forward conv of
// the output gradient with these weights.
__global__ void k_flip_weights(const float* __restrict__ W, float* __restrict__ Wt, int O, int C) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= O * C * kTaps) return;
    const int j = i % kTaps;
    const int c = (i / kTaps) % C;
    const int o = i / (kTaps * C);
    Wt[((size_t)c * O + o) * kTaps + (kTaps - 1 - j)] = W[i];
}

// g *= (a > 0): ReLU backward against the pre-activation a.
__global__ void k_relu_mask(float* __restrict__ g, const float* __restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (!(a[i] > 0.f)) g[i] = 0.f;
}

// gW[o][c][j] = sum_n sum_t gy[n][o][t] x[n][c][t + d (j - 2)]; gb[o] = sum gy.
// One block per (o, c); fixed-order tree reduction.
__global__ __launch_bounds__(256) void k_conv_bwd_w(const float* __restrict__ x, const float* __restrict__ gy,
                                                    float* __restrict__ gW, float* __restrict__ gb, int N,
                                                    int C, int O, int T, int d) {
    __shared__ float sh[kTaps + 1][256];
    const int o = blockIdx.x, c = blockIdx.y;
    float acc[kTaps + 1];
#pragma unroll
    for (int j = 0; j <= kTaps; ++j) acc[j] = 0.f;
    const int64_t total = (int64_t)N * T;
    for (int64_t i = threadIdx.x; i < total; i += 256) {
        const int n = (int)(i / T), t = (int)(i - (int64_t)n * T);
        const float g = gy[((size_t)n * O + o) * T + t];
        const float* xr = x + ((size_t)n * C + c) * T;
#pragma unroll
        for (int j = 0; j < kTaps; ++j) {
            const int u = t + d * (j - kHalf);
            if (u >= 0 && u < T) acc[j] = fmaf(g, xr[u], acc[j]);
        }
        acc[kTaps] += g;
    }
#pragma unroll
    for (int j = 0; j <= kTaps; ++j) sh[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int j = 0; j <= kTaps; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < kTaps) gW[((size_t)o * C + c) * kTaps + threadIdx.x] = sh[threadIdx.x][0];
    if (threadIdx.x == 0 && c == 0) {
        // the bias gradient needs one pass only: recompute with c == 0's sum
        gb[o] = sh[kTaps][0];
    }
}

// Masked mean squared error: g = 2 (y - target) mask / count; partial sums per block.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ tgt,
                                             const float* __restrict__ mask, int N, int O, int T,
                                             float inv_count, float* __restrict__ g,
                                             double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    const int64_t total = (int64_t)N * O * T;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int t = (int)(i % T);
        const int n = (int)(i / ((int64_t)O * T));
        const float m = mask[(size_t)n * T + t];
        const float r = (y[i] - tgt[i]) * m;
        g[i] = 2.f * r * inv_count;
        acc += (double)r * r;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_parts(const double* __restrict__ part, int n, double scale, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s * scale;
    }
}

__device__ __forceinline__ float round_bf16(float v) {
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

// Adam with bias correction on FP32 master weights; writes the BF16-rounded
// weights the forward pass uses.
__global__ void k_adam(float* __restrict__ w, float* __restrict__ wq, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wq[i] = round_bf16(wi);
}

__global__ void k_round_bf16(const float* __restrict__ w, float* __restrict__ wq, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wq[i] = round_bf16(w[i]);
}

hipError_t conv_fwd(const float* x, const float* W, const float* b, float* y, int N, int C, int O, int T,
                    int d, int relu, hipStream_t s) {
    const int halo = d * kHalf;
    const size_t lds = (size_t)C * (64 + 2 * halo) * sizeof(float);
    if (lds > 65536) return hipErrorInvalidValue;
    if (O >= 64) {
        const dim3 grid(N, (T + 63) / 64, (O + 63) / 64);
        hipLaunchKernelGGL(k_conv_fwd<16>, grid, dim3(256), lds, s, x, W, b, y, C, O, T, d, relu);
    } else if (O >= 16) {
        const dim3 grid(N, (T + 63) / 64, (O + 15) / 16);
        hipLaunchKernelGGL(k_conv_fwd<4>, grid, dim3(256), lds, s, x, W, b, y, C, O, T, d, relu);
    } else {
        const dim3 grid(N, (T + 63) / 64, (O + 3) / 4);
        hipLaunchKernelGGL(k_conv_fwd<1>, grid, dim3(256), lds, s, x, W, b, y, C, O, T, d, relu);
    }
    return hipGetLastError();
}

}  // namespace

// Parameter layout (one FP32 vector): W1 [H][k][5], b1 [H], W2 [H][H][5],
// b2 [H], W3 [2][H][5], b3 [2].
int net_param_count(int k, int H) {
    return H * k * kTaps + H + H * H * kTaps + H + 2 * H * kTaps + 2;
}

static void offsets(int k, int H, int* o) {
    o[0] = 0;                          // W1
    o[1] = o[0] + H * k * kTaps;       // b1
    o[2] = o[1] + H;                   // W2
    o[3] = o[2] + H * H * kTaps;       // b2
    o[4] = o[3] + H;                   // W3
    o[5] = o[4] + 2 * H * kTaps;       // b3
}

hipError_t net_forward(const float* P, const float* x, int N, int k, int H, int T, float* a1, float* a2,
                       float* y, hipStream_t s) {
    int o[6];
    offsets(k, H, o);
    // a1, a2 hold post-ReLU activations; the ReLU masks come from them (h > 0 <=> a > 0)
    hipError_t e = conv_fwd(x, P + o[0], P + o[1], a1, N, k, H, T, kNetDil[0], 1, s);
    if (e == hipSuccess) e = conv_fwd(a1, P + o[2], P + o[3], a2, N, H, H, T, kNetDil[1], 1, s);
    if (e == hipSuccess) e = conv_fwd(a2, P + o[4], P + o[5], y, N, H, 2, T, kNetDil[2], 0, s);
    return e;
}

hipError_t net_backward(const float* P, const float* x, const float* a1, const float* a2, const float* gy,
                        int N, int k, int H, int T, float* G, float* g1, float* g2, float* wt, hipStream_t s) {
    int o[6];
    offsets(k, H, o);
    const int64_t nact = (int64_t)N * H * T;
    const unsigned gblk = (unsigned)std::min<int64_t>((nact + 255) / 256, 16384);
    // layer 3
    hipLaunchKernelGGL(k_conv_bwd_w, dim3(2, H), dim3(256), 0, s, a2, gy, G + o[4], G + o[5], N, H, 2, T,
                       kNetDil[2]);
    hipLaunchKernelGGL(k_flip_weights, dim3((2 * H * kTaps + 255) / 256), dim3(256), 0, s, P + o[4], wt, 2, H);
    hipError_t e = conv_fwd(gy, wt, nullptr, g2, N, 2, H, T, kNetDil[2], 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_relu_mask, dim3(gblk), dim3(256), 0, s, g2, a2, nact);
    // layer 2
    hipLaunchKernelGGL(k_conv_bwd_w, dim3(H, H), dim3(256), 0, s, a1, g2, G + o[2], G + o[3], N, H, H, T,
                       kNetDil[1]);
    hipLaunchKernelGGL(k_flip_weights, dim3((H * H * kTaps + 255) / 256), dim3(256), 0, s, P + o[2], wt, H, H);
    e = conv_fwd(g2, wt, nullptr, g1, N, H, H, T, kNetDil[1], 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_relu_mask, dim3(gblk), dim3(256), 0, s, g1, a1, nact);
    // layer 1 (no input gradient needed)
    hipLaunchKernelGGL(k_conv_bwd_w, dim3(H, k), dim3(256), 0, s, x, g1, G + o[0], G + o[1], N, k, H, T,
                       kNetDil[0]);
    return hipGetLastError();
}

hipError_t net_mse(const float* y, const float* tgt, const float* mask, int N, int T, float* gy,
                   double* part, int nparts, double* loss, float count, hipStream_t s) {
    hipLaunchKernelGGL(k_mse, dim3(nparts), dim3(256), 0, s, y, tgt, mask, N, 2, T, 1.f / count, gy, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, part, nparts, 1.0 / (double)count, loss);
    return hipGetLastError();
}

hipError_t net_adam(float* w, float* wq, const float* g, float* m, float* v, int n, int step, float lr,
                    float b1, float b2, float eps, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, w, wq, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t net_round_bf16(const float* w, float* wq, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_round_bf16, dim3((n + 255) / 256), dim3(256), 0, s, w, wq, n);
    return hipGetLastError();
}
