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
#include <type_traits>

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

// The same convolution for the network's dilations (1, 4, 16): 256 samples
// x (4 * OPT) outputs per block, four consecutive samples per thread, so that
// one tap of one channel is one aligned 16-byte LDS read for the thread's
// four samples (dilation 1: two reads cover all five taps) and every weight
// feeds four products.  The order of the sum (channel, then tap) is the one
// k_conv_fwd uses: both give the same bits.
template <int OPT, int D>
__global__ __launch_bounds__(256) void k_conv_fwd_q(const float* __restrict__ x, const float* __restrict__ W,
                                                    const float* __restrict__ b, float* __restrict__ y, int C,
                                                    int O, int T, int relu) {
    constexpr int HALO = D * kHalf;               // 2, 8, 32: rows stay 16-byte aligned
    constexpr int WR = 256 + 2 * HALO;            // floats per staged channel
    constexpr int NXV = D == 1 ? 8 : 4 * kTaps;
    extern __shared__ float4 xs4[];               // [C][WR]
    float* xs = reinterpret_cast<float*>(xs4);
    const int n = blockIdx.x;
    const int t0 = blockIdx.y * 256;
    const int og = __builtin_amdgcn_readfirstlane(blockIdx.z * 4 + (threadIdx.x >> 6));
    const int q = threadIdx.x & 63;
    const float* xn = x + (size_t)n * C * T;
    for (int i = threadIdx.x; i < C * WR; i += 256) {
        const int c = i / WR, u = i - c * WR;
        const int t = t0 - HALO + u;
        xs[i] = (t >= 0 && t < T) ? xn[(size_t)c * T + t] : 0.f;
    }
    __syncthreads();
    const int o0 = og * OPT;
    if (o0 >= O) return;
    float acc[OPT][4];
#pragma unroll
    for (int i = 0; i < OPT; ++i) {
        const float bi = (o0 + i < O && b) ? b[o0 + i] : 0.f;
#pragma unroll
        for (int sm = 0; sm < 4; ++sm) acc[i][sm] = bi;
    }
    const int nout = min(OPT, O - o0);            // uniform
    for (int c = 0; c < C; ++c) {
        // sample t0 + 4q + sm, tap j reads staged x at 4q + sm + D j
        const float* xr = xs + c * WR + 4 * q;
        float xv[NXV];
        if constexpr (D == 1) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float4 v = *reinterpret_cast<const float4*>(xr + 4 * h);
                xv[4 * h] = v.x, xv[4 * h + 1] = v.y, xv[4 * h + 2] = v.z, xv[4 * h + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < kTaps; ++j) {
                const float4 v = *reinterpret_cast<const float4*>(xr + D * j);
                xv[4 * j] = v.x, xv[4 * j + 1] = v.y, xv[4 * j + 2] = v.z, xv[4 * j + 3] = v.w;
            }
        }
        auto xat = [&](int sm, int j) { return D == 1 ? xv[sm + j] : xv[4 * j + sm]; };
#pragma unroll
        for (int i = 0; i < OPT; ++i) {
            if (nout == OPT || i < nout) {
                const float* w5 = W + ((size_t)(o0 + i) * C + c) * kTaps;
#pragma unroll
                for (int j = 0; j < kTaps; ++j) {
                    const float wj = w5[j];
#pragma unroll
                    for (int sm = 0; sm < 4; ++sm) acc[i][sm] = fmaf(wj, xat(sm, j), acc[i][sm]);
                }
            }
        }
    }
    const int t = t0 + 4 * q;
#pragma unroll
    for (int i = 0; i < OPT; ++i) {
        if (o0 + i >= O) continue;
        float v[4];
#pragma unroll
        for (int sm = 0; sm < 4; ++sm) v[sm] = relu ? fmaxf(acc[i][sm], 0.f) : acc[i][sm];
        float* yr = y + ((size_t)n * O + o0 + i) * T;
        if ((T & 3) == 0 && (reinterpret_cast<uintptr_t>(y) & 15) == 0 && t + 3 < T) {
            *reinterpret_cast<float4*>(yr + t) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
#pragma unroll
            for (int sm = 0; sm < 4; ++sm)
                if (t + sm < T) yr[t + sm] = v[sm];
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

template <int D>
hipError_t conv_fwd_q(const float* x, const float* W, const float* b, float* y, int N, int C, int O, int T,
                      int relu, size_t lds, hipStream_t s) {
    const int gt = (T + 255) / 256;
    if (O >= 64) {
        hipLaunchKernelGGL((k_conv_fwd_q<16, D>), dim3(N, gt, (O + 63) / 64), dim3(256), lds, s, x, W, b, y, C, O,
                           T, relu);
    } else if (O >= 16) {
        hipLaunchKernelGGL((k_conv_fwd_q<4, D>), dim3(N, gt, (O + 15) / 16), dim3(256), lds, s, x, W, b, y, C, O,
                           T, relu);
    } else {
        hipLaunchKernelGGL((k_conv_fwd_q<1, D>), dim3(N, gt, (O + 3) / 4), dim3(256), lds, s, x, W, b, y, C, O, T,
                           relu);
    }
    return hipGetLastError();
}

hipError_t conv_fwd(const float* x, const float* W, const float* b, float* y, int N, int C, int O, int T,
                    int d, int relu, hipStream_t s) {
    if (d == 1 || d == 4 || d == 16) {
        const size_t lq = (size_t)C * (256 + 2 * d * kHalf) * sizeof(float);
        if (lq <= 65536) {
            if (d == 1) return conv_fwd_q<1>(x, W, b, y, N, C, O, T, relu, lq, s);
            if (d == 4) return conv_fwd_q<4>(x, W, b, y, N, C, O, T, relu, lq, s);
            return conv_fwd_q<16>(x, W, b, y, N, C, O, T, relu, lq, s);
        }
    }
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

// ---------------------------------------------------------------------------
// The whole network on one 256-sample tile of one trace (hidden width 16),
// in its inference form with half-precision activations, with the tail it
// predicts added to f1+ and f1- on the spot.  Each layer's output stays in
// LDS over the span the next layer reads,
//
//   y on [t0, t0 + 256), a2 on [t0 - 32, t0 + 288), a1 on [t0 - 40, t0 + 296),
//   x on [t0 - 42, t0 + 298),
//
// zero outside [0, T) exactly as the layer-by-layer form pads each input.
// The input and both hidden activations are stored as halves (round to
// nearest even, saturating at 65504); the weights (BF16-rounded FP32 values,
// exact in half precision within its range) are converted once.  Each layer
// is a product of a 16 x 5C weight block with a 5C x 16 block of shifted
// samples on v_mfma_f32_16x16x32_f16 with FP32 accumulation (a product of two
// halves is exact in FP32).  Activations are stored sample-major, channels
// contiguous, so the eight K values a lane feeds (eight channels at one tap,
// or four channels at two adjacent taps) are one or two LDS reads.  A tile
// that shares no sample with the trace's mute window is skipped: the tail is
// only used inside the window, and two tiles never touch the same f1 sample.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));

constexpr int kFH = 16;                        // hidden width of this form
constexpr int kFT = 256;                       // output samples per block
constexpr int kX0 = 42, kA10 = 40, kA20 = 32;  // reach of x, a1, a2 left of t0
constexpr int kXN = kFT + 2 * kX0;             // 340 staged input samples
constexpr int kA1N = kFT + 2 * kA10;           // 336 = 21 tiles of 16
constexpr int kA2N = kFT + 2 * kA20;           // 320 = 20 tiles of 16
constexpr int kHP = 16;                        // halves per sample row of 16 channels: 32-byte
                                               // rows, so the eight lanes a 16-byte read serves per
                                               // cycle hit distinct banks

__device__ __forceinline__ _Float16 to_half_sat(float v) {
    return (_Float16)fminf(fmaxf(v, -65504.f), 65504.f);
}

// K pairing of one matrix-core step of a C-channel layer: lane group g,
// element e -> (channel, tap).  C = 16: tap 2m + g/2, channels 8 (g & 1) + e;
// C = 8: tap 4m + g, channel e; C = 4: taps 8m + 2g + e/4, channel e & 3.
template <int C>
__device__ __forceinline__ void kpair(int m, int g, int e, int& c, int& j) {
    if constexpr (C == 16) { j = 2 * m + (g >> 1); c = 8 * (g & 1) + e; }
    else if constexpr (C == 8) { j = 4 * m + g; c = e; }
    else { j = 8 * m + 2 * g + (e >> 2); c = e & 3; }
}
template <int C> constexpr int ksteps() { return C == 16 ? 3 : C == 8 ? 2 : 1; }

// A operand of step m for output row i16 (rows >= nout and pairs past the
// five taps or the cin real channels are zero): W [nout][cin][5] FP32
template <int C>
__device__ __forceinline__ h8 weights_a(const float* __restrict__ W, int cin, int nout, int i16, int g, int m) {
    h8 a;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        int c, j;
        kpair<C>(m, g, e, c, j);
        const bool ok = i16 < nout && c < cin && j < kTaps;
        a[e] = ok ? (_Float16)W[(i16 * cin + c) * kTaps + j] : (_Float16)0.f;
    }
    return a;
}

// B operand of step m: the activation rows act[(s + d j) * pitch + c] of
// sample s of the tile (taps past the fifth read tap 4: their weights are 0)
template <int C, int D, int PITCH>
__device__ __forceinline__ h8 acts_b(const _Float16* act, int s, int g, int m) {
    if constexpr (C == 4) {
        const int j0 = min(8 * m + 2 * g, kTaps - 1), j1 = min(8 * m + 2 * g + 1, kTaps - 1);
        const h4 lo = *reinterpret_cast<const h4*>(act + (s + D * j0) * PITCH);
        const h4 hi = *reinterpret_cast<const h4*>(act + (s + D * j1) * PITCH);
        return h8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    } else {
        int c, j;
        kpair<C>(m, g, 0, c, j);
        j = min(j, kTaps - 1);
        return *reinterpret_cast<const h8*>(act + (s + D * j) * PITCH + c);
    }
}

// The three layers' A operands in the per-lane order the matrix cores take
// them, written once per loaded network: step q of the table holds 64 lanes
// x 8 halves, so a block reads each step with one 16-byte load per lane.
// Steps: layer 1 (ksteps<KP>), layer 2 (3), layer 3 (3).
template <int KP>
__global__ __launch_bounds__(64) void k_pack_tail(const float* __restrict__ P, int k, h8* __restrict__ out) {
    constexpr int S1 = ksteps<KP>(), S2 = ksteps<kFH>();
    const int lane = threadIdx.x, i16 = lane & 15, g = lane >> 4, q = blockIdx.x;
    const float* W1 = P;
    const float* W2 = W1 + kFH * k * kTaps + kFH;
    const float* W3 = W2 + kFH * kFH * kTaps + kFH;
    h8 a;
    if (q < S1) a = weights_a<KP>(W1, k, kFH, i16, g, q);
    else if (q < S1 + S2) a = weights_a<kFH>(W2, kFH, kFH, i16, g, q - S1);
    else a = weights_a<kFH>(W3, kFH, 2, i16, g, q - S1 - S2);
    out[q * 64 + lane] = a;
}

template <int KP>
__global__ __launch_bounds__(256) void k_net_tail(const float* __restrict__ P, const h8* __restrict__ wpk,
                                                  const float* __restrict__ hist,
                                                  const float* __restrict__ scale, const int32_t* __restrict__ itd,
                                                  int shift, int k, int T, int nt, float* __restrict__ f1p,
                                                  Ext3 ext) {
    constexpr int XP = KP == 16 ? kHP : KP;    // halves per staged input sample
    constexpr int S1 = ksteps<KP>(), S2 = ksteps<kFH>();
    constexpr int U2 = kXN * XP > kA2N * kHP ? kXN * XP : kA2N * kHP;
    __shared__ __attribute__((aligned(16))) _Float16 a1s[kA1N * kHP];
    __shared__ __attribute__((aligned(16))) _Float16 u2[U2];     // x, then a2
    const int tr = blockIdx.x;
    const int t0 = blockIdx.y * kFT;
    const int hT = T >> 1;
    // a tile that shares no sample with the mute window |t| < L leaves before
    // it loads anything (one round trip for itd first; the other blocks on
    // the CU cover it)
    const int L = itd[tr] - shift;
    if (L <= 0 || t0 >= hT + L || t0 + kFT <= hT - L + 1) return;
    // checked build: this trace's recorded iterates and its f1+
    MK_DCHECK((int64_t)(tr + 1) * k * T * 4 <= ext.r && (int64_t)(tr + 1) * nt * 4 <= ext.y);
    const float se = scale[tr];
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int i16 = lane & 15, g = lane >> 4;
    const float* B1 = P + kFH * k * kTaps;
    const float* B2 = B1 + kFH + kFH * kFH * kTaps;
    const float* B3 = B2 + kFH + 2 * kFH * kTaps;

    // layer 1's weights now; layers 2 and 3 load theirs where they start
    // (cache hits), so that fewer registers stay live
    h8 w1[S1];
#pragma unroll
    for (int m = 0; m < S1; ++m) w1[m] = wpk[m * 64 + lane];
    v4f bias1, bias2, bias3;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        bias1[r] = B1[4 * g + r];
        bias2[r] = B2[4 * g + r];
        // unconditional loads, masked: a selected load becomes a branch that waits for it
        const float v3 = B3[min(4 * g + r, 1)];
        bias3[r] = __uint_as_float(__float_as_uint(v3) & (4 * g + r < 2 ? 0xFFFFFFFFu : 0u));
    }

    // Every global load of the block is issued here, before any use: the
    // input samples (one thread per sample, all channels) and the f1 samples
    // this block updates (tile wv + 4 m, sample i16; lanes of every group
    // load the same addresses as group 0, which alone stores).
    const float* h = hist + (size_t)tr * k * T;
    constexpr int NU = (kXN + 255) / 256;
    float xv[NU][KP];
#pragma unroll
    for (int it = 0; it < NU; ++it) {
        const int u = threadIdx.x + 256 * it;
        const int t = t0 - kX0 + u;
        const bool in = u < kXN && t >= 0 && t < T;
        const float* hc = h + (in ? t : 0);
#pragma unroll
        for (int c = 0; c < KP; ++c) {
            // always a valid address; the value is masked, not selected (a
            // selected load becomes a branch that waits for it)
            const float v = hc[(size_t)(c < k ? c : 0) * T];
            xv[it][c] = __uint_as_float(__float_as_uint(v) & ((in && c < k) ? 0xFFFFFFFFu : 0u));
        }
    }
    float* fp = f1p + (size_t)tr * nt;
    // |t| <= T/2 <= nt/2 for u < T: one wrap at most
    auto f1_ip = [&](int m) {
        const int u = t0 + 16 * (wv + 4 * m) + i16;
        const int t = u - hT;
        return u < T ? (t < 0 ? t + nt : t) : 0;
    };
    float pv[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) pv[m] = fp[f1_ip(m)];
    const float inv = se > 0.f ? 1.f / se : 0.f;
    // output samples s = u - t0 of this tile the tail is used at: [lo3, hi3]
    // (not empty: the window test passed); layer 2 is needed on [lo3, hi3 + 64]
    // and layer 1 on [lo3, hi3 + 80] of their own spans.  A 16-sample tile of
    // a layer outside its range is not computed: only outputs that are never
    // used would read it.
    const int lo3 = max(hT - L + 1 - t0, 0), hi3 = min(hT + L - 1 - t0, kFT - 1);
    auto needed = [&](int tile, int hi) { return 16 * tile + 15 >= lo3 && 16 * tile <= hi; };
    bool upd[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int u = t0 + 16 * (wv + 4 * m) + i16;
        const int t = u - hT;
        upd[m] = u < T && t < L && -t < L && t != nt / 2 && -t != nt / 2;
    }

    // stage x = hist * inv as halves, sample-major; padding channels are zero
    _Float16* xs = u2;
#pragma unroll
    for (int it = 0; it < NU; ++it) {
        const int u = threadIdx.x + 256 * it;
        if (u < kXN) {
#pragma unroll
            for (int c0 = 0; c0 < KP; c0 += 4)
                *reinterpret_cast<h4*>(xs + u * XP + c0) =
                    h4{to_half_sat(xv[it][c0] * inv), to_half_sat(xv[it][c0 + 1] * inv),
                       to_half_sat(xv[it][c0 + 2] * inv), to_half_sat(xv[it][c0 + 3] * inv)};
        }
    }
    __syncthreads();

    // NT tiles of a hidden layer at once (tiles wv + 4 i): every operand read
    // is issued before the first product, the products of different tiles
    // interleave, and rows 4 g + r of each result go to LDS as halves
    auto hidden_layer = [&](auto cin_tag, auto d_tag, auto pitch_tag, auto nt_tag, const _Float16* in, const h8* w,
                            v4f bias, _Float16* out, int tile0, int tstep, int tfirst) {
        constexpr int C = decltype(cin_tag)::value, D = decltype(d_tag)::value, PIN = decltype(pitch_tag)::value;
        constexpr int NTL = decltype(nt_tag)::value, NS = ksteps<C>();
        h8 b[NTL][NS];
#pragma unroll
        for (int i = 0; i < NTL; ++i)
#pragma unroll
            for (int q = 0; q < NS; ++q) b[i][q] = acts_b<C, D, PIN>(in, 16 * (tile0 + tstep * i) + i16, g, q);
        v4f acc[NTL];
#pragma unroll
        for (int i = 0; i < NTL; ++i) acc[i] = bias;
#pragma unroll
        for (int q = 0; q < NS; ++q)
#pragma unroll
            for (int i = 0; i < NTL; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_f16(w[q], b[i][q], acc[i], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < NTL; ++i) {
            const int sidx = 16 * (tile0 + tstep * i) + i16;
            const int t = tfirst + sidx;
            const bool ok = t >= 0 && t < T;
            h4 o;
#pragma unroll
            for (int r = 0; r < 4; ++r) o[r] = ok ? to_half_sat(fmaxf(acc[i][r], 0.f)) : (_Float16)0.f;
            *reinterpret_cast<h4*>(out + sidx * kHP + 4 * g) = o;
        }
    };

    // layer 1: 21 tiles; layer 2: 20 tiles (x is dead: a2 takes its place)
    // (one 16-sample tile at a time, each only where it is needed)
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const int tile = wv + 4 * m;
        if (tile < kA1N / 16 && needed(tile, hi3 + 80))
            hidden_layer(std::integral_constant<int, KP>{}, std::integral_constant<int, 1>{},
                         std::integral_constant<int, XP>{}, std::integral_constant<int, 1>{}, xs, w1, bias1, a1s, tile,
                         0, t0 - kA10);
    }
    __syncthreads();
    _Float16* a2s = u2;
    h8 w2[S2];
#pragma unroll
    for (int m = 0; m < S2; ++m) w2[m] = wpk[(S1 + m) * 64 + lane];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        const int tile = wv + 4 * m;
        if (needed(tile, hi3 + 64))
            hidden_layer(std::integral_constant<int, kFH>{}, std::integral_constant<int, 4>{},
                         std::integral_constant<int, kHP>{}, std::integral_constant<int, 1>{}, a1s, w2, bias2, a2s,
                         tile, 0, t0 - kA20);
    }
    __syncthreads();

    // layer 3 (rows 0 and 1 of a padded 16-row product) and the tail
    // f1+ += s y_odd inside the window.  The even-pass tail (row 0) is not
    // applied: the restart that judges the estimate rebuilds f1- from f1+
    // alone (f1- := theta S f1+), so nothing would read it.
    h8 w3[S2];
#pragma unroll
    for (int m = 0; m < S2; ++m) w3[m] = wpk[(S1 + S2 + m) * 64 + lane];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        if (!needed(wv + 4 * m, hi3)) continue;
        v4f y = bias3;
#pragma unroll
        for (int q = 0; q < S2; ++q)
            y = __builtin_amdgcn_mfma_f32_16x16x32_f16(w3[q], acts_b<kFH, 16, kHP>(a2s, 16 * (wv + 4 * m) + i16, g, q),
                                                       y, 0, 0, 0);
        if (g == 0 && upd[m]) fp[f1_ip(m)] = pv[m] + se * y[1];
    }
}

}  // namespace

MK_CHECK_TAKE(check_take_net)

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

bool net_tail_fused(int k, int H) { return H == kFH && k >= 1 && k <= 16; }

size_t net_tail_pack_bytes(int k) {
    const int s1 = k <= 4 ? ksteps<4>() : k <= 8 ? ksteps<8>() : ksteps<16>();
    return (size_t)(s1 + 2 * ksteps<kFH>()) * 64 * sizeof(h8);
}

hipError_t net_tail_pack(const float* P, int k, int H, void* out, hipStream_t s) {
    if (!net_tail_fused(k, H)) return hipErrorInvalidValue;
    h8* o = static_cast<h8*>(out);
    const int s2 = 2 * ksteps<kFH>();
    if (k <= 4)
        hipLaunchKernelGGL(k_pack_tail<4>, dim3(ksteps<4>() + s2), dim3(64), 0, s, P, k, o);
    else if (k <= 8)
        hipLaunchKernelGGL(k_pack_tail<8>, dim3(ksteps<8>() + s2), dim3(64), 0, s, P, k, o);
    else
        hipLaunchKernelGGL(k_pack_tail<16>, dim3(ksteps<16>() + s2), dim3(64), 0, s, P, k, o);
    return hipGetLastError();
}

hipError_t net_tail_apply(const float* P, const void* wpack, const float* hist, const float* scale,
                          const int32_t* itd, int shift, int ntr, int k, int H, int T, int nt, float* f1p,
                          hipStream_t s) {
    if (!net_tail_fused(k, H)) return hipErrorInvalidValue;
    if (ntr <= 0 || T <= 0) return hipSuccess;
    const h8* w = static_cast<const h8*>(wpack);
    const dim3 grid(ntr, (T + kFT - 1) / kFT);
    const Ext3 ext{device_extent(hist), kExtentUnknown, device_extent(f1p)};
    if (k <= 4)
        hipLaunchKernelGGL(k_net_tail<4>, grid, dim3(256), 0, s, P, w, hist, scale, itd, shift, k, T, nt, f1p, ext);
    else if (k <= 8)
        hipLaunchKernelGGL(k_net_tail<8>, grid, dim3(256), 0, s, P, w, hist, scale, itd, shift, k, T, nt, f1p, ext);
    else
        hipLaunchKernelGGL(k_net_tail<16>, grid, dim3(256), 0, s, P, w, hist, scale, itd, shift, k, T, nt, f1p,
                           ext);
    return hipGetLastError();
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
