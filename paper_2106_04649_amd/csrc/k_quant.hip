// Reduced-precision storage of R: FP16 or BF16 pairs with one FP32 scale per
// frequency, R[w][r][s] ~= rscale[w] * q[w][r][s].  The scale maps the largest
// component of each frequency slice to 2^14, which keeps every FP16 value in
// the normal range down to 2^-14 of the slice maximum.
#include "mk_internal.h"

namespace {

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);     // round to nearest, ties to even (inputs are finite)
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint16_t f32_to_f16_rne(float x) {
    _Float16 h = (_Float16)x;           // v_cvt_f16_f32: round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}

// Per-frequency max |component| of the caller's [nr][B][ns] complex64 input.
__global__ __launch_bounds__(256) void k_rmax(const float2* __restrict__ in, int nr, int B, int ns,
                                              float* __restrict__ rmax, int* __restrict__ flag) {
    __shared__ float sh[256];
    const int w = blockIdx.x;
    float m = 0.f;
    for (int r = 0; r < nr; ++r) {
        const float2* row = in + ((int64_t)r * B + w) * ns;
        for (int s = threadIdx.x; s < ns; s += 256) {
            const float2 v = row[s];
            if (!isfinite(v.x) || !isfinite(v.y)) *flag = 1;
            m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
        }
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // a slice whose largest value is below 2^-100 quantises to zero with unit scale
        // (its scale would underflow FP32 and make the quotient infinite)
        const float mx = sh[0];
        rmax[w] = (mx >= 0x1p-100f && isfinite(mx)) ? mx * (1.0f / 16384.0f) : 1.0f;
    }
}

// out[w][r][s] = q(in[r][w][s] / rscale[w]) as 16-bit pairs; zero padding s >= ns.
template <int PREC>
__global__ void k_repack_q(const float2* __restrict__ in, uint32_t* __restrict__ out,
                           const float* __restrict__ rscale, int nr, int B, int ns, int ns_pad) {
    const int64_t total = (int64_t)B * nr * ns_pad;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(i % ns_pad);
        const int64_t wr = i / ns_pad;
        const int r = (int)(wr % nr);
        const int w = (int)(wr / nr);
        uint32_t v = 0;
        if (s < ns) {
            const float2 x = in[((int64_t)r * B + w) * ns + s];
            const float inv = 1.0f / rscale[w];
            const float a = x.x * inv, b = x.y * inv;
            uint16_t lo, hi;
            if (PREC == 1) {
                lo = f32_to_f16_rne(a);
                hi = f32_to_f16_rne(b);
            } else {
                lo = f32_to_bf16_rne(a);
                hi = f32_to_bf16_rne(b);
            }
            v = (uint32_t)lo | ((uint32_t)hi << 16);
        }
        out[i] = v;
    }
}

// One thread per 16-byte piece of the tiled layout (see mk_internal.h).
template <int PREC>
__global__ void k_repack_tiled(const float2* __restrict__ in, uint4* __restrict__ out,
                               const float* __restrict__ rscale, int nr, int B, int ns, int ng, int nch,
                               int* __restrict__ flag) {
    constexpr int EB = PREC == MK_R_C64 ? 8 : 4;       // bytes per complex element
    constexpr int PER = 16 / EB;                       // complex elements per piece
    const int64_t total = (int64_t)B * ng * nch * 128;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(o & 63), h = (int)((o >> 6) & 1);
        const int64_t t = o >> 7;
        const int c = (int)(t % nch);
        const int64_t t2 = t / nch;
        const int rg = (int)(t2 % ng);
        const int w = (int)(t2 / ng);
        const int r = rg * kTileRows + (lane & 15);
        const int s0 = (c * kTileChunkBytes + (lane >> 4) * 32 + h * 16) / EB;
        uint32_t word[4] = {0u, 0u, 0u, 0u};
        const float inv = PREC == MK_R_C64 ? 1.f : 1.0f / rscale[w];
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int sidx = s0 + e;
            float2 v = make_float2(0.f, 0.f);
            if (r < nr && sidx < ns) {
                v = in[((int64_t)r * B + w) * ns + sidx];
                if (PREC == MK_R_C64 && (!isfinite(v.x) || !isfinite(v.y))) *flag = 1;
            }
            if constexpr (PREC == MK_R_C64) {
                word[2 * e] = __float_as_uint(v.x);
                word[2 * e + 1] = __float_as_uint(v.y);
            } else if constexpr (PREC == MK_R_F16S) {
                word[e] = (uint32_t)f32_to_f16_rne(v.x * inv) | ((uint32_t)f32_to_f16_rne(v.y * inv) << 16);
            } else {
                word[e] = (uint32_t)f32_to_bf16_rne(v.x * inv) | ((uint32_t)f32_to_bf16_rne(v.y * inv) << 16);
            }
        }
        out[o] = make_uint4(word[0], word[1], word[2], word[3]);
    }
}

}  // namespace

size_t tiled_R_bytes(int prec, int nr, int B, int ns_pad) {
    const int eb = prec == MK_R_C64 ? 8 : 4;
    const size_t ng = (size_t)((nr + kTileRows - 1) / kTileRows);
    const size_t nch = (size_t)ns_pad * eb / kTileChunkBytes;
    return (size_t)B * ng * nch * 2048;
}

hipError_t launch_repack_tiled(int prec, const float* Rin, void* Rout, const float* rscale, int nr, int B,
                               int ns, int ns_pad, int* flag, hipStream_t s) {
    const int eb = prec == MK_R_C64 ? 8 : 4;
    if ((ns_pad * eb) % kTileChunkBytes != 0) return hipErrorInvalidValue;
    const int ng = (nr + kTileRows - 1) / kTileRows;
    const int nch = ns_pad * eb / kTileChunkBytes;
    const int64_t total = (int64_t)B * ng * nch * 128;
    const int64_t blocks = (total + 255) / 256;
    const unsigned g = (unsigned)(blocks < 65536 * 4 ? blocks : 65536 * 4);
    const float2* in = reinterpret_cast<const float2*>(Rin);
    uint4* out = reinterpret_cast<uint4*>(Rout);
    if (prec == MK_R_C64)
        hipLaunchKernelGGL(k_repack_tiled<MK_R_C64>, dim3(g), dim3(256), 0, s, in, out, rscale, nr, B, ns, ng, nch, flag);
    else if (prec == MK_R_F16S)
        hipLaunchKernelGGL(k_repack_tiled<MK_R_F16S>, dim3(g), dim3(256), 0, s, in, out, rscale, nr, B, ns, ng, nch, flag);
    else
        hipLaunchKernelGGL(k_repack_tiled<MK_R_BF16S>, dim3(g), dim3(256), 0, s, in, out, rscale, nr, B, ns, ng, nch, flag);
    return hipGetLastError();
}

hipError_t launch_rscale(const float* Rin, float* rscale, int nr, int B, int ns, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_rmax, dim3(B), dim3(256), 0, s, reinterpret_cast<const float2*>(Rin), nr, B,
                       ns, rscale, flag);
    return hipGetLastError();
}

hipError_t launch_quantize_R(int prec, const float* Rin, void* Rout, float* rscale, int nr, int B,
                             int ns, int ns_pad, int* flag, hipStream_t s) {
    hipError_t e = launch_rscale(Rin, rscale, nr, B, ns, flag, s);
    if (e != hipSuccess) return e;
    const int64_t total = (int64_t)B * nr * ns_pad;
    const int64_t blocks = (total + 255) / 256;
    const unsigned g = (unsigned)(blocks < 65536 * 4 ? blocks : 65536 * 4);
    if (prec == MK_R_F16S)
        hipLaunchKernelGGL(k_repack_q<1>, dim3(g), dim3(256), 0, s, reinterpret_cast<const float2*>(Rin),
                           reinterpret_cast<uint32_t*>(Rout), rscale, nr, B, ns, ns_pad);
    else
        hipLaunchKernelGGL(k_repack_q<2>, dim3(g), dim3(256), 0, s, reinterpret_cast<const float2*>(Rin),
                           reinterpret_cast<uint32_t*>(Rout), rscale, nr, B, ns, ns_pad);
    return hipGetLastError();
}
