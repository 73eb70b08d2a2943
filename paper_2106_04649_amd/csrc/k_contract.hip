// The space integral of Eq. (1) in the frequency domain:
//   Y[f][w][r] = sum_s R[w][r][s] * X[f][w][s]
// for every stored bin w, receiver r and focal column f (the Riemann weight
// c is applied by the per-trace kernel).  This is the paper's segmented dot
// product (Algorithm 2: pointwise multiply + segmented reduction), done in
// one pass so that R crosses HBM exactly once per pass.
//
// R is held frequency-major, [B][nr][ns_pad] complex64, so the rows of one
// frequency slice are contiguous.  A wavefront owns a run of consecutive
// rows q = w * nr + r; it keeps X[f][w][:] in registers (reloaded only when
// the run crosses into the next frequency), streams its rows with
// non-temporal 16-byte loads (two complex values per lane per load), reduces
// each row across the wave with DPP adds, and stores the run's results with
// one coalesced store per focal column.
#include "mk_internal.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;          // waves per block
constexpr int kRowsPerWave = 32;   // rows per wave run (<= 64)

// Sum over the 64 lanes; the total lands in lane 63.
__device__ __forceinline__ float wave_sum_to63(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));  // quad_perm 1,0,3,2
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));  // quad_perm 2,3,0,1
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false)); // row_half_mirror
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false)); // row_mirror
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false)); // row_bcast15
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false)); // row_bcast31
    return v;
}

template <int J, int NF>
__global__ __launch_bounds__(kWaves * 64) void k_contract_c64(
    const v4f* __restrict__ R, const v4f* __restrict__ X, float2* __restrict__ Y,
    int nr, int n4, int nload4, int64_t nrows, int64_t xstride4, int64_t ystride) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    const int64_t q0 = wave * kRowsPerWave;
    if (q0 >= nrows) return;
    const int64_t q1 = q0 + kRowsPerWave < nrows ? q0 + kRowsPerWave : nrows;

    int w = (int)(q0 / nr);
    v4f xr[NF][J];
    auto load_x = [&](int wq) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const v4f* xp = X + f * xstride4 + (int64_t)wq * n4;
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int i = lane + 64 * j;
                xr[f][j] = i < nload4 ? xp[i] : v4f{0.f, 0.f, 0.f, 0.f};
            }
        }
    };
    load_x(w);

    float2 mine[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) mine[f] = make_float2(0.f, 0.f);

    for (int64_t q = q0; q < q1; ++q) {
        const int wq = (int)(q / nr);
        if (wq != w) {
            w = wq;
            load_x(w);
        }
        const v4f* row = R + q * n4;
        v4f a[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int i = lane + 64 * j;
            a[j] = i < nload4 ? __builtin_nontemporal_load(row + i) : v4f{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const v4f r4 = a[j], x4 = xr[f][j];
                re = fmaf(r4.x, x4.x, re);
                re = fmaf(-r4.y, x4.y, re);
                re = fmaf(r4.z, x4.z, re);
                re = fmaf(-r4.w, x4.w, re);
                im = fmaf(r4.x, x4.y, im);
                im = fmaf(r4.y, x4.x, im);
                im = fmaf(r4.z, x4.w, im);
                im = fmaf(r4.w, x4.z, im);
            }
            re = wave_sum_to63(re);
            im = wave_sum_to63(im);
            const float sre = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(re), 63));
            const float sim = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(im), 63));
            if (lane == (int)(q - q0)) mine[f] = make_float2(sre, sim);
        }
    }
    if (q0 + lane < q1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) Y[f * ystride + q0 + lane] = mine[f];
    }
}

template <int J>
hipError_t launch_j(const float2* R, const float2* X, float2* Y, int nr, int B, int ns, int ns_pad,
                    int ncols, hipStream_t s) {
    const int n4 = ns_pad / 2;
    const int nload4 = (ns + 1) / 2;
    const int64_t nrows = (int64_t)B * nr;
    const int64_t xstride4 = (int64_t)B * n4;
    const int64_t ystride = (int64_t)B * nr;
    const int64_t waves = (nrows + kRowsPerWave - 1) / kRowsPerWave;
    const dim3 grid((unsigned)((waves + kWaves - 1) / kWaves)), block(kWaves * 64);
    const v4f* R4 = reinterpret_cast<const v4f*>(R);
    for (int c0 = 0; c0 < ncols;) {
        const int left = ncols - c0;
        const v4f* X4 = reinterpret_cast<const v4f*>(X) + c0 * xstride4;
        float2* Yc = Y + c0 * ystride;
        if (left >= 4) {
            hipLaunchKernelGGL((k_contract_c64<J, 4>), grid, block, 0, s, R4, X4, Yc, nr, n4, nload4,
                               nrows, xstride4, ystride);
            c0 += 4;
        } else if (left >= 2) {
            hipLaunchKernelGGL((k_contract_c64<J, 2>), grid, block, 0, s, R4, X4, Yc, nr, n4, nload4,
                               nrows, xstride4, ystride);
            c0 += 2;
        } else {
            hipLaunchKernelGGL((k_contract_c64<J, 1>), grid, block, 0, s, R4, X4, Yc, nr, n4, nload4,
                               nrows, xstride4, ystride);
            c0 += 1;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

__global__ void k_repack_c64(const float2* __restrict__ in, float2* __restrict__ out, int nr, int B,
                             int ns, int ns_pad, int* __restrict__ flag) {
    // out[w][r][s] = in[r][w][s]; zero in the padding s >= ns
    const int64_t total = (int64_t)B * nr * ns_pad;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(i % ns_pad);
        const int64_t wr = i / ns_pad;
        const int r = (int)(wr % nr);
        const int w = (int)(wr / nr);
        float2 v = make_float2(0.f, 0.f);
        if (s < ns) {
            v = in[((int64_t)r * B + w) * ns + s];
            if (!isfinite(v.x) || !isfinite(v.y)) *flag = 1;
        }
        out[i] = v;
    }
}

__global__ void k_check_finite(const float* __restrict__ x, int64_t n, int* __restrict__ flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (!isfinite(x[i])) *flag = 1;
    }
}

}  // namespace

hipError_t launch_contract_c64(const float2* R, const float2* X, float2* Y, int nr, int B, int ns,
                               int ns_pad, int ncols, hipStream_t s) {
    const int nload4 = (ns + 1) / 2;
    const int J = (nload4 + 63) / 64;
    switch (J) {
        case 1: return launch_j<1>(R, X, Y, nr, B, ns, ns_pad, ncols, s);
        case 2: return launch_j<2>(R, X, Y, nr, B, ns, ns_pad, ncols, s);
        case 3: return launch_j<3>(R, X, Y, nr, B, ns, ns_pad, ncols, s);
        case 4: return launch_j<4>(R, X, Y, nr, B, ns, ns_pad, ncols, s);
        case 5: return launch_j<5>(R, X, Y, nr, B, ns, ns_pad, ncols, s);
        case 6: return launch_j<6>(R, X, Y, nr, B, ns, ns_pad, ncols, s);
        case 7: return launch_j<7>(R, X, Y, nr, B, ns, ns_pad, ncols, s);
        case 8: return launch_j<8>(R, X, Y, nr, B, ns, ns_pad, ncols, s);
        case 9: case 10: return launch_j<10>(R, X, Y, nr, B, ns, ns_pad, ncols, s);
        case 11: case 12: return launch_j<12>(R, X, Y, nr, B, ns, ns_pad, ncols, s);
        case 13: case 14: case 15: case 16: return launch_j<16>(R, X, Y, nr, B, ns, ns_pad, ncols, s);
        default: return hipErrorInvalidValue;   // ns > 2048
    }
}

hipError_t launch_repack_c64(const float* Rin, float2* Rout, int nr, int B, int ns, int ns_pad,
                             int* flag, hipStream_t s) {
    const int64_t total = (int64_t)B * nr * ns_pad;
    const int64_t blocks = (total + 255) / 256;
    const unsigned g = (unsigned)(blocks < 65536 * 4 ? blocks : 65536 * 4);
    hipLaunchKernelGGL(k_repack_c64, dim3(g), dim3(256), 0, s, reinterpret_cast<const float2*>(Rin),
                       Rout, nr, B, ns, ns_pad, flag);
    return hipGetLastError();
}

hipError_t launch_check_finite(const float* x, int64_t n, int* flag, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    const unsigned g = (unsigned)(blocks < 8192 ? blocks : 8192);
    hipLaunchKernelGGL(k_check_finite, dim3(g), dim3(256), 0, s, x, n, flag);
    return hipGetLastError();
}
