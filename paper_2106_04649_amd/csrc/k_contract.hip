// The space integral of Eq. (1) in the frequency domain, few focal columns:
//   Y[f][w][r] = rscale[w] * sum_s R[w][r][s] * X[f][w][s]
// for every stored bin w, receiver r and focal column f (the Riemann weight
// c is applied by the per-trace kernel).  This is the paper's segmented dot
// product (Algorithm 2: pointwise multiply + segmented reduction), done in
// one pass so that R crosses HBM exactly once per pass.
//
// R is held frequency-major, [B][nr][ns_pad], as complex64 or as FP16/BF16
// pairs with a per-frequency scale.  A wavefront owns a run of consecutive
// rows q = w * nr + r; it keeps X[f][w][:] (FP32) in registers (reloaded only
// when the run crosses into the next frequency), streams its rows with
// non-temporal 16-byte loads, reduces each row across the wave with DPP adds,
// and stores the run's results with one coalesced store per focal column.
// The run length depends on the number of focal columns (RunShape below).
#include "mk_internal.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Rows per wave run (<= 64) and waves per block, by precision and focal
// columns.  Short runs make short-lived waves, and the waves resident at any
// moment then read a dense window of R, which streams faster than a few
// thousand long runs spread over the whole matrix; but each run loads its
// bin's X (from L2), which long runs amortise.  Measured at 601 x 601 x 1025
// bins (us per launch, against 32-row runs of four waves): complex64 with one
// column, one row per wave (405 against 447); with two, 4-row runs of eight
// waves (440 against 467); 16-bit R with one column, 4-row runs (216 against
// 238).  Four columns, and 16-bit R with two, keep 32-row runs.
template <int PREC, int NF>
struct RunShape {
    static constexpr bool c64 = PREC == MK_R_C64;
    static constexpr int rows = NF == 1 ? (c64 ? 1 : 4) : (NF == 2 && c64 ? 4 : 32);
    static constexpr int waves = NF == 2 && c64 ? 8 : 4;
};

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

// Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous run
// of row chunks, so the frequencies (and their X) it touches stay in its L2.
__device__ __forceinline__ int64_t xcd_block(int64_t per_xcd) {
    const int64_t b = blockIdx.x;
    return (b & 7) * per_xcd + (b >> 3);
}

// (re, im) of one 16-bit complex pair
template <int PREC>
__device__ __forceinline__ float2 unpack16(uint32_t u) {
    if constexpr (PREC == MK_R_F16S) {
        const _Float16 lo = __builtin_bit_cast(_Float16, (uint16_t)(u & 0xFFFFu));
        const _Float16 hi = __builtin_bit_cast(_Float16, (uint16_t)(u >> 16));
        return make_float2((float)lo, (float)hi);
    } else {
        return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xFFFF0000u));
    }
}

// Complex64 R: one 16-byte load = 2 complex values.
template <int J, int NF, int RPW, int WPB>
__global__ __launch_bounds__(WPB * 64) void k_contract_c64(
    const v4f* __restrict__ R, const v4f* __restrict__ X, float2* __restrict__ Y,
    int nr, int n4, int nload4, int64_t nrows, int64_t xstride4, int64_t ystride, int64_t per_xcd, Ext3 ext) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = xcd_block(per_xcd) * WPB + (threadIdx.x >> 6);
    const int64_t q0 = wave * RPW;
    if (q0 >= nrows) return;
    const int64_t q1 = q0 + RPW < nrows ? q0 + RPW : nrows;
    // checked build: this run's rows of R, its X slabs and its Y entries
    MK_DCHECK(((q1 - 1) * n4 + nload4) * 16 <= ext.r);
    MK_DCHECK(((NF - 1) * xstride4 + (q1 - 1) / nr * n4 + nload4) * 16 <= ext.x);
    MK_DCHECK(((NF - 1) * ystride + q1) * 8 <= ext.y);

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

// FP16/BF16 R with per-frequency scale: one 16-byte load = 4 complex values.
template <int J, int NF, int PREC, int RPW, int WPB>
__global__ __launch_bounds__(WPB * 64) void k_contract_q16(
    const v4u* __restrict__ R, const v4f* __restrict__ X, const float* __restrict__ rscale,
    float2* __restrict__ Y, int nr, int n16, int nload16, int n4, int64_t nrows, int64_t xstride4,
    int64_t ystride, int64_t per_xcd, Ext3 ext) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = xcd_block(per_xcd) * WPB + (threadIdx.x >> 6);
    const int64_t q0 = wave * RPW;
    if (q0 >= nrows) return;
    const int64_t q1 = q0 + RPW < nrows ? q0 + RPW : nrows;
    // checked build: this run's rows of R, its X slabs and its Y entries
    MK_DCHECK(((q1 - 1) * n16 + nload16) * 16 <= ext.r);
    MK_DCHECK(((NF - 1) * xstride4 + (q1 - 1) / nr * n4 + 2 * nload16) * 16 <= ext.x);
    MK_DCHECK(((NF - 1) * ystride + q1) * 8 <= ext.y);

    int w = (int)(q0 / nr);
    v4f xr[NF][J][2];
    auto load_x = [&](int wq) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const v4f* xp = X + f * xstride4 + (int64_t)wq * n4;
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int i = lane + 64 * j;
                xr[f][j][0] = i < nload16 ? xp[2 * i] : v4f{0.f, 0.f, 0.f, 0.f};
                xr[f][j][1] = i < nload16 ? xp[2 * i + 1] : v4f{0.f, 0.f, 0.f, 0.f};
            }
        }
    };
    load_x(w);
    float sc = rscale[w];

    float2 mine[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) mine[f] = make_float2(0.f, 0.f);

    for (int64_t q = q0; q < q1; ++q) {
        const int wq = (int)(q / nr);
        if (wq != w) {
            w = wq;
            load_x(w);
            sc = rscale[w];
        }
        const v4u* row = R + q * n16;
        v4u a[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int i = lane + 64 * j;
            a[j] = i < nload16 ? __builtin_nontemporal_load(row + i) : v4u{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int j = 0; j < J; ++j) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float2 r0 = unpack16<PREC>(a[j][2 * h]);
                    const float2 r1 = unpack16<PREC>(a[j][2 * h + 1]);
                    const v4f x4 = xr[f][j][h];
                    re = fmaf(r0.x, x4.x, re);
                    re = fmaf(-r0.y, x4.y, re);
                    re = fmaf(r1.x, x4.z, re);
                    re = fmaf(-r1.y, x4.w, re);
                    im = fmaf(r0.x, x4.y, im);
                    im = fmaf(r0.y, x4.x, im);
                    im = fmaf(r1.x, x4.w, im);
                    im = fmaf(r1.y, x4.z, im);
                }
            }
            re = wave_sum_to63(re);
            im = wave_sum_to63(im);
            const float sre = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(re), 63));
            const float sim = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(im), 63));
            if (lane == (int)(q - q0)) mine[f] = make_float2(sre * sc, sim * sc);
        }
    }
    if (q0 + lane < q1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) Y[f * ystride + q0 + lane] = mine[f];
    }
}

// grid of a launch over nrows rows in runs of rpw rows, wpb waves per block
struct RunGrid {
    dim3 grid, block;
    int64_t per_xcd;
};
RunGrid run_grid(int64_t nrows, int rpw, int wpb) {
    const int64_t waves = (nrows + rpw - 1) / rpw;
    const int64_t blocks = (waves + wpb - 1) / wpb;
    const int64_t per_xcd = (blocks + 7) / 8;
    return {dim3((unsigned)(8 * per_xcd)), dim3(wpb * 64), per_xcd};
}

template <int J, int NF>
void launch_one(const ContractArgs& c, const float2* X, float2* Yc, hipStream_t s) {
    const int64_t nrows = (int64_t)c.nb * c.nr;
    const int64_t xstride4 = (int64_t)c.B * (c.ns_pad / 2);
    const int64_t ystride = (int64_t)c.B * c.nr;
    // this column group's X and Y start past the launch's pointers
    const Ext3 ext{c.ext_r,
                   c.ext_x - (int64_t)(reinterpret_cast<const char*>(X) - static_cast<const char*>(c.X)),
                   c.ext_y - (int64_t)(reinterpret_cast<const char*>(Yc) - reinterpret_cast<const char*>(c.Y))};
    const v4f* X4 = reinterpret_cast<const v4f*>(X);
    const v4u* R16 = reinterpret_cast<const v4u*>(c.R);
    if (c.prec == MK_R_C64) {
        using S = RunShape<MK_R_C64, NF>;
        const RunGrid g = run_grid(nrows, S::rows, S::waves);
        hipLaunchKernelGGL((k_contract_c64<J, NF, S::rows, S::waves>), g.grid, g.block, 0, s,
                           reinterpret_cast<const v4f*>(c.R), X4, Yc, c.nr, c.ns_pad / 2, (c.ns + 1) / 2, nrows,
                           xstride4, ystride, g.per_xcd, ext);
    } else if (c.prec == MK_R_F16S) {
        using S = RunShape<MK_R_F16S, NF>;
        const RunGrid g = run_grid(nrows, S::rows, S::waves);
        hipLaunchKernelGGL((k_contract_q16<J, NF, MK_R_F16S, S::rows, S::waves>), g.grid, g.block, 0, s, R16, X4,
                           c.rscale, Yc, c.nr, c.ns_pad / 4, (c.ns + 3) / 4, c.ns_pad / 2, nrows, xstride4,
                           ystride, g.per_xcd, ext);
    } else {
        using S = RunShape<MK_R_BF16S, NF>;
        const RunGrid g = run_grid(nrows, S::rows, S::waves);
        hipLaunchKernelGGL((k_contract_q16<J, NF, MK_R_BF16S, S::rows, S::waves>), g.grid, g.block, 0, s, R16, X4,
                           c.rscale, Yc, c.nr, c.ns_pad / 4, (c.ns + 3) / 4, c.ns_pad / 2, nrows, xstride4,
                           ystride, g.per_xcd, ext);
    }
}

template <int J>
hipError_t launch_j(const ContractArgs& c, hipStream_t s) {
    const int64_t xslab = (int64_t)c.B * c.ns_pad;     // complex elements per focal slab
    const int64_t yslab = (int64_t)c.B * c.nr;
    for (int c0 = 0; c0 < c.ncols;) {
        const int left = c.ncols - c0;
        const float2* X = reinterpret_cast<const float2*>(c.X) + c0 * xslab;
        float2* Yc = c.Y + c0 * yslab;
        if (left >= 4) {
            launch_one<J, 4>(c, X, Yc, s);
            c0 += 4;
        } else if (left >= 2) {
            launch_one<J, 2>(c, X, Yc, s);
            c0 += 2;
        } else {
            launch_one<J, 1>(c, X, Yc, s);
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

MK_CHECK_TAKE(check_take_contract)


hipError_t launch_contract_gemv(const ContractArgs& c, hipStream_t s) {
    // 16-byte chunks per row: 2 complex (complex64) or 4 complex (16-bit)
    const int per = c.prec == MK_R_C64 ? 2 : 4;
    const int nload = (c.ns + per - 1) / per;
    const int J = (nload + 63) / 64;
    switch (J) {
        case 1: return launch_j<1>(c, s);
        case 2: return launch_j<2>(c, s);
        case 3: return launch_j<3>(c, s);
        case 4: return launch_j<4>(c, s);
        case 5: return launch_j<5>(c, s);
        case 6: return launch_j<6>(c, s);
        case 7: return launch_j<7>(c, s);
        case 8: return launch_j<8>(c, s);
        case 9: case 10: return launch_j<10>(c, s);
        case 11: case 12: return launch_j<12>(c, s);
        case 13: case 14: case 15: case 16: return launch_j<16>(c, s);
        default: return hipErrorInvalidValue;   // ns > 2048 (complex64) / 4096 (16-bit)
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
