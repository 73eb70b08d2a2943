// The space integral of Eq. (1) for a batch of focal points on the matrix
// cores: for every stored bin w, a complex GEMM
//     Y[f][w][r] = scale * sum_s R[w][r][s] * X[f][w][s].
// This is the paper's observation (Implementation and Results sections) that
// one batch of R serves many focal points; here one R tile in cache serves
// every focal column of the batch.
//
// Complex arithmetic on real MFMA: with n = 2 f + c (c = 0 real, 1 imaginary
// part of focal column f) and k = 2 s + c' (c' = 0/1 real/imaginary part of
// shot s), the product is the real GEMM D[n][r] = sum_k A[n][k] B[k][r] with
//     B[k][r]        = component c' of R[w][r][s]             (R as stored)
//     A[2f][2s..]    = ( Re X, -Im X)                          (row c = 0)
//     A[2f+1][2s..]  = ( Im X,  Re X)                          (row c = 1)
// so D[2f][r] = Re Y and D[2f+1][r] = Im Y.  A is formed in registers from
// the stored complex X (a sign flip or a swap of each pair), so X needs no
// expanded copy in memory, and the output tile is contiguous along r.
//
// Precisions: complex64 R and X on v_mfma_f32_16x16x4_f32; FP16 or BF16 R
// and X (per-frequency scale of R, per-focal scale of X) on
// v_mfma_f32_16x16x32_{f16,bf16}, accumulating in FP32.
//
// Tiling: a block of 4 waves (2 x 2) owns 32*WM focal-real rows x 32*WN
// receivers of one bin; each wave owns 16*WM x 16*WN.  Fragments are loaded
// straight from global memory with 16-byte loads.  Tiles are dealt to the
// 8 XCDs in contiguous runs (focal tiles fastest), so the focal tiles that
// reuse one R tile run on the same XCD and hit its L2.  Bins whose active
// focal count (uneven per-focal bands, focal points sorted by band end)
// ends before a tile skip it.
#include "mk_internal.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v4f a_row_f32(v4f x, int c) {
    // x = (Re x0, Im x0, Re x1, Im x1) -> row c of the real embedding
    return c == 0 ? v4f{x.x, -x.y, x.z, -x.w} : v4f{x.y, x.x, x.w, x.z};
}

__device__ __forceinline__ v4u a_row_16(v4u x, int c) {
    // each 32-bit word is (Re | Im << 16); c = 0: (Re, -Im); c = 1: (Im, Re)
    if (c == 0) return x ^ v4u{0x80000000u, 0x80000000u, 0x80000000u, 0x80000000u};
    return (x >> 16) | (x << 16);
}

template <int PREC, int WM, int WN, bool SPLIT>
__global__ __launch_bounds__(256) void k_contract_mfma(
    const void* __restrict__ Rv, const float* __restrict__ rscale, const void* __restrict__ Xv,
    const float* __restrict__ xscale, float2* __restrict__ Y, const int* __restrict__ ncols_w,
    int ncols_mul, int nr, int ns_pad, int B, int nfc, int ftiles, int rtiles, int64_t ntiles,
    int64_t per_xcd) {
    constexpr int FT = 32 * WM;      // focal-real rows per block
    constexpr int RT = 32 * WN;      // receivers per block
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int wm = wv & 1, wn = wv >> 1;
    const int64_t bid = blockIdx.x;
    const int64_t t = (bid & 7) * per_xcd + (bid >> 3);
    if (t >= ntiles) return;
    const int ft = (int)(t % ftiles);
    const int64_t t2 = t / ftiles;
    const int rt = (int)(t2 % rtiles);
    const int w = (int)(t2 / rtiles);
    const int nact = ncols_w ? min(ncols_w[w] * ncols_mul, nfc) : nfc;
    if (ft * (FT / 2) >= nact) return;

    const int i16 = lane & 15, g = lane >> 4;
    const int n0 = ft * FT + wm * 16 * WM;
    const int r0 = rt * RT + wn * 16 * WN;

    v4f acc[WM][WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    int cfl[WM];
    bool xok[WM];
    bool rok[WN];
    if constexpr (PREC == MK_R_C64) {
        const v4f* Xp[WM];
        const v4f* Rp[WN];
#pragma unroll
        for (int a = 0; a < WM; ++a) {
            const int n = n0 + 16 * a + i16;
            const int f = n >> 1;
            cfl[a] = n & 1;
            xok[a] = f < nact;
            Xp[a] = reinterpret_cast<const v4f*>(Xv) + (((int64_t)(xok[a] ? f : 0) * B + w) * ns_pad >> 1);
        }
#pragma unroll
        for (int b = 0; b < WN; ++b) {
            const int r = r0 + 16 * b + i16;
            rok[b] = r < nr;
            Rp[b] = reinterpret_cast<const v4f*>(Rv) + (((int64_t)w * nr + (rok[b] ? r : 0)) * ns_pad >> 1);
        }
        // 8 complex shots per step: lane group g covers shots s + 2g, s + 2g + 1
        const int nsteps = ns_pad >> 3;
        for (int st = 0; st < nsteps; ++st) {
            const int idx = 4 * st + g;
            v4f av[WM], bv[WN];
#pragma unroll
            for (int a = 0; a < WM; ++a) av[a] = xok[a] ? a_row_f32(Xp[a][idx], cfl[a]) : v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int b = 0; b < WN; ++b) bv[b] = rok[b] ? Rp[b][idx] : v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int a = 0; a < WM; ++a)
#pragma unroll
                    for (int b = 0; b < WN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][e], bv[b][e], acc[a][b], 0, 0, 0);
        }
    } else {
        const v4u* Xp[WM];
        const v4u* Rp[WN];
#pragma unroll
        for (int a = 0; a < WM; ++a) {
            const int n = n0 + 16 * a + i16;
            const int f = n >> 1;
            cfl[a] = n & 1;
            xok[a] = f < nact;
            Xp[a] = reinterpret_cast<const v4u*>(Xv) + (((int64_t)(xok[a] ? f : 0) * B + w) * ns_pad >> 2);
        }
#pragma unroll
        for (int b = 0; b < WN; ++b) {
            const int r = r0 + 16 * b + i16;
            rok[b] = r < nr;
            Rp[b] = reinterpret_cast<const v4u*>(Rv) + (((int64_t)w * nr + (rok[b] ? r : 0)) * ns_pad >> 2);
        }
        // 16 complex shots per step: lane group g covers shots s + 4g .. s + 4g + 3
        const int nsteps = ns_pad >> 4;
        const int64_t xlo4 = ((int64_t)nfc * B * ns_pad) >> 2;      // low plane, in 16-byte units
        for (int st = 0; st < nsteps; ++st) {
            const int idx = 4 * st + g;
            v4u av[WM], bv[WN];
#pragma unroll
            for (int a = 0; a < WM; ++a) av[a] = xok[a] ? a_row_16(Xp[a][idx], cfl[a]) : v4u{0u, 0u, 0u, 0u};
#pragma unroll
            for (int b = 0; b < WN; ++b) bv[b] = rok[b] ? Rp[b][idx] : v4u{0u, 0u, 0u, 0u};
#pragma unroll
            for (int a = 0; a < WM; ++a)
#pragma unroll
                for (int b = 0; b < WN; ++b) {
                    if constexpr (PREC == MK_R_F16S)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                            __builtin_bit_cast(h8, av[a]), __builtin_bit_cast(h8, bv[b]), acc[a][b], 0, 0, 0);
                    else
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(b8, av[a]), __builtin_bit_cast(b8, bv[b]), acc[a][b], 0, 0, 0);
                }
            if constexpr (SPLIT) {
                // the low plane of X: x = hi + lo recovers about twice the 16-bit precision
#pragma unroll
                for (int a = 0; a < WM; ++a) av[a] = xok[a] ? a_row_16(Xp[a][idx + xlo4], cfl[a]) : v4u{0u, 0u, 0u, 0u};
#pragma unroll
                for (int a = 0; a < WM; ++a)
#pragma unroll
                    for (int b = 0; b < WN; ++b) {
                        if constexpr (PREC == MK_R_F16S)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                __builtin_bit_cast(h8, av[a]), __builtin_bit_cast(h8, bv[b]), acc[a][b], 0, 0, 0);
                        else
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(b8, av[a]), __builtin_bit_cast(b8, bv[b]), acc[a][b], 0, 0, 0);
                    }
            }
        }
    }

    // D rows n0 + 16a + 4g + v (v = 0..3) are (Re, Im) of focal f0 and f0 + 1
    const float rs = PREC == MK_R_C64 ? 1.f : rscale[w];
#pragma unroll
    for (int a = 0; a < WM; ++a) {
        const int f0 = (n0 + 16 * a + 4 * g) >> 1;
#pragma unroll
        for (int b = 0; b < WN; ++b) {
            const int r = r0 + 16 * b + i16;
            if (r >= nr) continue;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int f = f0 + h;
                if (f >= nact) continue;
                const float sc = PREC == MK_R_C64 ? 1.f : rs * xscale[f];
                Y[((int64_t)f * B + w) * nr + r] = make_float2(acc[a][b][2 * h] * sc, acc[a][b][2 * h + 1] * sc);
            }
        }
    }
}

// LDS-staged variant for wide focal batches.  A block of 4 waves owns
// 16*RA focal-real rows (8*RA focal columns) x 256 receivers of one bin;
// wave v owns all of the block's rows x receivers [64 v, 64 v + 64), that is
// RA x 4 accumulator tiles.
//
// X for the block's focal columns goes through LDS in chunks of kChunk
// complex shots, double-buffered: chunk c + 1 is loaded into registers when
// chunk c starts and stored into the other buffer when it ends, one barrier
// per chunk, so its latency hides behind a whole chunk of matrix-core work.
//
// R, the streamed operand, goes straight from memory into registers, each R
// byte to exactly one wave, PD K steps ahead of its use (a shift register of
// PD fragments).  The K order is permuted so that a lane's two consecutive
// K steps read 32 contiguous bytes (lane group g holds bytes [32 g, 32 g + 32)
// of each 128-byte super-step, K step h of the pair the h-th half; a final
// lone K step keeps the plain order), and the four lane groups cover whole
// 128-byte lines; A is read from LDS in the same order, which leaves the sum
// unchanged.
constexpr int kChunk = 64;          // complex shots per staged chunk
constexpr int kLdsRcv = 256;        // receivers per block

template <int PREC, int RA, bool SPLIT, int PD>
__global__ __launch_bounds__(256, 2) void k_contract_lds(
    const void* __restrict__ Rv, const float* __restrict__ rscale, const void* __restrict__ Xv,
    const float* __restrict__ xscale, float2* __restrict__ Y, const int* __restrict__ ncols_w,
    int ncols_mul, int nr, int ns_pad, int B, int nfc, int ftiles, int rtiles, int64_t ntiles,
    int64_t per_xcd) {
    constexpr bool C64 = PREC == MK_R_C64;
    constexpr int PLANES = SPLIT ? 2 : 1;
    constexpr int NFB = 8 * RA;                   // focal columns per block
    constexpr int ROWS = NFB * PLANES;            // staged X rows
    constexpr int EB = C64 ? 8 : 4;               // bytes per complex element
    constexpr int ROWB = kChunk * EB + 16;        // padded LDS row: rows 4 banks apart
    constexpr int KS = C64 ? 8 : 16;              // complex shots per K step (64 bytes of a row)
    constexpr int SPC = kChunk / KS;              // K steps per full chunk
    constexpr int VPR = kChunk * EB / 16;         // 16-byte vectors per full chunk row
    constexpr int NV = (ROWS * VPR + 255) / 256;  // staging vectors per thread per chunk
    __shared__ __attribute__((aligned(16))) unsigned char lds[2][ROWS * ROWB];

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t bid = blockIdx.x;
    const int64_t t = (bid & 7) * per_xcd + (bid >> 3);
    if (t >= ntiles) return;
    const int ft = (int)(t % ftiles);
    const int64_t t2 = t / ftiles;
    const int rt = (int)(t2 % rtiles);
    const int w = (int)(t2 / rtiles);
    const int nact = ncols_w ? min(ncols_w[w] * ncols_mul, nfc) : nfc;
    const int fbase = ft * NFB;
    if (fbase >= nact) return;                    // uniform over the block

    const int i16 = lane & 15, g = lane >> 4;
    const int r0 = rt * kLdsRcv + wv * 64;
    const bool active = r0 < nr;                  // waves past nr only help stage X
    const int nsteps = ns_pad / KS;
    const int nch = (ns_pad + kChunk - 1) / kChunk;
    const int64_t lo_bytes = (int64_t)nfc * B * ns_pad * EB;
    const bool odd = (nsteps & 1) != 0;

    // byte offset of this lane's 16 bytes of K step st inside a row (or a chunk row)
    auto koff = [&](int st, bool lone) { return (st >> 1) * 128 + (lone ? g * 16 : g * 32 + (st & 1) * 16); };

    // ---- X staging: chunk c -> registers -> LDS buffer -------------------
    v4u xr[NV];
    auto stage_load = [&](int c) {
        const int sb = c * kChunk;
        const int vpr = (min(kChunk, ns_pad - sb) * EB) >> 4;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int v = threadIdx.x + 256 * i;
            const int row = v / VPR, col = v % VPR;
            const int f = fbase + row % NFB;
            xr[i] = v4u{0u, 0u, 0u, 0u};
            if (row < ROWS && col < vpr && f < nact)
                xr[i] = *reinterpret_cast<const v4u*>(reinterpret_cast<const unsigned char*>(Xv) +
                                                      (row / NFB) * lo_bytes +
                                                      (((int64_t)f * B + w) * ns_pad + sb) * EB + col * 16);
        }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int v = threadIdx.x + 256 * i;
            const int row = v / VPR, col = v % VPR;
            if (row < ROWS) *reinterpret_cast<v4u*>(&lds[buf][row * ROWB + col * 16]) = xr[i];
        }
    };

    // ---- R rows of this wave ----------------------------------------------
    const unsigned char* Rrow[4];
    bool rok[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int r = r0 + 16 * b + i16;
        rok[b] = active && r < nr;
        Rrow[b] = reinterpret_cast<const unsigned char*>(Rv) + ((int64_t)w * nr + (rok[b] ? r : 0)) * ns_pad * EB;
    }
    auto load_b = [&](int st, v4u (&bv)[4]) {
        const int off = koff(st, odd && st == nsteps - 1);
#pragma unroll
        for (int b = 0; b < 4; ++b)
            bv[b] = rok[b] ? *reinterpret_cast<const v4u*>(Rrow[b] + off) : v4u{0u, 0u, 0u, 0u};
    };

    v4f acc[RA][4];
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    // one K step: A from LDS (row pair 8a + i16/2 of buffer buf at byte offset off), B from bv
    auto kstep = [&](const unsigned char* buf, int off, const v4u (&bv)[4]) {
        const int c = i16 & 1;
#pragma unroll
        for (int a = 0; a < RA; ++a) {
            const int rl = 8 * a + (i16 >> 1);
            const v4u xa = *reinterpret_cast<const v4u*>(buf + rl * ROWB + off);
            if constexpr (C64) {
                const v4f av = a_row_f32(__builtin_bit_cast(v4f, xa), c);
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            av[e], __builtin_bit_cast(v4f, bv[b])[e], acc[a][b], 0, 0, 0);
            } else {
                v4u av[PLANES];
                av[0] = a_row_16(xa, c);
                if constexpr (SPLIT)
                    av[1] = a_row_16(*reinterpret_cast<const v4u*>(buf + (NFB + rl) * ROWB + off), c);
#pragma unroll
                for (int pl = 0; pl < PLANES; ++pl)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        if constexpr (PREC == MK_R_F16S)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                __builtin_bit_cast(h8, av[pl]), __builtin_bit_cast(h8, bv[b]), acc[a][b], 0, 0, 0);
                        else
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(b8, av[pl]), __builtin_bit_cast(b8, bv[b]), acc[a][b], 0, 0, 0);
                    }
            }
        }
    };

    stage_load(0);
    stage_store(0);
    v4u bq[PD][4];                                  // bq[0]: this K step; bq[p]: p steps ahead
#pragma unroll
    for (int p = 0; p < PD; ++p)
        if (p < nsteps) load_b(p, bq[p]);
    __syncthreads();
    int c = 0, j = 0;                               // chunk, K step within the chunk
    for (int st = 0; st < nsteps; ++st) {
        if (j == 0 && c + 1 < nch) stage_load(c + 1);
        if (active) kstep(lds[c & 1], koff(j, odd && st == nsteps - 1), bq[0]);
#pragma unroll
        for (int p = 0; p + 1 < PD; ++p)
#pragma unroll
            for (int b = 0; b < 4; ++b) bq[p][b] = bq[p + 1][b];
        if (st + PD < nsteps) load_b(st + PD, bq[PD - 1]);
        if (++j == SPC || st + 1 == nsteps) {       // end of chunk c
            if (c + 1 < nch) {
                stage_store((c + 1) & 1);
                __syncthreads();
            }
            ++c;
            j = 0;
        }
    }
    if (!active) return;

    // D rows 16a + 4g + v (v = 0..3) are (Re, Im) of focal fbase + 8a + 2g and the next one
    const float rs = C64 ? 1.f : rscale[w];
#pragma unroll
    for (int a = 0; a < RA; ++a) {
        const int f0 = fbase + 8 * a + 2 * g;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r = r0 + 16 * b + i16;
            if (r >= nr) continue;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int f = f0 + h;
                if (f >= nact) continue;
                const float sc = C64 ? 1.f : rs * xscale[f];
                Y[((int64_t)f * B + w) * nr + r] = make_float2(acc[a][b][2 * h] * sc, acc[a][b][2 * h + 1] * sc);
            }
        }
    }
}

template <int PREC, int RA, bool SPLIT, int PD>
hipError_t launch_l(const ContractArgs& c, hipStream_t s) {
    constexpr int NFB = 8 * RA;
    const int ftiles = (c.ncols + NFB - 1) / NFB;
    const int rtiles = (c.nr + kLdsRcv - 1) / kLdsRcv;
    const int64_t ntiles = (int64_t)ftiles * rtiles * c.B;
    const int64_t per_xcd = (ntiles + 7) / 8;
    hipLaunchKernelGGL((k_contract_lds<PREC, RA, SPLIT, PD>), dim3((unsigned)(8 * per_xcd)), dim3(256), 0, s,
                       c.R, c.rscale, c.X, c.xscale, c.Y, c.ncols_w, c.ncols_mul, c.nr, c.ns_pad, c.B, c.ncols,
                       ftiles, rtiles, ntiles, per_xcd);
    return hipGetLastError();
}

template <int PREC, int WM, int WN, bool SPLIT>
hipError_t launch_v(const ContractArgs& c, hipStream_t s) {
    constexpr int FT = 32 * WM, RT = 32 * WN;
    const int ftiles = (2 * c.ncols + FT - 1) / FT;
    const int rtiles = (c.nr + RT - 1) / RT;
    const int64_t ntiles = (int64_t)ftiles * rtiles * c.B;
    const int64_t per_xcd = (ntiles + 7) / 8;
    hipLaunchKernelGGL((k_contract_mfma<PREC, WM, WN, SPLIT>), dim3((unsigned)(8 * per_xcd)), dim3(256), 0, s,
                       c.R, c.rscale, c.X, c.xscale, c.Y, c.ncols_w, c.ncols_mul, c.nr, c.ns_pad, c.B, c.ncols,
                       ftiles, rtiles, ntiles, per_xcd);
    return hipGetLastError();
}

template <int PREC, bool SPLIT>
hipError_t launch_p(const ContractArgs& c, int variant, hipStream_t s) {
    switch (variant) {
        case 0: return launch_v<PREC, 4, 2, SPLIT>(c, s);
        case 1: return launch_v<PREC, 2, 2, SPLIT>(c, s);
        case 2: return launch_v<PREC, 2, 4, SPLIT>(c, s);
        case 3: return launch_v<PREC, 1, 4, SPLIT>(c, s);
        case 4: return launch_v<PREC, 4, 1, SPLIT>(c, s);
        case 5: return launch_l<PREC, 8, SPLIT, 2>(c, s);
        case 6: return launch_l<PREC, 4, SPLIT, 4>(c, s);
        case 7: return launch_l<PREC, 2, SPLIT, 4>(c, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int contract_mfma_variants() { return 8; }

hipError_t launch_contract_mfma(const ContractArgs& c, int variant, hipStream_t s) {
    if (c.ncols <= 0) return hipSuccess;
    if (c.ns_pad % 16 != 0) return hipErrorInvalidValue;
    switch (c.prec) {
        case MK_R_C64: return launch_p<MK_R_C64, false>(c, variant, s);
        case MK_R_F16S:
            return c.xsplit ? launch_p<MK_R_F16S, true>(c, variant, s) : launch_p<MK_R_F16S, false>(c, variant, s);
        case MK_R_BF16S:
            return c.xsplit ? launch_p<MK_R_BF16S, true>(c, variant, s) : launch_p<MK_R_BF16S, false>(c, variant, s);
        default: return hipErrorInvalidValue;
    }
}
