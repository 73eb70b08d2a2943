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
#include <type_traits>
#include <utility>

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

// Block barrier that orders LDS only: global loads in flight (prefetches)
// stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ v4u a_row_16(v4u x, int c) {
    // each 32-bit word is (Re | Im << 16); c = 0: (Re, -Im); c = 1: (Im, Re)
    if (c == 0) return x ^ v4u{0x80000000u, 0x80000000u, 0x80000000u, 0x80000000u};
    return (x >> 16) | (x << 16);
}

// Branch-free form of a_row_16 for a lane-dependent c: rotate each word by
// rot = 16 c and flip bit 31 when c = 0 (sgn = 0x80000000 (1 - c)).
__device__ __forceinline__ v4u a_row_16_sel(v4u x, uint32_t rot, uint32_t sgn) {
    v4u r;
#pragma unroll
    for (int e = 0; e < 4; ++e) r[e] = __builtin_amdgcn_alignbit(x[e], x[e], rot) ^ sgn;
    return r;
}

// Branch-free form of a_row_f32: c = 1 swaps each pair, c = 0 negates the odd entries.
__device__ __forceinline__ v4f a_row_f32_sel(v4f x, bool c) {
    const uint32_t sgn = c ? 0u : 0x80000000u;
    v4f r;
    r[0] = c ? x[1] : x[0];
    r[1] = __uint_as_float(__float_as_uint(c ? x[0] : x[1]) ^ sgn);
    r[2] = c ? x[3] : x[2];
    r[3] = __uint_as_float(__float_as_uint(c ? x[2] : x[3]) ^ sgn);
    return r;
}

template <int PREC, int WM, int WN, bool SPLIT>
__global__ __launch_bounds__(256) void k_contract_mfma(
    const void* __restrict__ Rv, const float* __restrict__ rscale, const void* __restrict__ Xv,
    const float* __restrict__ xscale, float2* __restrict__ Y, const int* __restrict__ ncols_w,
    int ncols_mul, int nr, int ns_pad, int B, int nfc, int ftiles, int rtiles, int64_t ntiles,
    int64_t per_xcd, Ext3 ext) {
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
    {
        // checked build: the rows of R and X this tile reads and the Y it writes
        constexpr int64_t EB = PREC == MK_R_C64 ? 8 : 4;
        const int64_t fmax = min(ft * (FT / 2) + FT / 2, nact) - 1;
        const int64_t rmax = min(rt * RT + RT, nr) - 1;
        MK_DCHECK(((int64_t)w * nr + rmax + 1) * ns_pad * EB <= ext.r);
        MK_DCHECK(((SPLIT ? (int64_t)nfc * B * ns_pad : 0) + (fmax * B + w + 1) * ns_pad) * EB <= ext.x);
        MK_DCHECK(((fmax * B + w) * nr + nr) * 8 <= ext.y);
    }

    const int i16 = lane & 15, g = lane >> 4;
    const int n0 = ft * FT + wm * 16 * WM;
    const int r0 = rt * RT + wn * 16 * WN;

    v4f acc[WM][WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    // output scales of this lane's focal columns, loaded before the K loop so
    // that the stores at the end wait for nothing (a load inside the
    // conditional store loop is waited for one at a time)
    float osc[WM][2];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int f = min(((n0 + 16 * a + 4 * g) >> 1) + h, nfc - 1);
            osc[a][h] = PREC == MK_R_C64 ? 1.f : rscale[w] * xscale[f];
        }

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
                const float sc = osc[a][h];
                Y[((int64_t)f * B + w) * nr + r] = make_float2(acc[a][b][2 * h] * sc, acc[a][b][2 * h + 1] * sc);
            }
        }
    }
}

// LDS-staged variant for wide focal batches.  A block of 4 (or 2, see
// lds_block_waves) waves owns 16*RA focal-real rows (8*RA focal columns) x
// 256 (128) receivers of one bin; wave v owns all of the block's rows x
// receivers [64 v, 64 v + 64), that is RA x 4 accumulator tiles.
//
// The shot axis is cut into chunks of 128 bytes of every row (32 complex
// shots in 16 bits, 16 in complex64), two matrix-core K steps each.  At the
// top of chunk c every wave issues its loads for chunk c + 2 -- its share of
// the X slice (into registers, stored into LDS at the end of chunk c + 1)
// and its own R fragments -- and only then runs chunk c's K steps; a barrier
// that orders LDS only closes the chunk, so loads stay in flight across it
// and each wave keeps two chunks of R in flight.  Three LDS buffers and three
// register sets rotate with the chunk index; the chunk loop is unrolled by
// three so that they rotate by name: no load is conditional or copied while
// in flight, which keeps the compiler's wait counts exact.  The 128-row tiles
// (one wave per SIMD, where a barrier costs most) close only every other
// chunk, with four LDS buffers.  Rows are whole chunks: ns_pad is a multiple
// of 32 shots.
//
// X is stored into LDS in both forms of the real embedding, (Re, -Im) and
// (Im, Re), so a lane reads its A fragment ready to use; the 16 lanes of a
// fragment read 16 different rows, 36 banks apart, without conflicts.
//
// Within a chunk the K order is permuted: lane group g holds bytes
// [32 g, 32 g + 32) of the 128, K step h the h-th half, so that the four lane
// groups read whole 128-byte lines of R; A is read from LDS in the same
// order, which leaves the sum unchanged.
//
// Loads are unconditional: a receiver row past nr reads row nr - 1 and a
// focal row past the active count reads the last active one.  Those values
// only reach output columns or rows that are never stored (the product's
// columns and rows are independent), so no masking or branching is needed
// and every address stays inside the buffers.
constexpr int kChunkBytes = 128;    // bytes of every row per chunk

// f(integral_constant<int, J>) for every J of the sequence, in order
template <int... J, typename F>
__device__ __forceinline__ void for_each_index(std::integer_sequence<int, J...>, F&& f) {
    (f(std::integral_constant<int, J>{}), ...);
}

// both embedding forms of a 16-byte X vector: form 0 (Re, -Im), form 1 (Im, Re)
template <bool C64>
__device__ __forceinline__ void x_forms(v4u x, v4u& f0, v4u& f1) {
    if constexpr (C64) {        // two complex64 values (Re0, Im0, Re1, Im1)
        f0 = v4u{x[0], x[1] ^ 0x80000000u, x[2], x[3] ^ 0x80000000u};
        f1 = v4u{x[1], x[0], x[3], x[2]};
    } else {                    // four (Re | Im << 16) words
        f0 = x ^ v4u{0x80000000u, 0x80000000u, 0x80000000u, 0x80000000u};
        f1 = (x >> 16) | (x << 16);
    }
}

// LDS bytes of one block of the LDS-staged tiles
constexpr int lds_tile_bytes(int RA, bool SPLIT) {
    return (RA >= 8 ? 4 : 3) * 2 * (8 * RA * (SPLIT ? 2 : 1)) * (kChunkBytes + 16);
}

// Waves per block (64 receivers each) of the LDS-staged tiles for nr
// receivers: four, or two where 128-receiver blocks pad fewer rows than
// 256-receiver ones (601 receivers: 640 against 768 rows, the last block's
// idle waves otherwise holding a SIMD each for the block's whole life), for
// the tiles that run two waves per SIMD and whose LDS still fits four of the
// smaller blocks per CU.  The 128-row tiles (one wave per SIMD) keep four
// waves: measured at 601 receivers, two-wave blocks made the 16-bit one-plane
// launch slower (445 against 436 us), while the complex64 32-column tiles
// gained 12 % (1599 against 1805 us).
constexpr bool lds_two_wave_fits(int RA, bool SPLIT) {
    return RA < 8 && 4 * lds_tile_bytes(RA, SPLIT) <= 160 * 1024;
}
int lds_block_waves(int RA, bool SPLIT, int nr) {
    const bool saves = (nr + 127) / 128 * 128 < (nr + 255) / 256 * 256;
    return lds_two_wave_fits(RA, SPLIT) && saves ? 2 : 4;
}

// One tile of the LDS-staged contraction: tile index t = (w * rtiles + rt)
// * ftiles + ft, on the block's LDS.  Every thread of the block calls it
// with the same t; it returns early (block-uniformly) when the tile's focal
// columns are past the bin's active count.
template <int PREC, int RA, bool SPLIT, bool TILED, int WV>
__device__ __forceinline__ void contract_lds_tile(
    const void* __restrict__ Rv, const float* __restrict__ rscale, const void* __restrict__ Xv,
    const float* __restrict__ xscale, float2* __restrict__ Y, const int* __restrict__ ncols_w,
    int ncols_mul, int nr, int ns_pad, int B, int nfc, int ftiles, int rtiles, int64_t t,
    unsigned char* __restrict__ lds, const Ext3& ext) {
    constexpr bool C64 = PREC == MK_R_C64;
    constexpr int PLANES = SPLIT ? 2 : 1;
    constexpr int NFB = 8 * RA;                   // focal columns per block
    constexpr int ROWS = NFB * PLANES;            // staged X rows (one form)
    constexpr int EB = C64 ? 8 : 4;               // bytes per complex element
    constexpr int CB = kChunkBytes;
    constexpr int ROWB = CB + 16;                 // padded LDS row: rows 36 banks apart
    constexpr int BUFB = 2 * ROWS * ROWB;         // one buffer: both forms of every row
    constexpr int VPR = CB / 16;                  // 16-byte vectors per chunk row
    constexpr int NVEC = ROWS * VPR;              // staging vectors per chunk
    constexpr int TB = 64 * WV;                   // threads per block
    constexpr int NV = (NVEC + TB - 1) / TB;      // per thread
    static_assert(NVEC % TB == 0 || NVEC < TB, "staging vectors fill whole sweeps");
    // RA = 8 (one wave per SIMD) puts a barrier after every other chunk, which
    // takes four LDS buffers; the others close every chunk with one (three)
    constexpr bool PAIRED = RA >= 8;

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int ft = (int)(t % ftiles);
    const int64_t t2 = t / ftiles;
    const int rt = (int)(t2 % rtiles);
    const int w = (int)(t2 / rtiles);
    const int nact = ncols_w ? min(ncols_w[w] * ncols_mul, nfc) : nfc;
    const int fbase = ft * NFB;
    if (fbase >= nact) return;                    // uniform over the block

    const int i16 = lane & 15, g = lane >> 4;
    const int r0 = rt * TB + wv * 64;             // 64 receivers per wave
    const int rowbytes = ns_pad * EB;
    const int nch = rowbytes / CB;                // rows are whole chunks (checked at launch)
    const int64_t lo_bytes = (int64_t)nfc * B * rowbytes;
    {
        // checked build: the bin's R, the tile's rows of X (both planes) and its Y
        const int64_t fmax = min(fbase + NFB, nact) - 1;
        const int64_t rbin = TILED ? (int64_t)((nr + kTileRows - 1) / kTileRows) * nch * 2048 : (int64_t)nr * rowbytes;
        MK_DCHECK((int64_t)(w + 1) * rbin <= ext.r);
        MK_DCHECK((PLANES - 1) * lo_bytes + (fmax * B + w + 1) * rowbytes <= ext.x);
        MK_DCHECK(((fmax * B + w) * nr + nr) * 8 <= ext.y);
    }

    // ---- X staging: chunk c -> registers -> LDS buffer (both forms) --------
    auto stage_load = [&](int c, v4u (&xr)[NV]) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int v = min((int)threadIdx.x + TB * i, NVEC - 1);   // extra threads repeat the last vector
            const int row = v / VPR, col = v % VPR;
            const int f = min(fbase + row % NFB, nact - 1);
            xr[i] = *reinterpret_cast<const v4u*>(reinterpret_cast<const unsigned char*>(Xv) + (row / NFB) * lo_bytes +
                                                  ((int64_t)f * B + w) * rowbytes + c * CB + col * 16);
        }
    };
    // staged row `row` (plane row / NFB, focal row % NFB) -> LDS rows 2 row (form 0), 2 row + 1 (form 1)
    auto stage_store = [&](int buf, const v4u (&xr)[NV]) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int v = min((int)threadIdx.x + TB * i, NVEC - 1);   // same value, same place
            const int row = v / VPR, col = v % VPR;
            v4u f0, f1;
            x_forms<C64>(xr[i], f0, f1);
            unsigned char* d = lds + buf * BUFB + (2 * row) * ROWB + col * 16;
            *reinterpret_cast<v4u*>(d) = f0;
            *reinterpret_cast<v4u*>(d + ROWB) = f1;
        }
    };

    // ---- R fragments of this wave: 32-bit offsets from the bin's slab ------
    // Row-major R: receiver row min(r, nr - 1), bytes c*128 + 32 g + 16 h.
    // Tiled R: 16-receiver group min(r0 / 16 + b, ng - 1), tile c, half h --
    // the same bytes, each wave load one contiguous kilobyte.
    const int lane_off = g * 32;
    const int ng = (nr + kTileRows - 1) / kTileRows;
    const unsigned char* Rw = reinterpret_cast<const unsigned char*>(Rv) +
                              (TILED ? (int64_t)w * ng * nch * 2048 : (int64_t)w * nr * rowbytes);
    uint32_t ro[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if constexpr (TILED)
            ro[b] = (uint32_t)min(r0 / kTileRows + b, ng - 1) * (uint32_t)(nch * 2048) + (uint32_t)lane * 16u;
        else
            ro[b] = (uint32_t)min(r0 + 16 * b + i16, nr - 1) * (uint32_t)rowbytes + (uint32_t)lane_off;
    }
    // both K steps of chunk c
    auto load_chunk = [&](int c, v4u (&bv)[2][4]) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t off = TILED ? (uint32_t)(c * 2048 + h * 1024) : (uint32_t)(c * CB + 16 * h);
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[h][b] = *reinterpret_cast<const v4u*>(Rw + (ro[b] + off));
        }
    };

    v4f acc[RA][4];
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    // output scales of this lane's focal columns (fbase + 8a + 2g + h),
    // loaded before the chunk loop: the stores at the end wait for nothing
    float osc[RA][2];
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int h = 0; h < 2; ++h)
            osc[a][h] = C64 ? 1.f : rscale[w] * xscale[min(fbase + 8 * a + 2 * g + h, nfc - 1)];

    // one K step: lane (i16, g) reads LDS row 16 a + i16 of each plane (focal
    // 8 a + i16 / 2 in form i16 % 2) at byte offset off; B from bv.  All A
    // fragments are read first and the products run plane by plane (or K
    // element by K element), so that updates of one accumulator are RA x 4
    // instructions apart.
    auto kstep = [&](int buf, int off, const v4u (&bv)[4]) {
        const unsigned char* base = lds + buf * BUFB + i16 * ROWB + off;
        v4u av[PLANES][RA];
#pragma unroll
        for (int pl = 0; pl < PLANES; ++pl)
#pragma unroll
            for (int a = 0; a < RA; ++a)
                av[pl][a] = *reinterpret_cast<const v4u*>(base + (2 * pl * NFB + 16 * a) * ROWB);
        if constexpr (C64) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int a = 0; a < RA; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(__builtin_bit_cast(v4f, av[0][a])[e],
                                                                         __builtin_bit_cast(v4f, bv[b])[e],
                                                                         acc[a][b], 0, 0, 0);
        } else {
#pragma unroll
            for (int pl = 0; pl < PLANES; ++pl)
#pragma unroll
                for (int a = 0; a < RA; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        if constexpr (PREC == MK_R_F16S)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                __builtin_bit_cast(h8, av[pl][a]), __builtin_bit_cast(h8, bv[b]), acc[a][b], 0, 0, 0);
                        else
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(b8, av[pl][a]), __builtin_bit_cast(b8, bv[b]), acc[a][b], 0, 0, 0);
                    }
        }
    };

    // The chunk loop, in two copies: waves with receivers (ACT) and waves
    // past nr, which only help stage X and keep the barriers.  Chunk c reads
    // LDS buffer c % 3 and R registers rb[c % 3]; at its top it loads X and R
    // of chunk c + 2 into xs[(c + 2) % 3] and rb[(c + 2) % 3] (both freed by
    // chunk c - 1); at its end it stores X of chunk c + 1 from xs[(c + 1) % 3]
    // into buffer (c + 1) % 3, which chunk c - 2 freed.
    auto run = [&](auto act_tag) {
        constexpr bool ACT = decltype(act_tag)::value;
        v4u rb[3][2][4];
        if constexpr (!PAIRED) {
            v4u xs[3][NV];
            auto chunk = [&](int c, auto q_tag) {
                constexpr int Q = decltype(q_tag)::value;      // c % 3
                constexpr int Q1 = (Q + 1) % 3, Q2 = (Q + 2) % 3;
                const int c2 = min(c + 2, nch - 1);           // past the end: reload the last chunk (unused)
                stage_load(c2, xs[Q2]);
                if constexpr (ACT) load_chunk(c2, rb[Q2]);
                __builtin_amdgcn_sched_barrier(0);            // keep the loads ahead of the K steps
                if constexpr (ACT) {
                    kstep(Q, lane_off, rb[Q][0]);
                    kstep(Q, lane_off + 16, rb[Q][1]);
                }
                stage_store(Q1, xs[Q1]);
                lds_barrier();
            };
            stage_load(0, xs[0]);
            stage_store(0, xs[0]);
            stage_load(min(1, nch - 1), xs[1]);
            if constexpr (ACT) {
                load_chunk(0, rb[0]);
                load_chunk(min(1, nch - 1), rb[1]);
            }
            lds_barrier();
            int c = 0;
            for (; c + 3 <= nch; c += 3) {
                chunk(c, std::integral_constant<int, 0>{});
                chunk(c + 1, std::integral_constant<int, 1>{});
                chunk(c + 2, std::integral_constant<int, 2>{});
            }
            if (c < nch) chunk(c, std::integral_constant<int, 0>{});
            if (c + 1 < nch) chunk(c + 1, std::integral_constant<int, 1>{});
        } else {
            // chunk j: X(j + 3) -> registers, R(j + 2) -> registers, the K
            // steps of chunk j (LDS buffer j % 4, R registers j % 3), X(j + 2)
            // -> buffer (j + 2) % 4; a barrier after odd chunks only.  Buffer
            // (j + 2) % 4 was last read in chunk j - 2, and every wave has
            // passed the barrier after chunk j - 2 or j - 1 (whichever is odd)
            // before any wave writes it; the barrier after chunk 2i + 1
            // publishes X(2i + 2) and X(2i + 3).  J = j mod 12 names every
            // ring slot at compile time.
            v4u xs[4][NV];
            auto chunk = [&](int j, auto jt) {
                constexpr int J = decltype(jt)::value;
                const int cx = min(j + 3, nch - 1), cr = min(j + 2, nch - 1);   // past the end: unused
                stage_load(cx, xs[(J + 3) % 4]);
                if constexpr (ACT) load_chunk(cr, rb[(J + 2) % 3]);
                __builtin_amdgcn_sched_barrier(0);            // keep the loads ahead of the K steps
                if constexpr (ACT) {
                    kstep(J % 4, lane_off, rb[J % 3][0]);
                    kstep(J % 4, lane_off + 16, rb[J % 3][1]);
                }
                stage_store((J + 2) % 4, xs[(J + 2) % 4]);
                if constexpr ((J & 1) != 0) lds_barrier();
            };
            stage_load(0, xs[0]);
            stage_store(0, xs[0]);
            stage_load(min(1, nch - 1), xs[1]);
            stage_store(1, xs[1]);
            stage_load(min(2, nch - 1), xs[2]);
            if constexpr (ACT) {
                load_chunk(0, rb[0]);
                load_chunk(min(1, nch - 1), rb[1]);
            }
            lds_barrier();
            int c = 0;
            for (; c + 12 <= nch; c += 12)
                for_each_index(std::make_integer_sequence<int, 12>{},
                               [&](auto jt) { chunk(c + decltype(jt)::value, jt); });
            for_each_index(std::make_integer_sequence<int, 11>{}, [&](auto jt) {
                if (c + decltype(jt)::value < nch) chunk(c + decltype(jt)::value, jt);
            });
        }
    };
    if (r0 < nr) run(std::true_type{});
    else run(std::false_type{});
    if (r0 >= nr) return;

    // D rows 16a + 4g + v (v = 0..3) are (Re, Im) of focal fbase + 8a + 2g and the next one
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
                const float sc = osc[a][h];
                Y[((int64_t)f * B + w) * nr + r] = make_float2(acc[a][b][2 * h] * sc, acc[a][b][2 * h + 1] * sc);
            }
        }
    }
}

// RA = 8 needs more than half the register file (one wave per SIMD);
// smaller tiles run two waves per SIMD.  Grid form: one block per tile,
// tiles dealt to the 8 XCDs in contiguous runs (focal tiles fastest, so the
// focal tiles that share an R tile meet in one L2).
template <int PREC, int RA, bool SPLIT, bool TILED, int WV>
__global__ __launch_bounds__(64 * WV, RA >= 8 ? 1 : 2) void k_contract_lds(
    const void* __restrict__ Rv, const float* __restrict__ rscale, const void* __restrict__ Xv,
    const float* __restrict__ xscale, float2* __restrict__ Y, const int* __restrict__ ncols_w,
    int ncols_mul, int nr, int ns_pad, int B, int nfc, int ftiles, int rtiles, int64_t ntiles,
    int64_t per_xcd, Ext3 ext) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[lds_tile_bytes(RA, SPLIT)];
    const int64_t bid = blockIdx.x;
    const int64_t t = (bid & 7) * per_xcd + (bid >> 3);
    if (t >= ntiles) return;
    contract_lds_tile<PREC, RA, SPLIT, TILED, WV>(Rv, rscale, Xv, xscale, Y, ncols_w, ncols_mul, nr, ns_pad, B,
                                                  nfc, ftiles, rtiles, t, lds, ext);
}

// Persistent form: a fixed grid (every block resident at once) walks a list
// of the active tiles -- those whose focal columns some focal point's band
// reaches at their bin -- so bins past most bands cost no block launch.  The
// list (ascending tile indices) is cut into 8 contiguous runs, one per XCD;
// the blocks of an XCD stride through its run.  Every block leaves the loop
// when its run is exhausted.
template <int PREC, int RA, bool SPLIT, bool TILED, int WV>
__global__ __launch_bounds__(64 * WV, RA >= 8 ? 1 : 2) void k_contract_lds_walk(
    const void* __restrict__ Rv, const float* __restrict__ rscale, const void* __restrict__ Xv,
    const float* __restrict__ xscale, float2* __restrict__ Y, const int* __restrict__ ncols_w,
    int ncols_mul, int nr, int ns_pad, int B, int nfc, int ftiles, int rtiles,
    const int* __restrict__ items, Ext3 ext) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[lds_tile_bytes(RA, SPLIT)];
    const int nitems = items[0];                  // the list: [count, tiles...]
    const int x = (int)(blockIdx.x & 7);
    const int per_xcd = (nitems + 7) >> 3;
    const int lo = x * per_xcd, hi = min(lo + per_xcd, nitems);
    const int step = (int)(gridDim.x >> 3);
    for (int i = lo + (int)(blockIdx.x >> 3); i < hi; i += step) {
        contract_lds_tile<PREC, RA, SPLIT, TILED, WV>(Rv, rscale, Xv, xscale, Y, ncols_w, ncols_mul, nr, ns_pad, B,
                                                      nfc, ftiles, rtiles, items[1 + i], lds, ext);
        __syncthreads();                          // the next tile restages the LDS buffers
    }
}

template <int PREC, int RA, bool SPLIT, bool TILED, int WV>
hipError_t launch_lw(const ContractArgs& c, hipStream_t s) {
    constexpr int NFB = 8 * RA;
    const int ftiles = (c.ncols + NFB - 1) / NFB;
    const int rtiles = (c.nr + 64 * WV - 1) / (64 * WV);
    if (c.items) {          // persistent form over the list of active tiles
        // walk_blocks_per_xcd counts blocks of four waves, two waves per SIMD
        const int blocks = c.walk_blocks_per_xcd * (4 / WV) / (RA >= 8 ? 2 : 1);
        const int grid = 8 * std::max(1, blocks);
        hipLaunchKernelGGL((k_contract_lds_walk<PREC, RA, SPLIT, TILED, WV>), dim3((unsigned)grid), dim3(64 * WV), 0,
                           s, c.R, c.rscale, c.X, c.xscale, c.Y, c.ncols_w, c.ncols_mul, c.nr, c.ns_pad, c.B,
                           c.ncols, ftiles, rtiles, c.items, Ext3{c.ext_r, c.ext_x, c.ext_y});
        return hipGetLastError();
    }
    const int64_t ntiles = (int64_t)ftiles * rtiles * c.nb;
    const int64_t per_xcd = (ntiles + 7) / 8;
    hipLaunchKernelGGL((k_contract_lds<PREC, RA, SPLIT, TILED, WV>), dim3((unsigned)(8 * per_xcd)), dim3(64 * WV), 0,
                       s, c.R, c.rscale, c.X, c.xscale, c.Y, c.ncols_w, c.ncols_mul, c.nr, c.ns_pad, c.B, c.ncols,
                       ftiles, rtiles, ntiles, per_xcd, Ext3{c.ext_r, c.ext_x, c.ext_y});
    return hipGetLastError();
}

template <int PREC, int RA, bool SPLIT, bool TILED>
hipError_t launch_l(const ContractArgs& c, hipStream_t s) {
    if ((c.ns_pad * (PREC == MK_R_C64 ? 8 : 4)) % kChunkBytes != 0) return hipErrorInvalidValue;
    if constexpr (lds_two_wave_fits(RA, SPLIT)) {
        if (lds_block_waves(RA, SPLIT, c.nr) == 2) return launch_lw<PREC, RA, SPLIT, TILED, 2>(c, s);
    }
    return launch_lw<PREC, RA, SPLIT, TILED, 4>(c, s);
}

template <int PREC, int WM, int WN, bool SPLIT>
hipError_t launch_v(const ContractArgs& c, hipStream_t s) {
    constexpr int FT = 32 * WM, RT = 32 * WN;
    const int ftiles = (2 * c.ncols + FT - 1) / FT;
    const int rtiles = (c.nr + RT - 1) / RT;
    const int64_t ntiles = (int64_t)ftiles * rtiles * c.nb;
    const int64_t per_xcd = (ntiles + 7) / 8;
    hipLaunchKernelGGL((k_contract_mfma<PREC, WM, WN, SPLIT>), dim3((unsigned)(8 * per_xcd)), dim3(256), 0, s,
                       c.R, c.rscale, c.X, c.xscale, c.Y, c.ncols_w, c.ncols_mul, c.nr, c.ns_pad, c.B, c.ncols,
                       ftiles, rtiles, ntiles, per_xcd, Ext3{c.ext_r, c.ext_x, c.ext_y});
    return hipGetLastError();
}

template <int PREC, bool SPLIT>
hipError_t launch_p(const ContractArgs& c, int variant, hipStream_t s) {
    if (c.tiled) {          // tiled R: only the LDS-staged kernels read it
        switch (variant) {
            case 5: return launch_l<PREC, 8, SPLIT, true>(c, s);
            case 6: return launch_l<PREC, 4, SPLIT, true>(c, s);
            case 7: return launch_l<PREC, 2, SPLIT, true>(c, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (variant) {
        case 0: return launch_v<PREC, 4, 2, SPLIT>(c, s);
        case 1: return launch_v<PREC, 2, 2, SPLIT>(c, s);
        case 2: return launch_v<PREC, 2, 4, SPLIT>(c, s);
        case 3: return launch_v<PREC, 1, 4, SPLIT>(c, s);
        case 4: return launch_v<PREC, 4, 1, SPLIT>(c, s);
        case 5: return launch_l<PREC, 8, SPLIT, false>(c, s);
        case 6: return launch_l<PREC, 4, SPLIT, false>(c, s);
        case 7: return launch_l<PREC, 2, SPLIT, false>(c, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

MK_CHECK_TAKE(check_take_mfma)


// contraction variant v (0 = GEMV, 1 + i = matrix-core shape i) reads tiled R
bool contract_variant_reads_tiled(int variant) { return variant >= 6 && variant <= 8; }

int contract_mfma_variants() { return 8; }

// focal columns per tile of LDS-staged variant v (6, 7, 8), 0 for the others
int contract_variant_focal_tile(int variant) {
    return variant == 6 ? 64 : variant == 7 ? 32 : variant == 8 ? 16 : 0;
}

int contract_lds_receivers(int variant, bool xsplit, int nr) {
    const int nfb = contract_variant_focal_tile(variant);
    return nfb == 0 ? 0 : 64 * lds_block_waves(nfb / 8, xsplit, nr);
}

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
