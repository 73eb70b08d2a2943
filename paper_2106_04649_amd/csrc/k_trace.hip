// Per-trace kernels: everything between two contractions of the Neumann
// series, fused so that a trace of nt samples never leaves LDS.
//
// One wavefront owns one trace (f, r); a 256-thread block holds four traces.
// The real transforms of length nt use one complex transform of length
// M = nt/2 on packed even/odd samples (Stockham autosort: radix-16 passes
// when a wave owns the trace, radix 4 (with one radix-2 pass when log2 M is
// odd) when the whole block does), with exact twiddles from a table of
// exp(-2 pi i k / nt) computed in double on the host.
//
// TM_ITER implements one pass of Algorithm 1 after the space integral of
// Eq. (1): inverse transform with zero-filled out-of-band bins ("padding"),
// time reversal with a sign flip, the mute theta_t, the accumulation of
// f1- (even passes) or f1+ (odd passes), the FP64 norm of N_i, and the
// forward transform of N_i that feeds the next contraction.
#include "mk_internal.h"

namespace {

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Twiddle exp(DIR 2 pi i idx / nt), idx in [0, nt), from a quarter table
// tq[r] = exp(-2 pi i r / nt), r < nt/4, held in LDS: with idx = qd nt/4 + r,
// exp(-2 pi i idx / nt) = (-i)^qd tq[r] (an exact swap and sign change).
template <int DIR, int NT>
__device__ __forceinline__ float2 twid(const float2* tq, int idx) {
    constexpr int Q = NT / 4;
    const int qd = (idx / Q) & 3, r = idx & (Q - 1);
    const float2 w = tq[r];
    const bool sw = (qd & 1) != 0;                         // odd quadrant: swap
    const float x = sw ? w.y : w.x, y = sw ? w.x : w.y;
    const float sx = (qd == 2 || qd == 3) ? -1.f : 1.f;    // (-i)^qd = (1,0) (0,-1) (-1,0) (0,1) on (x, y)
    const float sy = (qd == 1 || qd == 2) ? -1.f : 1.f;
    float2 t = make_float2(sx * x, sy * y);
    if (DIR > 0) t.y = -t.y;
    return t;
}

// LDS slot of element k of a trace's packed spectrum: one float2 of padding
// after every 16, so that the stride-16 accesses of the radix-16 passes (and
// the neighbouring traces of the cooperative phases) spread over all banks.
__device__ __forceinline__ int zi(int k) { return k + (k >> 4); }

// zi(base + q S): for S a multiple of 16 this is zi(base) + q (S + S/16), a
// constant offset from one address (the form the LDS instructions take).
template <int S>
__device__ __forceinline__ int zstep(int base, int q) {
    if constexpr (S % 16 == 0) return zi(base) + q * (S + S / 16);
    else return zi(base + q * S);
}

// Barrier among the threads that own one trace: the whole block, or one
// wave, whose lanes run in lockstep and whose LDS accesses complete in
// issue order, so that only the compiler has to be kept from reordering.
template <int TPT>
__device__ __forceinline__ void trace_sync() {
    if constexpr (TPT > 64) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// In-place complex transform of M = NT/2 points held in LDS by the TPT
// threads that own one trace (one wave, or the whole block).
// DIR = -1: forward (exp(-i...)), DIR = +1: inverse, both unnormalised.
template <int NT, int DIR, int TPT>
__device__ __forceinline__ void fft_lds(float2* z, const float2* __restrict__ tw, int lane) {
    constexpr int M = NT / 2;
    constexpr int LOG2M = ilog2c(M);
    constexpr int N4 = LOG2M / 2;
    constexpr int Q = M / 4;
    constexpr int PER4 = (Q + TPT - 1) / TPT;
#pragma unroll
    for (int st = 0; st < N4; ++st) {
        const int lns = 2 * st;          // log2 of the current sub-transform span Ns
        const int Ns = 1 << lns;
        float2 v[PER4][4];
#pragma unroll
        for (int p = 0; p < PER4; ++p) {
            const int j = lane + TPT * p;
            if (j < Q) {
#pragma unroll
                for (int q = 0; q < 4; ++q) v[p][q] = z[zi(j + q * Q)];
            }
        }
        trace_sync<TPT>();
#pragma unroll
        for (int p = 0; p < PER4; ++p) {
            const int j = lane + TPT * p;
            if (j < Q) {
                const int k = j & (Ns - 1);
                const int base = k * (NT >> (lns + 2));     // k * NT / (4 Ns)
                const float2 a0 = v[p][0];
                const float2 a1 = st == 0 ? v[p][1] : cmul(v[p][1], twid<DIR, NT>(tw, base));
                const float2 a2 = st == 0 ? v[p][2] : cmul(v[p][2], twid<DIR, NT>(tw, 2 * base));
                const float2 a3 = st == 0 ? v[p][3] : cmul(v[p][3], twid<DIR, NT>(tw, 3 * base));
                const float2 s02 = make_float2(a0.x + a2.x, a0.y + a2.y);
                const float2 d02 = make_float2(a0.x - a2.x, a0.y - a2.y);
                const float2 s13 = make_float2(a1.x + a3.x, a1.y + a3.y);
                const float2 d13 = make_float2(a1.x - a3.x, a1.y - a3.y);
                float2 y1, y3;
                if (DIR < 0) {   // y1 = d02 - i d13, y3 = d02 + i d13
                    y1 = make_float2(d02.x + d13.y, d02.y - d13.x);
                    y3 = make_float2(d02.x - d13.y, d02.y + d13.x);
                } else {         // y1 = d02 + i d13, y3 = d02 - i d13
                    y1 = make_float2(d02.x - d13.y, d02.y + d13.x);
                    y3 = make_float2(d02.x + d13.y, d02.y - d13.x);
                }
                const int idxD = ((j - k) << 2) + k;
                z[zi(idxD)] = make_float2(s02.x + s13.x, s02.y + s13.y);
                z[zi(idxD + Ns)] = y1;
                z[zi(idxD + 2 * Ns)] = make_float2(s02.x - s13.x, s02.y - s13.y);
                z[zi(idxD + 3 * Ns)] = y3;
            }
        }
        trace_sync<TPT>();
    }
    if constexpr ((LOG2M & 1) != 0) {
        constexpr int H = M / 2;
        constexpr int PER2 = (H + TPT - 1) / TPT;
        constexpr int lns = 2 * N4;
        constexpr int Ns = 1 << lns;
        float2 v[PER2][2];
#pragma unroll
        for (int p = 0; p < PER2; ++p) {
            const int j = lane + TPT * p;
            if (j < H) {
                v[p][0] = z[zi(j)];
                v[p][1] = z[zi(j + H)];
            }
        }
        trace_sync<TPT>();
#pragma unroll
        for (int p = 0; p < PER2; ++p) {
            const int j = lane + TPT * p;
            if (j < H) {
                const int k = j & (Ns - 1);
                const float2 a0 = v[p][0];
                const float2 a1 = lns == 0 ? v[p][1] : cmul(v[p][1], twid<DIR, NT>(tw, k * (NT >> (lns + 1))));
                const int idxD = ((j - k) << 1) + k;
                z[zi(idxD)] = make_float2(a0.x + a1.x, a0.y + a1.y);
                z[zi(idxD + Ns)] = make_float2(a0.x - a1.x, a0.y - a1.y);
            }
        }
        trace_sync<TPT>();
    }
}

// ---- radix-16 Stockham transform (one wave per trace) --------------------
// Passes of radix 16 and one final pass of radix 2, 4 or 8 (1024 points:
// 16 x 16 x 4), each lane holding whole butterflies in registers, so a
// transform makes three LDS round trips instead of five.  Pass with span Ns
// and radix R: butterfly j (k = j mod Ns) takes z[j + q M/R], q < R,
// multiplies input q by W_{Ns R}^{q k}, transforms, and writes output m to
// z[(j - k) R + k + m Ns].

// exp(2 pi i n / 16) for n = 0..15, and its sine
__device__ __forceinline__ float c16(int n) {
    constexpr float c[16] = {1.f, 0.92387953251128676f, 0.70710678118654752f, 0.38268343236508977f,
                             0.f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128676f,
                             -1.f, -0.92387953251128676f, -0.70710678118654752f, -0.38268343236508977f,
                             0.f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128676f};
    return c[n & 15];
}
__device__ __forceinline__ float s16(int n) { return c16(n + 12); }     // sin(x) = cos(x - pi/2)

// v * exp(DIR 2 pi i n / 16)
template <int DIR>
__device__ __forceinline__ float2 rot16(float2 v, int n) {
    const float c = c16(n), sn = DIR * s16(n);
    return make_float2(v.x * c - v.y * sn, v.x * sn + v.y * c);
}

template <int DIR>
__device__ __forceinline__ void dft2(float2& a0, float2& a1) {
    const float2 t = a0;
    a0 = make_float2(t.x + a1.x, t.y + a1.y);
    a1 = make_float2(t.x - a1.x, t.y - a1.y);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
    const float2 s02 = make_float2(a0.x + a2.x, a0.y + a2.y), d02 = make_float2(a0.x - a2.x, a0.y - a2.y);
    const float2 s13 = make_float2(a1.x + a3.x, a1.y + a3.y), d13 = make_float2(a1.x - a3.x, a1.y - a3.y);
    a0 = make_float2(s02.x + s13.x, s02.y + s13.y);
    a2 = make_float2(s02.x - s13.x, s02.y - s13.y);
    if (DIR < 0) {       // y1 = d02 - i d13, y3 = d02 + i d13
        a1 = make_float2(d02.x + d13.y, d02.y - d13.x);
        a3 = make_float2(d02.x - d13.y, d02.y + d13.x);
    } else {             // y1 = d02 + i d13, y3 = d02 - i d13
        a1 = make_float2(d02.x - d13.y, d02.y + d13.x);
        a3 = make_float2(d02.x + d13.y, d02.y - d13.x);
    }
}

// In-register DFT of R points (R = 2, 4, 8, 16).  R = R1 R2 with input
// q = R2 a + b: DFT_R1 over a, twiddle W_R^{b k1}, DFT_R2 over b; output
// X[k1 + R1 k2] ends in register R2 k1 + k2 (see out_reg).
template <int R, int DIR>
__device__ __forceinline__ void dft_reg(float2 (&v)[R]) {
    if constexpr (R == 2) {
        dft2<DIR>(v[0], v[1]);
    } else if constexpr (R == 4) {
        dft4<DIR>(v[0], v[1], v[2], v[3]);
    } else {
        constexpr int R1 = R == 16 ? 4 : 2, R2 = 4;
#pragma unroll
        for (int b = 0; b < R2; ++b) {
            if constexpr (R1 == 4) dft4<DIR>(v[b], v[4 + b], v[8 + b], v[12 + b]);
            else dft2<DIR>(v[b], v[4 + b]);
#pragma unroll
            for (int k1 = 1; k1 < R1; ++k1) v[R2 * k1 + b] = rot16<DIR>(v[R2 * k1 + b], (16 / R) * b * k1);
        }
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) dft4<DIR>(v[R2 * k1], v[R2 * k1 + 1], v[R2 * k1 + 2], v[R2 * k1 + 3]);
    }
}

// register holding output m of dft_reg
template <int R>
__device__ __forceinline__ constexpr int out_reg(int m) {
    return R == 16 ? 4 * (m & 3) + (m >> 2) : R == 8 ? 4 * (m & 1) + (m >> 1) : m;
}

// Twiddles of a pass.  Span 16 (W_{16 R}^{q k}, k < 16): read from a 16 x 16
// table of W_256^{q k} that sits in the padding slots of the block's four
// trace regions (ZS > 0: t16 is this lane's row).  Last pass of radix 4 or 8
// (W_M^{q k}): powers of W_M^k, which is entry 2 k of the first quadrant.
// Otherwise decoded from the quarter table.
template <int ZS>
__device__ __forceinline__ float2 t16_at(const float2* t16, int qq) {
    return t16[(qq >> 2) * ZS + 17 * 16 * (qq & 3)];
}

template <int NT, int DIR, int NS, int R, int ZS>
__device__ __forceinline__ void fft16_pass(float2* z, const float2* __restrict__ tw, const float2* t16, int lane) {
    constexpr int M = NT / 2;
    constexpr int NB = M / R;                // butterflies
    constexpr int PB = (NB + 63) / 64;       // per lane
    constexpr int TWS = NT / (NS * R);       // twiddle index step: W_{NS R}^{q k} = twid(q k TWS)
    float2 v[PB][R];
#pragma unroll
    for (int p = 0; p < PB; ++p) {
        const int j = lane + 64 * p;
        if (j < NB) {
#pragma unroll
            for (int q = 0; q < R; ++q) v[p][q] = z[zstep<NB>(j, q)];
        }
    }
    trace_sync<64>();
#pragma unroll
    for (int p = 0; p < PB; ++p) {
        const int j = lane + 64 * p;
        if (j < NB) {
            const int k = j & (NS - 1);
            if constexpr (NS == 16 && ZS > 0) {
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    float2 t = t16_at<ZS>(t16, (16 / R) * q);
                    if (DIR > 0) t.y = -t.y;
                    v[p][q] = cmul(v[p][q], t);
                }
            } else if constexpr (NS * R == M && (R == 4 || R == 8) && NS > 16) {
                float2 w[R];
                w[1] = tw[2 * k];
                if (DIR > 0) w[1].y = -w[1].y;
                w[2] = cmul(w[1], w[1]);
                w[3] = cmul(w[2], w[1]);
                if constexpr (R == 8) {
                    w[4] = cmul(w[2], w[2]);
                    w[5] = cmul(w[4], w[1]);
                    w[6] = cmul(w[4], w[2]);
                    w[7] = cmul(w[4], w[3]);
                }
#pragma unroll
                for (int q = 1; q < R; ++q) v[p][q] = cmul(v[p][q], w[q]);
            } else if constexpr (NS > 1) {
#pragma unroll
                for (int q = 1; q < R; ++q) v[p][q] = cmul(v[p][q], twid<DIR, NT>(tw, q * k * TWS));
            }
            dft_reg<R, DIR>(v[p]);
            const int base = (j - k) * R + k;
            if constexpr (NS == 1 && R == 16) {      // base = 16 j: zi(base + m) = zi(base) + m
                float2* zb = z + zi(base);
#pragma unroll
                for (int m = 0; m < R; ++m) zb[m] = v[p][out_reg<R>(m)];
            } else {
#pragma unroll
                for (int m = 0; m < R; ++m) z[zstep<NS>(base, m)] = v[p][out_reg<R>(m)];
            }
        }
    }
    trace_sync<64>();
}

template <int NT, int DIR, int NS, int BITS, int ZS>
__device__ __forceinline__ void fft16_passes(float2* z, const float2* __restrict__ tw, const float2* t16, int lane) {
    if constexpr (BITS >= 4) {
        fft16_pass<NT, DIR, NS, 16, ZS>(z, tw, t16, lane);
        fft16_passes<NT, DIR, NS * 16, BITS - 4, ZS>(z, tw, t16, lane);
    } else if constexpr (BITS > 0) {
        fft16_pass<NT, DIR, NS, (1 << BITS), ZS>(z, tw, t16, lane);
    }
}

// the transform of M = NT/2 points for TPT threads per trace: radix 16 when
// a wave owns the trace, radix 4 when the whole block does (more butterflies
// to spread over 256 threads)
template <int NT, int DIR, int TPT, int ZS>
__device__ __forceinline__ void fft_trace(float2* z, const float2* __restrict__ tw, const float2* t16, int lane) {
    if constexpr (TPT == 64 && NT >= 16) fft16_passes<NT, DIR, 1, ilog2c(NT / 2), ZS>(z, tw, t16, lane);
    else fft_lds<NT, DIR, TPT>(z, tw, lane);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Packed spectrum Z[k] = E[k] + i O[k] of the even/odd samples, from bins
// xk = X[k] and xm = X[M - k] of the real trace's spectrum; t = W^k.
__device__ __forceinline__ float2 pack_bins(float2 xk, float2 xm, float2 t) {
    const float2 e = make_float2(0.5f * (xk.x + xm.x), 0.5f * (xk.y - xm.y));
    const float2 d = make_float2(0.5f * (xk.x - xm.x), 0.5f * (xk.y + xm.y));
    const float2 o = make_float2(d.x * t.x + d.y * t.y, d.y * t.x - d.x * t.y);   // d * conj(t)
    return make_float2(e.x - o.y, e.y + o.x);
}

// Barrier for LDS traffic only: outstanding global loads stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---- the fused pass (one wave per trace, M = 1024 or 2048) ----------------
// The inverse transform's first pass packs its inputs on load, its last pass
// leaves the time samples in registers, and the forward transform's first
// pass starts from those registers: lane l holds element l + 64 e of the
// trace after the inverse transform, which is exactly the set of inputs its
// first forward butterflies take.

// First inverse pass (span 1, radix 16) fed from the half spectrum in LDS:
// input i is packed from bins i and M - i (slot 0 holds the real DC and
// Nyquist values).
template <int NT>
__device__ __forceinline__ void inv_first_pass(float2* z, const float2* tq, int lane) {
    constexpr int M = NT / 2, NB = M / 16, PB = NB / 64;
    static_assert(NB % 64 == 0, "whole butterflies per lane");
    float2 v[PB][16];
#pragma unroll
    for (int p = 0; p < PB; ++p) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int j = lane + 64 * p, i = j + q * NB;
            // bin M - i sits at zi(M - q NB) - (j + ceil(j / 16)); for i = 0 this
            // reads padding, replaced below
            const int jr = j + ((j + 15) >> 4);
            float2 xk = z[zstep<NB>(j, q)], xm = (z - jr)[(M - q * NB) + (M - q * NB) / 16];
            if (i == 0) {
                xm = make_float2(xk.y, 0.f);
                xk.y = 0.f;
            }
            v[p][q] = pack_bins(xk, xm, twid<-1, NT>(tq, i));
        }
    }
    trace_sync<64>();
#pragma unroll
    for (int p = 0; p < PB; ++p) {
        dft_reg<16, +1>(v[p]);
        float2* zb = z + zi(16 * (lane + 64 * p));
#pragma unroll
        for (int m = 0; m < 16; ++m) zb[m] = v[p][out_reg<16>(m)];
    }
    trace_sync<64>();
}

// Last inverse pass (radix R, span M / R) kept in registers: output m of
// butterfly p is element lane + 64 (p + PB m).
template <int NT, int R>
__device__ __forceinline__ void inv_last_pass(const float2* z, const float2* tq, int lane,
                                              float2 (&v)[NT / 2 / (64 * R)][R]) {
    constexpr int M = NT / 2, NB = M / R, PB = NB / 64;
    static_assert(R == 4 || R == 8, "last pass of 1024 or 2048 points");
#pragma unroll
    for (int p = 0; p < PB; ++p) {
#pragma unroll
        for (int q = 0; q < R; ++q) v[p][q] = z[zstep<NB>(lane + 64 * p, q)];
    }
    trace_sync<64>();
#pragma unroll
    for (int p = 0; p < PB; ++p) {
        const int k = lane + 64 * p;                 // < span: k = j
        // W_M^{-q k} as powers of conj(W_M^k) = conj(W_NT^{2k}), first quadrant
        float2 w[R];
        w[1] = tq[2 * k];
        w[1].y = -w[1].y;
        w[2] = cmul(w[1], w[1]);
        w[3] = cmul(w[2], w[1]);
        if constexpr (R == 8) {
            w[4] = cmul(w[2], w[2]);
            w[5] = cmul(w[4], w[1]);
            w[6] = cmul(w[4], w[2]);
            w[7] = cmul(w[4], w[3]);
        }
#pragma unroll
        for (int q = 1; q < R; ++q) v[p][q] = cmul(v[p][q], w[q]);
        dft_reg<R, +1>(v[p]);
    }
}

// First forward pass (span 1, radix 16) on registers: x[e] is element lane + 64 e.
template <int NT>
__device__ __forceinline__ void fwd_first_pass(float2* z, const float2 (&x)[NT / 128], int lane) {
    constexpr int M = NT / 2, NB = M / 16, PB = NB / 64;
#pragma unroll
    for (int p = 0; p < PB; ++p) {
        float2 v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = x[p + PB * q];    // input lane + 64 p + q NB
        dft_reg<16, -1>(v);
        float2* zb = z + zi(16 * (lane + 64 * p));
#pragma unroll
        for (int m = 0; m < 16; ++m) zb[m] = v[out_reg<16>(m)];
    }
}

// The time reverse of a trace, (x[(nt - 2m) mod nt], x[nt - 2m - 1]) for
// m = lane + 64 p, read as aligned pairs (one wave per trace): pair M - 1 - m
// holds x[nt - 2m - 1] and the even sample of element m + 1, which moves one
// lane up (lane 63 of p feeds lane 0 of p + 1, and of p = 0 from the last p).
template <int NT>
__device__ __forceinline__ void load_reversed(const float* __restrict__ x, int lane, float2 (&out)[NT / 128]) {
    constexpr int M = NT / 2, PM = M / 64;
    const float2* x2 = reinterpret_cast<const float2*>(x);
    float2 v[PM];
#pragma unroll
    for (int p = 0; p < PM; ++p) v[p] = x2[M - 1 - (lane + 64 * p)];
#pragma unroll
    for (int p = 0; p < PM; ++p) {
        const float xa = __shfl(v[p].x, (lane + 63) & 63, 64);
        const float xb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[(p + PM - 1) % PM].x), 63));
        out[p] = make_float2(lane == 0 ? xb : xa, v[p].y);
    }
}

// TPT threads own one trace: 64 (one wave, four traces per block) when the
// launch has many traces, 256 (the whole block) when it has few, so that a
// one-focal pass still spreads over every CU.  The traces of a block are
// consecutive receivers of one output column, and the block moves their
// spectra between HBM and LDS together: neighbouring lanes take neighbouring
// receivers of one bin, so each bin of Y is read and each bin of X written
// as one contiguous run of TPB elements.  Every global load a phase needs is
// issued before the first of them is used.
template <int NT, int MODE, int TPT>
__global__ __launch_bounds__(256, (TPT == 64 && NT <= 2048) ? 4 : 1) void k_trace(TraceArgs a) {
    constexpr int M = NT / 2;
    constexpr int TPB = 256 / TPT;          // traces per block
    constexpr int KSTR = 256 / TPB;         // bins per cooperative sweep
    constexpr int NY = (M + KSTR - 1) / KSTR;
    // float2 per trace region: padded (see zi), plus 8 so that the traces of
    // a block start 16 banks apart
    constexpr int ZS = M + M / 16 + 8;
    constexpr int PM = (M + TPT - 1) / TPT;
    constexpr int TQN = NT / 4, TQP = (TQN + 255) / 256;
    constexpr bool GMODE = MODE == TM_GFWD || MODE == TM_GOUT;
    constexpr bool YIN = MODE == TM_ITER || MODE == TM_GOUT || MODE == TM_RST1 || MODE == TM_RST2 || MODE == TM_POUT;
    constexpr bool FUSED = (MODE == TM_ITER || MODE == TM_RST1 || MODE == TM_RST2) && TPT == 64 &&
                           (M == 1024 || M == 2048);
    constexpr bool NEGCONJ = FUSED && MODE != TM_RST2;    // the next field is a time reverse
    // the span-16 twiddle table lives in the padding of the four trace regions
    constexpr int ZT = (TPT == 64 && M >= 1024) ? ZS : 0;
    __shared__ float2 lds[TPB * ZS];
    __shared__ float2 tq[TQN];               // quarter twiddle table (see twid)
    __shared__ double red[TPT > 64 ? 4 : 1];
    const int wv = TPT == 64 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64) : 0;   // trace slot
    const int lane = threadIdx.x % TPT;     // thread within the trace
    float2* z = lds + wv * ZS;
    // entry (q, k) of the span-16 table, n = 16 q + k, is padding slot n mod 64
    // (index 17 slot + 16) of region n / 64; a lane reads row k = lane mod 16
    const float2* t16 = lds + 17 * (lane & 15) + 16;

    // blocks are dealt to the 8 XCDs in contiguous runs, so that neighbouring
    // receivers (which share cache lines of Y and X) meet in one L2
    const int nrg = (a.nr + TPB - 1) / TPB; // receiver groups per column
    const int nblk = a.nfo * nrg;
    const int per_xcd = (nblk + 7) >> 3;
    const int blk = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
    if (blk >= nblk) return;                // uniform over the block
    const int fo = blk / nrg;               // output column
    const int r0 = (blk - fo * nrg) * TPB;  // first receiver of the block
    const bool valid = r0 + wv < a.nr;
    const int r = valid ? r0 + wv : a.nr - 1;   // a slot past nr computes on a copy, stores nothing
    // cooperative HBM <-> LDS moves: slot cs, bins ck, ck + KSTR, ...
    const int cs = threadIdx.x % TPB, ck = threadIdx.x / TPB;
    const bool cvalid = r0 + cs < a.nr;
    const int rc = cvalid ? r0 + cs : a.nr - 1;
    const int f = GMODE ? (fo >> 1) : fo;   // focal point (G columns interleave f1+ and f1-(-t))
    const int hi = a.lo + a.B - 1;
    int flo = a.lo, fhi = hi;
    if (a.fband) {
        flo = max(flo, a.fband[2 * f]);
        fhi = min(fhi, a.fband[2 * f + 1]);
    }
    const size_t tbase = ((size_t)f * a.nr + r) * NT;
    const float s = a.scale;
    {
        // checked build: every range this trace addresses ends inside its buffer
        const int64_t tend = (int64_t)(tbase + NT) * 4;           // per-trace fields, float
        if constexpr (YIN) MK_DCHECK((int64_t)(fo + 1) * a.B * a.nr * 8 <= a.ext[TE_Y]);
        if constexpr (MODE == TM_INIT) {
            MK_DCHECK(tend <= a.ext[TE_SRC] && tend <= a.ext[TE_F1P] && tend <= a.ext[TE_F1M]);
            if (a.n0) MK_DCHECK(tend <= a.ext[TE_N0]);
        } else if constexpr (MODE == TM_ITER) {
            MK_DCHECK(tend <= a.ext[a.parity == 0 ? TE_F1M : TE_F1P]);
            if (a.hist && a.rec_slot >= 0)
                MK_DCHECK((((int64_t)f * a.nr + r) * a.hist_k + a.rec_slot + 1) * a.hist_T * 4 <= a.ext[TE_HIST]);
        } else if constexpr (MODE == TM_GFWD || MODE == TM_GOUT) {
            MK_DCHECK(tend <= a.ext[TE_F1P] && tend <= a.ext[TE_F1M]);
            if constexpr (MODE == TM_GOUT) MK_DCHECK(tend <= a.ext[TE_GP] && tend <= a.ext[TE_GM]);
        } else if constexpr (MODE == TM_FWDF) {
            MK_DCHECK(tend <= a.ext[TE_F1P]);
        } else if constexpr (MODE == TM_RST1) {
            MK_DCHECK(tend <= a.ext[TE_F1M]);
        } else if constexpr (MODE == TM_RST2) {
            MK_DCHECK(tend <= a.ext[TE_N0] && tend <= a.ext[TE_F1P]);
        } else if constexpr (MODE == TM_POUT) {
            MK_DCHECK(tend <= a.ext[TE_F1P] && tend <= a.ext[TE_F1M] && tend <= a.ext[TE_GP] &&
                      tend <= a.ext[TE_GM] && tend <= a.ext[TE_AUX]);
        }
        if constexpr (MODE != TM_GOUT && MODE != TM_POUT) {       // X out: [planes][nfo][B][ns_pad]
            const bool x16 = a.xprec != XP_F32, split = a.xprec == XP_F16X2 || a.xprec == XP_BF16X2;
            MK_DCHECK(a.nr <= a.ns_pad && (int64_t)((split ? a.nfo : 0) + fo + 1) * a.B * a.ns_pad * (x16 ? 4 : 8) <=
                                              a.ext[TE_X]);
        }
    }
    // window of the mute, |t| < L (loaded first: the f1 addresses depend on it)
    [[maybe_unused]] int L = 0;
    if constexpr (MODE == TM_ITER || MODE == TM_RST1 || MODE == TM_RST2 || MODE == TM_GOUT)
        L = min(a.itd[f * a.nr + r] - a.shift, M);     // |t| < L; t = -M is never kept
    float2 tqv[TQP];
#pragma unroll
    for (int i = 0; i < TQP; ++i) tqv[i] = a.tw[min((int)threadIdx.x + 256 * i, TQN - 1)];
    [[maybe_unused]] float2 t16v;
    if constexpr (ZT > 0) t16v = a.tw[NT + threadIdx.x];

    // Y bins in [flo, fhi]; the others are zero (clamped, always valid, address)
    float2 yv[NY];
    float ynyq = 0.f;
    if constexpr (YIN) {
        const float2* Yt = a.Y + (size_t)fo * a.B * a.nr + rc;
        auto yload = [&](int k) {
            // the load is unconditional and its bits are masked: a selected
            // load would be sunk into a branch and waited for on its own
            const float2 v = Yt[(size_t)(min(max(k, a.lo), hi) - a.lo) * a.nr];
            const uint32_t msk = ((k >= flo) & (k <= fhi)) ? 0xFFFFFFFFu : 0u;
            return make_float2(__uint_as_float(__float_as_uint(v.x) & msk),
                               __uint_as_float(__float_as_uint(v.y) & msk));
        };
#pragma unroll
        for (int i = 0; i < NY; ++i) yv[i] = yload(ck + KSTR * i);
        ynyq = yload(M).x;
    }

    auto win = [&](int u) -> bool {         // sample u (signed time u or u - nt) inside the window
        return (u < L) | (u > NT - L);      // with L <= M; no short circuit: no branches
    };
    float* acc = (a.parity == 0) ? a.f1m : a.f1p;

#pragma unroll
    for (int i = 0; i < TQP; ++i) {
        if constexpr (TQN % 256 == 0) tq[threadIdx.x + 256 * i] = tqv[i];      // unconditional: the load stays early
        else if ((int)threadIdx.x + 256 * i < TQN) tq[threadIdx.x + 256 * i] = tqv[i];
    }
    if constexpr (ZT > 0) {
        const int n = threadIdx.x, q = n >> 4;
        lds[(q >> 2) * ZS + 17 * (16 * (q & 3) + (n & 15)) + 16] = t16v;
    }
    if constexpr (YIN) {
        // every stored bin is read once: slot k holds bin k, slot 0 the real
        // parts of DC and Nyquist (both real: their imaginary parts are dropped)
        float2* zc = lds + cs * ZS;
#pragma unroll
        for (int i = 0; i < NY; ++i) {
            const int k = ck + KSTR * i;
            if (k < M) {
                float2 v = yv[i];
                if (k == 0) v.y = ynyq;
                zc[zi(k)] = v;
            }
        }
    }
    lds_barrier();

    double nacc = 0.0;
    if constexpr (FUSED) {
        // ---- spectrum -> time -> mute -> spectrum, one LDS trip saved ----
        constexpr int LOG2M = ilog2c(M);
        constexpr int LOG2RL = (LOG2M % 4) == 0 ? 4 : LOG2M % 4;
        constexpr int RL = 1 << LOG2RL, PBL = M / (64 * RL), QN = M / 64;
        inv_first_pass<NT>(z, tq, lane);
        fft16_passes<NT, +1, 16, LOG2M - 4 - LOG2RL, ZT>(z, tq, t16, lane);
        float2 x[QN];                           // element lane + 64 e: (RN[2 idx], RN[2 idx + 1]) / s
        {
            float2 v[PBL][RL];
            inv_last_pass<NT, RL>(z, tq, lane, v);
#pragma unroll
            for (int p = 0; p < PBL; ++p) {
#pragma unroll
                for (int m = 0; m < RL; ++m) x[p + PBL * m] = v[p][out_reg<RL>(m)];
            }
        }
        // The window is symmetric (theta(-t) = theta(t)), so the next field
        // N = -theta RN(-t) is the time reverse of -Q with Q = theta RN: Q is
        // transformed, and the reversal becomes X = -conj(FFT Q) at the end.
#pragma unroll
        for (int e = 0; e < QN; ++e) {
            const int idx = lane + 64 * e;
            const float q0 = win(2 * idx) ? s * x[e].x : 0.f;
            const float q1 = win(2 * idx + 1) ? s * x[e].y : 0.f;
            x[e] = make_float2(q0, q1);
            if constexpr (MODE != TM_RST2) nacc += (double)q0 * q0 + (double)q1 * q1;
        }
        if constexpr (MODE == TM_ITER) {
            // Even passes add Q to f1- element by element.  Odd passes
            // subtract Q(-t) from f1+: the pair at (M - idx) mod M holds
            // samples -2 idx (element idx, x) and -(2 idx - 1) (element
            // idx - 1, y).  The pairs outside the window are neither read
            // nor written; all reads are issued before the first update.
            float2* ap = reinterpret_cast<float2*>(acc + tbase);
            const bool odd = a.parity != 0;
            auto gidx = [&](int idx) { return odd ? (M - idx) & (M - 1) : idx; };
            auto inw = [&](int idx) -> bool {
                return valid & (win(2 * idx) | win(odd ? (2 * idx - 1) & (NT - 1) : 2 * idx + 1));
            };
            const float ylast = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[QN - 1].y), 63));
            constexpr int FCH = 8;              // elements whose reads are in flight together
#pragma unroll
            for (int e0 = 0; e0 < QN; e0 += FCH) {
                float2 o[FCH];
#pragma unroll
                for (int c = 0; c < FCH; ++c) {
                    const int idx = lane + 64 * (e0 + c);
                    o[c] = ap[inw(idx) ? gidx(idx) : 0];
                }
#pragma unroll
                for (int c = 0; c < FCH; ++c) {
                    const int e = e0 + c, idx = lane + 64 * e;
                    // y of element idx - 1: lane - 1, or lane 63 of the previous e
                    const float ya = __shfl(x[e].y, (lane + 63) & 63, 64);
                    const float yb = e == 0 ? ylast
                                            : __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[e - 1].y), 63));
                    const float2 dd = odd ? make_float2(-x[e].x, -(lane == 0 ? yb : ya)) : x[e];
                    if (inw(idx)) ap[gidx(idx)] = make_float2(o[c].x + dd.x, o[c].y + dd.y);
                }
            }
            const int hT = a.hist_T >> 1;
            float* hrow = (a.hist && a.rec_slot >= 0)
                              ? a.hist + (((size_t)f * a.nr + r) * a.hist_k + a.rec_slot) * a.hist_T
                              : nullptr;
            if (hrow && valid) {                // record N_i on the window |t| < T/2
#pragma unroll
                for (int e = 0; e < QN; ++e) {
                    const int idx = lane + 64 * e;
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const int u = 2 * idx + c;
                        const int sr = u == M ? -M : (u < M ? -u : NT - u);   // signed time of -u
                        if (sr < hT && -sr <= hT) hrow[sr + hT] = -(c ? x[e].y : x[e].x);
                    }
                }
            }
        } else if constexpr (MODE == TM_RST1) {  // f1- := theta S f1+ = Q
            // Q is zero outside the window, where f1- already is: only the
            // pairs that meet the window are written
#pragma unroll
            for (int e = 0; e < QN; ++e) {
                const int idx = lane + 64 * e;
                if (valid & (win(2 * idx) | win(2 * idx + 1))) reinterpret_cast<float2*>(a.f1m + tbase)[idx] = x[e];
            }
        } else {
            // TM_RST2: N'' = -Q(-t); f1+ := N_-1 + N''; the residual rho = N_-1 + N'' - f1+
            // (old) feeds the next pass, unreversed.  Sample 2 idx of element
            // idx = l + 64 e reverses to element M - idx (x): lane 64 - l of
            // e' = QN - 1 - e, or lane 0 of (QN - e) mod QN; sample 2 idx + 1 to
            // element M - idx - 1 (y): lane 63 - l of QN - 1 - e.
            const float2* n0p = reinterpret_cast<const float2*>(a.n0 + tbase);
            float2* fpp = reinterpret_cast<float2*>(a.f1p + tbase);
            float2 xr[QN];
#pragma unroll
            for (int e = 0; e < QN; ++e) {
                const float ra = __shfl(x[QN - 1 - e].x, (64 - lane) & 63, 64);
                const float rb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[(QN - e) % QN].x), 0));
                const float ry = __shfl(x[QN - 1 - e].y, 63 - lane, 64);
                xr[e] = make_float2(lane == 0 ? rb : ra, ry);
            }
            // Outside the window N'' is zero and f1+ still holds N_-1 (no pass,
            // tail or restart writes there), so f1+ keeps its value and rho is
            // zero: only the pairs that meet the window are read and written.
            auto inw = [&](int idx) -> bool { return valid & (win(2 * idx) | win(2 * idx + 1)); };
            constexpr int FCH = 8;              // elements whose reads are in flight together
#pragma unroll
            for (int e0 = 0; e0 < QN; e0 += FCH) {
                float2 b0[FCH], fo[FCH];
#pragma unroll
                for (int c = 0; c < FCH; ++c) {
                    const int idx = lane + 64 * (e0 + c);
                    b0[c] = n0p[inw(idx) ? idx : 0];
                    fo[c] = fpp[inw(idx) ? idx : 0];
                }
#pragma unroll
                for (int c = 0; c < FCH; ++c) {
                    const int e = e0 + c, idx = lane + 64 * e;
                    const float2 nf2 = make_float2(b0[c].x - xr[e].x, b0[c].y - xr[e].y);
                    float2 rho = make_float2(nf2.x - fo[c].x, nf2.y - fo[c].y);
                    if (inw(idx)) {
                        fpp[idx] = nf2;
                    } else {
                        rho = make_float2(0.f, 0.f);
                    }
                    nacc += (double)rho.x * rho.x + (double)rho.y * rho.y;
                    x[e] = rho;
                }
            }
        }
        fwd_first_pass<NT>(z, x, lane);
        trace_sync<64>();
        fft16_passes<NT, -1, 16, LOG2M - 4, ZT>(z, tq, t16, lane);
    } else {
        // ---- spectrum -> time (TM_ITER, TM_GOUT, TM_RST1, TM_RST2) ------------
        if constexpr (YIN && TPT == 64 && M >= 1024) {
            constexpr int LOG2M = ilog2c(M);
            inv_first_pass<NT>(z, tq, lane);
            fft16_passes<NT, +1, 16, LOG2M - 4, ZT>(z, tq, t16, lane);
        } else if constexpr (YIN) {
            // packed spectrum from bins k and M - k; each thread rewrites its own pair in place
            for (int k = lane; k <= M / 2; k += TPT) {
                const float2 zk = z[zi(k)], zm = z[zi((M - k) & (M - 1))];
                if (k == 0) {
                    z[zi(0)] = pack_bins(make_float2(zk.x, 0.f), make_float2(zk.y, 0.f), make_float2(1.f, 0.f));
                } else {
                    z[zi(k)] = pack_bins(zk, zm, twid<-1, NT>(tq, k));
                    if (k != M - k) z[zi(M - k)] = pack_bins(zm, zk, twid<-1, NT>(tq, M - k));
                }
            }
            trace_sync<TPT>();
            fft_trace<NT, +1, TPT, ZT>(z, tq, t16, lane);
            // z[m] = (RN[2m], RN[2m+1]) / s
        }

        float2 out[PM];
        if constexpr (MODE == TM_ITER || MODE == TM_RST1 || MODE == TM_RST2) {
            const int hT = a.hist_T >> 1;
            float* hrow = (MODE == TM_ITER && a.hist && a.rec_slot >= 0)
                              ? a.hist + (((size_t)f * a.nr + r) * a.hist_k + a.rec_slot) * a.hist_T
                              : nullptr;
            // global operands first (clamped to the trace's first pair when unused)
            float2 g0[PM], g1[PM];
#pragma unroll
            for (int p = 0; p < PM; ++p) {
                const int m = min(lane + TPT * p, M - 1);
                if constexpr (MODE == TM_ITER) {
                    const bool w = valid && (win(2 * m) || win(2 * m + 1));
                    g0[p] = reinterpret_cast<const float2*>(acc + tbase)[w ? m : 0];
                } else if constexpr (MODE == TM_RST2) {
                    g0[p] = reinterpret_cast<const float2*>(a.n0 + tbase)[m];
                    g1[p] = reinterpret_cast<const float2*>(a.f1p + tbase)[m];
                }
            }
#pragma unroll
            for (int p = 0; p < PM; ++p) {
                const int m = lane + TPT * p;
                if (m < M) {
                    const int t0 = 2 * m, t1 = 2 * m + 1;
                    const int s0 = t0 < M ? t0 : t0 - NT;
                    const int s1 = t1 < M ? t1 : t1 - NT;
                    const bool k0 = win(t0), k1 = win(t1);
                    // N[t] = -RN[(nt - t) mod nt] inside the window
                    const float n0 = k0 ? -s * z[zi((M - m) & (M - 1))].x : 0.f;
                    const float n1 = k1 ? -s * z[zi(M - 1 - m)].y : 0.f;
                    if constexpr (MODE == TM_ITER) {
                        nacc += (double)n0 * n0 + (double)n1 * n1;
                        if (valid && (k0 || k1)) {
                            float2 o = g0[p];
                            if (a.parity == 0) {             // f1- -= N(-t)  ==  f1- += theta RN
                                const float2 zm = z[zi(m)];
                                if (k0) o.x += s * zm.x;
                                if (k1) o.y += s * zm.y;
                            } else {                          // f1+ += N
                                o.x += n0;
                                o.y += n1;
                            }
                            reinterpret_cast<float2*>(acc + tbase)[m] = o;
                        }
                        if (hrow && valid) {                  // record N_i on the window |t| < T/2
                            if (s0 < hT && -s0 <= hT) hrow[s0 + hT] = n0;
                            if (s1 < hT && -s1 <= hT) hrow[s1 + hT] = n1;
                        }
                        out[p] = make_float2(n0, n1);
                    } else if constexpr (MODE == TM_RST1) {
                        // f1- := theta S f1+ (overwrite); the field fed on is N' = -(theta RN)(-t)
                        nacc += (double)n0 * n0 + (double)n1 * n1;
                        if (valid) {
                            const float2 zm = z[zi(m)];
                            reinterpret_cast<float2*>(a.f1m + tbase)[m] =
                                make_float2(k0 ? s * zm.x : 0.f, k1 ? s * zm.y : 0.f);
                        }
                        out[p] = make_float2(n0, n1);
                    } else {
                        // N'' = A^2 f1+; rho = N_-1 + N'' - f1+; f1+ := N_-1 + N''
                        const float2 b0 = g0[p], fp = g1[p];
                        const float2 nf2 = make_float2(b0.x + n0, b0.y + n1);
                        const float2 rho = make_float2(nf2.x - fp.x, nf2.y - fp.y);
                        nacc += (double)rho.x * rho.x + (double)rho.y * rho.y;
                        if (valid) reinterpret_cast<float2*>(a.f1p + tbase)[m] = nf2;
                        out[p] = rho;
                    }
                }
            }
            trace_sync<TPT>();
#pragma unroll
            for (int p = 0; p < PM; ++p) {
                const int m = lane + TPT * p;
                if (m < M) z[zi(m)] = out[p];
            }
        } else if constexpr (MODE == TM_INIT) {
            const float* g = a.src + tbase;                // N_-1[t] = Gd[(nt - t) mod nt]
            if constexpr (TPT == 64 && M >= 64) {
                load_reversed<NT>(g, lane, out);
            } else {
#pragma unroll
                for (int p = 0; p < PM; ++p) {
                    const int m = min(lane + TPT * p, M - 1);
                    out[p] = make_float2(g[(NT - 2 * m) & (NT - 1)], g[NT - 2 * m - 1]);
                }
            }
#pragma unroll
            for (int p = 0; p < PM; ++p) {
                const int m = lane + TPT * p;
                if (m < M) {
                    const float n0 = out[p].x, n1 = out[p].y;
                    nacc += (double)n0 * n0 + (double)n1 * n1;
                    if (valid) {
                        reinterpret_cast<float2*>(a.f1p + tbase)[m] = make_float2(n0, n1);
                        reinterpret_cast<float2*>(a.f1m + tbase)[m] = make_float2(0.f, 0.f);
                        if (a.n0) reinterpret_cast<float2*>(a.n0 + tbase)[m] = make_float2(n0, n1);
                    }
                    z[zi(m)] = make_float2(n0, n1);
                }
            }
        } else if constexpr (MODE == TM_FWDF) {
#pragma unroll
            for (int p = 0; p < PM; ++p)
                out[p] = reinterpret_cast<const float2*>(a.f1p + tbase)[min(lane + TPT * p, M - 1)];
#pragma unroll
            for (int p = 0; p < PM; ++p) {
                const int m = lane + TPT * p;
                if (m < M) z[zi(m)] = out[p];
            }
        } else if constexpr (MODE == TM_GFWD) {
            const bool minus = (fo & 1) != 0;
            if constexpr (TPT == 64 && M >= 64) {
                if (!minus) {
#pragma unroll
                    for (int p = 0; p < PM; ++p) out[p] = reinterpret_cast<const float2*>(a.f1p + tbase)[lane + 64 * p];
                } else {
                    load_reversed<NT>(a.f1m + tbase, lane, out);     // f1-(-t)
                }
            } else {
#pragma unroll
                for (int p = 0; p < PM; ++p) {
                    const int m = min(lane + TPT * p, M - 1);
                    if (!minus) {
                        out[p] = reinterpret_cast<const float2*>(a.f1p + tbase)[m];
                    } else {                             // f1-(-t)
                        const float* q = a.f1m + tbase;
                        out[p] = make_float2(q[(NT - 2 * m) & (NT - 1)], q[NT - 2 * m - 1]);
                    }
                }
            }
#pragma unroll
            for (int p = 0; p < PM; ++p) {
                const int m = lane + TPT * p;
                if (m < M) z[zi(m)] = out[p];
            }
        } else if constexpr (MODE == TM_GOUT) {
            const bool plus = (fo & 1) != 0;
            if constexpr (TPT == 64 && M >= 64) {
                if (!plus) {
                    // f1- is zero outside the window: only the pairs that meet
                    // it are read (the others load the trace's first pair and
                    // mask the bits)
#pragma unroll
                    for (int p = 0; p < PM; ++p) {
                        const int m = lane + 64 * p;
                        const bool w = win(2 * m) | win(2 * m + 1);
                        const float2 v = reinterpret_cast<const float2*>(a.f1m + tbase)[w ? m : 0];
                        const uint32_t msk = w ? 0xFFFFFFFFu : 0u;
                        out[p] = make_float2(__uint_as_float(__float_as_uint(v.x) & msk),
                                             __uint_as_float(__float_as_uint(v.y) & msk));
                    }
                } else {
                    load_reversed<NT>(a.f1p + tbase, lane, out);     // f1+(-t)
                }
            } else {
#pragma unroll
                for (int p = 0; p < PM; ++p) {
                    const int m = min(lane + TPT * p, M - 1);
                    if (!plus) {
                        out[p] = reinterpret_cast<const float2*>(a.f1m + tbase)[m];
                    } else {
                        const float* q = a.f1p + tbase;
                        out[p] = make_float2(q[(NT - 2 * m) & (NT - 1)], q[NT - 2 * m - 1]);
                    }
                }
            }
#pragma unroll
            for (int p = 0; p < PM; ++p) {
                const int m = lane + TPT * p;
                if (m < M && valid) {
                    const float2 zm = z[zi(m)];
                    const double rn0 = (double)(s * zm.x), rn1 = (double)(s * zm.y);
                    if (!plus) {                          // G- = S[f1+] - f1-
                        reinterpret_cast<float2*>(a.gm + tbase)[m] =
                            make_float2((float)(rn0 - (double)out[p].x), (float)(rn1 - (double)out[p].y));
                    } else {                              // G+ = f1+(-t) - S[f1-(-t)]
                        reinterpret_cast<float2*>(a.gp + tbase)[m] =
                            make_float2((float)((double)out[p].x - rn0), (float)((double)out[p].y - rn1));
                    }
                }
            }
            return;
        } else if constexpr (MODE == TM_POUT) {
            // p- = sum of the syntheses RN_0 .. RN_{n-1} = S[f2+ - N_last] with
            // f2+ = f1+ - f1-(-t): S f1+ = G- + f1-, S f1-(-t) = f1+(-t) - G+,
            // and this launch's Y is S N_last.  Combined in FP64.
            float2 fpr[PM];
            if constexpr (TPT == 64 && M >= 64) {
                load_reversed<NT>(a.f1p + tbase, lane, fpr);      // f1+(-t)
            } else {
#pragma unroll
                for (int p = 0; p < PM; ++p) {
                    const int m = min(lane + TPT * p, M - 1);
                    const float* q = a.f1p + tbase;
                    fpr[p] = make_float2(q[(NT - 2 * m) & (NT - 1)], q[NT - 2 * m - 1]);
                }
            }
#pragma unroll
            for (int p = 0; p < PM; ++p) {
                const int m = lane + TPT * p;
                if (m < M && valid) {
                    const float2 zm = z[zi(m)];
                    const float2 gm2 = reinterpret_cast<const float2*>(a.gm + tbase)[m];
                    const float2 gp2 = reinterpret_cast<const float2*>(a.gp + tbase)[m];
                    const float2 fm2 = reinterpret_cast<const float2*>(a.f1m + tbase)[m];
                    const double v0 = ((double)gm2.x + fm2.x) + ((double)gp2.x - fpr[p].x) - (double)(s * zm.x);
                    const double v1 = ((double)gm2.y + fm2.y) + ((double)gp2.y - fpr[p].y) - (double)(s * zm.y);
                    reinterpret_cast<float2*>(a.aux + tbase)[m] = make_float2((float)v0, (float)v1);
                }
            }
            return;
        }

        // ---- time -> spectrum (TM_INIT, TM_ITER, TM_GFWD, TM_FWDF, restart) ----
        trace_sync<TPT>();
        fft_trace<NT, -1, TPT, ZT>(z, tq, t16, lane);
    }
    lds_barrier();                            // every trace of the block transformed
    // rfft bins kb + KSTR i of slot cs, unrolled: the LDS slots of bins k and
    // M - k step by a constant, W^k = W^kb W^{KSTR i} (the second factor at a
    // constant index), and the halves of E and D are folded into the scale
    constexpr int NXI = M / KSTR + 1;         // bins up to M
    constexpr int ZK = KSTR + KSTR / 16;      // slot step of KSTR bins
    const float2* zc = lds + cs * ZS;
    const int kend = a.skip_outband ? fhi : hi;
    const int kb = a.lo + ck;
    const int zkb = zi(kb), zmb = zi(M - kb);
    const float2 wb = twid<-1, NT>(tq, kb & (NT - 1));
    const size_t xoff = (size_t)fo * a.B * a.ns_pad + rc + (size_t)ck * a.ns_pad;
    const size_t xstep = (size_t)KSTR * a.ns_pad;
    auto bin2 = [&](int i) -> float2 {        // 2 X[k] (0 outside the focal band)
        const int k = kb + KSTR * i;
        const bool past = k >= M;             // k = M reads slot 0; beyond M nothing is stored
        const float2 zk = zc[past ? 0 : zkb + ZK * i];
        const float2 zm = zc[(past || (i == 0 && k == 0)) ? 0 : zmb - ZK * i];
        const float2 w = cmul(wb, twid<-1, NT>(tq, (KSTR * i) & (NT - 1)));
        const float2 e2 = make_float2(zk.x + zm.x, zk.y - zm.y);
        const float2 d2 = make_float2(zk.x - zm.x, zk.y + zm.y);
        const float2 wd = cmul(w, d2);
        const bool in = (k >= flo) & (k <= fhi);
        return make_float2(in ? e2.x + wd.y : 0.f, in ? e2.y - wd.x : 0.f);
    };
    const float cj = NEGCONJ ? -1.f : 1.f;    // fused pass: X = -conj(FFT Q)
    if (a.xprec == XP_F32) {
        float2* Xt = reinterpret_cast<float2*>(a.X) + xoff;
#pragma unroll
        for (int i = 0; i < NXI; ++i) {
            float2 v = bin2(i);
            v.x *= 0.5f * cj;
            v.y *= 0.5f;
            if (cvalid & (kb + KSTR * i <= kend)) Xt[i * xstep] = v;
        }
    } else {
        // 16-bit X scaled per focal point by the RMS trace norm of the previous field
        const double nrm = a.xs_in ? a.xs_in[f] : 0.0;
        float xs = (float)(nrm / sqrt((double)a.nr));
        if (!(xs >= 0x1p-100f) || !isfinite(xs)) xs = 1.f;
        const float inv = 0.5f / xs;
        uint32_t* Xt = reinterpret_cast<uint32_t*>(a.X) + xoff;
        const bool bf = a.xprec == XP_BF16 || a.xprec == XP_BF16X2;
        const bool split = a.xprec == XP_F16X2 || a.xprec == XP_BF16X2;
        const size_t lo_off = (size_t)a.nfo * a.B * a.ns_pad;       // second plane
#pragma unroll
        for (int i = 0; i < NXI; ++i) {
            float2 v = bin2(i);
            v.x *= cj * inv;
            v.y *= inv;
            uint32_t u, ul = 0;
            if (!bf) {
                const _Float16 hx = (_Float16)v.x, hy = (_Float16)v.y;
                u = (uint32_t)__builtin_bit_cast(uint16_t, hx) | ((uint32_t)__builtin_bit_cast(uint16_t, hy) << 16);
                if (split) {
                    const _Float16 lx = (_Float16)(v.x - (float)hx), ly = (_Float16)(v.y - (float)hy);
                    ul = (uint32_t)__builtin_bit_cast(uint16_t, lx) |
                         ((uint32_t)__builtin_bit_cast(uint16_t, ly) << 16);
                }
            } else {
                uint32_t ux = __float_as_uint(v.x), uy = __float_as_uint(v.y);
                ux = (ux + 0x7FFFu + ((ux >> 16) & 1u)) & 0xFFFF0000u;
                uy = (uy + 0x7FFFu + ((uy >> 16) & 1u)) & 0xFFFF0000u;
                u = (ux >> 16) | uy;
                if (split) {
                    uint32_t lx = __float_as_uint(v.x - __uint_as_float(ux));
                    uint32_t ly = __float_as_uint(v.y - __uint_as_float(uy));
                    lx += 0x7FFFu + ((lx >> 16) & 1u);
                    ly += 0x7FFFu + ((ly >> 16) & 1u);
                    ul = (lx >> 16) | (ly & 0xFFFF0000u);
                }
            }
            if (cvalid & (kb + KSTR * i <= kend)) {
                Xt[i * xstep] = u;
                if (split) Xt[lo_off + i * xstep] = ul;
            }
        }
        if (r0 == 0 && threadIdx.x == 0) a.xs_out[fo] = xs;
    }
    if constexpr (MODE == TM_ITER || MODE == TM_RST1 || MODE == TM_RST2) {
        nacc = wave_sum_d(nacc);
        if constexpr (TPT > 64) {            // combine the block's waves in a fixed order
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nacc;
            __syncthreads();
            nacc = red[0] + red[1] + red[2] + red[3];
        }
        if (valid && lane == 0) a.npart[(size_t)fo * a.nr + r] = nacc;
    }
}

// Sum of squares of each trace (FP64), one wave per trace: the norm of G_d.
// FP64 sum of squares of every trace: npart[j] for trace j of x0 (j < n0)
// and for trace j - n0 of x1 (j >= n0), so two fields reduce in one launch.
// One wave per trace, 16-byte loads, eight of a lane's loads in flight
// together (addresses clamped, out-of-range values dropped after the load).
// WIN 1: only the samples inside the trace's mute window |t| < L,
// L = min(itd - shift, nt / 2) (sample k is inside when k < L or k > nt - L),
// read alone: the f1 samples a pass can change.  WIN 2: the whole trace into
// npart and the samples outside the window into npart2.  Trace i of x1 is
// trace i - n0 of the window table.
template <int WIN>
__global__ __launch_bounds__(256) void k_sumsq(const float* __restrict__ x0, const float* __restrict__ x1, int n0,
                                               int ntr, int nt, const int32_t* __restrict__ itd, int shift,
                                               double* __restrict__ npart, double* __restrict__ npart2) {
    const int lane = threadIdx.x & 63;
    const int trace = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (trace >= ntr) return;
    const float4* p = reinterpret_cast<const float4*>(trace < n0 ? x0 + (size_t)trace * nt
                                                                 : x1 + (size_t)(trace - n0) * nt);
    const int n4 = nt >> 2;
    const int L = min(itd[trace < n0 ? trace : trace - n0] - shift, nt >> 1);
    auto inwin = [&](int k) { return k < L || k > nt - L; };
    // WIN 1 visits the float4 runs [0, a1) and [b2, n4), which hold the window
    int a1 = n4, b2 = n4, cnt = n4;
    if constexpr (WIN == 1) {
        a1 = (max(L, 0) + 3) >> 2;
        b2 = min((nt - max(L, 0) + 1) >> 2, n4);
        cnt = b2 <= a1 ? n4 : a1 + (n4 - b2);
        if (L <= 0) cnt = 0;
    }
    double acc = 0.0, acco = 0.0;
    for (int i0 = 0; i0 < cnt; i0 += 64 * 8) {
        float4 v[8];
        int q[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int u = min(i0 + lane + 64 * j, cnt - 1);
            q[j] = (WIN == 1 && b2 > a1 && u >= a1) ? b2 + (u - a1) : u;
            v[j] = p[q[j]];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const bool live = i0 + lane + 64 * j < cnt;
            const float e[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double sq = (double)e[c] * e[c];
                if constexpr (WIN == 1) {
                    acc += (live && inwin(4 * q[j] + c)) ? sq : 0.0;
                } else {
                    acc += live ? sq : 0.0;
                    acco += (live && !inwin(4 * q[j] + c)) ? sq : 0.0;
                }
            }
        }
    }
    acc = wave_sum_d(acc);
    if constexpr (WIN == 2) acco = wave_sum_d(acco);
    if (lane == 0) {
        npart[trace] = acc;
        if constexpr (WIN == 2) npart2[trace] = acco;
    }
}

// f2+ = N_-1 + sum of every pass's N_i (Algorithm 1, second loop): the odd
// passes are in f1+ and f1- holds minus the time reverse of the even ones,
// so f2+(t) = f1+(t) - f1-(-t).  One thread per sample.
__global__ __launch_bounds__(256) void k_f2p(const float* __restrict__ f1p, const float* __restrict__ f1m,
                                             int64_t ntr, int nt, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= ntr * nt) return;
    const int64_t tr = i / nt;
    const int k = (int)(i - tr * nt);
    out[i] = f1p[i] - f1m[tr * nt + (k == 0 ? 0 : nt - k)];
}

// The total Green's function G = G+ + G-, one rounding per sample.
__global__ __launch_bounds__(256) void k_gsum(const float* __restrict__ gp, const float* __restrict__ gm, int64_t n,
                                              float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = gp[i] + gm[i];
}

// Double-focusing image (Theory section, imaging): the zero-time sample of
// G- convolved in time with f1+ and integrated over the receivers.  First
// stage, one wave per trace: sum_k G-[k] f1+[(-k) mod nt] in FP64 (a product
// of two FP32 values is exact in FP64).  Eight loads of each field in flight
// per lane; f1+ is read backwards, which still fills whole lines.
__global__ __launch_bounds__(256) void k_image_part(const float* __restrict__ gm, const float* __restrict__ f1p,
                                                    int ntr, int nt, double* __restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int trace = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (trace >= ntr) return;
    const float* g = gm + (size_t)trace * nt;
    const float* f = f1p + (size_t)trace * nt;
    constexpr int U = 8;
    double acc = 0.0;
    for (int k0 = 0; k0 < nt; k0 += 64 * U) {
        float gv[U], fv[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int k = min(k0 + lane + 64 * j, nt - 1);
            gv[j] = g[k];
            fv[j] = f[k == 0 ? 0 : nt - k];
        }
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (k0 + lane + 64 * j < nt) acc = fma((double)gv[j], (double)fv[j], acc);
    }
    acc = wave_sum_d(acc);
    if (lane == 0) part[trace] = acc;
}

// Second stage: out[f] = scale * sum_r part[f][r], one block per focal point,
// in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_image_reduce(const double* __restrict__ part, int nr, double scale,
                                                      double* __restrict__ out) {
    __shared__ double sh[256];
    const double* p = part + (size_t)blockIdx.x * nr;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nr; i += 256) acc += p[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = scale * sh[0];
}

// dst[j] = src[perm[j]] for blocks of `per` elements of type T; block row
// blockIdx.y is block j.
template <typename T>
__global__ __launch_bounds__(256) void k_gather(const T* __restrict__ src, T* __restrict__ dst,
                                                const int* __restrict__ perm, int64_t per) {
    const int j = blockIdx.y;
    const T* s = src + (int64_t)perm[j] * per;
    T* d = dst + (int64_t)j * per;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < per; i += (int64_t)gridDim.x * 256) d[i] = s[i];
}

__global__ __launch_bounds__(256) void k_norm_reduce(const double* __restrict__ npart, int nr,
                                                     double* __restrict__ out, double* __restrict__ out2) {
    __shared__ double sh[256];
    const double* p = npart + (size_t)blockIdx.x * nr;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nr; i += 256) acc += p[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = sqrt(sh[0]);
        out[blockIdx.x] = v;
        if (out2) out2[blockIdx.x] = v;
    }
}

template <int NT, int TPT>
hipError_t launch_trace_tpt(int mode, const TraceArgs& a, hipStream_t s) {
    constexpr int TPB = 256 / TPT;
    const int nblk = a.nfo * ((a.nr + TPB - 1) / TPB);
    const dim3 grid(8 * ((nblk + 7) / 8)), block(256);
    switch (mode) {
        case TM_INIT: hipLaunchKernelGGL((k_trace<NT, TM_INIT, TPT>), grid, block, 0, s, a); break;
        case TM_ITER: hipLaunchKernelGGL((k_trace<NT, TM_ITER, TPT>), grid, block, 0, s, a); break;
        case TM_GFWD: hipLaunchKernelGGL((k_trace<NT, TM_GFWD, TPT>), grid, block, 0, s, a); break;
        case TM_GOUT: hipLaunchKernelGGL((k_trace<NT, TM_GOUT, TPT>), grid, block, 0, s, a); break;
        case TM_FWDF: hipLaunchKernelGGL((k_trace<NT, TM_FWDF, TPT>), grid, block, 0, s, a); break;
        case TM_RST1: hipLaunchKernelGGL((k_trace<NT, TM_RST1, TPT>), grid, block, 0, s, a); break;
        case TM_RST2: hipLaunchKernelGGL((k_trace<NT, TM_RST2, TPT>), grid, block, 0, s, a); break;
        case TM_POUT: hipLaunchKernelGGL((k_trace<NT, TM_POUT, TPT>), grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Few traces (fewer than 8 per CU): a whole block per trace; otherwise one wave.
constexpr int kWholeBlockTraces = 2048;

template <int NT>
hipError_t launch_trace_nt(int mode, const TraceArgs& a, hipStream_t s) {
    if (a.nfo * a.nr < kWholeBlockTraces) return launch_trace_tpt<NT, 256>(mode, a, s);
    return launch_trace_tpt<NT, 64>(mode, a, s);
}

}  // namespace

MK_CHECK_TAKE(check_take_trace)


hipError_t launch_trace(int mode, int nt, const TraceArgs& a, hipStream_t s) {
    if (a.nfo * a.nr <= 0) return hipSuccess;
    switch (nt) {
        case 16: return launch_trace_nt<16>(mode, a, s);
        case 32: return launch_trace_nt<32>(mode, a, s);
        case 64: return launch_trace_nt<64>(mode, a, s);
        case 128: return launch_trace_nt<128>(mode, a, s);
        case 256: return launch_trace_nt<256>(mode, a, s);
        case 512: return launch_trace_nt<512>(mode, a, s);
        case 1024: return launch_trace_nt<1024>(mode, a, s);
        case 2048: return launch_trace_nt<2048>(mode, a, s);
        case 4096: return launch_trace_nt<4096>(mode, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_norm_reduce(const double* npart, int nr, int nfo, double* out, double* out2,
                              hipStream_t s) {
    if (nfo <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_norm_reduce, dim3(nfo), dim3(256), 0, s, npart, nr, out, out2);
    return hipGetLastError();
}

hipError_t launch_sumsq_out(const float* x, int ntr, int nt, const int32_t* itd, int shift, double* npart,
                            double* npart_out, hipStream_t s) {
    if (ntr <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sumsq<2>, dim3((ntr + 3) / 4), dim3(256), 0, s, x, x, ntr, ntr, nt, itd, shift, npart,
                       npart_out);
    return hipGetLastError();
}

hipError_t launch_sumsq2_win(const float* x0, const float* x1, int ntr, int nt, const int32_t* itd, int shift,
                             double* npart, hipStream_t s) {
    if (ntr <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sumsq<1>, dim3((2 * ntr + 3) / 4), dim3(256), 0, s, x0, x1, ntr, 2 * ntr, nt, itd, shift,
                       npart, nullptr);
    return hipGetLastError();
}

hipError_t launch_f2p(const float* f1p, const float* f1m, int64_t ntr, int nt, float* out, hipStream_t s) {
    if (ntr <= 0) return hipSuccess;
    const int64_t n = ntr * nt;
    hipLaunchKernelGGL(k_f2p, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f1p, f1m, ntr, nt, out);
    return hipGetLastError();
}

hipError_t launch_gsum(const float* gp, const float* gm, int64_t n, float* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gsum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, gp, gm, n, out);
    return hipGetLastError();
}

hipError_t launch_image(const float* gm, const float* f1p, int nf, int nr, int nt, double scale, double* part,
                        double* out, hipStream_t s) {
    if (nf <= 0 || nr <= 0) return hipSuccess;
    const int ntr = nf * nr;
    hipLaunchKernelGGL(k_image_part, dim3((ntr + 3) / 4), dim3(256), 0, s, gm, f1p, ntr, nt, part);
    hipLaunchKernelGGL(k_image_reduce, dim3(nf), dim3(256), 0, s, part, nr, scale, out);
    return hipGetLastError();
}

hipError_t launch_gather(const float* src, float* dst, const int* perm, int nf, int64_t per,
                         hipStream_t s) {
    if (nf <= 0 || per <= 0) return hipSuccess;
    const bool v4 = per % 4 == 0 && reinterpret_cast<uintptr_t>(src) % 16 == 0 &&
                    reinterpret_cast<uintptr_t>(dst) % 16 == 0;
    const int64_t n = v4 ? per / 4 : per;
    const int64_t blocks = (n + 255) / 256;
    const dim3 grid((unsigned)(blocks < 512 ? blocks : 512), (unsigned)nf);
    if (v4)
        hipLaunchKernelGGL(k_gather<float4>, grid, dim3(256), 0, s, reinterpret_cast<const float4*>(src),
                           reinterpret_cast<float4*>(dst), perm, n);
    else
        hipLaunchKernelGGL(k_gather<float>, grid, dim3(256), 0, s, src, dst, perm, n);
    return hipGetLastError();
}
