// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "mk.h"
#include "mk_check.h"

// Per-trace kernel modes (one wave per trace of nt samples).
enum TraceMode : int {
    TM_INIT = 0,   // N_-1 = Gd(-t); f1+ = N_-1; f1- = 0; X = rfft(N_-1)
    TM_ITER = 1,   // RN = irfft(Y); N = mute(-RN(-t)); accumulate; X = rfft(N)
    TM_GFWD = 2,   // X[2f] = rfft(f1+[f]); X[2f+1] = rfft(f1-[f](-t))
    TM_GOUT = 3,   // G- = irfft(Y[2f]) - f1-;  G+ = f1+(-t) - irfft(Y[2f+1])
    TM_FWDF = 4,   // X[f] = rfft(f1+[f])                      (restart, first synthesis)
    TM_RST1 = 5,   // RN = irfft(Y); f1- := theta RN; N' = -RN(-t) windowed; X = rfft(N')
    TM_RST2 = 6,   // N'' = mute(-RN(-t)); rho = N_-1 + N'' - f1+; f1+ := N_-1 + N''; X = rfft(rho)
    TM_POUT = 7    // aux = p- = (G- + f1-) + (G+ - f1+(-t)) - irfft(Y), Y = S N_last
};

// Storage of the contraction input X.  The X2 forms keep a 16-bit "hi" plane
// and a 16-bit "lo" plane (x ~ hi + lo) for two matrix-core products.
enum XPrec : int { XP_F32 = 0, XP_F16 = 1, XP_BF16 = 2, XP_F16X2 = 3, XP_BF16X2 = 4 };

// Buffers of the per-trace kernel whose extents the checked build tests.
enum TraceExt : int { TE_Y, TE_X, TE_SRC, TE_F1P, TE_F1M, TE_GP, TE_GM, TE_AUX, TE_N0, TE_HIST, TE_COUNT };

// Arguments of the per-trace kernel.  Layouts (all row-major):
//   Y   [nfo][B][nr]        complex, contraction output (unscaled sum over s)
//   X   [nfo][B][ns_pad]    complex, next contraction input
//   src [nf][nr][nt]        float, G_d for TM_INIT
//   f1p, f1m, gp, gm [nf][nr][nt] float
//   itd [nf][nr], fband [nf][2] (or null), npart [nfo][nr] double
//   tw  [nt + 256] complex: exp(-2 pi i k / nt), then exp(-2 pi i q k / 256) at 16 q + k
struct TraceArgs {
    const float2* Y;
    void* X;           // float2 (XP_F32) or 16-bit pairs (XP_F16 / XP_BF16)
    const float* src;
    float* f1p;
    float* f1m;
    float* gp;
    float* gm;
    float* aux;        // [nf][nr][nt] TM_POUT output
    const int32_t* itd;
    const int32_t* fband;
    double* npart;
    const float2* tw;
    const double* xs_in;   // [nf] norm setting the scale of 16-bit X (per focal point)
    float* xs_out;         // [nfo] scale written next to 16-bit X (X = xs_out * stored)
    int xprec;             // XPrec
    int skip_outband;      // X above the focal band end is never read: do not write it
    float* n0;             // [nf][nr][nt] N_-1 = G_d(-t), kept for the restart
    float* hist;           // [nf][nr][hist_k][hist_T] recorded iterates (or null)
    int hist_k, hist_T;
    int rec_slot;          // iterate index this pass records, or -1
    int nr;
    int nf;        // focal points of the series
    int nfo;       // traces are nfo x nr (nf, or 2 nf for the G modes)
    int lo;        // first stored bin
    int B;         // stored bins
    int ns_pad;    // row pitch of X (complex elements)
    int shift;
    int parity;    // pass index & 1 (TM_ITER)
    float scale;   // c / (nt / 2): Riemann weight and inverse-FFT normalisation
    // bytes from each pointer to the end of its allocation (checked build)
    int64_t ext[TE_COUNT];
};

struct ProfileSlot {
    double ms = 0.0;
    int64_t launches = 0;
};

// One contraction choice: the GEMV (variant 0) or an MFMA tile shape (1 + v).
struct ContractChoice {
    int variant = 0;
    int xprec = XP_F32;   // storage of X this choice consumes
};

struct mk_plan_s {
    mk_plan_desc d{};
    int B = 0;          // stored bins
    int M = 0;          // nt / 2
    int ns_pad = 0;     // padded row length of R and X (complex elements, multiple of 32)
    bool r_tiled = false;   // R in the LDS-staged contraction's tiles (nf_max > 4, no MK_FLAG_ROW_R)
    int device = 0;
    hipStream_t stream = nullptr;

    // device memory (plan-owned)
    void* R = nullptr;         // [B][nr][ns_pad] complex64 or 16-bit pairs, or tiled (r_tiled)
    float* rscale = nullptr;   // [B] per-frequency scale of 16-bit R
    float2* X = nullptr;       // [3 nf_max][B][ns_pad]: series slabs, then G-assembly slabs
    float2* Y = nullptr;       // [2 nf_max][B][nr]
    float* f1p = nullptr;      // [nf_max][nr][nt]  (focal points in the plan's sorted order)
    float* f1m = nullptr;
    float* gp = nullptr;
    float* gm = nullptr;
    float* stage = nullptr;    // [nf_max][nr][nt] staging for permuted inputs and outputs
    int32_t* itd = nullptr;    // [nf_max][nr]
    int32_t* fband = nullptr;  // [nf_max][2]
    int32_t* perm = nullptr;   // [nf_max] sorted position -> caller's focal index
    int32_t* iperm = nullptr;  // [nf_max] caller's focal index -> sorted position
    int32_t* ncols = nullptr;  // [B] active focal count per bin (sorted order)
    double* npart = nullptr;   // [2 nf_max][nr]
    double* norm0 = nullptr;   // [nf_max] norm the 16-bit X of the series is scaled by (||G_d||, then ||rho||)
    double* gdnorm = nullptr;  // [nf_max] ||G_d||: scale of the 16-bit X of the G assembly (f1 fields)
    double* nlast = nullptr;   // [nf_max] norm of the last N (scales 16-bit X)
    double* img = nullptr;     // [nf_max] double-focusing image, sorted focal order
    float* aux = nullptr;      // [nf_max][nr][nt] f2+ or p- for mk_get (allocated on first request)
    float* xscale = nullptr;   // [3 nf_max] scale stored with 16-bit X
    double* norms = nullptr;   // [norm_cap][nf_max]
    int norm_cap = 0;
    // norms of every term since mk_set_focal, [log_cap][nf] (row e holds one
    // term for every focal point, sorted order): the first row of each series
    // is its starting field (N_-1, or the restart residual), then one row per
    // pass; the stopping rule of mk_iterate_tol reads the current series
    double* norm_log = nullptr;
    int log_cap = 0, log_len = 0, series_start = 0, prev_series_start = 0;
    double* fnorm = nullptr;   // [2 nf_max] ||f1+||, ||f1-|| for the stopping rule
    double* hpin = nullptr;    // pinned host buffer for small device-to-host reads
    size_t hpin_cap = 0;       // its capacity in doubles
    // MK_FLAG_WALK: lists of active tiles for the persistent LDS-staged
    // contraction, [0] the series (nf columns), [1] the G assembly (2 nf)
    // ([count, tiles...] on the device; buffers sized once for the largest
    // list, so that captured graphs keep valid pointers)
    int* walk_items[2] = {nullptr, nullptr};
    int walk_variant[2] = {-1, -1};
    int walk_blocks_per_xcd = 0;
    std::vector<int32_t> ncols_host;   // active focal count per bin (sorted order) when bands are set
    // R streamed from pinned host memory (r_dev_bytes below the size of R):
    // the whole of R in the device layout on the host, two device buffers of
    // slab_bins bins each, a copy stream and the events that order the ring
    bool r_stream = false;
    unsigned char* R_host = nullptr;
    void* rbuf[2] = {nullptr, nullptr};
    size_t bin_bytes = 0;      // bytes of one bin of R in the device layout
    int slab_bins = 0, nslabs = 0;
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_copied[2] = {nullptr, nullptr}, ev_consumed[2] = {nullptr, nullptr};
    int buf_slab[2] = {-1, -1};  // slab each buffer holds (or is receiving)
    int64_t slab_use = 0;        // slab contractions so far; use u reads buffer u % 2
    float2* tw = nullptr;      // [nt + 256]
    int* flag = nullptr;       // device scratch flag (non-finite input detection)
    float* n0 = nullptr;       // [nf_max][nr][nt] N_-1 = G_d(-t)

    // series tail: recorded iterates and the network
    float* hist = nullptr;     // [nf_max][nr][hist_k][hist_T]
    int hist_k = 0, hist_T = 0;
    float* tail_w = nullptr;   // BF16-rounded parameters
    void* tail_wpk = nullptr;  // the same weights packed for the one-kernel form
    int tail_nw = 0;
    float* tail_x = nullptr;   // [chunk][k][T] normalised input (layer-by-layer form only)
    float* tail_work = nullptr;   // [2][chunk][hidden][T] (layer-by-layer form only)
    float* tail_y = nullptr;   // [chunk][2][T] (layer-by-layer form only)
    float* tail_scale = nullptr;  // [nf_max][nr]
    int tail_chunk = 0;
    int pass_base = 0;         // passes before the current series (a restart starts a new one)
    bool tail_applied = false;
    int tail_hidden = 0;       // hidden width tail_work is sized for
    int tail_net_hidden = 0;   // hidden width of the loaded network
    std::vector<double> gd_norm_host;   // ||G_d|| per focal point (caller order)

    // series state
    int nf = 0;
    int shift = 0;
    int passes = 0;
    bool has_fband = false;
    bool R_loaded = false;
    bool focal_set = false;
    bool g_valid = false;
    std::vector<double> norm0_host;
    // sum of squares of N_-1 outside the mute window per focal point (plan
    // order): f1+ keeps those samples of N_-1, f1- is zero there
    std::vector<double> f1p_out2_host;
    std::vector<int> perm_host;
    ContractChoice series_choice, g_choice;

    // graph replay (MK_FLAG_GRAPH): one executable per (passes, start parity)
    // and per state the captured launches hold by value (batch width, bands,
    // mute margin, contraction choice)
    struct GraphEntry {
        int niter;
        int parity;
        int nf;
        bool fband;
        int shift;
        int variant;
        int xprec;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t capture_stream = nullptr;   // private stream used when the plan stream is NULL

    // contraction selection: -1 heuristic, -2 autotune, >= 0 forced variant
    int tune_mode = -1;
    std::vector<std::pair<int, int>> tuned;   // (ncols, variant) chosen by the autotuner

    // profiling (MK_FLAG_PROFILE)
    struct Pending {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    ProfileSlot prof[6];

    std::string err;
};

// Arguments of the contraction kernels (GEMV and MFMA).
//   R  [B][nr][ns_pad] complex64 or 16-bit pairs, rscale [B] (16-bit only)
//   X  [ncols][B][ns_pad] complex64 (GEMV, MFMA-f32) or 16-bit pairs (MFMA-16)
//   xscale [ncols] (MFMA-16 only), Y [ncols][B][nr] complex64
//   ncols_w [B]: active columns per bin (times ncols_mul), or null for all
struct ContractArgs {
    const void* R;
    const float* rscale;
    int prec;              // mk_rprec of R
    const void* X;
    const float* xscale;
    float2* Y;
    const int* ncols_w;
    int ncols_mul;
    int xsplit;            // 16-bit X held as hi and lo planes (two products)
    int tiled;             // R in the LDS-staged contraction's tiles
    int nr, ns, ns_pad, B, ncols;
    int nb;                // bins this launch covers (R, rscale, X, Y, ncols_w start at its first bin;
                           // X and Y keep the B-bin strides of the whole band)
    // LDS-staged variants only: when items is set, the persistent form walks
    // the tile list items = [count, tile indices (ascending)...] with
    // walk_blocks_per_xcd four-wave blocks (two waves per SIMD) on each of
    // the 8 XCDs: half as many for the one-wave 128-row tiles, twice as many
    // two-wave blocks where the tiles use those
    const int* items = nullptr;
    int walk_blocks_per_xcd = 0;
    // bytes from R, X and Y to the end of their allocations (checked build)
    int64_t ext_r = kExtentUnknown, ext_x = kExtentUnknown, ext_y = kExtentUnknown;
};

// extents (bytes from the pointer to the end of its allocation) of a
// contraction launch's R, X and Y, for the checked build
struct Ext3 {
    int64_t r, x, y;
};

// bytes from ptr to the end of the device allocation behind it (checked
// build; 0 for NULL; kExtentUnknown in the normal build)
int64_t device_extent(const void* ptr);

// the checked build's bounds-check words, one per translation unit (read
// and cleared; always 0 in the normal build)
hipError_t check_take_trace(unsigned* out);
hipError_t check_take_contract(unsigned* out);
hipError_t check_take_mfma(unsigned* out);
hipError_t check_take_net(unsigned* out);
hipError_t check_take_tail(unsigned* out);

// kernel launchers (return hipSuccess or the launch error)
hipError_t launch_trace(int mode, int nt, const TraceArgs& a, hipStream_t s);
hipError_t launch_norm_reduce(const double* npart, int nr, int nfo, double* out, double* out2,
                              hipStream_t s);
// the sums of squares of two fields of ntr traces each, over the samples
// inside each trace's mute window only (itd [ntr]), in one launch: npart [2 ntr]
hipError_t launch_sumsq2_win(const float* x0, const float* x1, int ntr, int nt, const int32_t* itd, int shift,
                             double* npart, hipStream_t s);
// whole traces into npart, the samples outside the mute window into npart_out
hipError_t launch_sumsq_out(const float* x, int ntr, int nt, const int32_t* itd, int shift, double* npart,
                            double* npart_out, hipStream_t s);
// out = f1p(t) - f1m(-t) per trace (f2+)
hipError_t launch_f2p(const float* f1p, const float* f1m, int64_t ntr, int nt, float* out, hipStream_t s);
// out = gp + gm elementwise (the total G)
hipError_t launch_gsum(const float* gp, const float* gm, int64_t n, float* out, hipStream_t s);
// out[f] = scale * sum_r sum_k gm[f][r][k] f1p[f][r][(-k) mod nt] (FP64); part holds nf * nr doubles
hipError_t launch_image(const float* gm, const float* f1p, int nf, int nr, int nt, double scale, double* part,
                        double* out, hipStream_t s);
hipError_t launch_gather(const float* src, float* dst, const int* perm, int nf, int64_t per,
                         hipStream_t s);
hipError_t launch_contract_gemv(const ContractArgs& c, hipStream_t s);
hipError_t launch_contract_mfma(const ContractArgs& c, int variant, hipStream_t s);
int contract_mfma_variants();
hipError_t launch_repack_c64(const float* Rin, float2* Rout, int nr, int B, int ns, int ns_pad,
                             int* flag, hipStream_t s);
hipError_t launch_quantize_R(int prec, const float* Rin, void* Rout, float* rscale, int nr, int B,
                             int ns, int ns_pad, int* flag, hipStream_t s);
// per-frequency scales of 16-bit R (k_rmax); the tiled repack below uses them
hipError_t launch_rscale(const float* Rin, float* rscale, int nr, int B, int ns, int* flag, hipStream_t s);
// Tiled R for the LDS-staged contraction: for bin w, 16-receiver group rg and
// 128-byte chunk c of the rows, a 2 KB tile [h][lane] of 16-byte pieces where
// lane = 16 g + i holds receiver 16 rg + i, row bytes c*128 + 32 g + 16 h; the
// tiles follow in (w, rg, c) order, so one wave load of 64 x 16 bytes is 1 KB
// of contiguous memory.  Receivers past nr and shots past ns are zero.
constexpr int kTileRows = 16;
constexpr int kTileChunkBytes = 128;
// R into the tiles of the LDS-staged contraction (any precision)
hipError_t launch_repack_tiled(int prec, const float* Rin, void* Rout, const float* rscale, int nr, int B,
                               int ns, int ns_pad, int* flag, hipStream_t s);
size_t tiled_R_bytes(int prec, int nr, int B, int ns_pad);
bool contract_variant_reads_tiled(int variant);
// focal columns per tile of LDS-staged contraction variant v (6, 7, 8); 0 for the others
int contract_variant_focal_tile(int variant);
// receivers per block (and per tile of the walk's list) of LDS-staged
// variant v for nr receivers and one or two planes of X: 256 or 128; 0 for
// the other variants
int contract_lds_receivers(int variant, bool xsplit, int nr);
hipError_t launch_check_finite(const float* x, int64_t n, int* flag, hipStream_t s);
// x may be NULL: then only the per-trace scales are written
hipError_t launch_tail_prep(const float* hist, int ntr, int k, int T, float* x, float* scale, hipStream_t s);
// the odd-pass tail into f1+ (the restart that follows rebuilds f1- from f1+)
hipError_t launch_tail_apply(const float* hist, const float* y, const float* scale, const int32_t* itd, int shift,
                             int ntr, int k, int T, int nt, int mode, float* f1p, hipStream_t s);

// series-tail network (k -> H -> H -> 2 channels, 5 taps, H hidden channels)
constexpr int kNetHiddenMax = 128;      // widest hidden layer the ABI accepts
constexpr int kNetDil[3] = {1, 4, 16};
int net_param_count(int k, int H);
hipError_t net_forward(const float* P, const float* x, int N, int k, int H, int T, float* a1, float* a2,
                       float* y, hipStream_t s);
// the whole network plus the tail's application in one kernel per 256-sample
// tile (hidden width 16, k <= 16); other widths go layer by layer
bool net_tail_fused(int k, int H);
// the weights in the matrix cores' per-lane order (net_tail_pack_bytes(k) bytes), written once per network
size_t net_tail_pack_bytes(int k);
hipError_t net_tail_pack(const float* P, int k, int H, void* out, hipStream_t s);
hipError_t net_tail_apply(const float* P, const void* wpack, const float* hist, const float* scale,
                          const int32_t* itd, int shift, int ntr, int k, int H, int T, int nt, float* f1p,
                          hipStream_t s);
hipError_t net_backward(const float* P, const float* x, const float* a1, const float* a2, const float* gy,
                        int N, int k, int H, int T, float* G, float* g1, float* g2, float* wt, hipStream_t s);
hipError_t net_mse(const float* y, const float* tgt, const float* mask, int N, int T, float* gy,
                   double* part, int nparts, double* loss, float count, hipStream_t s);
hipError_t net_adam(float* w, float* wq, const float* g, float* m, float* v, int n, int step, float lr,
                    float b1, float b2, float eps, hipStream_t s);
hipError_t net_round_bf16(const float* w, float* wq, int n, hipStream_t s);
