/*
 * mk.h -- C ABI of the MI355X (gfx950) Marchenko synthesis library.
 *
 * The library runs the iterative (Neumann-series) Marchenko scheme of
 * Koehne et al., "A multi-GPU benchmark for 2D Marchenko Imaging"
 * (arXiv 2106.04649): Eq. (1) of the Theory section and Algorithm 1, with
 * the synthesis of Algorithm 2 as hand-written HIP kernels on one GPU.
 *
 * Conventions shared by every call:
 *   - Time axis: nt samples, periodic, t = 0 at sample 0.  Time reversal
 *     maps sample k to (nt - k) mod nt.
 *   - Frequency: numpy rfft convention, kernel exp(-2 pi i k n / nt),
 *     unnormalised; bins w = 0 .. nt/2.  Complex values are interleaved
 *     (re, im) float pairs.
 *   - Mute theta_t of Eq. (1): sample k of trace (f, r) is kept when
 *     |t_k| < itd[f][r] - shift, with t_k = k for k < nt/2 and k - nt above;
 *     the sample nt/2 is never kept.
 *   - One synthesis: S(x)[r](t) = c * sum_s (R[r][s] * x[s])(t), circular
 *     time convolution evaluated in the frequency domain over the stored
 *     band, with c = dx * dt (Riemann weight of the double integral).
 *     Bins outside the band are zero before the inverse transform.
 *   - Sources and receivers share one grid (nr == ns), since each output
 *     trace of a synthesis is an integration position of the next one.
 *   - "on_device" arguments: 0 = host pointer, 1 = device pointer (HIP
 *     device memory of the current device).  Device inputs are read only
 *     during the call; the caller owns every buffer it passes.
 *   - All GPU work is ordered on the plan's stream.  Calls that return data
 *     to host memory synchronise that stream.
 *   - Errors are reported by status code; nothing aborts or throws across
 *     the ABI.  mk_last_error() gives a message for the last failure.
 *   - A plan is not thread-safe: one plan per host thread and stream.
 */
#ifndef MK_H
#define MK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mk_plan_s* mk_plan_t;

typedef enum {
    MK_OK = 0,
    MK_ERR_ARG = 1,          /* invalid argument (null, size, range, NaN input) */
    MK_ERR_STATE = 2,        /* call out of order (e.g. iterate before load_R)  */
    MK_ERR_OOM = 3,          /* device allocation failed                        */
    MK_ERR_HIP = 4,          /* a HIP runtime call failed                       */
    MK_ERR_UNSUPPORTED = 5,  /* valid request the library does not implement     */
    MK_ERR_DIVERGED = 6      /* series norms non-finite or above div_factor     */
} mk_status;

/* Storage precision of R inside the plan. */
typedef enum {
    MK_R_C64 = 0,    /* complex64 (FP32 pairs)                                 */
    MK_R_F16S = 1,   /* FP16 pairs with one FP32 scale per frequency           */
    MK_R_BF16S = 2   /* BF16 pairs with one FP32 scale per frequency           */
} mk_rprec;

/* Fields returned by mk_get, each [nf][nr][nt] float32. */
typedef enum {
    MK_F1PLUS = 0,   /* f1+ : N_{-1} plus the odd-pass terms  (Algorithm 1)    */
    MK_F1MINUS = 1,  /* f1- : minus the time-reversed even-pass terms          */
    MK_GPLUS = 2,    /* G+  : f1+(-t) - S[f1-(-t)]   (one extra synthesis)     */
    MK_GMINUS = 3,   /* G-  : S[f1+] - f1-           (last lines of Alg. 1)    */
    MK_F2PLUS = 4,   /* f2+ : N_{-1} plus every pass's N_i (Alg. 1, second loop) */
    MK_PMINUS = 5,   /* p-  : sum of every pass's synthesis RN_i (Alg. 1)        */
    MK_GTOTAL = 6    /* G   : the total Green's function, which the Theory
                        section obtains from f2+ and p- (p-(t) + S[N_last](t)
                        + f2+(-t)); with Algorithm 1's signs that is G+ + G-,
                        formed here as their sum                              */
} mk_field;

/* Plan flags. */
#define MK_FLAG_GRAPH    0x1u  /* replay the per-pass kernels as a HIP graph   */
#define MK_FLAG_PROFILE  0x2u  /* time every kernel with HIP events            */
#define MK_FLAG_AUTOTUNE 0x4u  /* time the contraction variants on first use   */
#define MK_FLAG_FAST_X   0x8u  /* 16-bit R on matrix cores: one 16-bit plane of X
                                  instead of the default hi + lo planes (half the
                                  products, about 2x the rounding error)        */
#define MK_FLAG_WALK     0x20u /* run the LDS-staged contraction (variants 6..8)
                                  as a persistent kernel that walks a list of
                                  its active tiles, spread evenly over the
                                  XCDs, also without per-focal bands (with
                                  bands the plan walks by default); not with
                                  MK_FLAG_AUTOTUNE, MK_FLAG_GRID or streamed R */
#define MK_FLAG_GRID     0x40u /* launch one block per tile of the LDS-staged
                                  contraction even with per-focal bands (out-of-
                                  band tiles then exit at once): the form the
                                  walk replaces, kept for comparison; not with
                                  MK_FLAG_WALK                                 */
#define MK_FLAG_ROW_R    0x10u /* keep R frequency-major and row-major even when
                                  nf_max > 4 (by default such plans store R in
                                  the tiles of the LDS-staged matrix-core
                                  contraction, variants 6..8, the only ones that
                                  read that layout)                             */

typedef struct {
    int32_t nr;          /* receivers (output positions x_R)                    */
    int32_t ns;          /* shots (integration positions x); must equal nr      */
    int32_t nt;          /* time samples = FFT length; power of two, 16..4096   */
    int32_t iw_lo;       /* first stored rfft bin (inclusive), >= 0             */
    int32_t iw_hi;       /* last stored rfft bin (inclusive), <= nt/2           */
    int32_t nf_max;      /* largest focal batch mk_set_focal will be given      */
    double dt;           /* time sampling (s), > 0                              */
    double dx;           /* receiver spacing (m), > 0                           */
    double div_factor;   /* divergence threshold on ||N_i|| / ||N_-1||; <= 0 -> 1e3 */
    int32_t rprec;       /* mk_rprec                                            */
    uint32_t flags;      /* MK_FLAG_*                                           */
    void* stream;        /* hipStream_t to order work on; NULL = null stream    */
    int64_t r_dev_bytes; /* cap on the device memory that holds R; <= 0 or at
                            least R's size: R resident.  Below R's size, R
                            stays in pinned host memory and crosses to the
                            device in slabs of frequency bins on every
                            synthesis, two slab buffers of at most half the
                            cap each, the copy of one slab overlapping the
                            contraction of the previous one (the pipelined
                            batches of Algorithm 2, for R larger than HBM) */
} mk_plan_desc;

/*
 * mk_plan -- validate the problem description and create a plan.
 * Follows the problem statement of the Theory section (R, G_d, the mute and
 * niter are the inputs) and the batching of Algorithm 2.  Allocates the
 * plan's device workspace for nf_max focal points.
 * rprec selects the storage of R: MK_R_C64 keeps complex64; MK_R_F16S and
 * MK_R_BF16S keep 16-bit pairs with one FP32 scale per frequency (the
 * contraction accumulates in FP32; the norms and the final G subtraction
 * stay in FP64).
 * With r_dev_bytes below the size of R in the plan's storage, the plan
 * holds R in pinned host memory (hipHostMalloc) and two device slab buffers
 * instead of a resident copy; results are the same bits as the resident
 * plan's (the same kernels per bin), at PCIe speed.
 * Errors: MK_ERR_ARG (null pointers, nr != ns, nt not a power of two in
 * [16, 4096], band outside [0, nt/2], nf_max < 1, dt or dx not positive,
 * unknown rprec or flag, r_dev_bytes positive but below two bins of R),
 * MK_ERR_UNSUPPORTED (ns > 2048 with MK_R_C64, ns > 4096, MK_FLAG_GRAPH or
 * MK_FLAG_AUTOTUNE with streamed R, MK_FLAG_WALK with MK_FLAG_AUTOTUNE or
 * streamed R), MK_ERR_OOM, MK_ERR_HIP.  *out is NULL on failure.
 */
mk_status mk_plan(const mk_plan_desc* desc, mk_plan_t* out);

/*
 * mk_load_R -- copy the frequency-domain reflection response into the plan.
 * R: interleaved complex float32, layout receivers x frequencies x shots,
 * R[r][w - iw_lo][s] for w in [iw_lo, iw_hi] (the layout of the
 * Introduction and Implementation sections: the space integral runs over
 * the fastest axis).  The plan repacks it frequency-major (and quantises it
 * for MK_R_F16S / MK_R_BF16S); the caller may free R on return.  A plan
 * with streamed R (r_dev_bytes) repacks one slab of bins at a time on the
 * device and keeps the result in its pinned host copy.
 * Errors: MK_ERR_ARG (null, non-finite value), MK_ERR_HIP.
 */
mk_status mk_load_R(mk_plan_t plan, const float* R, int on_device);

/*
 * mk_set_focal -- start a new series for nf focal points.
 * Gd: float32 [nf][nr][nt], the first-arrival field G_d(x_R, x_F, t) of the
 * Theory section; the series starts from N_{-1} = f1+ = G_d(-t), f1- = 0.
 * itd: int32 [nf][nr], first-arrival time in samples (the mute window of
 * Algorithm 1's applyMute); shift: mute margin in samples (>= 0).
 * band: int32 [nf][2] per-focal inclusive rfft-bin band inside the plan
 * band, or NULL for the plan band.  All four arrays are host or device per
 * on_device.  Runs the first forward transform on the GPU.  With bands, the
 * plan orders the focal points by band end internally (the batch active at
 * a bin is then a prefix, and the batched contraction skips the rest);
 * every output and norm comes back in the caller's order.
 * Errors: MK_ERR_ARG (nf outside [1, nf_max], null Gd or itd, negative
 * shift, band outside the plan band, non-finite Gd), MK_ERR_STATE (R not
 * loaded), MK_ERR_HIP.  The argument checks leave the plan as it was; a
 * non-finite device Gd (found from its norm, after the arrays were taken in)
 * and MK_ERR_HIP leave no focal points set.
 */
mk_status mk_set_focal(mk_plan_t plan, int32_t nf, const float* Gd, const int32_t* itd,
                       int32_t shift, const int32_t* band, int on_device);

/*
 * mk_iterate -- run niter more passes of Algorithm 1's loop.
 * Pass i: RN_i = S(N_{i-1}); N_i = theta(-RN_i(-t)); even i: f1- -= N_i(-t);
 * odd i: f1+ += N_i.  Continues the series across calls.  With
 * MK_FLAG_GRAPH the passes of one call are captured once per (niter, parity
 * of the first pass) as a HIP graph of kernel launches and replayed on later
 * calls (not while the autotuner still has to time the batch, and not with
 * MK_FLAG_PROFILE).
 * norms: host double [niter][nf] receiving ||N_i||_2 (FP64 reduction), or
 * NULL.  With norms != NULL the call synchronises and returns
 * MK_ERR_DIVERGED when a norm is non-finite or exceeds div_factor times
 * ||N_-1||; the passes have still been applied.
 * Errors: MK_ERR_ARG (niter < 0), MK_ERR_STATE (no focal set), MK_ERR_HIP,
 * MK_ERR_DIVERGED.
 */
mk_status mk_iterate(mk_plan_t plan, int32_t niter, double* norms);

/*
 * mk_iterate_tol -- run passes of the current series until the library's own
 * estimate of the remaining error of every output is within tol (relative
 * L2), or max_passes passes have run.  The judge is the plain iteration
 * itself: the series converges like a geometric series whose ratio q per
 * pass is read from the FP64 norms of its last terms (the largest of the
 * last two term-to-term ratios; right after mk_tail_apply, the ratio of the
 * series before it, whose operator A = theta Rev S is the same), so the
 * terms not yet added sum to about rest = ||N_last|| q / (1 - q).  Every
 * output's error is a part of that sum: the odd terms belong to f1+ and the
 * even ones to f1- (Algorithm 1), and G+ and G- are syntheses of f1+ and f1-
 * with S a contraction.  The estimate is rest / min(||f1+||, ||f1-||), with
 * the field norms reduced in FP64 on the GPU; q is capped at 0.95.  From it
 * the call predicts how many passes reach tol, runs them as one batch, and
 * judges again.  With fewer than two terms and no earlier series, it first
 * runs two passes.
 * passes_run: passes this call ran (may be NULL).  est: host double [nf],
 * the final estimate per focal point in the caller's order (may be NULL);
 * an estimate above tol after max_passes means the budget ran out, which is
 * not an error.  Synchronises.
 * Errors: MK_ERR_ARG (tol not positive and finite, max_passes < 0),
 * MK_ERR_STATE (no focal set), MK_ERR_HIP, MK_ERR_DIVERGED (as mk_iterate).
 */
mk_status mk_iterate_tol(mk_plan_t plan, double tol, int32_t max_passes, int32_t* passes_run, double* est);

/*
 * mk_get -- copy one field, float32 [nf][nr][nt], into out.
 * MK_GPLUS / MK_GMINUS run the G assembly of the Theory section and the
 * last lines of Algorithm 1: both are formed together from one batched
 * synthesis of f1+ and f1-(-t), with the final subtraction in FP64; the
 * result is cached until the series changes.  MK_F2PLUS and MK_PMINUS are
 * the auxiliary fields of Algorithm 1's second loop (the Theory section
 * names them as the route to the total G): f2+ = f1+(t) - f1-(-t), which
 * holds N_{-1} and every N_i; p- = S[f2+ - N_last], formed from the G
 * assembly and one more synthesis of the last N (so it costs one pass's
 * contraction).  Both are defined for a plain series only.  MK_GTOTAL is
 * the total G = G+ + G- (after the G assembly, one add per sample).  The
 * first request of any of the three allocates an nf_max x nr x nt buffer.
 * Synchronises when out is a host pointer.
 * Errors: MK_ERR_ARG (null out, unknown field), MK_ERR_STATE (no focal
 * set; MK_F2PLUS or MK_PMINUS after mk_tail_apply), MK_ERR_OOM, MK_ERR_HIP.
 */
mk_status mk_get(mk_plan_t plan, int32_t field, float* out, int on_device);

/*
 * mk_image -- the double-focusing image of every focal point (Theory
 * section, imaging paragraph; the last step of Algorithm 1): G- and f1+ of a
 * focal point convolved in time and integrated over the receivers give
 * G^{-,+}(x_F, x_F, t), whose zero-time sample is the local reflectivity,
 *     image[f] = dx * dt * sum_r sum_k G-[f][r][k] * f1+[f][r][(-k) mod nt].
 * Runs the G assembly first when G- is not current.  Products and sums in
 * FP64 (each product of two FP32 samples is exact), summed in a fixed order.
 * image: host array of nf doubles, in the caller's focal order; the caller
 * owns it.  Synchronises.
 * Errors: MK_ERR_ARG (null plan or image), MK_ERR_STATE (no focal set),
 * MK_ERR_HIP.
 */
mk_status mk_image(mk_plan_t plan, double* image);

/*
 * mk_tune -- choose how the contraction (the space integral of Eq. (1),
 * segmented dot products of Algorithm 2) runs.  mode -1: built-in
 * heuristic; -2: autotune (time every variant once per column count at its
 * first use and keep the fastest; with the environment variable
 * MK_TUNE_CACHE naming a file, choices are read from and appended to it);
 * 0: the streaming GEMV; 1..5: matrix-core tiles loaded straight from
 * memory (focal-real rows x receivers per block: 128x64, 64x64, 64x128,
 * 32x128, 128x32); 6..8: matrix-core tiles with X staged through LDS
 * (128, 64, 32 focal-real rows x 256 receivers per block).  Plans with
 * nf_max > 4 store R tiled for variants 6..8 (unless MK_FLAG_ROW_R) and
 * accept only those.  The storage of X follows from the choice, so the
 * focal points must be set again after this call (MK_ERR_STATE otherwise).
 * Errors: MK_ERR_ARG (null plan, mode outside [-2, 8], or a variant that
 * cannot read the plan's layout of R).
 */
mk_status mk_tune(mk_plan_t plan, int32_t mode);

/*
 * mk_contract_variant -- the contraction variant (0 GEMV, v >= 1 MFMA shape
 * v - 1) the plan uses, or has tuned, for ncols focal columns.
 * Errors: MK_ERR_ARG (null, ncols < 1).
 */
mk_status mk_contract_variant(mk_plan_t plan, int32_t ncols, int32_t* variant);

/*
 * mk_passes -- number of passes applied since the last mk_set_focal.
 * Errors: MK_ERR_ARG (null).
 */
mk_status mk_passes(mk_plan_t plan, int32_t* passes);

/*
 * mk_profile -- accumulated time of one kernel class, recorded with HIP
 * events on the plan's stream when the plan has MK_FLAG_PROFILE.
 * kind: 0 contraction (the space integral of Eq. (1)), 1 per-pass epilogue
 * (inverse FFT, reverse, mute, accumulate, forward FFT), 2 norm reduction,
 * 3 first forward transform, 4 G assembly, 5 image.  Synchronises.  reset != 0
 * clears the counters after reading.
 * Errors: MK_ERR_ARG, MK_ERR_UNSUPPORTED (plan without MK_FLAG_PROFILE).
 */
mk_status mk_profile(mk_plan_t plan, int32_t kind, double* total_ms, int64_t* launches,
                     int reset);

/*
 * Series-tail network (learned extension of the Neumann series; not in the
 * paper).  A fixed 3-layer dilated 1D convolution maps the first k iterates
 * N_0 .. N_{k-1} of one trace (k channels over a window of T samples centred
 * on t = 0, normalised per trace) to two channels: the even-pass and the
 * odd-pass sums of the remaining terms of the series.
 *   conv(k -> H, 5 taps, dilation 1), ReLU, conv(H -> H, 5, dilation 4),
 *   ReLU, conv(H -> 2, 5, dilation 16); zero padding outside the window;
 *   H ("hidden", 1..128) hidden channels.
 * Parameters: one FP32 vector, W1 [H][k][5], b1 [H], W2 [H][H][5],
 * b2 [H], W3 [2][H][5], b3 [2].  The forward pass is meant to run on
 * BF16-rounded parameters (mk_net_round / the wq output of mk_net_adam).
 * Every pointer below is device memory owned by the caller; work is
 * enqueued on `stream` (hipStream_t, NULL = null stream) and not
 * synchronised.  Errors: MK_ERR_ARG (NULL, bad sizes), MK_ERR_HIP; the
 * message is in mk_net_last_error().
 */
int32_t mk_net_param_count(int32_t k, int32_t hidden);   /* -1 when k or hidden is out of range */
const char* mk_net_last_error(void);

/* Forward pass: x [N][k][T] -> y [N][2][T]; work [2][N][hidden][T] keeps the
 * hidden activations for mk_net_backward. */
mk_status mk_net_forward(const float* params, const float* x, int32_t N, int32_t k, int32_t hidden, int32_t T,
                         float* work, float* y, void* stream);

/* Gradient of sum(gy * y) with respect to every parameter -> grads (same
 * layout as params); work as left by mk_net_forward; work2 holds
 * 2 N hidden T + hidden * hidden * 5 floats of scratch. */
mk_status mk_net_backward(const float* params, const float* x, const float* work, const float* gy,
                          int32_t N, int32_t k, int32_t hidden, int32_t T, float* grads, float* work2,
                          void* stream);

/* Masked mean squared error over both output channels: loss (one double)
 * = sum(((y - target) mask)^2) / count, gy = 2 (y - target) mask / count;
 * mask [N][T]; part holds nparts doubles of scratch (fixed-order sum). */
mk_status mk_net_loss(const float* y, const float* target, const float* mask, int32_t N, int32_t T,
                      float count, float* gy, double* loss, double* part, int32_t nparts, void* stream);

/* mk_net_loss_noalloc -- mk_net_loss without the caller's scratch buffer,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight training or serving loops, harnesses that forbid
 * hipMalloc).  It allocates nothing: the nparts FP64 partial sums go to a
 * fixed array inside the library (1024 doubles per GPU, held until the
 * process ends).  Same arguments, results and stream ordering as
 * mk_net_loss with the same nparts (the same kernels, so the same bits).
 * Calls that overlap on one GPU (two streams, or two threads) share that
 * array and race; order them on one stream.  Errors: MK_ERR_ARG (NULL, bad
 * sizes, nparts outside [1, 1024]), MK_ERR_HIP. */
mk_status mk_net_loss_noalloc(const float* y, const float* target, const float* mask, int32_t N, int32_t T,
                              float count, float* gy, double* loss, int32_t nparts, void* stream);

/* One Adam step (Kingma and Ba) with bias correction on FP32 master weights
 * w with moments m, v; writes the BF16-rounded weights to wq. */
mk_status mk_net_adam(float* w, float* wq, const float* g, float* m, float* v, int32_t n, int32_t step,
                      float lr, float b1, float b2, float eps, void* stream);

/* wq = BF16 rounding (nearest, ties to even) of w. */
mk_status mk_net_round(const float* w, float* wq, int32_t n, void* stream);

/*
 * mk_tail_record -- record the first k iterates N_0 .. N_{k-1} of each new
 * series (after mk_set_focal) on the window of T samples centred on t = 0
 * (sample u holds t = u - T/2).  Needed by mk_tail_apply and for building
 * the tail network's training set.  Errors: MK_ERR_ARG (k outside [1, 16],
 * T odd or above nt), MK_ERR_OOM, MK_ERR_HIP.
 */
mk_status mk_tail_record(mk_plan_t plan, int32_t k, int32_t T);

/*
 * mk_tail_load -- load the tail network's parameters (host FP32, layout of
 * mk_net_param_count(k, hidden) for the recorded k; the hidden width follows
 * from count); they are rounded to BF16.  Recording again with another k or
 * T drops the loaded network.
 * Errors: MK_ERR_ARG (NULL, a count that fits no hidden width, non-finite),
 * MK_ERR_STATE (no mk_tail_record), MK_ERR_OOM, MK_ERR_HIP.
 */
mk_status mk_tail_load(mk_plan_t plan, const float* params, int32_t count);

/*
 * mk_tail_history -- copy the recorded iterates, float [nf][nr][k][T] in
 * the caller's focal order.  Errors: MK_ERR_ARG, MK_ERR_STATE (nothing
 * recorded), MK_ERR_HIP.
 */
mk_status mk_tail_history(mk_plan_t plan, float* out, int on_device);

/*
 * mk_tail_apply -- after exactly k passes of a fresh series: add an estimate
 * of the rest of the series, T_odd = sum_{i>=k odd} N_i, to f1+ inside the
 * mute window (the rule of Algorithm 1 loop 2 for odd passes), then judge
 * it with plain synthesis: one fixed-point step f1- <- theta S f1+,
 * f1+ <- G_d(-t) + A^2 f1+ (A = theta Rev S; two syntheses, counted as two
 * passes), whose residual rho starts a new series carrying the remaining
 * error; later mk_iterate calls continue that series.  (The even-pass tail
 * T_even would feed f1-, which the judging step rebuilds from f1+ alone, so
 * it is not applied.)  mode 0: the loaded network
 * (inputs normalised by the RMS of N_0 per trace; with hidden width 16 it
 * runs as one kernel in its half-precision inference form -- input and
 * hidden activations stored as IEEE halves, FP32 accumulation -- and only
 * on the 256-sample tiles that meet the mute window; other widths run layer
 * by layer in FP32); 1: geometric
 * extrapolation of the last two odd iterates (needs an even k >= 4);
 * 2: no estimate (exactly two more passes of the plain series).
 * rel_resid: host double [nf] receiving ||rho|| / ||G_d|| per focal point
 * (the restart step's verdict on the estimate), or NULL.  Synchronises.
 * Errors: MK_ERR_ARG (mode), MK_ERR_STATE (not exactly k recorded passes
 * since mk_set_focal, already applied, no network for mode 0), MK_ERR_HIP.
 */
mk_status mk_tail_apply(mk_plan_t plan, int32_t mode, double* rel_resid);

/* mk_destroy -- free the plan and its device memory (NULL is a no-op). */
/*
 * Series state: checkpoint and resume of a running series (Algorithm 1's
 * loop state: the accumulated f1+ and f1-, the spectrum of the last term as
 * the next synthesis reads it, the pass counters, the focal set and the
 * norms the stopping rule reads).  The next synthesis depends on the last
 * term only through its stored in-band spectrum, so the blob holds that
 * spectrum (in the plan's X storage) rather than the time-domain term.
 *
 * mk_state_bytes -- size in bytes of the blob for the current series.
 * mk_get_state -- copy the state into blob (host memory of at least
 *   mk_state_bytes bytes).  Synchronises.
 * mk_set_state -- make blob the plan's current series.  The plan must have
 *   R loaded and the same nr, nt, band, rprec and MK_FLAG_FAST_X as the
 *   plan that saved it, nf_max >= the saved nf, and, when the saved series
 *   was recording iterates, mk_tail_record with the same k and T.  The
 *   series then continues exactly: mk_iterate after mk_set_state gives the
 *   same bits as the uninterrupted plan (same R and contraction choice).
 *   Synchronises.
 * Errors: MK_ERR_ARG (NULL, short blob, a blob of another shape or storage,
 * inconsistent counters), MK_ERR_STATE (no focal points set; R not loaded;
 * recording mismatch), MK_ERR_OOM, MK_ERR_HIP.
 */
mk_status mk_state_bytes(mk_plan_t plan, size_t* bytes);
mk_status mk_get_state(mk_plan_t plan, void* blob, size_t bytes);
mk_status mk_set_state(mk_plan_t plan, const void* blob, size_t bytes);

mk_status mk_destroy(mk_plan_t plan);

/* mk_strerror -- static description of a status code (an mk_status value;
 * any other value gives "unknown status"). */
const char* mk_strerror(int32_t status);

/* mk_last_error -- message of the plan's last failure ("" if none); with a
 * NULL plan, the message of the last failed mk_plan on this thread. */
const char* mk_last_error(mk_plan_t plan);

/* mk_device_checks -- the device-side bounds checks of the checked build
 * (the same library compiled with -DMK_DEVICE_CHECKS: every kernel compares
 * the end of each range of a buffer it reads or writes with the end of the
 * allocation behind the pointer it was given).  Waits for the device, then
 * writes to *violations a bit mask of the kernel files whose checks failed
 * since the last call (bit 0: per-trace kernels, 1: streaming contraction,
 * 2: matrix-core contraction, 3: network, 4: series tail) and clears them.
 * MK_ERR_UNSUPPORTED from a library built without the checks; MK_ERR_ARG if
 * violations is NULL; MK_ERR_HIP if the device reports an error.  It reads
 * no plan; it is for debugging runs, as the host sanitizer build is for the
 * host code. */
mk_status mk_device_checks(uint32_t* violations);

#ifdef __cplusplus
}
#endif

#endif /* MK_H */
