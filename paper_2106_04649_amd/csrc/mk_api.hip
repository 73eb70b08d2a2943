// Host side of the C ABI declared in include/mk.h: plan validation, device
// memory, the order of kernel launches for Algorithm 1, contraction
// selection (heuristic, forced or autotuned) and status codes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <numeric>
#include <sstream>

#include "mk_internal.h"

// Bytes from `ptr` to the end of the device allocation behind it, for the
// checked build's kernel-side bounds checks (0 for a null pointer; unknown,
// which passes every check, in the normal build or when the runtime does not
// know the pointer).
int64_t device_extent(const void* ptr) {
#ifdef MK_DEVICE_CHECKS
    if (!ptr) return 0;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void*>(ptr)) != hipSuccess) {
        (void)hipGetLastError();
        return kExtentUnknown;
    }
    const int64_t ext = (int64_t)size - (int64_t)(static_cast<const char*>(ptr) - static_cast<const char*>(base));
    // a test hook: report extents this many bytes short, so that the checks
    // fire on accesses that are in bounds
    static const int64_t shrink = [] {
        const char* v = std::getenv("MK_CHECK_SHRINK");
        return v ? std::atoll(v) : 0LL;
    }();
    return ext - shrink;
#else
    (void)ptr;
    return kExtentUnknown;
#endif
}

namespace {

thread_local std::string g_plan_error;

const char* kStatusText[] = {
    "success",
    "invalid argument",
    "call out of order",
    "device memory exhausted",
    "HIP runtime error",
    "unsupported request",
    "series diverged (norm non-finite or above the divergence threshold)",
};

mk_status fail(mk_plan_t p, mk_status st, const std::string& msg) {
    if (p) p->err = msg; else g_plan_error = msg;
    return st;
}

mk_status hip_fail(mk_plan_t p, hipError_t e, const char* where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(p, e == hipErrorOutOfMemory ? MK_ERR_OOM : MK_ERR_HIP, m);
}

#define HIP_TRY(p, expr)                                          \
    do {                                                          \
        hipError_t e_ = (expr);                                   \
        if (e_ != hipSuccess) return hip_fail((p), e_, #expr);    \
    } while (0)

#define MK_TRY(expr)                          \
    do {                                      \
        mk_status st_ = (expr);               \
        if (st_ != MK_OK) return st_;         \
    } while (0)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

template <typename T>
hipError_t dalloc(T** ptr, size_t count) {
    *ptr = nullptr;
    if (count == 0) return hipSuccess;
    return hipMalloc(reinterpret_cast<void**>(ptr), count * sizeof(T));
}

void drop_graphs(mk_plan_t p) {
    for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
    p->graphs.clear();
}

void free_plan_memory(mk_plan_t p) {
    drop_graphs(p);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    if (p->copy_stream) {
        (void)hipStreamSynchronize(p->copy_stream);
        (void)hipStreamDestroy(p->copy_stream);
    }
    for (int b = 0; b < 2; ++b) {
        if (p->rbuf[b]) (void)hipFree(p->rbuf[b]);
        if (p->ev_copied[b]) (void)hipEventDestroy(p->ev_copied[b]);
        if (p->ev_consumed[b]) (void)hipEventDestroy(p->ev_consumed[b]);
    }
    if (p->R_host) (void)hipHostFree(p->R_host);
    if (p->hpin) (void)hipHostFree(p->hpin);
    void* bufs[] = {p->R, p->rscale, p->X, p->Y, p->f1p, p->f1m, p->gp, p->gm, p->stage, p->itd,
                    p->fband, p->perm, p->iperm, p->ncols, p->npart, p->norm0, p->gdnorm, p->nlast, p->xscale,
                    p->norms, p->tw, p->flag, p->n0, p->hist, p->tail_w, p->tail_x, p->tail_work,
                    p->tail_y, p->tail_scale, p->img, p->aux, p->tail_wpk, p->norm_log, p->fnorm,
                    p->walk_items[0], p->walk_items[1]};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (auto& pe : p->pending) {
        (void)hipEventDestroy(pe.a);
        (void)hipEventDestroy(pe.b);
    }
    for (auto e : p->event_pool) (void)hipEventDestroy(e);
}

// --- profiling ------------------------------------------------------------

hipError_t prof_begin(mk_plan_t p, hipEvent_t* a) {
    if (!(p->d.flags & MK_FLAG_PROFILE)) return hipSuccess;
    if (p->event_pool.empty()) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        p->event_pool.push_back(e);
    }
    *a = p->event_pool.back();
    p->event_pool.pop_back();
    return hipEventRecord(*a, p->stream);
}

hipError_t prof_end(mk_plan_t p, hipEvent_t a, int kind) {
    if (!(p->d.flags & MK_FLAG_PROFILE)) return hipSuccess;
    hipEvent_t b;
    if (p->event_pool.empty()) {
        hipError_t err = hipEventCreate(&b);
        if (err != hipSuccess) return err;
    } else {
        b = p->event_pool.back();
        p->event_pool.pop_back();
    }
    hipError_t err = hipEventRecord(b, p->stream);
    p->pending.push_back({a, b, kind});
    return err;
}

hipError_t prof_resolve(mk_plan_t p) {
    if (p->pending.empty()) return hipSuccess;
    hipError_t err = hipStreamSynchronize(p->stream);
    if (err != hipSuccess) return err;
    for (auto& pe : p->pending) {
        float ms = 0.f;
        err = hipEventElapsedTime(&ms, pe.a, pe.b);
        if (err != hipSuccess) return err;
        p->prof[pe.kind].ms += ms;
        p->prof[pe.kind].launches += 1;
        p->event_pool.push_back(pe.a);
        p->event_pool.push_back(pe.b);
    }
    p->pending.clear();
    return hipSuccess;
}

// --- contraction selection -------------------------------------------------

constexpr int kGemvMaxCols = 4;

int xprec_of(int rprec, int variant, bool fast_x = false) {
    if (variant == 0) return XP_F32;                     // GEMV keeps X in FP32
    if (rprec == MK_R_F16S) return fast_x ? XP_F16 : XP_F16X2;
    if (rprec == MK_R_BF16S) return fast_x ? XP_BF16 : XP_BF16X2;
    return XP_F32;
}

int heuristic_variant(mk_plan_t p, int ncols) {
    if (p->r_tiled) {                    // LDS-staged tiles, the only readers of tiled R
        if (ncols <= 16) return 1 + 7;   // 32 focal-real rows x 256 receivers
        // one 16-bit plane of X leaves room for 128 x 256 tiles (barrier after
        // every other chunk): 451 against 475 us at 601^2 and 64 columns, 9.36
        // against 9.76 ms at 2001^2 and 256 columns
        if (ncols >= 48 && p->d.rprec != MK_R_C64 && (p->d.flags & MK_FLAG_FAST_X)) return 1 + 5;
        return 1 + 6;                    // 64 x 256
    }
    if (ncols <= kGemvMaxCols) return 0;
    if (ncols <= 16) return 1 + 3;       // 32 focal-real rows x 128 receivers
    return 1 + 6;                        // LDS-staged, 64 focal-real rows x 256 receivers
}

// whether contraction variant v can read the plan's layout of R
bool variant_fits(mk_plan_t p, int v) { return contract_variant_reads_tiled(v) || !p->r_tiled; }

void set_contract_extents(ContractArgs& c) {
    c.ext_r = device_extent(c.R);
    c.ext_x = device_extent(c.X);
    c.ext_y = device_extent(c.Y);
}

ContractArgs contract_args(mk_plan_t p, const void* X, int ncols, int ncols_mul) {
    ContractArgs c{};
    c.R = p->R;
    c.rscale = p->rscale;
    c.prec = p->d.rprec;
    c.X = X;
    c.Y = p->Y;
    c.ncols_w = p->has_fband ? p->ncols : nullptr;
    c.ncols_mul = ncols_mul;
    c.xsplit = 0;
    c.tiled = p->r_tiled ? 1 : 0;
    c.nr = p->d.nr;
    c.ns = p->d.ns;
    c.ns_pad = p->ns_pad;
    c.B = p->B;
    c.ncols = ncols;
    c.nb = p->B;
    set_contract_extents(c);
    return c;
}

hipError_t launch_choice(ContractArgs c, int variant, hipStream_t s) {
    if (variant == 0) return c.tiled ? hipErrorInvalidValue : launch_contract_gemv(c, s);
    return launch_contract_mfma(c, variant - 1, s);
}

std::string tune_key(mk_plan_t p, int ncols) {
    char buf[160];
    std::snprintf(buf, sizeof(buf), "gfx950 nr=%d ns_pad=%d B=%d prec=%d ncols=%d banded=%d",
                  p->d.nr, p->ns_pad, p->B, p->d.rprec, ncols, p->has_fband ? 1 : 0);
    return buf;
}

// Time every candidate that consumes the same X storage on the plan's
// current X (the results are overwritten by the real launch that follows)
// and keep the fastest.  The choice is cached in the plan and, when the
// environment variable MK_TUNE_CACHE names a file, appended to that file.
mk_status autotune(mk_plan_t p, const void* Xbuf, const float* xs, int ncols, int ncols_mul,
                   int xprec, int* out) {
    for (auto& kv : p->tuned)
        if (kv.first == ncols) {
            *out = kv.second;
            return MK_OK;
        }
    const char* path = std::getenv("MK_TUNE_CACHE");
    const std::string key = tune_key(p, ncols);
    if (path) {
        std::ifstream in(path);
        std::string line;
        while (std::getline(in, line)) {
            const size_t bar = line.rfind('|');
            if (bar != std::string::npos && line.substr(0, bar) == key) {
                const int v = std::atoi(line.c_str() + bar + 1);
                if (v >= 0 && v <= contract_mfma_variants() && variant_fits(p, v) &&
                    xprec_of(p->d.rprec, v, (p->d.flags & MK_FLAG_FAST_X) != 0) == xprec) {
                    p->tuned.push_back({ncols, v});
                    *out = v;
                    return MK_OK;
                }
            }
        }
    }
    std::vector<int> cands;
    const bool fast = (p->d.flags & MK_FLAG_FAST_X) != 0;
    if (xprec_of(p->d.rprec, 0, fast) == xprec && ncols <= 2 * kGemvMaxCols && variant_fits(p, 0))
        cands.push_back(0);
    for (int v = 0; v < contract_mfma_variants(); ++v)
        if (xprec_of(p->d.rprec, 1 + v, fast) == xprec && variant_fits(p, 1 + v)) cands.push_back(1 + v);
    hipEvent_t e0, e1;
    HIP_TRY(p, hipEventCreate(&e0));
    HIP_TRY(p, hipEventCreate(&e1));
    float best = 1e30f;
    int best_v = cands.empty() ? 0 : cands[0];
    for (int v : cands) {
        ContractArgs c = contract_args(p, Xbuf, ncols, ncols_mul);
        c.xscale = xs;
        c.xsplit = (xprec == XP_F16X2 || xprec == XP_BF16X2) ? 1 : 0;
        HIP_TRY(p, launch_choice(c, v, p->stream));     // warm
        HIP_TRY(p, hipEventRecord(e0, p->stream));
        for (int rep = 0; rep < 2; ++rep) HIP_TRY(p, launch_choice(c, v, p->stream));
        HIP_TRY(p, hipEventRecord(e1, p->stream));
        HIP_TRY(p, hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(p, hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
            best = ms;
            best_v = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->tuned.push_back({ncols, best_v});
    if (path) {
        std::ofstream o(path, std::ios::app);
        if (o) o << key << "|" << best_v << "\n";
    }
    *out = best_v;
    return MK_OK;
}

// The contraction used for ncols columns; the X storage follows from it.
ContractChoice choose(mk_plan_t p, int ncols) {
    ContractChoice ch;
    ch.variant = p->tune_mode >= 0 ? p->tune_mode : heuristic_variant(p, ncols);
    ch.xprec = xprec_of(p->d.rprec, ch.variant, (p->d.flags & MK_FLAG_FAST_X) != 0);
    return ch;
}

// --- pieces of the series -------------------------------------------------

TraceArgs trace_args(mk_plan_t p, int nfo) {
    TraceArgs a{};
    a.Y = p->Y;
    a.X = p->X;
    a.f1p = p->f1p;
    a.f1m = p->f1m;
    a.gp = p->gp;
    a.gm = p->gm;
    a.aux = p->aux;
    a.itd = p->itd;
    a.fband = p->has_fband ? p->fband : nullptr;
    a.npart = p->npart;
    a.tw = p->tw;
    a.xs_in = nullptr;
    a.xs_out = p->xscale;
    a.xprec = XP_F32;
    a.skip_outband = 0;
    a.n0 = p->n0;
    a.hist = nullptr;
    a.hist_k = p->hist_k;
    a.hist_T = p->hist_T;
    a.rec_slot = -1;
    a.nr = p->d.nr;
    a.nf = p->nf;
    a.nfo = nfo;
    a.lo = p->d.iw_lo;
    a.B = p->B;
    a.ns_pad = p->ns_pad;
    a.shift = p->shift;
    a.scale = (float)(p->d.dx * p->d.dt / (double)p->M);
    return a;
}

// Streamed R: slab `slab` (bins [slab * slab_bins, ...)) into device buffer
// `buf` on the copy stream, after the last contraction that read that buffer;
// nothing to do when the buffer already holds it or is receiving it.
mk_status slab_in(mk_plan_t p, int slab, int buf) {
    if (p->buf_slab[buf] == slab) return MK_OK;
    const int w0 = slab * p->slab_bins;
    const int nb = std::min(p->slab_bins, p->B - w0);
    HIP_TRY(p, hipStreamWaitEvent(p->copy_stream, p->ev_consumed[buf], 0));
    HIP_TRY(p, hipMemcpyAsync(p->rbuf[buf], p->R_host + (size_t)w0 * p->bin_bytes, (size_t)nb * p->bin_bytes,
                              hipMemcpyHostToDevice, p->copy_stream));
    HIP_TRY(p, hipEventRecord(p->ev_copied[buf], p->copy_stream));
    p->buf_slab[buf] = slab;
    return MK_OK;
}

// One contraction over streamed R, slab by slab: each slab's launch covers
// its bins (R, scales, X, Y and the active counts offset to its first bin,
// X and Y keeping the strides of the whole band) and waits for its copy;
// the next slab (after the last, the first one of the next contraction)
// is copied into the other buffer meanwhile.  The per-bin arithmetic is that
// of the resident plan.
mk_status contract_streamed(mk_plan_t p, const ContractArgs& c, int variant, int xprec) {
    const size_t xbin = (size_t)p->ns_pad * (xprec == XP_F32 ? sizeof(float2) : sizeof(uint32_t));
    for (int j = 0; j < p->nslabs; ++j) {
        const int buf = (int)(p->slab_use & 1);
        const int w0 = j * p->slab_bins;
        MK_TRY(slab_in(p, j, buf));
        HIP_TRY(p, hipStreamWaitEvent(p->stream, p->ev_copied[buf], 0));
        ContractArgs cj = c;
        cj.R = p->rbuf[buf];
        cj.rscale = c.rscale + w0;
        cj.X = static_cast<const unsigned char*>(c.X) + (size_t)w0 * xbin;
        cj.Y = c.Y + (size_t)w0 * c.nr;
        cj.ncols_w = c.ncols_w ? c.ncols_w + w0 : nullptr;
        cj.nb = std::min(p->slab_bins, p->B - w0);
        set_contract_extents(cj);
        HIP_TRY(p, launch_choice(cj, variant, p->stream));
        HIP_TRY(p, hipEventRecord(p->ev_consumed[buf], p->stream));
        ++p->slab_use;
        MK_TRY(slab_in(p, (j + 1) % p->nslabs, buf ^ 1));
    }
    return MK_OK;
}

mk_status run_contract(mk_plan_t p, const ContractChoice& ch, const void* Xbuf, const float* xs,
                       int ncols, int ncols_mul, int kind) {
    int variant = ch.variant;
    if (p->tune_mode == -2) MK_TRY(autotune(p, Xbuf, xs, ncols, ncols_mul, ch.xprec, &variant));
    ContractArgs c = contract_args(p, Xbuf, ncols, ncols_mul);
    c.xscale = xs;
    c.xsplit = (ch.xprec == XP_F16X2 || ch.xprec == XP_BF16X2) ? 1 : 0;
    const int wk = ncols_mul == 2 ? 1 : 0;      // the series' list, or the G assembly's
    if (p->walk_variant[wk] == variant && ncols == (wk + 1) * p->nf) {
        c.items = p->walk_items[wk];
        c.walk_blocks_per_xcd = p->walk_blocks_per_xcd;
    }
    hipEvent_t ev = nullptr;
    HIP_TRY(p, prof_begin(p, &ev));
    if (p->r_stream) MK_TRY(contract_streamed(p, c, variant, ch.xprec));
    else HIP_TRY(p, launch_choice(c, variant, p->stream));
    HIP_TRY(p, prof_end(p, ev, kind));
    return MK_OK;
}

mk_status run_trace(mk_plan_t p, int mode, const TraceArgs& a0, int kind) {
    TraceArgs a = a0;
    const void* bufs[TE_COUNT] = {a.Y, a.X, a.src, a.f1p, a.f1m, a.gp, a.gm, a.aux, a.n0, a.hist};
    for (int i = 0; i < TE_COUNT; ++i) a.ext[i] = device_extent(bufs[i]);
    hipEvent_t ev = nullptr;
    HIP_TRY(p, prof_begin(p, &ev));
    HIP_TRY(p, launch_trace(mode, p->d.nt, a, p->stream));
    HIP_TRY(p, prof_end(p, ev, kind));
    return MK_OK;
}

mk_status run_norms(mk_plan_t p, double* out) {
    hipEvent_t ev = nullptr;
    HIP_TRY(p, prof_begin(p, &ev));
    HIP_TRY(p, launch_norm_reduce(p->npart, p->d.nr, p->nf, out, p->nlast, p->stream));
    HIP_TRY(p, prof_end(p, ev, 2));
    return MK_OK;
}

mk_status ensure_norm_cap(mk_plan_t p, int niter) {
    if (niter <= p->norm_cap) return MK_OK;
    int cap = p->norm_cap > 0 ? p->norm_cap : 64;
    while (cap < niter) cap *= 2;
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    drop_graphs(p);                    // captured passes point into the old buffer
    if (p->norms) HIP_TRY(p, hipFree(p->norms));
    p->norms = nullptr;
    p->norm_cap = 0;
    HIP_TRY(p, dalloc(&p->norms, (size_t)cap * p->d.nf_max));
    p->norm_cap = cap;
    return MK_OK;
}

// Room for `rows` more rows of the norm log (copied over when it grows).
mk_status ensure_log_cap(mk_plan_t p, int rows) {
    const int need = p->log_len + rows;
    if (need <= p->log_cap) return MK_OK;
    int cap = p->log_cap > 0 ? p->log_cap : 128;
    while (cap < need) cap *= 2;
    double* fresh = nullptr;
    HIP_TRY(p, dalloc(&fresh, (size_t)cap * p->d.nf_max));
    if (p->norm_log) {
        if (p->log_len > 0) {
            hipError_t e = hipMemcpyAsync(fresh, p->norm_log, (size_t)p->log_len * p->nf * sizeof(double),
                                          hipMemcpyDeviceToDevice, p->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
            if (e != hipSuccess) {
                (void)hipFree(fresh);
                return hip_fail(p, e, "norm log copy");
            }
        }
        HIP_TRY(p, hipFree(p->norm_log));
    }
    p->norm_log = fresh;
    p->log_cap = cap;
    return MK_OK;
}

// Small device-to-host reads go through a pinned buffer: into pageable
// memory the runtime completes every copy on its own before the call
// returns, into pinned memory several copies queue behind one
// synchronisation.  Returns the buffer, grown to hold `doubles` values.
mk_status pinned(mk_plan_t p, size_t doubles, double** out) {
    if (doubles > p->hpin_cap) {
        HIP_TRY(p, hipStreamSynchronize(p->stream));
        if (p->hpin) HIP_TRY(p, hipHostFree(p->hpin));
        p->hpin = nullptr;
        p->hpin_cap = 0;
        const size_t cap = std::max<size_t>(doubles, 4096);
        HIP_TRY(p, hipHostMalloc(reinterpret_cast<void**>(&p->hpin), cap * sizeof(double), hipHostMallocDefault));
        p->hpin_cap = cap;
    }
    *out = p->hpin;
    return MK_OK;
}

// Append `rows` rows of nf norms from device memory to the log.
mk_status log_rows(mk_plan_t p, const double* src, int rows) {
    if (rows <= 0) return MK_OK;
    MK_TRY(ensure_log_cap(p, rows));
    HIP_TRY(p, hipMemcpyAsync(p->norm_log + (size_t)p->log_len * p->nf, src, (size_t)rows * p->nf * sizeof(double),
                              hipMemcpyDeviceToDevice, p->stream));
    p->log_len += rows;
    return MK_OK;
}

// A new series starts from the field whose norms (nf, device) are `start`.
mk_status log_series_start(mk_plan_t p, const double* start) {
    p->prev_series_start = p->series_start;
    p->series_start = p->log_len;
    return log_rows(p, start, 1);
}

// Outside its mute window f1+ keeps N_-1 and f1- stays zero (every pass,
// tail and restart writes inside the window only), so the judge reads the
// windows alone and adds these sums of squares of N_-1 outside them.
// `src`: N_-1 or G_d (the window is symmetric in t), plan order.  Leaves
// ||src|| per focal point in p->norm0 and p->nlast (whole traces).
mk_status outside_window_norms(mk_plan_t p, const float* src, int nf, int32_t shift) {
    const int nr = p->d.nr, ntr = nf * nr;
    HIP_TRY(p, launch_sumsq_out(src, ntr, p->d.nt, p->itd, shift, p->npart, p->npart + ntr, p->stream));
    HIP_TRY(p, launch_norm_reduce(p->npart, nr, nf, p->norm0, p->nlast, p->stream));
    HIP_TRY(p, launch_norm_reduce(p->npart + ntr, nr, nf, p->fnorm, nullptr, p->stream));
    return MK_OK;
}

// The stopping rule.  a[0..n) are the norms of one focal point's terms in the
// current series (a[0] its starting field); a[n-1] is the last term added.
// The series contracts by q per pass: the largest of the last two
// term-to-term ratios, or `q_prior` (the previous series' value, the same
// operator) while this series holds fewer than two terms.  If the remaining
// terms keep shrinking by q, their norms sum to at most
//     rest = a[n-1] q / (1 - q),
// and every output's error is a part of that sum (the odd terms go to f1+,
// the even ones to f1-, and G+ and G- are syntheses of f1+-, with S a
// contraction).  q is capped at 0.95; a negative q means "not known yet".
struct RestEstimate {
    double rest;
    double q;
};

RestEstimate estimate_rest(const double* a, int n, double q_prior) {
    double q = -1.0;
    for (int j = std::max(1, n - 2); j < n; ++j)
        if (a[j - 1] > 0.0) q = std::max(q, a[j] / a[j - 1]);
    if (q < 0.0) q = q_prior;
    if (a[n - 1] == 0.0) return {0.0, std::max(q, 0.0)};
    if (q < 0.0) return {HUGE_VAL, -1.0};
    q = std::min(q, 0.95);
    return {a[n - 1] * q / (1.0 - q), q};
}

// The rule for every focal point: est[j] = rest / min(||f1+||, ||f1-||) in the
// plan's sorted order, and the passes still needed, predicted from q (0 when
// every estimate is within tol, -1 when some q is not known yet).
mk_status judge_series(mk_plan_t p, double tol, std::vector<double>& est, int* more, int check_from) {
    const int nf = p->nf, nr = p->d.nr, nt = p->d.nt;
    HIP_TRY(p, launch_sumsq2_win(p->f1p, p->f1m, nf * nr, nt, p->itd, p->shift, p->npart, p->stream));
    HIP_TRY(p, launch_norm_reduce(p->npart, nr, 2 * nf, p->fnorm, nullptr, p->stream));
    double* h = nullptr;
    MK_TRY(pinned(p, 2 * (size_t)nf + (size_t)p->log_len * nf, &h));
    const double* fn = h;
    const double* log = h + 2 * nf;
    HIP_TRY(p, hipMemcpyAsync(h, p->fnorm, 2 * (size_t)nf * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    if (p->log_len > 0)
        HIP_TRY(p, hipMemcpyAsync(h + 2 * nf, p->norm_log, (size_t)p->log_len * nf * sizeof(double),
                                  hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    // the divergence check of the passes since row check_from (mk_iterate's,
    // on the same rows of the log)
    for (int e = std::max(check_from, 0); check_from >= 0 && e < p->log_len; ++e)
        for (int j = 0; j < nf; ++j) {
            const double v = log[(size_t)e * nf + j];
            const int f = p->perm_host[j];
            if (!std::isfinite(v) || v > p->d.div_factor * p->norm0_host[f]) {
                char buf[160];
                std::snprintf(buf, sizeof(buf), "mk_iterate_tol: ||N|| = %g at pass %d, focal %d (||N_-1|| = %g)", v,
                              p->passes - (p->log_len - e), f, p->norm0_host[f]);
                return fail(p, MK_ERR_DIVERGED, buf);
            }
        }
    est.assign(nf, 0.0);
    *more = 0;
    const int n = p->log_len - p->series_start;
    std::vector<double> a;
    for (int j = 0; j < nf; ++j) {
        double q_prior = -1.0;
        if (p->series_start >= 2) {         // the previous series' last ratios
            a.clear();
            for (int e = p->prev_series_start; e < p->series_start; ++e) a.push_back(log[(size_t)e * nf + j]);
            q_prior = estimate_rest(a.data(), (int)a.size(), -1.0).q;
        }
        a.clear();
        for (int e = p->series_start; e < p->log_len; ++e) a.push_back(log[(size_t)e * nf + j]);
        const RestEstimate r = estimate_rest(a.data(), n, q_prior);
        const double fp = std::sqrt(fn[j] * fn[j] + p->f1p_out2_host[j]);     // ||f1+||, ||f1-||
        const double den = std::min(fp, fn[nf + j]);
        if (r.rest == 0.0) {
            est[j] = 0.0;
            continue;
        }
        est[j] = den > 0.0 ? r.rest / den : HUGE_VAL;
        if (est[j] <= tol) continue;
        if (r.q < 0.0 || !(den > 0.0)) {
            *more = -1;
            continue;
        }
        // passes m with a[n-1] q^m q / (1 - q) <= tol den
        const int m = r.q > 0.0 ? (int)std::ceil(std::log(tol * den / r.rest) / std::log(r.q)) : 1;
        if (*more >= 0) *more = std::max(*more, std::max(m, 1));
    }
    return MK_OK;
}

template <typename T>
mk_status copy_in(mk_plan_t p, T* dst, const T* src, size_t n, int on_device, const char* what) {
    if (n == 0) return MK_OK;
    hipError_t e = hipMemcpyAsync(dst, src, n * sizeof(T),
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                  p->stream);
    if (e != hipSuccess) return hip_fail(p, e, what);
    return MK_OK;
}

// G+ and G- from one batched synthesis of the interleaved columns
// [f1+[0], f1-(-t)[0], f1+[1], ...].  Their spectra go to X slabs
// [nf, 3 nf): slabs [0, nf) hold the spectrum of the last N_i, which the
// next pass of the series still needs.
mk_status assemble_G(mk_plan_t p) {
    const int nf = p->nf;
    TraceArgs a = trace_args(p, 2 * nf);
    float2* Xg = p->X + (size_t)nf * p->B * p->ns_pad;
    a.X = Xg;
    a.xprec = p->g_choice.xprec;
    a.xs_in = p->gdnorm;      // f1+ and f1- stay on the scale of G_d (norm0 may hold a restart residual)
    a.xs_out = p->xscale + nf;
    a.skip_outband = (p->g_choice.variant != 0 && p->has_fband) ? 1 : 0;
    MK_TRY(run_trace(p, TM_GFWD, a, 4));
    MK_TRY(run_contract(p, p->g_choice, Xg, p->xscale + nf, 2 * nf, 2, 4));
    MK_TRY(run_trace(p, TM_GOUT, a, 4));
    p->g_valid = true;
    return MK_OK;
}

// f2+ and p- (Algorithm 1, second loop) into p->aux.  f2+ = f1+ - f1-(-t)
// holds every N_i; p- = S[f2+ - N_last] comes from the G assembly's two
// syntheses and one synthesis of the last N, whose spectrum X still holds.
// After a tail or restart the fields are no longer partial sums of one
// series, so both are refused there.
mk_status aux_field(mk_plan_t p, int field) {
    if (p->tail_applied && field != MK_GTOTAL)
        return fail(p, MK_ERR_STATE, "mk_get: f2+ and p- are defined for a plain series (no tail applied)");
    if (!p->aux) {
        HIP_TRY(p, hipStreamSynchronize(p->stream));
        HIP_TRY(p, dalloc(&p->aux, (size_t)p->d.nf_max * p->d.nr * p->d.nt));
    }
    if (field == MK_GTOTAL) {
        // p- + S[N_last] + f2+(-t) = G+ + G- (Algorithm 1's signs): the sum of
        // the two assembled fields, without a third synthesis
        if (!p->g_valid) MK_TRY(assemble_G(p));
        HIP_TRY(p, launch_gsum(p->gp, p->gm, (int64_t)p->nf * p->d.nr * p->d.nt, p->aux, p->stream));
        return MK_OK;
    }
    if (field == MK_F2PLUS) {
        HIP_TRY(p, launch_f2p(p->f1p, p->f1m, (int64_t)p->nf * p->d.nr, p->d.nt, p->aux, p->stream));
        return MK_OK;
    }
    if (!p->g_valid) MK_TRY(assemble_G(p));
    MK_TRY(run_contract(p, p->series_choice, p->X, p->xscale, p->nf, 1, 4));
    TraceArgs a = trace_args(p, p->nf);
    MK_TRY(run_trace(p, TM_POUT, a, 4));
    return MK_OK;
}

// The lists of active tiles for the series' and the G
// assembly's contraction choices (when they are LDS-staged tiles): tile
// (w, rt, ft) is active when focal tile ft starts below the bin's active
// column count (all nf, or the band prefix ncols_host[w]).  Ascending tile
// indices, (w rtiles + rt) ftiles + ft, the order of the grid form.
mk_status build_walk(mk_plan_t p) {
    p->walk_variant[0] = p->walk_variant[1] = -1;
    // always with MK_FLAG_WALK; by default whenever per-focal bands are set,
    // where it also balances the XCDs (the grid form deals contiguous runs of
    // bins to them, and the low bins hold most of the active tiles)
    const bool walk = (p->d.flags & MK_FLAG_WALK) ||
                      (p->has_fband && !p->r_stream && !(p->d.flags & MK_FLAG_GRID));
    if (!walk) return MK_OK;
    const ContractChoice* ch[2] = {&p->series_choice, &p->g_choice};
    for (int k = 0; k < 2; ++k) {
        const int nfb = contract_variant_focal_tile(ch[k]->variant);
        if (nfb == 0) continue;                   // not an LDS-staged choice
        const bool xsplit = ch[k]->xprec == XP_F16X2 || ch[k]->xprec == XP_BF16X2;
        const int rcv = contract_lds_receivers(ch[k]->variant, xsplit, p->d.nr);
        const int rtiles = (p->d.nr + rcv - 1) / rcv;
        if (!p->walk_items[k]) {
            // sized once for the largest list (every tile of the narrowest
            // LDS-staged tiles, 16 focal columns x 128 receivers), so
            // captured graphs keep a valid address across focal sets
            const size_t rmax = (size_t)(p->d.nr + 127) / 128;
            const size_t cap = 1 + (size_t)p->B * rmax * (((size_t)(k + 1) * p->d.nf_max + 15) / 16);
            HIP_TRY(p, hipStreamSynchronize(p->stream));
            HIP_TRY(p, dalloc(&p->walk_items[k], cap));
        }
        const int mul = k + 1, ncols = mul * p->nf;
        const int ftiles = (ncols + nfb - 1) / nfb;
        std::vector<int32_t> items(1, 0);
        for (int w = 0; w < p->B; ++w) {
            const int nact = p->has_fband ? std::min(p->ncols_host[w] * mul, ncols) : ncols;
            const int fa = (nact + nfb - 1) / nfb;
            for (int rt = 0; rt < rtiles; ++rt)
                for (int ft = 0; ft < fa; ++ft) items.push_back((w * rtiles + rt) * ftiles + ft);
        }
        items[0] = (int32_t)(items.size() - 1);
        HIP_TRY(p, hipMemcpyAsync(p->walk_items[k], items.data(), items.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, p->stream));
        HIP_TRY(p, hipStreamSynchronize(p->stream));      // the host list goes out of scope
        p->walk_variant[k] = ch[k]->variant;
    }
    return MK_OK;
}

// mk_load_R for streamed R: one slab of bins at a time, the caller's rows of
// those bins (a 2D region of R[r][w][s]) go to a device staging buffer, the
// resident path's repack / quantisation kernels write the slab's device
// layout into slab buffer 0 (the per-frequency scales need only the slab's
// own bins), and the slab goes down to its place in the pinned host copy.
mk_status load_R_streamed(mk_plan_t p, const float* R, int on_device) {
    const mk_plan_desc& d = p->d;
    HIP_TRY(p, hipStreamSynchronize(p->copy_stream));      // no copy may still read the slab buffers
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    p->buf_slab[0] = p->buf_slab[1] = -1;
    float* staging = nullptr;
    HIP_TRY(p, dalloc(&staging, 2 * (size_t)d.nr * p->slab_bins * d.ns));
    const size_t pitch = (size_t)p->B * d.ns * sizeof(float2);      // one receiver row of the caller's R
    hipError_t e = hipMemsetAsync(p->flag, 0, sizeof(int), p->stream);
    for (int j = 0; j < p->nslabs && e == hipSuccess; ++j) {
        const int w0 = j * p->slab_bins;
        const int nb = std::min(p->slab_bins, p->B - w0);
        const size_t width = (size_t)nb * d.ns * sizeof(float2);
        e = hipMemcpy2DAsync(staging, width, R + (size_t)w0 * d.ns * 2, pitch, width, d.nr,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, p->stream);
        if (e != hipSuccess) break;
        if (p->r_tiled) {
            if (d.rprec != MK_R_C64) e = launch_rscale(staging, p->rscale + w0, d.nr, nb, d.ns, p->flag, p->stream);
            if (e == hipSuccess)
                e = launch_repack_tiled(d.rprec, staging, p->rbuf[0], p->rscale + w0, d.nr, nb, d.ns, p->ns_pad,
                                        p->flag, p->stream);
        } else if (d.rprec == MK_R_C64) {
            e = launch_repack_c64(staging, reinterpret_cast<float2*>(p->rbuf[0]), d.nr, nb, d.ns, p->ns_pad,
                                  p->flag, p->stream);
        } else {
            e = launch_quantize_R(d.rprec, staging, p->rbuf[0], p->rscale + w0, d.nr, nb, d.ns, p->ns_pad,
                                  p->flag, p->stream);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->R_host + (size_t)w0 * p->bin_bytes, p->rbuf[0], (size_t)nb * p->bin_bytes,
                               hipMemcpyDeviceToHost, p->stream);
    }
    int h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    (void)hipFree(staging);
    if (e != hipSuccess) return hip_fail(p, e, "mk_load_R: streamed repack");
    // the slab buffers were written by the compute stream: later copies into
    // them wait for that work (done: the stream is synchronised)
    for (int b = 0; b < 2; ++b) HIP_TRY(p, hipEventRecord(p->ev_consumed[b], p->stream));
    if (h) {
        p->R_loaded = false;
        return fail(p, MK_ERR_ARG, "mk_load_R: R holds a non-finite value");
    }
    p->R_loaded = true;
    p->focal_set = false;
    p->g_valid = false;
    return MK_OK;
}

}  // namespace

extern "C" {

const char* mk_strerror(int32_t status) {
    // an int, not the enum: a caller may pass a value no enumerator names
    const int i = status;
    if (i < 0 || i >= (int)(sizeof(kStatusText) / sizeof(kStatusText[0]))) return "unknown status";
    return kStatusText[i];
}

const char* mk_last_error(mk_plan_t plan) {
    return plan ? plan->err.c_str() : g_plan_error.c_str();
}

mk_status mk_plan(const mk_plan_desc* desc, mk_plan_t* out) {
    g_plan_error.clear();
    if (!out) return fail(nullptr, MK_ERR_ARG, "mk_plan: out is NULL");
    *out = nullptr;
    if (!desc) return fail(nullptr, MK_ERR_ARG, "mk_plan: desc is NULL");
    const mk_plan_desc& d = *desc;
    if (d.nr < 1 || d.ns < 1) return fail(nullptr, MK_ERR_ARG, "mk_plan: nr and ns must be >= 1");
    if (d.nr != d.ns)
        return fail(nullptr, MK_ERR_ARG, "mk_plan: nr must equal ns (one shared surface grid)");
    if (d.ns > 4096) return fail(nullptr, MK_ERR_UNSUPPORTED, "mk_plan: ns above 4096");
    if (!is_pow2(d.nt) || d.nt < 16 || d.nt > 4096)
        return fail(nullptr, MK_ERR_ARG, "mk_plan: nt must be a power of two in [16, 4096]");
    if (d.iw_lo < 0 || d.iw_hi < d.iw_lo || d.iw_hi > d.nt / 2)
        return fail(nullptr, MK_ERR_ARG, "mk_plan: band must satisfy 0 <= iw_lo <= iw_hi <= nt/2");
    if (d.nf_max < 1) return fail(nullptr, MK_ERR_ARG, "mk_plan: nf_max must be >= 1");
    if (!(d.dt > 0.0) || !(d.dx > 0.0) || !std::isfinite(d.dt) || !std::isfinite(d.dx))
        return fail(nullptr, MK_ERR_ARG, "mk_plan: dt and dx must be finite and positive");
    if (std::isnan(d.div_factor)) return fail(nullptr, MK_ERR_ARG, "mk_plan: div_factor is NaN");
    if (d.rprec != MK_R_C64 && d.rprec != MK_R_F16S && d.rprec != MK_R_BF16S)
        return fail(nullptr, MK_ERR_ARG, "mk_plan: unknown rprec");
    if (d.rprec == MK_R_C64 && d.ns > 2048)
        return fail(nullptr, MK_ERR_UNSUPPORTED, "mk_plan: complex64 R supports ns <= 2048");
    if (d.flags & ~(MK_FLAG_GRAPH | MK_FLAG_PROFILE | MK_FLAG_AUTOTUNE | MK_FLAG_FAST_X | MK_FLAG_ROW_R |
                    MK_FLAG_WALK | MK_FLAG_GRID))
        return fail(nullptr, MK_ERR_ARG, "mk_plan: unknown flag bits");
    if ((d.flags & MK_FLAG_WALK) && (d.flags & MK_FLAG_GRID))
        return fail(nullptr, MK_ERR_ARG, "mk_plan: MK_FLAG_WALK and MK_FLAG_GRID exclude each other");
    if ((d.flags & MK_FLAG_WALK) && (d.flags & MK_FLAG_AUTOTUNE))
        return fail(nullptr, MK_ERR_UNSUPPORTED, "mk_plan: MK_FLAG_WALK excludes MK_FLAG_AUTOTUNE");
    const int B = d.iw_hi - d.iw_lo + 1;
    const int ns_pad = (d.ns + 31) & ~31;      // rows of whole 128-byte chunks in every precision
    const bool r_tiled = d.nf_max > kGemvMaxCols && !(d.flags & MK_FLAG_ROW_R);
    const size_t relem = d.rprec == MK_R_C64 ? sizeof(float2) : sizeof(uint32_t);
    const size_t rbytes = r_tiled ? tiled_R_bytes(d.rprec, d.nr, B, ns_pad) : (size_t)B * d.nr * ns_pad * relem;
    const size_t bin_bytes = rbytes / (size_t)B;
    const bool r_stream = d.r_dev_bytes > 0 && (size_t)d.r_dev_bytes < rbytes;
    int slab_bins = 0;
    if (r_stream) {
        slab_bins = (int)std::min<size_t>((size_t)d.r_dev_bytes / 2 / bin_bytes, (size_t)B);
        if (slab_bins < 1)
            return fail(nullptr, MK_ERR_ARG, "mk_plan: r_dev_bytes holds fewer than two bins of R (" +
                                                 std::to_string(2 * bin_bytes) + " bytes)");
        if (d.flags & (MK_FLAG_GRAPH | MK_FLAG_AUTOTUNE | MK_FLAG_WALK))
            return fail(nullptr, MK_ERR_UNSUPPORTED,
                        "mk_plan: streamed R (r_dev_bytes below the size of R) excludes MK_FLAG_GRAPH, "
                        "MK_FLAG_AUTOTUNE and MK_FLAG_WALK");
    }

    mk_plan_t p = new (std::nothrow) mk_plan_s();
    if (!p) return fail(nullptr, MK_ERR_OOM, "mk_plan: host allocation failed");
    p->d = d;
    if (!(p->d.div_factor > 0.0)) p->d.div_factor = 1e3;
    p->B = B;
    p->M = d.nt / 2;
    p->ns_pad = ns_pad;
    p->r_tiled = r_tiled;
    p->r_stream = r_stream;
    p->bin_bytes = bin_bytes;
    p->slab_bins = slab_bins;
    p->nslabs = r_stream ? (B + slab_bins - 1) / slab_bins : 0;
    p->stream = reinterpret_cast<hipStream_t>(d.stream);
    p->tune_mode = (d.flags & MK_FLAG_AUTOTUNE) ? -2 : -1;

    auto bail = [&](hipError_t e, const char* where) {
        std::string m = std::string("mk_plan: ") + where + ": " + hipGetErrorString(e);
        free_plan_memory(p);
        delete p;
        return fail(nullptr, e == hipErrorOutOfMemory ? MK_ERR_OOM : MK_ERR_HIP, m);
    };
    hipError_t e;
    if ((e = hipGetDevice(&p->device)) != hipSuccess) return bail(e, "hipGetDevice");
    if ((d.flags & MK_FLAG_GRAPH) && p->stream == nullptr) {
        // stream capture needs a non-null stream; the graph still runs on the null stream
        if ((e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking)) != hipSuccess)
            return bail(e, "capture stream");
    }
    const size_t nfm = (size_t)d.nf_max;
    const size_t trace = (size_t)d.nr * d.nt;
    if (r_stream) {
        if ((e = hipHostMalloc((void**)&p->R_host, rbytes, hipHostMallocDefault)) != hipSuccess)
            return bail(e, "pinned host R");
        for (int b = 0; b < 2; ++b) {
            if ((e = hipMalloc(&p->rbuf[b], (size_t)slab_bins * bin_bytes)) != hipSuccess)
                return bail(e, "R slab buffer");
            if ((e = hipEventCreateWithFlags(&p->ev_copied[b], hipEventDisableTiming)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&p->ev_consumed[b], hipEventDisableTiming)) != hipSuccess)
                return bail(e, "slab events");
        }
        // a second stream at the default priority carries the host-to-device copies
        if ((e = hipStreamCreateWithFlags(&p->copy_stream, hipStreamNonBlocking)) != hipSuccess)
            return bail(e, "copy stream");
        for (int b = 0; b < 2; ++b)
            if ((e = hipEventRecord(p->ev_consumed[b], p->stream)) != hipSuccess) return bail(e, "slab events");
    } else if ((e = hipMalloc(&p->R, rbytes)) != hipSuccess) {
        return bail(e, "R");
    }
    if ((e = dalloc(&p->rscale, (size_t)p->B)) != hipSuccess) return bail(e, "R scales");
    if ((e = dalloc(&p->X, 3 * nfm * p->B * p->ns_pad)) != hipSuccess) return bail(e, "X");
    if ((e = dalloc(&p->Y, 2 * nfm * p->B * d.nr)) != hipSuccess) return bail(e, "Y");
    if ((e = dalloc(&p->f1p, nfm * trace)) != hipSuccess) return bail(e, "f1+");
    if ((e = dalloc(&p->f1m, nfm * trace)) != hipSuccess) return bail(e, "f1-");
    if ((e = dalloc(&p->gp, nfm * trace)) != hipSuccess) return bail(e, "G+");
    if ((e = dalloc(&p->gm, nfm * trace)) != hipSuccess) return bail(e, "G-");
    if ((e = dalloc(&p->stage, nfm * trace)) != hipSuccess) return bail(e, "staging");
    if ((e = dalloc(&p->itd, 2 * nfm * d.nr)) != hipSuccess) return bail(e, "itd");
    if ((e = dalloc(&p->fband, nfm * 2)) != hipSuccess) return bail(e, "band");
    if ((e = dalloc(&p->perm, nfm)) != hipSuccess) return bail(e, "perm");
    if ((e = dalloc(&p->iperm, nfm)) != hipSuccess) return bail(e, "iperm");
    if ((e = dalloc(&p->ncols, (size_t)p->B)) != hipSuccess) return bail(e, "ncols");
    if ((e = dalloc(&p->npart, 2 * nfm * d.nr)) != hipSuccess) return bail(e, "norm partials");
    if ((e = dalloc(&p->norm0, nfm)) != hipSuccess) return bail(e, "norm0");
    if ((e = dalloc(&p->gdnorm, nfm)) != hipSuccess) return bail(e, "gdnorm");
    if ((e = dalloc(&p->nlast, nfm)) != hipSuccess) return bail(e, "nlast");
    if ((e = dalloc(&p->img, nfm)) != hipSuccess) return bail(e, "image");
    if ((e = dalloc(&p->fnorm, 2 * nfm)) != hipSuccess) return bail(e, "field norms");
    if ((e = dalloc(&p->xscale, 3 * nfm)) != hipSuccess) return bail(e, "X scales");
    if ((e = dalloc(&p->tw, (size_t)d.nt + 256)) != hipSuccess) return bail(e, "twiddles");
    if ((e = dalloc(&p->flag, 1)) != hipSuccess) return bail(e, "flag");
    if ((e = dalloc(&p->n0, nfm * trace)) != hipSuccess) return bail(e, "N_-1");
    {
        int cus = 0;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device)) != hipSuccess)
            return bail(e, "CU count");
        p->walk_blocks_per_xcd = 2 * std::max(1, cus / 8);     // two blocks of four waves per CU
    }
    // the padding columns of X (s >= ns) must read as zero
    if ((e = hipMemsetAsync(p->X, 0, 3 * nfm * p->B * p->ns_pad * sizeof(float2), p->stream)) !=
        hipSuccess)
        return bail(e, "clear X");
    if ((e = hipMemsetAsync(p->xscale, 0, 3 * nfm * sizeof(float), p->stream)) != hipSuccess)
        return bail(e, "clear X scales");
    std::vector<float2> tw(d.nt + 256);
    for (int k = 0; k < d.nt; ++k) {
        const double ang = -2.0 * M_PI * (double)k / (double)d.nt;
        tw[k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    for (int n = 0; n < 256; ++n) {          // W_256^{q k}, n = 16 q + k
        const double ang = -2.0 * M_PI * (double)((n >> 4) * (n & 15)) / 256.0;
        tw[d.nt + n] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    if ((e = hipMemcpyAsync(p->tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice,
                            p->stream)) != hipSuccess)
        return bail(e, "twiddle upload");
    if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return bail(e, "sync");
    *out = p;
    return MK_OK;
}

mk_status mk_load_R(mk_plan_t p, const float* R, int on_device) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_load_R: plan is NULL");
    if (!R) return fail(p, MK_ERR_ARG, "mk_load_R: R is NULL");
    if (p->r_stream) return load_R_streamed(p, R, on_device);
    const mk_plan_desc& d = p->d;
    const size_t n = (size_t)d.nr * p->B * d.ns;      // complex elements
    const float* src = R;
    float* staging = nullptr;
    if (!on_device) {
        HIP_TRY(p, dalloc(&staging, 2 * n));
        mk_status st = copy_in(p, staging, R, 2 * n, 0, "mk_load_R: upload");
        if (st != MK_OK) {
            (void)hipFree(staging);
            return st;
        }
        src = staging;
    }
    int h = 0;
    hipError_t e = hipMemsetAsync(p->flag, 0, sizeof(int), p->stream);
    if (e == hipSuccess) {
        if (p->r_tiled) {
            if (d.rprec != MK_R_C64) e = launch_rscale(src, p->rscale, d.nr, p->B, d.ns, p->flag, p->stream);
            if (e == hipSuccess)
                e = launch_repack_tiled(d.rprec, src, p->R, p->rscale, d.nr, p->B, d.ns, p->ns_pad, p->flag,
                                        p->stream);
        } else if (d.rprec == MK_R_C64) {
            e = launch_repack_c64(src, reinterpret_cast<float2*>(p->R), d.nr, p->B, d.ns, p->ns_pad,
                                  p->flag, p->stream);
        } else {
            e = launch_quantize_R(d.rprec, src, p->R, p->rscale, d.nr, p->B, d.ns, p->ns_pad, p->flag,
                                  p->stream);
        }
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&h, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (staging) (void)hipFree(staging);
    if (e != hipSuccess) return hip_fail(p, e, "mk_load_R: repack");
    if (h) {
        p->R_loaded = false;
        return fail(p, MK_ERR_ARG, "mk_load_R: R holds a non-finite value");
    }
    p->R_loaded = true;
    p->focal_set = false;
    p->g_valid = false;
    return MK_OK;
}

mk_status mk_set_focal(mk_plan_t p, int32_t nf, const float* Gd, const int32_t* itd, int32_t shift,
                       const int32_t* band, int on_device) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_set_focal: plan is NULL");
    const mk_plan_desc& d = p->d;
    if (nf < 1 || nf > d.nf_max) return fail(p, MK_ERR_ARG, "mk_set_focal: nf outside [1, nf_max]");
    if (!Gd || !itd) return fail(p, MK_ERR_ARG, "mk_set_focal: Gd or itd is NULL");
    if (shift < 0) return fail(p, MK_ERR_ARG, "mk_set_focal: shift must be >= 0");
    if (!p->R_loaded) return fail(p, MK_ERR_STATE, "mk_set_focal: R has not been loaded");
    const size_t ntr = (size_t)nf * d.nr;
    std::vector<int32_t> hb;
    if (band) {
        hb.resize(2 * (size_t)nf);
        if (on_device) {
            HIP_TRY(p, hipMemcpyAsync(hb.data(), band, hb.size() * sizeof(int32_t),
                                      hipMemcpyDeviceToHost, p->stream));
            HIP_TRY(p, hipStreamSynchronize(p->stream));
        } else {
            std::memcpy(hb.data(), band, hb.size() * sizeof(int32_t));
        }
        for (int f = 0; f < nf; ++f)
            if (hb[2 * f] < d.iw_lo || hb[2 * f + 1] > d.iw_hi || hb[2 * f] > hb[2 * f + 1])
                return fail(p, MK_ERR_ARG, "mk_set_focal: focal band outside the plan band");
    }
    if (!on_device) {
        for (size_t i = 0; i < ntr * d.nt; ++i)
            if (!std::isfinite(Gd[i])) return fail(p, MK_ERR_ARG, "mk_set_focal: Gd holds a non-finite value");
    }
    // focal order: by band end, descending (stable), so that the focal points
    // active at bin w are a prefix of the batch when all bands start at iw_lo
    std::vector<int> perm(nf);
    std::iota(perm.begin(), perm.end(), 0);
    if (band)
        std::stable_sort(perm.begin(), perm.end(),
                         [&](int a, int b) { return hb[2 * a + 1] > hb[2 * b + 1]; });
    std::vector<int> iperm(nf);
    for (int j = 0; j < nf; ++j) iperm[perm[j]] = j;
    HIP_TRY(p, hipMemcpyAsync(p->perm, perm.data(), nf * sizeof(int), hipMemcpyHostToDevice, p->stream));
    HIP_TRY(p, hipMemcpyAsync(p->iperm, iperm.data(), nf * sizeof(int), hipMemcpyHostToDevice, p->stream));
    // G_d and itd in sorted order (G_d lands in the G+ buffer, free until the G
    // assembly); device arrays are gathered in place, host arrays through the
    // staging buffers.  A non-finite device G_d shows up as a non-finite norm
    // below (the FP64 sum of squares of finite floats cannot overflow).
    p->focal_set = false;
    const float* gsrc = Gd;
    if (!on_device) {
        MK_TRY(copy_in(p, p->stage, Gd, ntr * d.nt, 0, "mk_set_focal: Gd"));
        gsrc = p->stage;
    }
    // in the caller's order INIT reads G_d where it is (this call waits for
    // INIT before it returns)
    bool identity = true;
    for (int j = 0; j < nf; ++j) identity = identity && perm[j] == j;
    if (!identity) {
        HIP_TRY(p, launch_gather(gsrc, p->gp, p->perm, nf, (int64_t)d.nr * d.nt, p->stream));
        gsrc = p->gp;
    }
    const int32_t* isrc = itd;
    if (!on_device) {
        int32_t* itd_stage = p->itd + (size_t)d.nf_max * d.nr;
        MK_TRY(copy_in(p, itd_stage, itd, ntr, 0, "mk_set_focal: itd"));
        isrc = itd_stage;
    }
    HIP_TRY(p, launch_gather(reinterpret_cast<const float*>(isrc), reinterpret_cast<float*>(p->itd),
                             p->perm, nf, d.nr, p->stream));
    if (band) {
        std::vector<int32_t> sb(2 * (size_t)nf);
        for (int j = 0; j < nf; ++j) {
            sb[2 * j] = hb[2 * perm[j]];
            sb[2 * j + 1] = hb[2 * perm[j] + 1];
        }
        std::vector<int32_t> nc(p->B, 0);
        for (int w = 0; w < p->B; ++w) {
            const int bin = d.iw_lo + w;
            for (int j = nf - 1; j >= 0; --j)
                if (sb[2 * j] <= bin && bin <= sb[2 * j + 1]) {
                    nc[w] = j + 1;
                    break;
                }
        }
        HIP_TRY(p, hipMemcpyAsync(p->fband, sb.data(), sb.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                  p->stream));
        HIP_TRY(p, hipMemcpyAsync(p->ncols, nc.data(), nc.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                  p->stream));
        HIP_TRY(p, hipStreamSynchronize(p->stream));    // host vectors go out of scope
        p->ncols_host = nc;
    }
    p->has_fband = band != nullptr;
    p->perm_host = perm;
    p->nf = nf;
    p->shift = shift;
    p->passes = 0;
    p->pass_base = 0;
    p->tail_applied = false;
    p->g_valid = false;
    p->series_choice = choose(p, nf);
    p->g_choice = choose(p, 2 * nf);
    MK_TRY(build_walk(p));
    // ||N_-1|| = ||G_d|| per focal point (also the scale of the first 16-bit X)
    MK_TRY(outside_window_norms(p, gsrc, nf, shift));
    HIP_TRY(p, hipMemcpyAsync(p->gdnorm, p->norm0, nf * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
    TraceArgs a = trace_args(p, nf);
    a.src = gsrc;
    a.xprec = p->series_choice.xprec;
    a.xs_in = p->norm0;
    a.xs_out = p->xscale;
    a.skip_outband = (p->series_choice.variant != 0 && p->has_fband) ? 1 : 0;
    MK_TRY(run_trace(p, TM_INIT, a, 3));
    double* n0 = nullptr;
    MK_TRY(pinned(p, 2 * (size_t)nf, &n0));
    HIP_TRY(p, hipMemcpyAsync(n0, p->norm0, nf * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipMemcpyAsync(n0 + nf, p->fnorm, nf * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    p->f1p_out2_host.resize(nf);
    for (int j = 0; j < nf; ++j) p->f1p_out2_host[j] = n0[nf + j] * n0[nf + j];
    for (int j = 0; j < nf; ++j)
        if (!std::isfinite(n0[j])) return fail(p, MK_ERR_ARG, "mk_set_focal: Gd holds a non-finite value");
    p->norm0_host.assign(nf, 0.0);
    for (int j = 0; j < nf; ++j) p->norm0_host[perm[j]] = n0[j];
    p->gd_norm_host = p->norm0_host;
    p->log_len = 0;
    p->series_start = 0;
    MK_TRY(log_series_start(p, p->norm0));
    p->focal_set = true;
    return MK_OK;
}

}  // extern "C"

namespace {

// Enqueue passes [i0, i0 + n) of one mk_iterate call; `parity0` is the
// parity of pass i0 in the series.
mk_status enqueue_passes(mk_plan_t p, int i0, int n, int parity0) {
    for (int i = i0; i < i0 + n; ++i) {
        MK_TRY(run_contract(p, p->series_choice, p->X, p->xscale, p->nf, 1, 0));
        TraceArgs a = trace_args(p, p->nf);
        a.parity = (parity0 + (i - i0)) & 1;
        const int idx = p->passes + (i - i0);          // pass index since mk_set_focal
        if (p->hist && !p->tail_applied && idx < p->hist_k) {
            a.hist = p->hist;
            a.rec_slot = idx;
        }
        a.xprec = p->series_choice.xprec;
        a.xs_in = p->nlast;
        a.xs_out = p->xscale;
        a.skip_outband = (p->series_choice.variant != 0 && p->has_fband) ? 1 : 0;
        MK_TRY(run_trace(p, TM_ITER, a, 1));
        MK_TRY(run_norms(p, p->norms + (size_t)i * p->nf));
    }
    return MK_OK;
}

// Passes [0, n) of one mk_iterate call as one HIP graph, captured on first
// use and replayed afterwards.  The captured work holds kernel launches only
// (no memset or copy nodes).
mk_status replay_passes(mk_plan_t p, int n, int parity0) {
    const int i0 = 0;
    hipGraphExec_t exec = nullptr;
    for (auto& g : p->graphs)
        if (g.niter == n && g.parity == parity0 && g.nf == p->nf && g.fband == p->has_fband &&
            g.shift == p->shift && g.variant == p->series_choice.variant && g.xprec == p->series_choice.xprec)
            exec = g.exec;
    if (!exec) {
        hipStream_t cs = p->capture_stream ? p->capture_stream : p->stream;
        hipStream_t keep = p->stream;
        p->stream = cs;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) {
            p->stream = keep;
            return hip_fail(p, e, "hipStreamBeginCapture");
        }
        mk_status st = enqueue_passes(p, i0, n, parity0);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        p->stream = keep;
        if (st != MK_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return hip_fail(p, e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(p, e, "hipGraphInstantiate");
        if (p->graphs.size() >= 32) drop_graphs(p);      // bound the cache of executables
        p->graphs.push_back({n, parity0, p->nf, p->has_fband, p->shift, p->series_choice.variant,
                             p->series_choice.xprec, exec});
    }
    hipError_t e = hipGraphLaunch(exec, p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "hipGraphLaunch");
    return MK_OK;
}

// ---- series state (checkpoint and resume) ----------------------------------
// The blob is a header followed by the plan's series state in a fixed order;
// every piece is a straight copy of what the plan holds, so a resumed series
// continues with the same bits as an uninterrupted one.
constexpr char kStateMagic[8] = {'M', 'K', 'S', 'T', 'A', 'T', 'E', '1'};

struct StateHeader {
    char magic[8];
    int32_t nr, nt, iw_lo, iw_hi, ns_pad, rprec, flags;
    int32_t nf, shift, passes, pass_base, tail_applied, has_fband;
    int32_t variant, xprec, log_len, series_start, prev_series_start;
    int32_t hist_k, hist_T, has_hist, reserved;
};

// One entry of the blob after the header: `bytes` bytes at device address
// `dev` (or host address `host` when dev is null).
struct StatePart {
    void* dev;
    void* host;
    size_t bytes;
};

std::vector<StatePart> state_parts(mk_plan_t p, const StateHeader& h, std::vector<double>& host_norms) {
    const size_t nf = (size_t)h.nf, nr = (size_t)p->d.nr, nt = (size_t)p->d.nt, B = (size_t)p->B;
    const size_t trace = nf * nr * nt;
    host_norms.resize(2 * nf);
    std::vector<StatePart> v = {
        {p->perm, nullptr, nf * sizeof(int32_t)},
        {p->iperm, nullptr, nf * sizeof(int32_t)},
        {p->fband, nullptr, 2 * nf * sizeof(int32_t)},
        {p->ncols, nullptr, B * sizeof(int32_t)},
        {p->itd, nullptr, nf * nr * sizeof(int32_t)},
        {p->n0, nullptr, trace * sizeof(float)},
        {p->f1p, nullptr, trace * sizeof(float)},
        {p->f1m, nullptr, trace * sizeof(float)},
        {p->X, nullptr, nf * B * (size_t)p->ns_pad * sizeof(float2)},   // the series' slab, any X storage
        {p->xscale, nullptr, nf * sizeof(float)},
        {p->norm0, nullptr, nf * sizeof(double)},
        {p->gdnorm, nullptr, nf * sizeof(double)},
        {p->nlast, nullptr, nf * sizeof(double)},
        {p->norm_log, nullptr, (size_t)h.log_len * nf * sizeof(double)},
        {nullptr, host_norms.data(), 2 * nf * sizeof(double)},          // norm0_host, gd_norm_host
    };
    if (h.has_hist) v.push_back({p->hist, nullptr, nf * nr * (size_t)h.hist_k * h.hist_T * sizeof(float)});
    return v;
}

size_t state_size(mk_plan_t p, const StateHeader& h) {
    std::vector<double> tmp;
    size_t n = sizeof(StateHeader);
    for (auto& part : state_parts(p, h, tmp)) n += part.bytes;
    return n;
}

StateHeader state_header(mk_plan_t p) {
    StateHeader h{};
    std::memcpy(h.magic, kStateMagic, sizeof(h.magic));
    h.nr = p->d.nr;
    h.nt = p->d.nt;
    h.iw_lo = p->d.iw_lo;
    h.iw_hi = p->d.iw_hi;
    h.ns_pad = p->ns_pad;
    h.rprec = p->d.rprec;
    h.flags = (int32_t)(p->d.flags & MK_FLAG_FAST_X);
    h.nf = p->nf;
    h.shift = p->shift;
    h.passes = p->passes;
    h.pass_base = p->pass_base;
    h.tail_applied = p->tail_applied ? 1 : 0;
    h.has_fband = p->has_fband ? 1 : 0;
    h.variant = p->series_choice.variant;
    h.xprec = p->series_choice.xprec;
    h.log_len = p->log_len;
    h.series_start = p->series_start;
    h.prev_series_start = p->prev_series_start;
    h.hist_k = p->hist_k;
    h.hist_T = p->hist_T;
    h.has_hist = p->hist ? 1 : 0;
    return h;
}

bool tune_pending(mk_plan_t p) {
    if (p->tune_mode != -2) return false;
    for (auto& kv : p->tuned)
        if (kv.first == p->nf) return false;
    return true;
}

}  // namespace

extern "C" {

mk_status mk_iterate(mk_plan_t p, int32_t niter, double* norms) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_iterate: plan is NULL");
    if (niter < 0) return fail(p, MK_ERR_ARG, "mk_iterate: niter must be >= 0");
    if (!p->focal_set) return fail(p, MK_ERR_STATE, "mk_iterate: no focal points set");
    if (niter == 0) return MK_OK;
    MK_TRY(ensure_norm_cap(p, niter));
    p->g_valid = false;
    // graphs replay passes whose contraction is already chosen: while the
    // autotuner still has to time this column count, the passes run eagerly
    // (and while the first passes are being recorded for the series tail)
    const bool recording = p->hist && !p->tail_applied && p->passes < p->hist_k;
    const bool graph = (p->d.flags & MK_FLAG_GRAPH) && !(p->d.flags & MK_FLAG_PROFILE) && !tune_pending(p) &&
                       !recording;
    const int parity0 = (p->passes - p->pass_base) & 1;
    if (graph) MK_TRY(replay_passes(p, niter, parity0));
    else MK_TRY(enqueue_passes(p, 0, niter, parity0));
    p->passes += niter;
    MK_TRY(log_rows(p, p->norms, niter));
    if (norms) {
        double* h = nullptr;
        MK_TRY(pinned(p, (size_t)niter * p->nf, &h));
        HIP_TRY(p, hipMemcpyAsync(h, p->norms, (size_t)niter * p->nf * sizeof(double), hipMemcpyDeviceToHost,
                                  p->stream));
        HIP_TRY(p, hipStreamSynchronize(p->stream));
        for (int i = 0; i < niter; ++i)
            for (int j = 0; j < p->nf; ++j) norms[(size_t)i * p->nf + p->perm_host[j]] = h[(size_t)i * p->nf + j];
        for (int i = 0; i < niter; ++i)
            for (int f = 0; f < p->nf; ++f) {
                const double v = norms[(size_t)i * p->nf + f];
                if (!std::isfinite(v) || v > p->d.div_factor * p->norm0_host[f]) {
                    char buf[160];
                    std::snprintf(buf, sizeof(buf),
                                  "mk_iterate: ||N|| = %g at pass %d, focal %d (||N_-1|| = %g)", v,
                                  p->passes - niter + i, f, p->norm0_host[f]);
                    return fail(p, MK_ERR_DIVERGED, buf);
                }
            }
    }
    return MK_OK;
}

mk_status mk_iterate_tol(mk_plan_t p, double tol, int32_t max_passes, int32_t* passes_run, double* est) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_iterate_tol: plan is NULL");
    if (passes_run) *passes_run = 0;
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(p, MK_ERR_ARG, "mk_iterate_tol: tol must be positive");
    if (max_passes < 0) return fail(p, MK_ERR_ARG, "mk_iterate_tol: max_passes must be >= 0");
    if (!p->focal_set) return fail(p, MK_ERR_STATE, "mk_iterate_tol: no focal points set");
    std::vector<double> e;
    int run = 0, check_from = -1;
    for (;;) {
        int more = 0;
        // the judge also reads the new passes' norms: it applies mk_iterate's
        // divergence check to them, so the passes return without a read
        MK_TRY(judge_series(p, tol, e, &more, check_from));
        if (more == 0 || run >= max_passes) break;
        // an unknown contraction factor needs two terms of this series first
        const int m = std::min(more < 0 ? 2 : more, max_passes - run);
        check_from = p->log_len;
        mk_status st = mk_iterate(p, m, nullptr);
        run += m;
        if (passes_run) *passes_run = run;
        if (st != MK_OK) return st;
    }
    if (est)
        for (int j = 0; j < p->nf; ++j) est[p->perm_host[j]] = e[j];
    return MK_OK;
}

mk_status mk_get(mk_plan_t p, int32_t field, float* out, int on_device) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_get: plan is NULL");
    if (!out) return fail(p, MK_ERR_ARG, "mk_get: out is NULL");
    if (field < MK_F1PLUS || field > MK_GTOTAL) return fail(p, MK_ERR_ARG, "mk_get: unknown field");
    if (!p->focal_set) return fail(p, MK_ERR_STATE, "mk_get: no focal points set");
    const float* src = nullptr;
    switch (field) {
        case MK_F1PLUS: src = p->f1p; break;
        case MK_F1MINUS: src = p->f1m; break;
        case MK_GPLUS: src = p->gp; break;
        case MK_GMINUS: src = p->gm; break;
        default: break;
    }
    if ((field == MK_GPLUS || field == MK_GMINUS) && !p->g_valid) MK_TRY(assemble_G(p));
    if (field == MK_F2PLUS || field == MK_PMINUS || field == MK_GTOTAL) {
        MK_TRY(aux_field(p, field));
        src = p->aux;
    }
    const size_t per = (size_t)p->d.nr * p->d.nt;
    const size_t n = (size_t)p->nf * per;
    // back to the caller's focal order: straight into a device destination,
    // through the staging buffer for a host one, a plain copy when the plan
    // kept the caller's order
    bool identity = true;
    for (int j = 0; j < p->nf; ++j) identity = identity && p->perm_host[j] == j;
    if (identity) {
        HIP_TRY(p, hipMemcpyAsync(out, src, n * sizeof(float),
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, p->stream));
    } else if (on_device) {
        HIP_TRY(p, launch_gather(src, out, p->iperm, p->nf, (int64_t)per, p->stream));
    } else {
        HIP_TRY(p, launch_gather(src, p->stage, p->iperm, p->nf, (int64_t)per, p->stream));
        HIP_TRY(p, hipMemcpyAsync(out, p->stage, n * sizeof(float), hipMemcpyDeviceToHost, p->stream));
    }
    if (!on_device) HIP_TRY(p, hipStreamSynchronize(p->stream));
    return MK_OK;
}

mk_status mk_image(mk_plan_t p, double* image) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_image: plan is NULL");
    if (!image) return fail(p, MK_ERR_ARG, "mk_image: image is NULL");
    if (!p->focal_set) return fail(p, MK_ERR_STATE, "mk_image: no focal points set");
    if (!p->g_valid) MK_TRY(assemble_G(p));
    hipEvent_t ev = nullptr;
    HIP_TRY(p, prof_begin(p, &ev));
    HIP_TRY(p, launch_image(p->gm, p->f1p, p->nf, p->d.nr, p->d.nt, p->d.dx * p->d.dt, p->npart, p->img,
                            p->stream));
    HIP_TRY(p, prof_end(p, ev, 5));
    std::vector<double> v(p->nf);
    HIP_TRY(p, hipMemcpyAsync(v.data(), p->img, p->nf * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    for (int j = 0; j < p->nf; ++j) image[p->perm_host[j]] = v[j];
    return MK_OK;
}

mk_status mk_passes(mk_plan_t p, int32_t* passes) {
    if (!p || !passes) return fail(p, MK_ERR_ARG, "mk_passes: NULL argument");
    *passes = p->passes;
    return MK_OK;
}

mk_status mk_tune(mk_plan_t p, int32_t mode) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_tune: plan is NULL");
    if (mode < -2 || mode > contract_mfma_variants())
        return fail(p, MK_ERR_ARG, "mk_tune: mode outside [-2, number of variants]");
    if (mode >= 0 && !variant_fits(p, mode))
        return fail(p, MK_ERR_ARG, "mk_tune: this variant reads row-major R; the plan keeps R tiled "
                                   "(nf_max > 4 without MK_FLAG_ROW_R)");
    p->tune_mode = mode;
    p->tuned.clear();
    drop_graphs(p);
    // the X storage is fixed when the focal points are set: the caller sets them again
    p->focal_set = false;
    p->g_valid = false;
    return MK_OK;
}

mk_status mk_contract_variant(mk_plan_t p, int32_t ncols, int32_t* variant) {
    if (!p || !variant || ncols < 1) return fail(p, MK_ERR_ARG, "mk_contract_variant: bad argument");
    for (auto& kv : p->tuned)
        if (kv.first == ncols) {
            *variant = kv.second;
            return MK_OK;
        }
    *variant = choose(p, ncols).variant;
    return MK_OK;
}


mk_status mk_tail_record(mk_plan_t p, int32_t k, int32_t T) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_tail_record: plan is NULL");
    if (k < 1 || k > 16 || T < 2 || (T & 1) || T > p->d.nt)
        return fail(p, MK_ERR_ARG, "mk_tail_record: need 1 <= k <= 16 and an even T <= nt");
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    if (p->hist) HIP_TRY(p, hipFree(p->hist));
    p->hist = nullptr;
    if (k != p->hist_k || T != p->hist_T) {      // network and its buffers were sized for the old (k, T)
        float** bufs[] = {&p->tail_w, &p->tail_x, &p->tail_work, &p->tail_y};
        for (float** b : bufs) {
            if (*b) HIP_TRY(p, hipFree(*b));
            *b = nullptr;
        }
        p->tail_nw = 0;
        p->tail_hidden = 0;
        p->tail_net_hidden = 0;
    }
    const size_t n = (size_t)p->d.nf_max * p->d.nr * k * T;
    HIP_TRY(p, dalloc(&p->hist, n));
    HIP_TRY(p, hipMemsetAsync(p->hist, 0, n * sizeof(float), p->stream));
    p->hist_k = k;
    p->hist_T = T;
    drop_graphs(p);
    return MK_OK;
}

mk_status mk_tail_load(mk_plan_t p, const float* params, int32_t count) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_tail_load: plan is NULL");
    if (!params) return fail(p, MK_ERR_ARG, "mk_tail_load: params is NULL");
    if (!p->hist) return fail(p, MK_ERR_STATE, "mk_tail_load: call mk_tail_record first");
    int H = 0;                                   // the hidden width follows from the count
    for (int h = 1; h <= kNetHiddenMax && !H; ++h)
        if (net_param_count(p->hist_k, h) == count) H = h;
    if (!H) return fail(p, MK_ERR_ARG, "mk_tail_load: parameter count fits no hidden width for this k");
    for (int i = 0; i < count; ++i)
        if (!std::isfinite(params[i])) return fail(p, MK_ERR_ARG, "mk_tail_load: non-finite parameter");
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    if (p->tail_w && p->tail_nw != count) {
        HIP_TRY(p, hipFree(p->tail_w));
        p->tail_w = nullptr;
    }
    if (!p->tail_w) HIP_TRY(p, dalloc(&p->tail_w, (size_t)count));
    HIP_TRY(p, hipMemcpyAsync(p->tail_w, params, count * sizeof(float), hipMemcpyHostToDevice, p->stream));
    HIP_TRY(p, net_round_bf16(p->tail_w, p->tail_w, count, p->stream));
    p->tail_nw = count;
    const int ntr = p->d.nf_max * p->d.nr;
    if (!net_tail_fused(p->hist_k, H)) {            // layer by layer: activations in HBM, in chunks
        if (p->tail_work && p->tail_hidden < H) {   // activations sized for a narrower network
            HIP_TRY(p, hipFree(p->tail_work));
            p->tail_work = nullptr;
        }
        p->tail_chunk = std::min(ntr, 4096);
        if (!p->tail_work) {
            HIP_TRY(p, dalloc(&p->tail_work, 2 * (size_t)p->tail_chunk * H * p->hist_T));
            p->tail_hidden = H;
        }
        if (!p->tail_x) {
            const size_t c = (size_t)p->tail_chunk, T = (size_t)p->hist_T;
            HIP_TRY(p, dalloc(&p->tail_x, c * 16 * T));             // room for k <= 16
            HIP_TRY(p, dalloc(&p->tail_y, c * 2 * T));
        }
    }
    p->tail_net_hidden = H;
    if (!p->tail_scale) HIP_TRY(p, dalloc(&p->tail_scale, (size_t)ntr));
    if (net_tail_fused(p->hist_k, H)) {
        if (!p->tail_wpk) HIP_TRY(p, hipMalloc(&p->tail_wpk, net_tail_pack_bytes(16)));   // room for any k
        HIP_TRY(p, net_tail_pack(p->tail_w, p->hist_k, H, p->tail_wpk, p->stream));
    }
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    return MK_OK;
}

mk_status mk_tail_history(mk_plan_t p, float* out, int on_device) {
    if (!p || !out) return fail(p, MK_ERR_ARG, "mk_tail_history: NULL argument");
    if (!p->hist || !p->focal_set) return fail(p, MK_ERR_STATE, "mk_tail_history: nothing recorded");
    const size_t per = (size_t)p->d.nr * p->hist_k * p->hist_T;
    const size_t n = per * p->nf;
    float* dst = out;
    float* tmp = nullptr;
    if (!on_device) {
        HIP_TRY(p, dalloc(&tmp, n));
        dst = tmp;
    }
    hipError_t e = launch_gather(p->hist, dst, p->iperm, p->nf, (int64_t)per, p->stream);
    if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(out, tmp, n * sizeof(float), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess && !on_device) e = hipStreamSynchronize(p->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(p, e, "mk_tail_history");
    return MK_OK;
}

mk_status mk_tail_apply(mk_plan_t p, int32_t mode, double* rel_resid) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_tail_apply: plan is NULL");
    if (mode < 0 || mode > 2) return fail(p, MK_ERR_ARG, "mk_tail_apply: mode must be 0, 1 or 2");
    if (!p->focal_set || !p->hist || p->tail_applied || p->passes - p->pass_base != p->hist_k)
        return fail(p, MK_ERR_STATE, "mk_tail_apply: needs exactly k recorded passes of a fresh series");
    if (mode == 0 && !p->tail_w) return fail(p, MK_ERR_STATE, "mk_tail_apply: no network loaded");
    if (mode == 1 && (p->hist_k < 4 || (p->hist_k & 1)))
        return fail(p, MK_ERR_ARG, "mk_tail_apply: geometric extrapolation needs an even k >= 4");
    const int nr = p->d.nr, nt = p->d.nt, k = p->hist_k, T = p->hist_T;
    const int ntr = p->nf * nr;
    if (mode == 0 && net_tail_fused(k, p->tail_net_hidden)) {
        HIP_TRY(p, launch_tail_prep(p->hist, ntr, k, T, nullptr, p->tail_scale, p->stream));
        HIP_TRY(p, net_tail_apply(p->tail_w, p->tail_wpk, p->hist, p->tail_scale, p->itd, p->shift, ntr, k,
                                  p->tail_net_hidden, T, nt, p->f1p, p->stream));
    } else if (mode == 0) {
        const int H = p->tail_net_hidden;
        const size_t act = (size_t)p->tail_chunk * H * T;
        for (int c0 = 0; c0 < ntr; c0 += p->tail_chunk) {
            const int n = std::min(p->tail_chunk, ntr - c0);
            const float* h = p->hist + (size_t)c0 * k * T;
            HIP_TRY(p, launch_tail_prep(h, n, k, T, p->tail_x, p->tail_scale + c0, p->stream));
            HIP_TRY(p, net_forward(p->tail_w, p->tail_x, n, k, H, T, p->tail_work, p->tail_work + act, p->tail_y,
                                   p->stream));
            HIP_TRY(p, launch_tail_apply(h, p->tail_y, p->tail_scale + c0, p->itd + c0, p->shift, n, k, T, nt, 0,
                                         p->f1p + (size_t)c0 * nt, p->stream));
        }
    } else if (mode == 1) {
        HIP_TRY(p, launch_tail_apply(p->hist, nullptr, nullptr, p->itd, p->shift, ntr, k, T, nt, 1, p->f1p,
                                     p->stream));
    }
    // the judge: one fixed-point step f1+ <- G_d(-t) + A^2 f1+ (two syntheses),
    // whose residual starts a new Neumann series for the remaining error
    TraceArgs a = trace_args(p, p->nf);
    a.xprec = p->series_choice.xprec;
    a.xs_in = p->norm0;
    a.xs_out = p->xscale;
    a.skip_outband = (p->series_choice.variant != 0 && p->has_fband) ? 1 : 0;
    MK_TRY(run_trace(p, TM_FWDF, a, 1));
    MK_TRY(run_contract(p, p->series_choice, p->X, p->xscale, p->nf, 1, 0));
    MK_TRY(run_trace(p, TM_RST1, a, 1));
    MK_TRY(run_contract(p, p->series_choice, p->X, p->xscale, p->nf, 1, 0));
    MK_TRY(run_trace(p, TM_RST2, a, 1));
    HIP_TRY(p, launch_norm_reduce(p->npart, nr, p->nf, p->norm0, p->nlast, p->stream));
    double* rn = nullptr;
    MK_TRY(pinned(p, p->nf, &rn));
    HIP_TRY(p, hipMemcpyAsync(rn, p->norm0, p->nf * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    for (int j = 0; j < p->nf; ++j) {
        const int f = p->perm_host[j];
        p->norm0_host[f] = rn[j];
        if (rel_resid) rel_resid[f] = p->gd_norm_host[f] > 0.0 ? rn[j] / p->gd_norm_host[f] : rn[j];
    }
    p->passes += 2;
    p->pass_base = p->passes;
    p->tail_applied = true;
    p->g_valid = false;
    MK_TRY(log_series_start(p, p->norm0));
    return MK_OK;
}

mk_status mk_profile(mk_plan_t p, int32_t kind, double* total_ms, int64_t* launches, int reset) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_profile: plan is NULL");
    if (kind < 0 || kind > 5) return fail(p, MK_ERR_ARG, "mk_profile: unknown kernel kind");
    if (!(p->d.flags & MK_FLAG_PROFILE))
        return fail(p, MK_ERR_UNSUPPORTED, "mk_profile: plan was created without MK_FLAG_PROFILE");
    HIP_TRY(p, prof_resolve(p));
    if (total_ms) *total_ms = p->prof[kind].ms;
    if (launches) *launches = p->prof[kind].launches;
    if (reset) p->prof[kind] = ProfileSlot{};
    return MK_OK;
}

mk_status mk_state_bytes(mk_plan_t p, size_t* bytes) {
    if (!p || !bytes) return fail(p, MK_ERR_ARG, "mk_state_bytes: NULL argument");
    if (!p->focal_set) return fail(p, MK_ERR_STATE, "mk_state_bytes: no focal points set");
    *bytes = state_size(p, state_header(p));
    return MK_OK;
}

mk_status mk_get_state(mk_plan_t p, void* blob, size_t bytes) {
    if (!p || !blob) return fail(p, MK_ERR_ARG, "mk_get_state: NULL argument");
    if (!p->focal_set) return fail(p, MK_ERR_STATE, "mk_get_state: no focal points set");
    const StateHeader h = state_header(p);
    if (bytes < state_size(p, h)) return fail(p, MK_ERR_ARG, "mk_get_state: blob smaller than mk_state_bytes");
    std::vector<double> hn;
    auto parts = state_parts(p, h, hn);
    for (int j = 0; j < p->nf; ++j) {            // caller order, as the plan keeps them
        hn[j] = p->norm0_host[j];
        hn[p->nf + j] = p->gd_norm_host[j];
    }
    unsigned char* o = static_cast<unsigned char*>(blob);
    std::memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    for (auto& part : parts) {
        if (part.bytes == 0) continue;
        if (part.dev)
            HIP_TRY(p, hipMemcpyAsync(o, part.dev, part.bytes, hipMemcpyDeviceToHost, p->stream));
        else
            std::memcpy(o, part.host, part.bytes);
        o += part.bytes;
    }
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    return MK_OK;
}

mk_status mk_set_state(mk_plan_t p, const void* blob, size_t bytes) {
    if (!p || !blob) return fail(p, MK_ERR_ARG, "mk_set_state: NULL argument");
    if (!p->R_loaded) return fail(p, MK_ERR_STATE, "mk_set_state: R has not been loaded");
    StateHeader h;
    if (bytes < sizeof(h)) return fail(p, MK_ERR_ARG, "mk_set_state: blob too small");
    std::memcpy(&h, blob, sizeof(h));
    if (std::memcmp(h.magic, kStateMagic, sizeof(h.magic)) != 0)
        return fail(p, MK_ERR_ARG, "mk_set_state: not a state blob of this library");
    if (h.nr != p->d.nr || h.nt != p->d.nt || h.iw_lo != p->d.iw_lo || h.iw_hi != p->d.iw_hi ||
        h.ns_pad != p->ns_pad || h.rprec != p->d.rprec || h.flags != (int32_t)(p->d.flags & MK_FLAG_FAST_X))
        return fail(p, MK_ERR_ARG, "mk_set_state: the blob was saved by a plan of another shape, band, "
                                   "precision or X storage");
    if (h.nf < 1 || h.nf > p->d.nf_max) return fail(p, MK_ERR_ARG, "mk_set_state: nf above this plan's nf_max");
    if (h.variant < 0 || h.variant > contract_mfma_variants() || !variant_fits(p, h.variant) ||
        xprec_of(p->d.rprec, h.variant, (p->d.flags & MK_FLAG_FAST_X) != 0) != h.xprec)
        return fail(p, MK_ERR_ARG, "mk_set_state: the saved contraction choice cannot read this plan's R");
    if (h.has_hist && (!p->hist || p->hist_k != h.hist_k || p->hist_T != h.hist_T))
        return fail(p, MK_ERR_STATE, "mk_set_state: the saved series records iterates: call mk_tail_record "
                                     "with the same k and T first");
    if (h.log_len < 1 || h.series_start < 0 || h.series_start >= h.log_len || h.prev_series_start < 0 ||
        h.prev_series_start > h.series_start || h.passes < h.pass_base || h.pass_base < 0)
        return fail(p, MK_ERR_ARG, "mk_set_state: inconsistent counters in the blob");
    if (bytes < state_size(p, h)) return fail(p, MK_ERR_ARG, "mk_set_state: blob truncated");
    p->focal_set = false;
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    p->log_len = 0;                              // room for the saved norm log
    MK_TRY(ensure_log_cap(p, h.log_len));
    std::vector<double> hn;
    auto parts = state_parts(p, h, hn);
    const unsigned char* in = static_cast<const unsigned char*>(blob) + sizeof(h);
    for (auto& part : parts) {
        if (part.bytes == 0) continue;
        if (part.dev)
            HIP_TRY(p, hipMemcpyAsync(part.dev, in, part.bytes, hipMemcpyHostToDevice, p->stream));
        else
            std::memcpy(part.host, in, part.bytes);
        in += part.bytes;
    }
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    p->nf = h.nf;
    p->shift = h.shift;
    p->passes = h.passes;
    p->pass_base = h.pass_base;
    p->tail_applied = h.tail_applied != 0;
    p->has_fband = h.has_fband != 0;
    p->series_choice.variant = h.variant;
    p->series_choice.xprec = h.xprec;
    p->g_choice = choose(p, 2 * h.nf);
    if (p->has_fband) {
        p->ncols_host.assign(p->B, 0);
        HIP_TRY(p, hipMemcpyAsync(p->ncols_host.data(), p->ncols, p->B * sizeof(int32_t), hipMemcpyDeviceToHost,
                                  p->stream));
        HIP_TRY(p, hipStreamSynchronize(p->stream));
    }
    MK_TRY(build_walk(p));
    {
        // the outside-window sums of N_-1; norm0 and nlast keep their saved values
        const int ntr = h.nf * p->d.nr;
        HIP_TRY(p, launch_sumsq_out(p->n0, ntr, p->d.nt, p->itd, h.shift, p->npart, p->npart + ntr, p->stream));
        HIP_TRY(p, launch_norm_reduce(p->npart + ntr, p->d.nr, h.nf, p->fnorm, nullptr, p->stream));
        double* o = nullptr;
        MK_TRY(pinned(p, h.nf, &o));
        HIP_TRY(p, hipMemcpyAsync(o, p->fnorm, h.nf * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        HIP_TRY(p, hipStreamSynchronize(p->stream));
        p->f1p_out2_host.resize(h.nf);
        for (int j = 0; j < h.nf; ++j) p->f1p_out2_host[j] = o[j] * o[j];
    }
    p->log_len = h.log_len;
    p->series_start = h.series_start;
    p->prev_series_start = h.prev_series_start;
    p->norm0_host.assign(hn.begin(), hn.begin() + h.nf);
    p->gd_norm_host.assign(hn.begin() + h.nf, hn.end());
    std::vector<int32_t> perm(h.nf);
    std::memcpy(perm.data(), static_cast<const unsigned char*>(blob) + sizeof(h), h.nf * sizeof(int32_t));
    p->perm_host.assign(perm.begin(), perm.end());
    p->g_valid = false;
    p->focal_set = true;
    return MK_OK;
}

mk_status mk_device_checks(uint32_t* violations) {
    if (!violations) return fail(nullptr, MK_ERR_ARG, "mk_device_checks: violations is NULL");
    *violations = 0;
#ifndef MK_DEVICE_CHECKS
    return fail(nullptr, MK_ERR_UNSUPPORTED, "mk_device_checks: this library was built without device checks");
#else
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail(nullptr, MK_ERR_HIP, std::string("mk_device_checks: ") + hipGetErrorString(e));
    hipError_t (*take[])(unsigned*) = {check_take_trace, check_take_contract, check_take_mfma, check_take_net,
                                       check_take_tail};
    for (int i = 0; i < 5; ++i) {
        unsigned v = 0;
        if ((e = take[i](&v)) != hipSuccess)
            return fail(nullptr, MK_ERR_HIP, std::string("mk_device_checks: ") + hipGetErrorString(e));
        if (v) *violations |= 1u << i;
    }
    return MK_OK;
#endif
}

mk_status mk_destroy(mk_plan_t p) {
    if (!p) return MK_OK;
    (void)hipStreamSynchronize(p->stream);
    free_plan_memory(p);
    delete p;
    return MK_OK;
}

}  // extern "C"
