// Host side of the C ABI declared in include/mk.h: plan validation, device
// memory, the order of kernel launches for Algorithm 1, and status codes.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "mk_internal.h"

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

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

template <typename T>
hipError_t dalloc(T** ptr, size_t count) {
    *ptr = nullptr;
    if (count == 0) return hipSuccess;
    return hipMalloc(reinterpret_cast<void**>(ptr), count * sizeof(T));
}

void free_plan_memory(mk_plan_t p) {
    void* bufs[] = {p->R, p->X, p->Y, p->f1p, p->f1m, p->gp, p->gm, p->itd, p->fband,
                    p->npart, p->norm0, p->norms, p->tw, p->flag};
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

// --- pieces of the series -------------------------------------------------

TraceArgs trace_args(mk_plan_t p, int nfo) {
    TraceArgs a{};
    a.Y = p->Y;
    a.X = p->X;
    a.f1p = p->f1p;
    a.f1m = p->f1m;
    a.gp = p->gp;
    a.gm = p->gm;
    a.itd = p->itd;
    a.fband = p->has_fband ? p->fband : nullptr;
    a.npart = p->npart;
    a.tw = p->tw;
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

mk_status run_contract(mk_plan_t p, int ncols) {
    hipEvent_t ev = nullptr;
    HIP_TRY(p, prof_begin(p, &ev));
    HIP_TRY(p, launch_contract_c64(p->R, p->X, p->Y, p->d.nr, p->B, p->d.ns, p->ns_pad, ncols,
                                   p->stream));
    HIP_TRY(p, prof_end(p, ev, 0));
    return MK_OK;
}

mk_status run_trace(mk_plan_t p, int mode, const TraceArgs& a, int kind) {
    hipEvent_t ev = nullptr;
    HIP_TRY(p, prof_begin(p, &ev));
    HIP_TRY(p, launch_trace(mode, p->d.nt, a, p->stream));
    HIP_TRY(p, prof_end(p, ev, kind));
    return MK_OK;
}

mk_status run_norms(mk_plan_t p, double* out) {
    hipEvent_t ev = nullptr;
    HIP_TRY(p, prof_begin(p, &ev));
    HIP_TRY(p, launch_norm_reduce(p->npart, p->d.nr, p->nf, out, p->stream));
    HIP_TRY(p, prof_end(p, ev, 2));
    return MK_OK;
}

mk_status ensure_norm_cap(mk_plan_t p, int niter) {
    if (niter <= p->norm_cap) return MK_OK;
    int cap = p->norm_cap > 0 ? p->norm_cap : 64;
    while (cap < niter) cap *= 2;
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    if (p->norms) HIP_TRY(p, hipFree(p->norms));
    p->norms = nullptr;
    p->norm_cap = 0;
    HIP_TRY(p, dalloc(&p->norms, (size_t)cap * p->d.nf_max));
    p->norm_cap = cap;
    return MK_OK;
}

// Copy n elements of a host or device input into plan memory.
template <typename T>
mk_status copy_in(mk_plan_t p, T* dst, const T* src, size_t n, int on_device, const char* what) {
    if (n == 0) return MK_OK;
    hipError_t e = hipMemcpyAsync(dst, src, n * sizeof(T),
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                  p->stream);
    if (e != hipSuccess) return hip_fail(p, e, what);
    return MK_OK;
}

mk_status device_all_finite(mk_plan_t p, const float* x, int64_t n, bool* ok) {
    int h = 0;
    HIP_TRY(p, hipMemsetAsync(p->flag, 0, sizeof(int), p->stream));
    HIP_TRY(p, launch_check_finite(x, n, p->flag, p->stream));
    HIP_TRY(p, hipMemcpyAsync(&h, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    *ok = (h == 0);
    return MK_OK;
}

// G+ and G- from one batched synthesis of [f1+, f1-(-t)].  The spectra go to
// X slabs [nf, 3 nf): slabs [0, nf) hold the spectrum of the last N_i, which
// the next pass of the series still needs.
mk_status assemble_G(mk_plan_t p) {
    const int nf = p->nf;
    TraceArgs a = trace_args(p, 2 * nf);
    float2* Xg = p->X + (size_t)nf * p->B * p->ns_pad;
    a.X = Xg;
    mk_status st = run_trace(p, TM_GFWD, a, 4);
    if (st != MK_OK) return st;
    hipEvent_t ev = nullptr;
    HIP_TRY(p, prof_begin(p, &ev));
    HIP_TRY(p, launch_contract_c64(p->R, Xg, p->Y, p->d.nr, p->B, p->d.ns, p->ns_pad, 2 * nf,
                                   p->stream));
    HIP_TRY(p, prof_end(p, ev, 4));
    st = run_trace(p, TM_GOUT, a, 4);
    if (st != MK_OK) return st;
    p->g_valid = true;
    return MK_OK;
}

}  // namespace

extern "C" {

const char* mk_strerror(mk_status status) {
    const int i = (int)status;
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
    if (d.rprec != MK_R_C64) {
        if (d.rprec == MK_R_F16S || d.rprec == MK_R_BF16S)
            return fail(nullptr, MK_ERR_UNSUPPORTED, "mk_plan: reduced-precision R is not built");
        return fail(nullptr, MK_ERR_ARG, "mk_plan: unknown rprec");
    }
    if (d.flags & ~(MK_FLAG_GRAPH | MK_FLAG_PROFILE))
        return fail(nullptr, MK_ERR_ARG, "mk_plan: unknown flag bits");
    if (d.flags & MK_FLAG_GRAPH)
        return fail(nullptr, MK_ERR_UNSUPPORTED, "mk_plan: graph replay is not built");

    mk_plan_t p = new (std::nothrow) mk_plan_s();
    if (!p) return fail(nullptr, MK_ERR_OOM, "mk_plan: host allocation failed");
    p->d = d;
    if (!(p->d.div_factor > 0.0)) p->d.div_factor = 1e3;
    p->B = d.iw_hi - d.iw_lo + 1;
    p->M = d.nt / 2;
    p->ns_pad = (d.ns + 3) & ~3;
    p->stream = reinterpret_cast<hipStream_t>(d.stream);

    auto bail = [&](hipError_t e, const char* where) {
        std::string m = std::string("mk_plan: ") + where + ": " + hipGetErrorString(e);
        free_plan_memory(p);
        delete p;
        return fail(nullptr, e == hipErrorOutOfMemory ? MK_ERR_OOM : MK_ERR_HIP, m);
    };
    hipError_t e;
    if ((e = hipGetDevice(&p->device)) != hipSuccess) return bail(e, "hipGetDevice");
    const size_t nfm = (size_t)d.nf_max;
    const size_t trace = (size_t)d.nr * d.nt;
    if ((e = dalloc(&p->R, (size_t)p->B * d.nr * p->ns_pad)) != hipSuccess) return bail(e, "R");
    if ((e = dalloc(&p->X, 3 * nfm * p->B * p->ns_pad)) != hipSuccess) return bail(e, "X");
    if ((e = dalloc(&p->Y, 2 * nfm * p->B * d.nr)) != hipSuccess) return bail(e, "Y");
    if ((e = dalloc(&p->f1p, nfm * trace)) != hipSuccess) return bail(e, "f1+");
    if ((e = dalloc(&p->f1m, nfm * trace)) != hipSuccess) return bail(e, "f1-");
    if ((e = dalloc(&p->gp, nfm * trace)) != hipSuccess) return bail(e, "G+");
    if ((e = dalloc(&p->gm, nfm * trace)) != hipSuccess) return bail(e, "G-");
    if ((e = dalloc(&p->itd, nfm * d.nr)) != hipSuccess) return bail(e, "itd");
    if ((e = dalloc(&p->fband, nfm * 2)) != hipSuccess) return bail(e, "band");
    if ((e = dalloc(&p->npart, 2 * nfm * d.nr)) != hipSuccess) return bail(e, "norm partials");
    if ((e = dalloc(&p->norm0, nfm)) != hipSuccess) return bail(e, "norm0");
    if ((e = dalloc(&p->tw, (size_t)d.nt)) != hipSuccess) return bail(e, "twiddles");
    if ((e = dalloc(&p->flag, 1)) != hipSuccess) return bail(e, "flag");
    // the padding columns of X (s >= ns) must read as zero
    if ((e = hipMemsetAsync(p->X, 0, 3 * nfm * p->B * p->ns_pad * sizeof(float2), p->stream)) !=
        hipSuccess)
        return bail(e, "clear X");
    std::vector<float2> tw(d.nt);
    for (int k = 0; k < d.nt; ++k) {
        const double ang = -2.0 * M_PI * (double)k / (double)d.nt;
        tw[k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
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
    if (e == hipSuccess) e = launch_repack_c64(src, p->R, d.nr, p->B, d.ns, p->ns_pad, p->flag, p->stream);
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
    // band check on the host (device bands are copied back: 2 nf integers)
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
    // Gd goes to the G+ buffer, which is free until the G assembly
    mk_status st = copy_in(p, p->gp, Gd, ntr * d.nt, on_device, "mk_set_focal: Gd");
    if (st != MK_OK) return st;
    if (on_device) {
        bool ok = true;
        st = device_all_finite(p, p->gp, (int64_t)(ntr * d.nt), &ok);
        if (st != MK_OK) return st;
        if (!ok) return fail(p, MK_ERR_ARG, "mk_set_focal: Gd holds a non-finite value");
    }
    st = copy_in(p, p->itd, itd, ntr, on_device, "mk_set_focal: itd");
    if (st != MK_OK) return st;
    if (band) {
        HIP_TRY(p, hipMemcpyAsync(p->fband, hb.data(), hb.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, p->stream));
    }
    p->has_fband = band != nullptr;
    p->nf = nf;
    p->shift = shift;
    p->passes = 0;
    p->g_valid = false;
    TraceArgs a = trace_args(p, nf);
    a.src = p->gp;
    st = run_trace(p, TM_INIT, a, 3);
    if (st != MK_OK) return st;
    HIP_TRY(p, launch_norm_reduce(p->npart, d.nr, nf, p->norm0, p->stream));
    p->norm0_host.assign(nf, 0.0);
    HIP_TRY(p, hipMemcpyAsync(p->norm0_host.data(), p->norm0, nf * sizeof(double),
                              hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    p->focal_set = true;
    return MK_OK;
}

mk_status mk_iterate(mk_plan_t p, int32_t niter, double* norms) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_iterate: plan is NULL");
    if (niter < 0) return fail(p, MK_ERR_ARG, "mk_iterate: niter must be >= 0");
    if (!p->focal_set) return fail(p, MK_ERR_STATE, "mk_iterate: no focal points set");
    if (niter == 0) return MK_OK;
    mk_status st = ensure_norm_cap(p, niter);
    if (st != MK_OK) return st;
    p->g_valid = false;
    for (int i = 0; i < niter; ++i) {
        st = run_contract(p, p->nf);
        if (st != MK_OK) return st;
        TraceArgs a = trace_args(p, p->nf);
        a.parity = p->passes & 1;
        st = run_trace(p, TM_ITER, a, 1);
        if (st != MK_OK) return st;
        st = run_norms(p, p->norms + (size_t)i * p->nf);
        if (st != MK_OK) return st;
        p->passes += 1;
    }
    if (norms) {
        HIP_TRY(p, hipMemcpyAsync(norms, p->norms, (size_t)niter * p->nf * sizeof(double),
                                  hipMemcpyDeviceToHost, p->stream));
        HIP_TRY(p, hipStreamSynchronize(p->stream));
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

mk_status mk_get(mk_plan_t p, int32_t field, float* out, int on_device) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_get: plan is NULL");
    if (!out) return fail(p, MK_ERR_ARG, "mk_get: out is NULL");
    if (field < MK_F1PLUS || field > MK_GMINUS) return fail(p, MK_ERR_ARG, "mk_get: unknown field");
    if (!p->focal_set) return fail(p, MK_ERR_STATE, "mk_get: no focal points set");
    const float* src = nullptr;
    switch (field) {
        case MK_F1PLUS: src = p->f1p; break;
        case MK_F1MINUS: src = p->f1m; break;
        case MK_GPLUS: src = p->gp; break;
        case MK_GMINUS: src = p->gm; break;
    }
    if ((field == MK_GPLUS || field == MK_GMINUS) && !p->g_valid) {
        mk_status st = assemble_G(p);
        if (st != MK_OK) return st;
    }
    const size_t n = (size_t)p->nf * p->d.nr * p->d.nt;
    HIP_TRY(p, hipMemcpyAsync(out, src, n * sizeof(float),
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, p->stream));
    if (!on_device) HIP_TRY(p, hipStreamSynchronize(p->stream));
    return MK_OK;
}

mk_status mk_passes(mk_plan_t p, int32_t* passes) {
    if (!p || !passes) return fail(p, MK_ERR_ARG, "mk_passes: NULL argument");
    *passes = p->passes;
    return MK_OK;
}

mk_status mk_profile(mk_plan_t p, int32_t kind, double* total_ms, int64_t* launches, int reset) {
    if (!p) return fail(nullptr, MK_ERR_ARG, "mk_profile: plan is NULL");
    if (kind < 0 || kind > 4) return fail(p, MK_ERR_ARG, "mk_profile: unknown kernel kind");
    if (!(p->d.flags & MK_FLAG_PROFILE))
        return fail(p, MK_ERR_UNSUPPORTED, "mk_profile: plan was created without MK_FLAG_PROFILE");
    HIP_TRY(p, prof_resolve(p));
    if (total_ms) *total_ms = p->prof[kind].ms;
    if (launches) *launches = p->prof[kind].launches;
    if (reset) p->prof[kind] = ProfileSlot{};
    return MK_OK;
}

mk_status mk_destroy(mk_plan_t p) {
    if (!p) return MK_OK;
    (void)hipStreamSynchronize(p->stream);
    free_plan_memory(p);
    delete p;
    return MK_OK;
}

}  // extern "C"
