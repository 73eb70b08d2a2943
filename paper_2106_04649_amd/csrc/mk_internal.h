// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mk.h"

// Per-trace kernel modes (one wave per trace of nt samples).
enum TraceMode : int {
    TM_INIT = 0,   // N_-1 = Gd(-t); f1+ = N_-1; f1- = 0; X = rfft(N_-1)
    TM_ITER = 1,   // RN = irfft(Y); N = mute(-RN(-t)); accumulate; X = rfft(N)
    TM_GFWD = 2,   // X[f] = rfft(f1+[f]); X[nf + f] = rfft(f1-[f](-t))
    TM_GOUT = 3    // G- = irfft(Y[f]) - f1-;  G+ = f1+(-t) - irfft(Y[nf + f])
};

// Arguments of the per-trace kernel.  Layouts (all row-major):
//   Y   [nfo][B][nr]        complex, contraction output (unscaled sum over s)
//   X   [nfo][B][ns_pad]    complex, next contraction input
//   src [nf][nr][nt]        float, G_d for TM_INIT
//   f1p, f1m, gp, gm [nf][nr][nt] float
//   itd [nf][nr], fband [nf][2] (or null), npart [nfo][nr] double
//   tw  [nt] complex: exp(-2 pi i k / nt)
struct TraceArgs {
    const float2* Y;
    float2* X;
    const float* src;
    float* f1p;
    float* f1m;
    float* gp;
    float* gm;
    const int32_t* itd;
    const int32_t* fband;
    double* npart;
    const float2* tw;
    int nr;
    int nf;        // focal points of the series
    int nfo;       // traces are nfo x nr (nf, or 2 nf for the G modes)
    int lo;        // first stored bin
    int B;         // stored bins
    int ns_pad;    // row pitch of X (complex elements)
    int shift;
    int parity;    // pass index & 1 (TM_ITER)
    float scale;   // c / (nt / 2): Riemann weight and inverse-FFT normalisation
};

struct ProfileSlot {
    double ms = 0.0;
    int64_t launches = 0;
};

struct mk_plan_s {
    mk_plan_desc d{};
    int B = 0;          // stored bins
    int M = 0;          // nt / 2
    int ns_pad = 0;     // padded row length of R and X (complex elements, multiple of 4)
    int device = 0;
    hipStream_t stream = nullptr;

    // device memory (plan-owned)
    float2* R = nullptr;       // [B][nr][ns_pad] complex64
    float2* X = nullptr;       // [3 nf_max][B][ns_pad]: series slabs, then G-assembly slabs
    float2* Y = nullptr;       // [2 nf_max][B][nr]
    float* f1p = nullptr;      // [nf_max][nr][nt]
    float* f1m = nullptr;
    float* gp = nullptr;
    float* gm = nullptr;
    int32_t* itd = nullptr;    // [nf_max][nr]
    int32_t* fband = nullptr;  // [nf_max][2]
    double* npart = nullptr;   // [2 nf_max][nr]
    double* norm0 = nullptr;   // [nf_max]
    double* norms = nullptr;   // [norm_cap][nf_max]
    int norm_cap = 0;
    float2* tw = nullptr;      // [nt]
    int* flag = nullptr;       // device scratch flag (non-finite input detection)

    // series state
    int nf = 0;
    int shift = 0;
    int passes = 0;
    bool has_fband = false;
    bool R_loaded = false;
    bool focal_set = false;
    bool g_valid = false;
    std::vector<double> norm0_host;

    // profiling (MK_FLAG_PROFILE)
    struct Pending {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    ProfileSlot prof[5];

    std::string err;
};

// kernel launchers (return hipSuccess or the launch error)
hipError_t launch_trace(int mode, int nt, const TraceArgs& a, hipStream_t s);
hipError_t launch_norm_reduce(const double* npart, int nr, int nfo, double* out, hipStream_t s);
hipError_t launch_contract_c64(const float2* R, const float2* X, float2* Y, int nr, int B,
                               int ns, int ns_pad, int ncols, hipStream_t s);
hipError_t launch_repack_c64(const float* Rin, float2* Rout, int nr, int B, int ns, int ns_pad,
                             int* flag, hipStream_t s);
hipError_t launch_check_finite(const float* x, int64_t n, int* flag, hipStream_t s);
