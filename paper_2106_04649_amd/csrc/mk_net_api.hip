// C ABI of the series-tail network kernels (training and inference on
// caller-owned device buffers).
#include <mutex>

#include "mk_internal.h"

// Partial sums of mk_net_loss_noalloc: one double per block of the loss
// kernel.  Every GPU the library runs on holds its own copy until the process
// ends; the host side reaches it only through the per-device address below
// (the array's own name is not a device address in host code).
constexpr int kLossScratchParts = 1024;
static __device__ __align__(256) double scratch[kLossScratchParts];

namespace {
thread_local std::string g_net_error;

mk_status net_fail(mk_status st, const std::string& m) {
    g_net_error = m;
    return st;
}

mk_status net_hip(hipError_t e, const char* where) {
    if (e == hipSuccess) return MK_OK;
    return net_fail(MK_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool net_dims_ok(int N, int k, int T) { return N >= 1 && k >= 1 && k <= 16 && T >= 1 && T <= 4096; }
bool hidden_ok(int H) { return H >= 1 && H <= kNetHiddenMax; }

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
mk_status scratch_on_current_device(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return net_hip(e, "mk_net_loss_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return net_fail(MK_ERR_UNSUPPORTED, "mk_net_loss_noalloc: device index");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return net_hip(e, "mk_net_loss_noalloc: hipGetSymbolAddress");
        if (!ptr) return net_fail(MK_ERR_HIP, "mk_net_loss_noalloc: no address for the scratch array");
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return MK_OK;
}
}  // namespace

extern "C" {

int32_t mk_net_param_count(int32_t k, int32_t hidden) {
    return k >= 1 && k <= 16 && hidden_ok(hidden) ? net_param_count(k, hidden) : -1;
}

const char* mk_net_last_error(void) { return g_net_error.c_str(); }

mk_status mk_net_forward(const float* params, const float* x, int32_t N, int32_t k, int32_t hidden, int32_t T,
                         float* work, float* y, void* stream) {
    if (!params || !x || !work || !y) return net_fail(MK_ERR_ARG, "mk_net_forward: NULL pointer");
    if (!net_dims_ok(N, k, T) || !hidden_ok(hidden))
        return net_fail(MK_ERR_ARG, "mk_net_forward: bad N, k, hidden or T");
    const size_t act = (size_t)N * hidden * T;
    return net_hip(net_forward(params, x, N, k, hidden, T, work, work + act, y, (hipStream_t)stream),
                   "mk_net_forward");
}

mk_status mk_net_backward(const float* params, const float* x, const float* work, const float* gy, int32_t N,
                          int32_t k, int32_t hidden, int32_t T, float* grads, float* work2, void* stream) {
    if (!params || !x || !work || !gy || !grads || !work2)
        return net_fail(MK_ERR_ARG, "mk_net_backward: NULL pointer");
    if (!net_dims_ok(N, k, T) || !hidden_ok(hidden))
        return net_fail(MK_ERR_ARG, "mk_net_backward: bad N, k, hidden or T");
    const size_t act = (size_t)N * hidden * T;
    return net_hip(net_backward(params, x, work, work + act, gy, N, k, hidden, T, grads, work2, work2 + act,
                                work2 + 2 * act, (hipStream_t)stream),
                   "mk_net_backward");
}

mk_status mk_net_loss(const float* y, const float* target, const float* mask, int32_t N, int32_t T,
                            float count, float* gy, double* loss, double* part, int32_t nparts,
                            void* stream) {
    if (!y || !target || !mask || !gy || !loss || !part || nparts < 1)
        return net_fail(MK_ERR_ARG, "mk_net_loss: NULL pointer or nparts < 1");
    if (!net_dims_ok(N, 1, T) || !(count > 0.f)) return net_fail(MK_ERR_ARG, "mk_net_loss: bad N, T or count");
    return net_hip(net_mse(y, target, mask, N, T, gy, part, nparts, loss, count, (hipStream_t)stream),
                   "mk_net_loss");
}

mk_status mk_net_loss_noalloc(const float* y, const float* target, const float* mask, int32_t N, int32_t T,
                              float count, float* gy, double* loss, int32_t nparts, void* stream) {
    if (!y || !target || !mask || !gy || !loss) return net_fail(MK_ERR_ARG, "mk_net_loss_noalloc: NULL pointer");
    if (nparts < 1 || nparts > kLossScratchParts)
        return net_fail(MK_ERR_ARG, "mk_net_loss_noalloc: nparts must be in [1, " +
                                        std::to_string(kLossScratchParts) + "]");
    if (!net_dims_ok(N, 1, T) || !(count > 0.f))
        return net_fail(MK_ERR_ARG, "mk_net_loss_noalloc: bad N, T or count");
    double* part = nullptr;
    const mk_status st = scratch_on_current_device(&part);
    if (st != MK_OK) return st;
    // every block of the loss kernel writes its own partial: nothing to clear
    return net_hip(net_mse(y, target, mask, N, T, gy, part, nparts, loss, count, (hipStream_t)stream),
                   "mk_net_loss_noalloc");
}

mk_status mk_net_adam(float* w, float* wq, const float* g, float* m, float* v, int32_t n, int32_t step, float lr,
                      float b1, float b2, float eps, void* stream) {
    if (!w || !wq || !g || !m || !v || n < 1 || step < 1) return net_fail(MK_ERR_ARG, "mk_net_adam: bad argument");
    return net_hip(net_adam(w, wq, g, m, v, n, step, lr, b1, b2, eps, (hipStream_t)stream), "mk_net_adam");
}

mk_status mk_net_round(const float* w, float* wq, int32_t n, void* stream) {
    if (!w || !wq || n < 1) return net_fail(MK_ERR_ARG, "mk_net_round: bad argument");
    return net_hip(net_round_bf16(w, wq, n, (hipStream_t)stream), "mk_net_round");
}

}  // extern "C"
