// C ABI of the series-tail network kernels (training and inference on
// caller-owned device buffers).
#include "mk_internal.h"

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
