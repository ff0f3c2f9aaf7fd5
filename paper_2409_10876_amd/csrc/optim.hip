// Total-variation term of Eq. jr and the Adam update of the pixel-grid SOS (Sec. 3.3).
//
// Both run one thread per node over as many workgroups as the grid needs.  The
// TV value is summed per workgroup in a fixed order and added to the loss with
// one float atomic per workgroup (so its last bits may vary between runs; the
// gradient does not).  Adam reads the device-side step counter t[0] in every
// workgroup; the last workgroup to finish (an arrival counter in t[1]) writes
// t[0] + 1 and resets t[1], so a captured step can be replayed.
#include "common.h"

namespace pact {
namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void tv_kernel(const float* __restrict__ v,
                                                      const unsigned char* __restrict__ mask, int Gy, int Gx,
                                                      float lambda, float* __restrict__ grad,
                                                      float* __restrict__ loss) {
    __shared__ float red[kThreads / 64];
    const int idx = blockIdx.x * kThreads + threadIdx.x;
    float tv = 0.0f;
    if (idx < Gy * Gx) {
        const int a = idx / Gx, b = idx - a * Gx;
        float g;
        tv_node(v, mask, idx, a, b, Gy, Gx, tv, g);
        grad[idx] = fmaf(lambda, g, grad[idx]);
    }
    tv = block_sum(tv, red);
    if (threadIdx.x == 0 && tv != 0.0f) atomicAdd(loss, lambda * tv);
}

// TV subgradient added to the data gradient, then Adam, reading sos_in and writing sos_out (so that every
// thread sees its neighbours' old values); fixed nodes are copied.
__global__ __launch_bounds__(kThreads) void tv_adam_kernel(const float* __restrict__ sos_in,
                                                           float* __restrict__ sos_out, float* __restrict__ m,
                                                           float* __restrict__ v, int* __restrict__ t,
                                                           const unsigned char* __restrict__ mask, int Gy, int Gx,
                                                           const float* __restrict__ grad, float lambda,
                                                           float* __restrict__ loss, float lr, float b1, float b2,
                                                           float eps) {
    __shared__ float red[kThreads / 64];
    const int step = t[0] + 1;
    const int idx = blockIdx.x * kThreads + threadIdx.x;
    float tv = 0.0f;
    if (idx < Gy * Gx) {
        const int a = idx / Gx, b = idx - a * Gx;
        // every load up front (m, v and the gradient also for fixed nodes, which leave them unchanged)
        const float gd = grad[idx];
        float mm = m[idx], vv = v[idx];
        float g_tv = 0.0f;
        if (lambda != 0.0f) tv_node(sos_in, mask, idx, a, b, Gy, Gx, tv, g_tv);
        float p = sos_in[idx];
        if (mask[idx]) {
            p = adam_node(p, fmaf(lambda, g_tv, gd), mm, vv, step, lr, b1, b2, eps);
            m[idx] = mm;
            v[idx] = vv;
        }
        sos_out[idx] = p;
    }
    if (loss) {
        tv = block_sum(tv, red);
        if (threadIdx.x == 0 && tv != 0.0f) atomicAdd(loss, lambda * tv);
    }
    advance_step(t, step);
}

__global__ __launch_bounds__(kThreads) void adam_kernel(float* __restrict__ p, float* __restrict__ m,
                                                        float* __restrict__ v, int* __restrict__ t,
                                                        const unsigned char* __restrict__ mask, int n,
                                                        const float* __restrict__ grad, float lr, float b1, float b2,
                                                        float eps) {
    const int step = t[0] + 1;
    const int idx = blockIdx.x * kThreads + threadIdx.x;
    if (idx < n && (!mask || mask[idx])) {
        float mm = m[idx], vv = v[idx];
        p[idx] = adam_node(p[idx], grad[idx], mm, vv, step, lr, b1, b2, eps);
        m[idx] = mm;
        v[idx] = vv;
    }
    advance_step(t, step);
}

}  // namespace
}  // namespace pact

extern "C" int pact_tv_grad(const float* sos, const unsigned char* mask, const pact_grid* sosg_, float lambda, float* grad,
                            float* loss, void* stream) {
    if (!sosg_) {
        pact::set_error("pact_tv_grad: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_grid sosg = *sosg_;
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(sos && mask && grad && loss, "pact_tv_grad: null pointer");
    if (int s = check_grid(sosg, "pact_tv_grad")) return s;
    PACT_CHECK_ARG(std::isfinite(lambda), "pact_tv_grad: lambda must be finite");
    tv_kernel<<<ceil_div(static_cast<long long>(sosg.ny) * sosg.nx, kThreads), kThreads, 0, as_stream(stream)>>>(
        sos, mask, sosg.ny, sosg.nx, lambda, grad, loss);
    return launch_status("pact_tv_grad");
}

extern "C" int pact_adam_step(float* sos, float* m, float* v, int* t, const unsigned char* mask, int n,
                              const float* grad, float lr, float b1, float b2, float eps, void* stream) {
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(sos && m && v && t && grad, "pact_adam_step: null pointer");
    PACT_CHECK_ARG(n > 0, "pact_adam_step: n must be positive");
    PACT_CHECK_ARG(b1 >= 0.0f && b1 < 1.0f && b2 >= 0.0f && b2 < 1.0f, "pact_adam_step: betas must be in [0, 1)");
    PACT_CHECK_ARG(eps > 0.0f && std::isfinite(lr), "pact_adam_step: eps must be positive and lr finite");
    adam_kernel<<<ceil_div(n, kThreads), kThreads, 0, as_stream(stream)>>>(sos, m, v, t, mask, n, grad, lr, b1, b2,
                                                                           eps);
    return launch_status("pact_adam_step");
}

extern "C" int pact_tv_adam_step(const float* sos_in, float* sos_out, float* m, float* v, int* t,
                                 const unsigned char* mask, const pact_grid* sosg_, const float* grad, float lambda,
                                 float* loss, float lr, float b1, float b2, float eps, void* stream) {
    if (!sosg_) {
        pact::set_error("pact_tv_adam_step: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_grid sosg = *sosg_;
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(sos_in && sos_out && m && v && t && mask && grad, "pact_tv_adam_step: null pointer");
    PACT_CHECK_ARG(sos_in != sos_out, "pact_tv_adam_step: sos_out must not be sos_in");
    if (int s = check_grid(sosg, "pact_tv_adam_step")) return s;
    PACT_CHECK_ARG(std::isfinite(lambda), "pact_tv_adam_step: lambda must be finite");
    PACT_CHECK_ARG(b1 >= 0.0f && b1 < 1.0f && b2 >= 0.0f && b2 < 1.0f, "pact_tv_adam_step: betas must be in [0, 1)");
    PACT_CHECK_ARG(eps > 0.0f && std::isfinite(lr), "pact_tv_adam_step: eps must be positive and lr finite");
    tv_adam_kernel<<<ceil_div(static_cast<long long>(sosg.ny) * sosg.nx, kThreads), kThreads, 0,
                     as_stream(stream)>>>(sos_in, sos_out, m, v, t, mask, sosg.ny, sosg.nx, grad, lambda, loss, lr,
                                          b1, b2, eps);
    return launch_status("pact_tv_adam_step");
}
