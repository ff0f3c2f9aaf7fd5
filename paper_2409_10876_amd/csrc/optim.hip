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

__device__ __forceinline__ float sgn(float x) { return x > 0.0f ? 1.0f : (x < 0.0f ? -1.0f : 0.0f); }

__global__ __launch_bounds__(kThreads) void tv_kernel(const float* __restrict__ v,
                                                      const unsigned char* __restrict__ mask, int Gy, int Gx,
                                                      float lambda, float* __restrict__ grad,
                                                      float* __restrict__ loss) {
    __shared__ float red[kThreads / 64];
    const int idx = blockIdx.x * kThreads + threadIdx.x;
    float tv = 0.0f;
    if (idx < Gy * Gx) {
        const int a = idx / Gx, b = idx - a * Gx;
        const float x = v[idx];
        const bool m = mask[idx] != 0;
        float g = 0.0f;
        // pair (a, b)-(a+1, b) and (a, b)-(a, b+1): counted once, by their first node
        if (a + 1 < Gy && (m || mask[idx + Gx])) {
            const float dv = v[idx + Gx] - x;
            tv += fabsf(dv);
            g -= sgn(dv);
        }
        if (b + 1 < Gx && (m || mask[idx + 1])) {
            const float dv = v[idx + 1] - x;
            tv += fabsf(dv);
            g -= sgn(dv);
        }
        // the same pairs seen from their second node
        if (a > 0 && (m || mask[idx - Gx])) g += sgn(x - v[idx - Gx]);
        if (b > 0 && (m || mask[idx - 1])) g += sgn(x - v[idx - 1]);
        grad[idx] = fmaf(lambda, g, grad[idx]);
    }
    tv = block_sum(tv, red);
    if (threadIdx.x == 0 && tv != 0.0f) atomicAdd(loss, lambda * tv);
}

__global__ __launch_bounds__(kThreads) void adam_kernel(float* __restrict__ p, float* __restrict__ m,
                                                        float* __restrict__ v, int* __restrict__ t,
                                                        const unsigned char* __restrict__ mask, int n,
                                                        const float* __restrict__ grad, float lr, float b1, float b2,
                                                        float eps) {
    const int step = t[0] + 1;
    const int idx = blockIdx.x * kThreads + threadIdx.x;
    if (idx < n && (!mask || mask[idx])) {
        const float bc1 = 1.0f - powf(b1, static_cast<float>(step));
        const float bc2 = 1.0f - powf(b2, static_cast<float>(step));
        const float g = grad[idx];
        const float mm = fmaf(b1, m[idx], (1.0f - b1) * g);
        const float vv = fmaf(b2, v[idx], (1.0f - b2) * g * g);
        m[idx] = mm;
        v[idx] = vv;
        p[idx] -= (lr / bc1) * mm / fmaf(sqrtf(vv), 1.0f / sqrtf(bc2), eps);
    }
    // every thread of this workgroup has read t[0] (above the barrier); the last workgroup to arrive
    // advances it
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = atomicAdd(reinterpret_cast<unsigned*>(t + 1), 1u);
        if (prev == gridDim.x - 1) {
            t[0] = step;
            t[1] = 0;
        }
    }
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
