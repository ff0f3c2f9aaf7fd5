// Multichannel deconvolution, Eq. fm_fourier / Eq. multi-deconv (Sec. 3.2), its adjoint, and the
// data term of Eq. jr for given H and X (the modular, H-materialising path).
//
// One thread per (patch, frequency bin); the M channels of a bin are strided by
// P^2 complex values, so each channel read is a coalesced row of the wave.
#include "common.h"

namespace pact {
namespace {

__global__ __launch_bounds__(256) void deconv_kernel(const float2* __restrict__ Y, const float2* __restrict__ H,
                                                     int M, int PP, float eps, float2* __restrict__ X) {
    const int bin = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (bin >= PP) return;
    float ar = 0.0f, ai = 0.0f, den = eps;
    for (int j = 0; j < M; ++j) {
        const size_t o = (static_cast<size_t>(i) * M + j) * PP + bin;
        const float2 h = H[o], y = Y[o];
        ar = fmaf(h.x, y.x, fmaf(h.y, y.y, ar));     // conj(h) y
        ai = fmaf(h.x, y.y, fmaf(-h.y, y.x, ai));
        den = fmaf(h.x, h.x, fmaf(h.y, h.y, den));
    }
    const float inv = 1.0f / den;
    X[static_cast<size_t>(i) * PP + bin] = make_float2(ar * inv, ai * inv);
}

// dL/dH_j = (conj(g) Y_j - 2 Re(conj(g) X) H_j) / B with X = A / B, A = sum conj(H) Y, B = sum |H|^2 + eps.
__global__ __launch_bounds__(256) void deconv_adj_kernel(const float2* __restrict__ Y, const float2* __restrict__ H,
                                                         int M, int PP, float eps, const float2* __restrict__ gX,
                                                         float2* __restrict__ gH) {
    const int bin = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (bin >= PP) return;
    float ar = 0.0f, ai = 0.0f, den = eps;
    for (int j = 0; j < M; ++j) {
        const size_t o = (static_cast<size_t>(i) * M + j) * PP + bin;
        const float2 h = H[o], y = Y[o];
        ar = fmaf(h.x, y.x, fmaf(h.y, y.y, ar));
        ai = fmaf(h.x, y.y, fmaf(-h.y, y.x, ai));
        den = fmaf(h.x, h.x, fmaf(h.y, h.y, den));
    }
    const float inv = 1.0f / den;
    const float xr = ar * inv, xi = ai * inv;
    const float2 g = gX[static_cast<size_t>(i) * PP + bin];
    const float re_gx = g.x * xr + g.y * xi;         // Re(conj(g) X)
    for (int j = 0; j < M; ++j) {
        const size_t o = (static_cast<size_t>(i) * M + j) * PP + bin;
        const float2 h = H[o], y = Y[o];
        // conj(g) y = (g.x y.x + g.y y.y) + j (g.x y.y - g.y y.x)
        const float cr = g.x * y.x + g.y * y.y - 2.0f * re_gx * h.x;
        const float ci = g.x * y.y - g.y * y.x - 2.0f * re_gx * h.y;
        gH[o] = make_float2(cr * inv, ci * inv);
    }
}

__global__ __launch_bounds__(256) void residual_kernel(const float2* __restrict__ Y, const float2* __restrict__ H,
                                                       const float2* __restrict__ X, int M, int P,
                                                       float two_pi_over_Ppx, float2* __restrict__ gH,
                                                       float2* __restrict__ gX, float* __restrict__ partial) {
    __shared__ float red[4];
    const int PP = P * P;
    const int bin = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    float l = 0.0f;
    if (bin < PP) {
        const float kx = fft_wavenumber(bin % P, P, two_pi_over_Ppx);
        const float ky = fft_wavenumber(bin / P, P, two_pi_over_Ppx);
        const float kabs = sqrtf(kx * kx + ky * ky);
        const float2 x = X[static_cast<size_t>(i) * PP + bin];
        float gxr = 0.0f, gxi = 0.0f;
        for (int j = 0; j < M; ++j) {
            const size_t o = (static_cast<size_t>(i) * M + j) * PP + bin;
            const float2 h = H[o], y = Y[o];
            const float rr = y.x - (h.x * x.x - h.y * x.y);
            const float ri = y.y - (h.x * x.y + h.y * x.x);
            l = fmaf(rr, rr, fmaf(ri, ri, l));
            if (gH) {   // -2|k| r conj(x)
                gH[o] = make_float2(-2.0f * kabs * (rr * x.x + ri * x.y), -2.0f * kabs * (ri * x.x - rr * x.y));
            }
            gxr += rr * h.x + ri * h.y;       // r conj(h)
            gxi += ri * h.x - rr * h.y;
        }
        l *= kabs;
        if (gX) gX[static_cast<size_t>(i) * PP + bin] = make_float2(-2.0f * kabs * gxr, -2.0f * kabs * gxi);
    }
    const float s = block_sum(l, red);
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void finish_sum_kernel(const float* __restrict__ partial, int n,
                                                         float* __restrict__ out) {
    __shared__ float red[4];
    // fixed assignment of partials to threads and a fixed reduction tree: deterministic
    float s = 0.0f;
    for (int k = threadIdx.x; k < n; k += blockDim.x) s += partial[k];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *out = s;
}

int check_spec(const void* a, const void* b, int N, int M, int P, const char* what) {
    PACT_CHECK_ARG(a && b, "%s: null pointer", what);
    PACT_CHECK_ARG(N > 0 && M > 0 && P > 0, "%s: N, M and P must be positive", what);
    return PACT_OK;
}

}  // namespace
}  // namespace pact

extern "C" int pact_multichannel_deconv(const float* Y, const float* H, int N, int M, int P, float eps, float* X,
                                        void* stream) {
    using namespace pact;
    clear_error();
    if (int s = check_spec(Y, H, N, M, P, "pact_multichannel_deconv")) return s;
    PACT_CHECK_ARG(X, "pact_multichannel_deconv: null output");
    PACT_CHECK_ARG(eps >= 0.0f && std::isfinite(eps), "pact_multichannel_deconv: eps must be >= 0");
    dim3 grid(ceil_div(P * P, 256), N);
    deconv_kernel<<<grid, 256, 0, as_stream(stream)>>>(reinterpret_cast<const float2*>(Y),
                                                       reinterpret_cast<const float2*>(H), M, P * P, eps,
                                                       reinterpret_cast<float2*>(X));
    return launch_status("pact_multichannel_deconv");
}

extern "C" int pact_multichannel_deconv_adjoint(const float* Y, const float* H, int N, int M, int P, float eps,
                                                const float* dL_dX, float* dL_dH, void* stream) {
    using namespace pact;
    clear_error();
    if (int s = check_spec(Y, H, N, M, P, "pact_multichannel_deconv_adjoint")) return s;
    PACT_CHECK_ARG(dL_dX && dL_dH, "pact_multichannel_deconv_adjoint: null pointer");
    PACT_CHECK_ARG(eps >= 0.0f && std::isfinite(eps), "pact_multichannel_deconv_adjoint: eps must be >= 0");
    dim3 grid(ceil_div(P * P, 256), N);
    deconv_adj_kernel<<<grid, 256, 0, as_stream(stream)>>>(
        reinterpret_cast<const float2*>(Y), reinterpret_cast<const float2*>(H), M, P * P, eps,
        reinterpret_cast<const float2*>(dL_dX), reinterpret_cast<float2*>(dL_dH));
    return launch_status("pact_multichannel_deconv_adjoint");
}

extern "C" size_t pact_residual_loss_workspace_size(int N, int P) {
    if (N <= 0 || P <= 0) return 0;
    return static_cast<size_t>(N) * pact::ceil_div(static_cast<long long>(P) * P, 256) * sizeof(float);
}

extern "C" int pact_residual_loss(const float* Y, const float* H, const float* X, int N, int M, int P, float px,
                                  float* loss, float* dL_dH, float* dL_dX, void* ws, size_t ws_bytes,
                                  void* stream) {
    using namespace pact;
    clear_error();
    if (int s = check_spec(Y, H, N, M, P, "pact_residual_loss")) return s;
    PACT_CHECK_ARG(X && loss, "pact_residual_loss: null pointer");
    PACT_CHECK_ARG(px > 0.0f, "pact_residual_loss: px must be positive");
    const size_t need = pact_residual_loss_workspace_size(N, P);
    if (!ws || ws_bytes < need) {
        set_error("pact_residual_loss: workspace of %zu bytes needed, %zu given", need, ws_bytes);
        return PACT_EWORKSPACE;
    }
    const float k0 = static_cast<float>(2.0 * M_PI / (static_cast<double>(P) * px));
    dim3 grid(ceil_div(P * P, 256), N);
    residual_kernel<<<grid, 256, 0, as_stream(stream)>>>(
        reinterpret_cast<const float2*>(Y), reinterpret_cast<const float2*>(H), reinterpret_cast<const float2*>(X),
        M, P, k0, reinterpret_cast<float2*>(dL_dH), reinterpret_cast<float2*>(dL_dX), static_cast<float*>(ws));
    if (int s = launch_status("pact_residual_loss")) return s;
    finish_sum_kernel<<<1, 256, 0, as_stream(stream)>>>(static_cast<float*>(ws), grid.x * grid.y, loss);
    return launch_status("pact_residual_loss (sum)");
}
