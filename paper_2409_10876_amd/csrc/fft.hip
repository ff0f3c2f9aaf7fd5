// Windowed patch spectra (Eq. conv / Sec. 3.3) and the inverse transform of patch spectra.
//
// One workgroup per (patch, delay) image.  The P x P patch (P <= 96, any P --
// the paper-scale 80 = 2^4 * 5 is not a power of two) is staged in LDS with its
// Gaussian window applied, then transformed as two passes of length-P DFTs
// (rows, then columns) against an LDS twiddle table e^{-2 pi i m / P}: P^2 (P/2+1)
// complex multiply-adds per pass for the half spectrum.  Once per scan, this is
// a few GFLOP at the paper scale; the loads of a patch row and the stores of a
// spectrum row are coalesced.
#include "common.h"

namespace pact {
namespace {

__global__ __launch_bounds__(256) void patch_dft_kernel(const float* __restrict__ stack, int M, int ny, int nx,
                                                        int P, int stride, int npx, float px, float inv_two_sigma2,
                                                        int Wout, float2* __restrict__ Y) {
    extern __shared__ float lds[];
    float* xs = lds;                       // [P][P] windowed patch
    float* zr = xs + P * P;                // [P][Wout] row transforms
    float* zi = zr + P * Wout;
    float* twc = zi + P * Wout;            // [P] cos(2 pi m / P)
    float* tws = twc + P;                  // [P] sin(2 pi m / P)
    float* g1 = tws + P;                   // [P] 1-D window factor

    const int img = blockIdx.x;            // = i * M + j
    const int i = img / M;
    const int j = img % M;
    const int r0 = (i / npx) * stride;
    const int c0 = (i % npx) * stride;
    const int tid = threadIdx.x;

    for (int m = tid; m < P; m += blockDim.x) {
        float s, c;
        sincospif(2.0f * m / P, &s, &c);
        twc[m] = c;
        tws[m] = s;
        const float u = (m - 0.5f * (P - 1)) * px;
        g1[m] = expf(-u * u * inv_two_sigma2);
    }
    __syncthreads();
    const float* src = stack + (static_cast<size_t>(j) * ny + r0) * nx + c0;
    for (int idx = tid; idx < P * P; idx += blockDim.x) {
        const int u = idx / P, v = idx % P;
        xs[idx] = src[static_cast<size_t>(u) * nx + v] * (g1[u] * g1[v]);
    }
    __syncthreads();
    // rows: z[u][kx] = sum_v x[u][v] e^{-2 pi i v kx / P}
    for (int idx = tid; idx < P * Wout; idx += blockDim.x) {
        const int u = idx / Wout, kx = idx % Wout;
        const float* row = xs + u * P;
        float ar = 0.0f, ai = 0.0f;
        int m = 0;
        for (int v = 0; v < P; ++v) {
            const float xv = row[v];
            ar = fmaf(xv, twc[m], ar);
            ai = fmaf(-xv, tws[m], ai);
            m += kx;
            if (m >= P) m -= P;
        }
        zr[idx] = ar;
        zi[idx] = ai;
    }
    __syncthreads();
    // columns: Y[ky][kx] = sum_u z[u][kx] e^{-2 pi i u ky / P}
    float2* dst = Y + static_cast<size_t>(img) * P * Wout;
    for (int idx = tid; idx < P * Wout; idx += blockDim.x) {
        const int ky = idx / Wout, kx = idx % Wout;
        float ar = 0.0f, ai = 0.0f;
        int m = 0;
        for (int u = 0; u < P; ++u) {
            const float a = zr[u * Wout + kx], b = zi[u * Wout + kx];
            const float c = twc[m], s = tws[m];
            ar = fmaf(a, c, fmaf(b, s, ar));
            ai = fmaf(b, c, fmaf(-a, s, ai));
            m += ky;
            if (m >= P) m -= P;
        }
        dst[idx] = make_float2(ar, ai);
    }
}

// x[b] = Re(IFFT2(X[b])) for full P x P spectra.
__global__ __launch_bounds__(256) void idft_real_kernel(const float2* __restrict__ X, int P,
                                                        float* __restrict__ x) {
    extern __shared__ float lds[];
    float* ar_ = lds;                      // [P][P] input re
    float* ai_ = ar_ + P * P;              // [P][P] input im
    float* zr = ai_ + P * P;               // [P][P] after the column pass (re)
    float* zi = zr + P * P;
    float* twc = zi + P * P;
    float* tws = twc + P;
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    for (int m = tid; m < P; m += blockDim.x) {
        float s, c;
        sincospif(2.0f * m / P, &s, &c);
        twc[m] = c;
        tws[m] = s;
    }
    const float2* src = X + static_cast<size_t>(b) * P * P;
    for (int idx = tid; idx < P * P; idx += blockDim.x) {
        const float2 v = src[idx];
        ar_[idx] = v.x;
        ai_[idx] = v.y;
    }
    __syncthreads();
    // z[u][kx] = sum_ky X[ky][kx] e^{+2 pi i ky u / P}
    for (int idx = tid; idx < P * P; idx += blockDim.x) {
        const int u = idx / P, kx = idx % P;
        float sr = 0.0f, si = 0.0f;
        int m = 0;
        for (int ky = 0; ky < P; ++ky) {
            const float a = ar_[ky * P + kx], bb = ai_[ky * P + kx];
            const float c = twc[m], s = tws[m];
            sr = fmaf(a, c, fmaf(-bb, s, sr));
            si = fmaf(a, s, fmaf(bb, c, si));
            m += u;
            if (m >= P) m -= P;
        }
        zr[idx] = sr;
        zi[idx] = si;
    }
    __syncthreads();
    // x[u][v] = Re(sum_kx z[u][kx] e^{+2 pi i kx v / P}) / P^2
    const float scale = 1.0f / (static_cast<float>(P) * P);
    float* dst = x + static_cast<size_t>(b) * P * P;
    for (int idx = tid; idx < P * P; idx += blockDim.x) {
        const int u = idx / P, v = idx % P;
        float sr = 0.0f;
        int m = 0;
        for (int kx = 0; kx < P; ++kx) {
            sr = fmaf(zr[u * P + kx], twc[m], fmaf(-zi[u * P + kx], tws[m], sr));
            m += v;
            if (m >= P) m -= P;
        }
        dst[idx] = sr * scale;
    }
}

}  // namespace

int launch_idft_real(const float* X, int B, int P, float* x, hipStream_t stream) {
    const size_t lds = (4 * static_cast<size_t>(P) * P + 2 * P) * sizeof(float);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(idft_real_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        attr = true;
    }
    idft_real_kernel<<<B, 256, lds, stream>>>(reinterpret_cast<const float2*>(X), P, x);
    return launch_status("pact_ifft2_real");
}

}  // namespace pact

extern "C" int pact_patch_fft(const float* stack, int M, const pact_grid* img_, const pact_patches* pp_, int half, float* Y,
                              void* stream) {
    if (!img_ || !pp_) {
        pact::set_error("pact_patch_fft: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_grid img = *img_;
    const pact_patches pp = *pp_;
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(stack && Y, "pact_patch_fft: null pointer");
    PACT_CHECK_ARG(M > 0, "pact_patch_fft: M must be positive");
    PACT_CHECK_ARG(pp.fwhm > 0.0f, "pact_patch_fft: fwhm must be positive");
    int npy = 0, npx = 0;
    if (int s = pact_patch_count(&img, &pp, &npy, &npx)) return s;
    PACT_CHECK_SUPPORTED(pp.P <= kMaxPatch, "pact_patch_fft: P = %d exceeds %d", pp.P, kMaxPatch);
    const int P = pp.P;
    const int Wout = half ? P / 2 + 1 : P;
    const double sigma = pp.fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    const float inv_two_sigma2 = static_cast<float>(1.0 / (2.0 * sigma * sigma));
    const size_t lds = (static_cast<size_t>(P) * P + 2 * static_cast<size_t>(P) * Wout + 3 * P) * sizeof(float);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(patch_dft_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        attr = true;
    }
    patch_dft_kernel<<<npy * npx * M, 256, lds, as_stream(stream)>>>(stack, M, img.ny, img.nx, P, pp.stride, npx,
                                                                   img.spacing, inv_two_sigma2, Wout,
                                                                   reinterpret_cast<float2*>(Y));
    return launch_status("pact_patch_fft");
}

extern "C" int pact_ifft2_real(const float* X, int B, int P, float* x, void* stream) {
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(X && x, "pact_ifft2_real: null pointer");
    PACT_CHECK_ARG(B > 0 && P > 0, "pact_ifft2_real: B and P must be positive");
    PACT_CHECK_SUPPORTED(P <= kMaxPatch, "pact_ifft2_real: P = %d exceeds %d", P, kMaxPatch);
    return launch_idft_real(X, B, P, x, as_stream(stream));
}
