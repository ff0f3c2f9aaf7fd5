// Transfer functions and PSFs from the wavefront table, Eq. TF (Sec. 3.1), and the adjoint.
//
// These standalone calls materialise H [N][M][P][P]; the optimisation step does
// not use them (the fused loss recomputes what it needs from w), they serve
// the modular path, diagnostics and the PSF images.
//
// Per frequency bin k of patch i: theta = angle of k, u = k / |k|.  The wavefront
// towards theta and theta + pi is read off the element table w[i] at the
// fractional element index where the ray from the patch centre along +u / -u
// meets the ring (linear between neighbouring elements).  Then for each delay
//   H = 1/2 (e^{+j|k|(d - W(theta))} + e^{-j|k|(d - W(theta + pi))})
// (the sign is that of the data's e^{-j k.r} forward transform).
#include "common.h"

namespace pact {

int launch_idft_real(const float* X, int B, int P, float* x, hipStream_t stream);

namespace {

struct BinGeo {
    float kabs;
    int n0a, n1a, n0b, n1b;
    float alpha_a, alpha_b;
};

__device__ __forceinline__ BinGeo bin_geometry(int bin, int P, float two_pi_over_Ppx, float cx, float cy,
                                               float R2mc2, float phi0, int n_elem) {
    BinGeo g;
    const int ky = bin / P, kx = bin % P;
    const float kyv = fft_wavenumber(ky, P, two_pi_over_Ppx);
    const float kxv = fft_wavenumber(kx, P, two_pi_over_Ppx);
    g.kabs = sqrtf(kxv * kxv + kyv * kyv);
    const float inv = g.kabs > 0.0f ? 1.0f / g.kabs : 0.0f;
    const float ux = g.kabs > 0.0f ? kxv * inv : 1.0f;
    const float uy = kyv * inv;
    const float nf = static_cast<float>(n_elem);
    const float n2pi = nf / kTwoPi;
    ring_cell(ring_hit_index(cx, cy, ux, uy, R2mc2, phi0, n2pi, nf), n_elem, g.n0a, g.n1a, g.alpha_a);
    ring_cell(ring_hit_index(cx, cy, -ux, -uy, R2mc2, phi0, n2pi, nf), n_elem, g.n0b, g.n1b, g.alpha_b);
    return g;
}

__global__ __launch_bounds__(256) void psf_kernel(const float* __restrict__ w, const float* __restrict__ centres,
                                                  int n_elem, float R, float phi0, const float* __restrict__ d, int M,
                                                  int P, float two_pi_over_Ppx, float2* __restrict__ H) {
    extern __shared__ float wl[];
    const int i = blockIdx.y;
    for (int n = threadIdx.x; n < n_elem; n += blockDim.x) wl[n] = w[static_cast<size_t>(i) * n_elem + n];
    __syncthreads();
    const int bin = blockIdx.x * blockDim.x + threadIdx.x;
    if (bin >= P * P) return;
    const float cx = centres[2 * i], cy = centres[2 * i + 1];
    const BinGeo g = bin_geometry(bin, P, two_pi_over_Ppx, cx, cy, R * R - (cx * cx + cy * cy), phi0, n_elem);
    const float Wa = fmaf(g.alpha_a, wl[g.n1a] - wl[g.n0a], wl[g.n0a]);
    const float Wb = fmaf(g.alpha_b, wl[g.n1b] - wl[g.n0b], wl[g.n0b]);
    for (int j = 0; j < M; ++j) {
        const float dj = d[j];
        float sa, ca, sb, cb;
        sincosf(g.kabs * (dj - Wa), &sa, &ca);
        sincosf(g.kabs * (dj - Wb), &sb, &cb);
        H[(static_cast<size_t>(i) * M + j) * P * P + bin] = make_float2(0.5f * (ca + cb), 0.5f * (sa - sb));
    }
}

// One workgroup per patch; the element gradient is accumulated in LDS and written once.
__global__ __launch_bounds__(256) void psf_adj_kernel(const float* __restrict__ w,
                                                      const float* __restrict__ centres, int n_elem, float R,
                                                      float phi0, const float* __restrict__ d, int M, int P,
                                                      float two_pi_over_Ppx, const float2* __restrict__ gH,
                                                      float* __restrict__ dL_dw) {
    extern __shared__ float lds[];
    float* wl = lds;
    float* gw = lds + n_elem;
    const int i = blockIdx.x;
    for (int n = threadIdx.x; n < n_elem; n += blockDim.x) {
        wl[n] = w[static_cast<size_t>(i) * n_elem + n];
        gw[n] = 0.0f;
    }
    __syncthreads();
    const float cx = centres[2 * i], cy = centres[2 * i + 1];
    const float R2mc2 = R * R - (cx * cx + cy * cy);
    for (int bin = threadIdx.x; bin < P * P; bin += blockDim.x) {
        const BinGeo g = bin_geometry(bin, P, two_pi_over_Ppx, cx, cy, R2mc2, phi0, n_elem);
        if (g.kabs == 0.0f) continue;
        const float Wa = fmaf(g.alpha_a, wl[g.n1a] - wl[g.n0a], wl[g.n0a]);
        const float Wb = fmaf(g.alpha_b, wl[g.n1b] - wl[g.n0b], wl[g.n0b]);
        float ga = 0.0f, gb = 0.0f;
        for (int j = 0; j < M; ++j) {
            const float2 g2 = gH[(static_cast<size_t>(i) * M + j) * P * P + bin];
            float sa, ca, sb, cb;
            sincosf(g.kabs * (d[j] - Wa), &sa, &ca);
            sincosf(g.kabs * (d[j] - Wb), &sb, &cb);
            // dH/dW(theta) = -j|k|/2 e^{j alpha};  dH/dW(theta+pi) = +j|k|/2 e^{-j beta}
            ga += g2.x * sa - g2.y * ca;
            gb += g2.x * sb + g2.y * cb;
        }
        ga *= 0.5f * g.kabs;
        gb *= 0.5f * g.kabs;
        atomicAdd(&gw[g.n0a], ga - g.alpha_a * ga);
        atomicAdd(&gw[g.n1a], g.alpha_a * ga);
        atomicAdd(&gw[g.n0b], gb - g.alpha_b * gb);
        atomicAdd(&gw[g.n1b], g.alpha_b * gb);
    }
    __syncthreads();
    for (int n = threadIdx.x; n < n_elem; n += blockDim.x) dL_dw[static_cast<size_t>(i) * n_elem + n] = gw[n];
}

int check_psf(const float* w, const float* centres, int N, pact_ring ring, const float* d, int M, int P, float px,
              const char* what) {
    PACT_CHECK_ARG(w && centres && d, "%s: null pointer", what);
    PACT_CHECK_ARG(N > 0 && M > 0 && P > 0, "%s: N, M and P must be positive", what);
    PACT_CHECK_ARG(px > 0.0f && std::isfinite(px), "%s: px must be positive", what);
    if (int s = check_ring(ring)) return s;
    PACT_CHECK_SUPPORTED(P <= kMaxPatch, "%s: P = %d exceeds %d", what, P, kMaxPatch);
    PACT_CHECK_SUPPORTED(2 * static_cast<size_t>(ring.n_elem) * sizeof(float) <= kLdsBytes,
                         "%s: n_elem = %d too large", what, ring.n_elem);
    return PACT_OK;
}

}  // namespace
}  // namespace pact

extern "C" int pact_delays_to_psf(const float* w, const float* centres, int N, const pact_ring* ring_, const float* d, int M,
                                  int P, float px, float* H, float* h_opt, void* stream) {
    if (!ring_) {
        pact::set_error("pact_delays_to_psf: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_ring ring = *ring_;
    using namespace pact;
    clear_error();
    if (int s = check_psf(w, centres, N, ring, d, M, P, px, "pact_delays_to_psf")) return s;
    PACT_CHECK_ARG(H, "pact_delays_to_psf: null output");
    const float k0 = static_cast<float>(2.0 * M_PI / (static_cast<double>(P) * px));
    dim3 grid(ceil_div(P * P, 256), N);
    psf_kernel<<<grid, 256, ring.n_elem * sizeof(float), as_stream(stream)>>>(
        w, centres, ring.n_elem, ring.radius, ring.phi0, d, M, P, k0, reinterpret_cast<float2*>(H));
    if (int s = launch_status("pact_delays_to_psf")) return s;
    if (h_opt) return launch_idft_real(H, N * M, P, h_opt, as_stream(stream));
    return PACT_OK;
}

extern "C" int pact_delays_to_psf_adjoint(const float* w, const float* centres, int N, const pact_ring* ring_,
                                          const float* d, int M, int P, float px, const float* dL_dH, float* dL_dw,
                                          void* stream) {
    if (!ring_) {
        pact::set_error("pact_delays_to_psf_adjoint: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_ring ring = *ring_;
    using namespace pact;
    clear_error();
    if (int s = check_psf(w, centres, N, ring, d, M, P, px, "pact_delays_to_psf_adjoint")) return s;
    PACT_CHECK_ARG(dL_dH && dL_dw, "pact_delays_to_psf_adjoint: null pointer");
    const float k0 = static_cast<float>(2.0 * M_PI / (static_cast<double>(P) * px));
    psf_adj_kernel<<<N, 256, 2 * ring.n_elem * sizeof(float), as_stream(stream)>>>(
        w, centres, ring.n_elem, ring.radius, ring.phi0, d, M, P, k0, reinterpret_cast<const float2*>(dL_dH), dL_dw);
    return launch_status("pact_delays_to_psf_adjoint");
}
