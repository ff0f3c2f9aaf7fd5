// Delay-and-sum stack, Eq. DAS (Sec. 3.1), for every extra delay of the stack (Sec. 3.2).
//
// One thread per pixel, 16 x 16 pixel tiles per workgroup, up to 16 delays per launch (the delay count is a
// template argument, so the per-delay loop is unrolled without guards).  Element positions are staged in
// LDS 256 at a time (FP64).  Per (pixel, element) the distance |p - r_n| and the sample position
// tb = fs (|p - r_n| / v0 - t0) are formed in FP64 -- a sample index near 4000 would lose ~5e-4 samples
// in FP32 -- and split into an integer ti and a fraction tf in [0, 1).  Each delay's position
// tb - fs d_j / v0 is then ti + (tf - e_j) with e_j = fs d_j / v0 in FP32: |tf - e_j| stays within a few
// tens of samples, so this costs about 1e-6 samples.  When every delay's pair of samples lies inside the
// record (tested once per element), the two loads per delay are unconditional and all of them are in
// flight together; else each is guarded.  Interpolation and the sum over elements run in FP32.  The
// records of one element are read by the 64 lanes of a wave at nearby sample positions, so the gathers
// hit the same few cache lines.
#include "common.h"

#include <algorithm>

namespace pact {
namespace {

constexpr int kTile = 16;
constexpr int kDelayChunk = 16;
constexpr int kElemChunk = 256;

template <int MC>
__global__ __launch_bounds__(256) void das_kernel(const float* __restrict__ S, int n_t, double base0,
                                                  double fs_over_v0, int n_elem, double R, double phi0,
                                                  const float* __restrict__ d, int j0, int ny, int nx, double px,
                                                  float* __restrict__ stack) {
    __shared__ double ex[kElemChunk];
    __shared__ double ey[kElemChunk];
    __shared__ float esh[MC];

    const int c = blockIdx.x * kTile + (threadIdx.x % kTile);
    const int r = blockIdx.y * kTile + (threadIdx.x / kTile);
    // clamped to +-1e6 samples (far beyond any record), so that the integer offsets below cannot overflow
    if (threadIdx.x < MC)
        esh[threadIdx.x] = fminf(fmaxf(static_cast<float>(static_cast<double>(d[j0 + threadIdx.x]) * fs_over_v0), -1.0e6f),
                                 1.0e6f);

    const double x = (c - 0.5 * (nx - 1)) * px;
    const double y = (r - 0.5 * (ny - 1)) * px;

    float acc[MC];
#pragma unroll
    for (int j = 0; j < MC; ++j) acc[j] = 0.0f;

    const double dphi = 2.0 * M_PI / n_elem;
    for (int e0 = 0; e0 < n_elem; e0 += kElemChunk) {
        const int ne = min(kElemChunk, n_elem - e0);
        __syncthreads();
        for (int e = threadIdx.x; e < ne; e += blockDim.x) {
            double sn, cs;
            sincos(phi0 + dphi * (e0 + e), &sn, &cs);
            ex[e] = R * cs;
            ey[e] = R * sn;
        }
        __syncthreads();
        // the offsets floor(tf - e_j) of the delays lie in [lo, hi] for every tf in [0, 1)
        float ej[MC];
        int lo = 0, hi = 0;
#pragma unroll
        for (int j = 0; j < MC; ++j) {
            ej[j] = esh[j];
            const int a0 = static_cast<int>(floorf(-ej[j])), a1 = static_cast<int>(floorf(1.0f - ej[j]));
            lo = j ? min(lo, a0) : a0;
            hi = j ? max(hi, a1) : a1;
        }
        for (int e = 0; e < ne; ++e) {
            const double dx = x - ex[e];
            const double dy = y - ey[e];
            const double tb = sqrt(dx * dx + dy * dy) * fs_over_v0 + base0;
            const double tfl = fmin(fmax(floor(tb), -1.0e9), 1.0e9);
            const int ti = static_cast<int>(tfl);
            const float tf = static_cast<float>(tb - tfl);
            const float* rec = S + static_cast<size_t>(e0 + e) * n_t;
            if (ti + lo >= 0 && ti + hi + 1 < n_t) {
#pragma unroll
                for (int j = 0; j < MC; ++j) {
                    const float u = tf - ej[j];
                    const float fl = floorf(u);
                    const float* p = rec + (ti + static_cast<int>(fl));
                    const float s0 = p[0], s1 = p[1];
                    acc[j] += fmaf(u - fl, s1 - s0, s0);
                }
            } else {
#pragma unroll
                for (int j = 0; j < MC; ++j) {
                    const float u = tf - ej[j];
                    const float fl = floorf(u);
                    const int i0 = ti + static_cast<int>(fl);
                    const float s0 = (i0 >= 0 && i0 < n_t) ? rec[i0] : 0.0f;
                    const float s1 = (i0 + 1 >= 0 && i0 + 1 < n_t) ? rec[i0 + 1] : 0.0f;
                    acc[j] += fmaf(u - fl, s1 - s0, s0);
                }
            }
        }
    }
    if (r < ny && c < nx) {
#pragma unroll
        for (int j = 0; j < MC; ++j) stack[(static_cast<size_t>(j0 + j) * ny + r) * nx + c] = acc[j];
    }
}

template <int MC>
void launch_das(dim3 grid, hipStream_t st, const float* S, int n_t, double base0, double fs_over_v0, int n_elem,
                double R, double phi0, const float* d, int j0, int ny, int nx, double px, float* stack) {
    das_kernel<MC><<<grid, 256, 0, st>>>(S, n_t, base0, fs_over_v0, n_elem, R, phi0, d, j0, ny, nx, px, stack);
}

using DasLaunch = void (*)(dim3, hipStream_t, const float*, int, double, double, int, double, double, const float*,
                           int, int, int, double, float*);
constexpr DasLaunch kDasLaunch[kDelayChunk] = {
    launch_das<1>,  launch_das<2>,  launch_das<3>,  launch_das<4>,  launch_das<5>,  launch_das<6>,
    launch_das<7>,  launch_das<8>,  launch_das<9>,  launch_das<10>, launch_das<11>, launch_das<12>,
    launch_das<13>, launch_das<14>, launch_das<15>, launch_das<16>};

}  // namespace
}  // namespace pact

extern "C" int pact_das_stack(const float* S, int n_t, float fs, float t0, const pact_ring* ring_, float v0,
                              const float* d, int M, const pact_grid* img_, float* stack, void* stream) {
    if (!ring_ || !img_) {
        pact::set_error("pact_das_stack: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_ring ring = *ring_;
    const pact_grid img = *img_;
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(S && d && stack, "pact_das_stack: null pointer");
    PACT_CHECK_ARG(n_t > 0 && M > 0, "pact_das_stack: n_t and M must be positive");
    PACT_CHECK_ARG(fs > 0.0f && v0 > 0.0f && std::isfinite(t0), "pact_das_stack: fs and v0 must be positive");
    if (int s = check_ring(ring)) return s;
    if (int s = check_grid(img, "pact_das_stack")) return s;
    const double fs_over_v0 = static_cast<double>(fs) / v0;
    const double base0 = -static_cast<double>(t0) * fs;
    const dim3 grid(ceil_div(img.nx, kTile), ceil_div(img.ny, kTile));
    for (int j0 = 0; j0 < M; j0 += kDelayChunk) {
        const int mc = std::min(kDelayChunk, M - j0);
        kDasLaunch[mc - 1](grid, as_stream(stream), S, n_t, base0, fs_over_v0, ring.n_elem, ring.radius, ring.phi0, d,
                           j0, img.ny, img.nx, img.spacing, stack);
        if (int s = launch_status("pact_das_stack")) return s;
    }
    return PACT_OK;
}
