// Delay-and-sum stack, Eq. DAS (Sec. 3.1), for every extra delay of the stack (Sec. 3.2).
//
// One thread per pixel, 16 x 16 pixel tiles per workgroup, up to 16 delays per
// launch slice (grid.z).  Element positions are staged in LDS 256 at a time
// (FP64).  The distance |p - r_n| and the fractional sample position are formed
// in FP64 -- a sample index near 4000 would lose ~5e-4 samples in FP32 -- and the
// linear interpolation and the sum over elements run in FP32.  The records of
// one element are read by the 64 lanes of a wave at nearby sample positions, so
// the gathers hit the same few cache lines.
#include "common.h"

namespace pact {
namespace {

constexpr int kTile = 16;
constexpr int kDelayChunk = 16;
constexpr int kElemChunk = 256;

__global__ __launch_bounds__(256) void das_kernel(const float* __restrict__ S, int n_t, double base0,
                                                  double fs_over_v0, int n_elem, double R, double phi0,
                                                  const float* __restrict__ d, int M, int ny, int nx, double px,
                                                  float* __restrict__ stack) {
    __shared__ double ex[kElemChunk];
    __shared__ double ey[kElemChunk];
    __shared__ double dsh[kDelayChunk];

    const int j0 = blockIdx.z * kDelayChunk;
    const int mc = min(kDelayChunk, M - j0);
    const int c = blockIdx.x * kTile + (threadIdx.x % kTile);
    const int r = blockIdx.y * kTile + (threadIdx.x / kTile);
    if (threadIdx.x < mc) dsh[threadIdx.x] = static_cast<double>(d[j0 + threadIdx.x]) * fs_over_v0;

    const double x = (c - 0.5 * (nx - 1)) * px;
    const double y = (r - 0.5 * (ny - 1)) * px;

    float acc[kDelayChunk];
#pragma unroll
    for (int j = 0; j < kDelayChunk; ++j) acc[j] = 0.0f;

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
        for (int e = 0; e < ne; ++e) {
            const double dx = x - ex[e];
            const double dy = y - ey[e];
            const double tb = sqrt(dx * dx + dy * dy) * fs_over_v0 + base0;
            const float* rec = S + static_cast<size_t>(e0 + e) * n_t;
#pragma unroll
            for (int j = 0; j < kDelayChunk; ++j) {
                if (j < mc) {
                    const double tau = tb - dsh[j];
                    const double fl = fmin(fmax(floor(tau), -2.0), static_cast<double>(n_t));
                    const int i0 = static_cast<int>(fl);
                    const float a = static_cast<float>(tau - fl);
                    const float s0 = (i0 >= 0 && i0 < n_t) ? rec[i0] : 0.0f;
                    const float s1 = (i0 + 1 >= 0 && i0 + 1 < n_t) ? rec[i0 + 1] : 0.0f;
                    acc[j] += fmaf(a, s1 - s0, s0);
                }
            }
        }
    }
    if (r < ny && c < nx) {
#pragma unroll
        for (int j = 0; j < kDelayChunk; ++j)
            if (j < mc) stack[(static_cast<size_t>(j0 + j) * ny + r) * nx + c] = acc[j];
    }
}

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
    dim3 grid(ceil_div(img.nx, kTile), ceil_div(img.ny, kTile), ceil_div(M, kDelayChunk));
    das_kernel<<<grid, 256, 0, as_stream(stream)>>>(S, n_t, base0, fs_over_v0, ring.n_elem, ring.radius, ring.phi0,
                                                   d, M, img.ny, img.nx, img.spacing, stack);
    return launch_status("pact_das_stack");
}
