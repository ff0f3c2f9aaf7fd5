// Gaussian-weighted stitching of the deconvolved patches into the image (Supp. S1.4):
//   image[y][x] = sum_i x_i[y - y_i][x - x_i] / sum_i g[y - y_i][x - x_i]   where the weight sum > floor,
// over the patches i whose footprint covers the pixel, g the analysis window of pact_patch_fft.  The
// deconvolved patch estimates the windowed clean patch, so the window enters the weight sum once.
//
// One thread per pixel gathers from the (at most ceil(P / stride)^2) patches that cover it, so the sum
// needs no atomics and is taken in a fixed order.  HBM-bound: it reads every patch pixel once (the
// overlap re-reads hit L2) and writes the image.
#include "common.h"

namespace pact {
namespace {

__global__ __launch_bounds__(256) void stitch_kernel(const float* __restrict__ patches, int ny, int nx, int P,
                                                    int stride, int npy, int npx, float px, float inv_two_sigma2,
                                                    float floor_w, float* __restrict__ image) {
    const int x = blockIdx.x * 16 + (threadIdx.x & 15);
    const int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= nx || y >= ny) return;
    const float c = 0.5f * static_cast<float>(P - 1);
    // patches a with a * stride <= y < a * stride + P
    const int a_hi = min(y / stride, npy - 1);
    const int a_lo = max(0, (y - P + stride) / stride);
    const int b_hi = min(x / stride, npx - 1);
    const int b_lo = max(0, (x - P + stride) / stride);
    float acc = 0.0f, wsum = 0.0f;
    for (int a = a_lo; a <= a_hi; ++a) {
        const int u = y - a * stride;
        if (u < 0 || u >= P) continue;
        const float du = (static_cast<float>(u) - c) * px;
        for (int b = b_lo; b <= b_hi; ++b) {
            const int v = x - b * stride;
            if (v < 0 || v >= P) continue;
            const float dv = (static_cast<float>(v) - c) * px;
            acc += patches[(static_cast<size_t>(a) * npx + b) * P * P + u * P + v];
            wsum += expf(-(du * du + dv * dv) * inv_two_sigma2);
        }
    }
    image[static_cast<size_t>(y) * nx + x] = wsum > floor_w ? acc / wsum : 0.0f;
}

}  // namespace
}  // namespace pact

extern "C" int pact_stitch(const float* patches, int N, const pact_grid* img_, const pact_patches* pp_, float* image,
                           void* stream) {
    if (!img_ || !pp_) {
        pact::set_error("pact_stitch: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_grid img = *img_;
    const pact_patches pp = *pp_;
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(patches && image, "pact_stitch: null pointer");
    if (int s = check_grid(img, "pact_stitch")) return s;
    PACT_CHECK_ARG(pp.P > 0 && pp.stride > 0 && pp.P <= img.ny && pp.P <= img.nx,
                   "pact_stitch: patch size %d / stride %d invalid for a %d x %d image", pp.P, pp.stride, img.ny,
                   img.nx);
    PACT_CHECK_ARG(pp.stride <= pp.P, "pact_stitch: stride larger than the patch leaves pixels uncovered");
    PACT_CHECK_ARG(pp.fwhm > 0.0f, "pact_stitch: fwhm must be positive");
    const int npy = (img.ny - pp.P) / pp.stride + 1, npx = (img.nx - pp.P) / pp.stride + 1;
    PACT_CHECK_ARG(N == npy * npx, "pact_stitch: %d patches given, the geometry has %d", N, npy * npx);
    const double sigma = pp.fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    const float inv_two_sigma2 = static_cast<float>(1.0 / (2.0 * sigma * sigma));
    dim3 grid(ceil_div(img.nx, 16), ceil_div(img.ny, 16));
    stitch_kernel<<<grid, 256, 0, as_stream(stream)>>>(patches, img.ny, img.nx, pp.P, pp.stride, npy, npx, img.spacing,
                                                      inv_two_sigma2, 1e-12f, image);
    return launch_status("pact_stitch");
}
