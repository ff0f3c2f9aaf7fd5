// Error reporting, argument checks and host-side geometry of libpact.
#include "common.h"

#include <cstring>

namespace pact {

namespace {
thread_local char g_err[512] = "";
}

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

int launch_status(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: HIP launch failed: %s", what, hipGetErrorString(e));
        return PACT_EHIP;
    }
    return PACT_OK;
}

int device_cu_count() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (cached[dev] <= 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

int check_ring(const pact_ring& r) {
    PACT_CHECK_ARG(r.n_elem > 0, "ring: n_elem must be positive (got %d)", r.n_elem);
    PACT_CHECK_ARG(r.radius > 0.0f && std::isfinite(r.radius), "ring: radius must be positive and finite");
    PACT_CHECK_ARG(std::isfinite(r.phi0), "ring: phi0 must be finite");
    return PACT_OK;
}

int check_grid(const pact_grid& g, const char* what) {
    PACT_CHECK_ARG(g.ny > 0 && g.nx > 0, "%s: grid sizes must be positive (got %d x %d)", what, g.ny, g.nx);
    PACT_CHECK_ARG(g.spacing > 0.0f && std::isfinite(g.spacing), "%s: grid spacing must be positive", what);
    return PACT_OK;
}

}  // namespace pact

extern "C" {

const char* pact_last_error(void) { return pact::g_err; }

int pact_version(void) { return 2; }

int pact_patch_count(const pact_grid* img_, const pact_patches* pp_, int* npy, int* npx) {
    pact::clear_error();
    PACT_CHECK_ARG(img_ && pp_, "pact_patch_count: null geometry pointer");
    const pact_grid img = *img_;
    const pact_patches pp = *pp_;
    if (int s = pact::check_grid(img, "pact_patch_count")) return s;
    PACT_CHECK_ARG(npy && npx, "pact_patch_count: null output pointer");
    PACT_CHECK_ARG(pp.P > 0 && pp.stride > 0, "pact_patch_count: P and stride must be positive");
    PACT_CHECK_ARG(pp.P <= img.ny && pp.P <= img.nx, "pact_patch_count: patch larger than the image");
    *npy = (img.ny - pp.P) / pp.stride + 1;
    *npx = (img.nx - pp.P) / pp.stride + 1;
    return PACT_OK;
}

int pact_patch_centres(const pact_grid* img_, const pact_patches* pp_, float* centres_host) {
    int npy = 0, npx = 0;
    if (int s = pact_patch_count(img_, pp_, &npy, &npx)) return s;
    const pact_grid img = *img_;
    const pact_patches pp = *pp_;
    PACT_CHECK_ARG(centres_host, "pact_patch_centres: null output pointer");
    // mean of the pixel centres of rows a*stride .. a*stride + P - 1 (same for columns)
    const double half = 0.5 * (pp.P - 1);
    for (int a = 0; a < npy; ++a) {
        for (int b = 0; b < npx; ++b) {
            const double x = (b * pp.stride + half - 0.5 * (img.nx - 1)) * img.spacing;
            const double y = (a * pp.stride + half - 0.5 * (img.ny - 1)) * img.spacing;
            centres_host[2 * (a * npx + b) + 0] = static_cast<float>(x);
            centres_host[2 * (a * npx + b) + 1] = static_cast<float>(y);
        }
    }
    return PACT_OK;
}

}  // extern "C"
