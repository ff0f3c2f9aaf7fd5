// Straight-ray wavefront errors, Eq. TOF / Eq. wf (Sec. 3.1), and their adjoint.
//
// The node grid of SOS contrasts delta = v - v0 is staged in LDS with a one-node
// ring of zeros (the fixed background), so that every midpoint sample inside
// the clipped ray reads its four bilinear neighbours without a bounds test:
// (G + 2)^2 floats, 80.6 KB at G = 140, two workgroups of 1024 threads per CU.
// A ray (patch i, element n) is owned by a group of kLanes consecutive lanes;
// lane l takes samples l, l + kLanes, ...; the group sums with cross-lane
// shuffles.  The integrand is evaluated as delta / (v0 + delta) = 1 - v0 / v,
// which keeps the contrast exact instead of cancelling 1 against v0 / v.
//
// Adjoint: each workgroup privatises the gradient grid in LDS next to the SOS
// grid (2 x 80.6 KB at G = 140, one workgroup per CU), scatters
// dL/dw * dl * v0 / v^2 * (bilinear weight) with LDS float atomics, and writes
// its partial grid; a second kernel sums the partials in a fixed order.
#include "common.h"

namespace pact {

int device_cu_count();

namespace {

constexpr int kLanes = 16;       // lanes per ray
constexpr int kThreads = 1024;

struct RayGeo {
    float inv_ds;       // 1 / node spacing
    float off_x;        // (Gx + 1) / 2: padded node coordinate of x = 0
    float off_y;
    float hx, hy;       // half-extent of the box where v differs from v0
    int Gx, Gy, W;      // W = Gx + 2 (padded row length)
};

__device__ __forceinline__ void load_contrast(float* vs, const float* __restrict__ sos, float v0, const RayGeo& g) {
    const int total = (g.Gy + 2) * g.W;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int a = idx / g.W - 1, b = idx % g.W - 1;
        vs[idx] = (a >= 0 && a < g.Gy && b >= 0 && b < g.Gx) ? sos[a * g.Gx + b] - v0 : 0.0f;
    }
}

// Geometry of ray (i, n): padded node coordinates of the start point, their increment per step,
// and the step length.
__device__ __forceinline__ void ray_setup(const float* __restrict__ centres, int i, int n, int n_elem, float R,
                                          float phi0, int Ns, const RayGeo& g, float& gx0, float& gy0, float& dgx,
                                          float& dgy, float& dl) {
    const float cx = centres[2 * i], cy = centres[2 * i + 1];
    float sn, cs;
    sincosf(phi0 + kTwoPi * (static_cast<float>(n) / n_elem), &sn, &cs);
    const float dx = R * cs - cx, dy = R * sn - cy;
    const float dist = sqrtf(dx * dx + dy * dy);
    const float ux = dx / dist, uy = dy / dist;
    float L = dist;
    if (ux > 0.0f) L = fminf(L, (g.hx - cx) / ux);
    if (ux < 0.0f) L = fminf(L, (-g.hx - cx) / ux);
    if (uy > 0.0f) L = fminf(L, (g.hy - cy) / uy);
    if (uy < 0.0f) L = fminf(L, (-g.hy - cy) / uy);
    L = fmaxf(L, 0.0f);
    dl = L / Ns;
    gx0 = fmaf(cx, g.inv_ds, g.off_x);
    gy0 = fmaf(cy, g.inv_ds, g.off_y);
    dgx = dl * ux * g.inv_ds;
    dgy = dl * uy * g.inv_ds;
}

// Padded cell index and fractions of a sample (clamped so that the 2 x 2 stencil stays in the grid).
__device__ __forceinline__ int sample_cell(float gx, float gy, const RayGeo& g, float& fx, float& fy) {
    const float bf = floorf(gx), af = floorf(gy);
    fx = gx - bf;
    fy = gy - af;
    const int b0 = min(max(static_cast<int>(bf), 0), g.Gx);
    const int a0 = min(max(static_cast<int>(af), 0), g.Gy);
    return a0 * g.W + b0;
}

__global__ __launch_bounds__(kThreads) void rays_fwd_kernel(const float* __restrict__ sos, float v0,
                                                            const float* __restrict__ centres, int N, int n_elem,
                                                            float R, float phi0, int Ns, RayGeo g,
                                                            float* __restrict__ w) {
    extern __shared__ float vs[];
    load_contrast(vs, sos, v0, g);
    __syncthreads();
    const int lane = threadIdx.x % kLanes;
    const long long n_rays = static_cast<long long>(N) * n_elem;
    const long long groups = static_cast<long long>(gridDim.x) * (blockDim.x / kLanes);
    for (long long ray = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) / kLanes; ray < n_rays;
         ray += groups) {
        const int i = static_cast<int>(ray / n_elem), n = static_cast<int>(ray % n_elem);
        float gx0, gy0, dgx, dgy, dl;
        ray_setup(centres, i, n, n_elem, R, phi0, Ns, g, gx0, gy0, dgx, dgy, dl);
        float acc = 0.0f;
        for (int s = lane; s < Ns; s += kLanes) {
            const float sf = static_cast<float>(s) + 0.5f;
            float fx, fy;
            const int c = sample_cell(fmaf(sf, dgx, gx0), fmaf(sf, dgy, gy0), g, fx, fy);
            const float v00 = vs[c], v01 = vs[c + 1], v10 = vs[c + g.W], v11 = vs[c + g.W + 1];
            const float top = fmaf(fx, v01 - v00, v00);
            const float bot = fmaf(fx, v11 - v10, v10);
            const float dv = fmaf(fy, bot - top, top);
            acc = fmaf(dv, __builtin_amdgcn_rcpf(v0 + dv), acc);
        }
#pragma unroll
        for (int off = kLanes / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kLanes);
        if (lane == 0) w[ray] = acc * dl;
    }
}

__global__ __launch_bounds__(kThreads) void rays_adj_kernel(const float* __restrict__ sos, float v0,
                                                            const float* __restrict__ centres, int N, int n_elem,
                                                            float R, float phi0, int Ns, RayGeo g,
                                                            const float* __restrict__ dL_dw,
                                                            float* __restrict__ partial) {
    extern __shared__ float lds[];
    float* vs = lds;
    float* gacc = lds + (g.Gy + 2) * g.W;
    load_contrast(vs, sos, v0, g);
    for (int idx = threadIdx.x; idx < (g.Gy + 2) * g.W; idx += blockDim.x) gacc[idx] = 0.0f;
    __syncthreads();
    const int lane = threadIdx.x % kLanes;
    const long long n_rays = static_cast<long long>(N) * n_elem;
    const long long groups = static_cast<long long>(gridDim.x) * (blockDim.x / kLanes);
    for (long long ray = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) / kLanes; ray < n_rays;
         ray += groups) {
        const float gw = dL_dw[ray];
        if (gw == 0.0f) continue;
        const int i = static_cast<int>(ray / n_elem), n = static_cast<int>(ray % n_elem);
        float gx0, gy0, dgx, dgy, dl;
        ray_setup(centres, i, n, n_elem, R, phi0, Ns, g, gx0, gy0, dgx, dgy, dl);
        const float scale = gw * dl * v0;
        for (int s = lane; s < Ns; s += kLanes) {
            const float sf = static_cast<float>(s) + 0.5f;
            float fx, fy;
            const int c = sample_cell(fmaf(sf, dgx, gx0), fmaf(sf, dgy, gy0), g, fx, fy);
            const float v00 = vs[c], v01 = vs[c + 1], v10 = vs[c + g.W], v11 = vs[c + g.W + 1];
            const float top = fmaf(fx, v01 - v00, v00);
            const float bot = fmaf(fx, v11 - v10, v10);
            const float r = __builtin_amdgcn_rcpf(v0 + fmaf(fy, bot - top, top));
            const float q = scale * r * r;                      // dL/dw * dl * v0 / v^2
            const float qy1 = q * fy, qy0 = q - qy1;
            atomicAdd(&gacc[c], qy0 - qy0 * fx);
            atomicAdd(&gacc[c + 1], qy0 * fx);
            atomicAdd(&gacc[c + g.W], qy1 - qy1 * fx);
            atomicAdd(&gacc[c + g.W + 1], qy1 * fx);
        }
    }
    __syncthreads();
    float* dst = partial + static_cast<size_t>(blockIdx.x) * g.Gy * g.Gx;
    for (int idx = threadIdx.x; idx < g.Gy * g.Gx; idx += blockDim.x) {
        const int a = idx / g.Gx, b = idx % g.Gx;
        dst[idx] = gacc[(a + 1) * g.W + b + 1];
    }
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const float* __restrict__ partial, int nparts, int n,
                                                           const float* __restrict__ scale, int accumulate,
                                                           float* __restrict__ out) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    float s = 0.0f;
    for (int p = 0; p < nparts; ++p) s += partial[static_cast<size_t>(p) * n + idx];
    if (scale) s *= *scale;
    out[idx] = accumulate ? out[idx] + s : s;
}

RayGeo make_geo(const pact_grid& sosg) {
    RayGeo g;
    g.inv_ds = 1.0f / sosg.spacing;
    g.off_x = 0.5f * (sosg.nx + 1);
    g.off_y = 0.5f * (sosg.ny + 1);
    g.hx = 0.5f * (sosg.nx + 1) * sosg.spacing;
    g.hy = 0.5f * (sosg.ny + 1) * sosg.spacing;
    g.Gx = sosg.nx;
    g.Gy = sosg.ny;
    g.W = sosg.nx + 2;
    return g;
}

int check_rays(const float* sos, pact_grid sosg, float v0, const float* centres, int N, pact_ring ring,
               int n_samples, const char* what) {
    PACT_CHECK_ARG(sos && centres, "%s: null pointer", what);
    PACT_CHECK_ARG(N > 0 && n_samples > 0, "%s: N and n_samples must be positive", what);
    PACT_CHECK_ARG(v0 > 0.0f && std::isfinite(v0), "%s: v0 must be positive", what);
    if (int s = check_ring(ring)) return s;
    if (int s = check_grid(sosg, what)) return s;
    return PACT_OK;
}

int adj_blocks() { return device_cu_count(); }

}  // namespace
}  // namespace pact

extern "C" int pact_sos_to_delays(const float* sos, const pact_grid* sosg_, float v0, const float* centres, int N,
                                  const pact_ring* ring_, int n_samples, float* w, void* stream) {
    if (!sosg_ || !ring_) {
        pact::set_error("pact_sos_to_delays: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_grid sosg = *sosg_;
    const pact_ring ring = *ring_;
    using namespace pact;
    clear_error();
    if (int s = check_rays(sos, sosg, v0, centres, N, ring, n_samples, "pact_sos_to_delays")) return s;
    PACT_CHECK_ARG(w, "pact_sos_to_delays: null output");
    const size_t lds = static_cast<size_t>(sosg.ny + 2) * (sosg.nx + 2) * sizeof(float);
    PACT_CHECK_SUPPORTED(lds <= kLdsBytes, "pact_sos_to_delays: SOS grid %d x %d does not fit in LDS", sosg.ny,
                         sosg.nx);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(rays_fwd_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        attr = true;
    }
    const long long n_rays = static_cast<long long>(N) * ring.n_elem;
    const int per_block = kThreads / kLanes;
    const int blocks = static_cast<int>(std::min<long long>((n_rays + per_block - 1) / per_block,
                                                            2LL * device_cu_count()));
    rays_fwd_kernel<<<blocks, kThreads, lds, as_stream(stream)>>>(sos, v0, centres, N, ring.n_elem, ring.radius,
                                                                 ring.phi0, n_samples, make_geo(sosg), w);
    return launch_status("pact_sos_to_delays");
}

extern "C" size_t pact_sos_to_delays_adjoint_workspace_size(const pact_grid* sosg_, int N, const pact_ring* ring_) {
    if (!sosg_ || !ring_) return 0;
    const pact_grid sosg = *sosg_;
    const pact_ring ring = *ring_;
    (void)N;
    (void)ring;
    if (sosg.ny <= 0 || sosg.nx <= 0) return 0;
    return static_cast<size_t>(pact::adj_blocks()) * sosg.ny * sosg.nx * sizeof(float);
}

extern "C" int pact_sos_to_delays_adjoint(const float* sos, const pact_grid* sosg_, float v0, const float* centres, int N,
                                          const pact_ring* ring_, int n_samples, const float* dL_dw, const float* scale,
                                          float* dL_dsos, int accumulate, void* ws, size_t ws_bytes,
                                          void* stream) {
    if (!sosg_ || !ring_) {
        pact::set_error("pact_sos_to_delays_adjoint: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_grid sosg = *sosg_;
    const pact_ring ring = *ring_;
    using namespace pact;
    clear_error();
    if (int s = check_rays(sos, sosg, v0, centres, N, ring, n_samples, "pact_sos_to_delays_adjoint")) return s;
    PACT_CHECK_ARG(dL_dw && dL_dsos, "pact_sos_to_delays_adjoint: null pointer");
    const size_t lds = 2 * static_cast<size_t>(sosg.ny + 2) * (sosg.nx + 2) * sizeof(float);
    PACT_CHECK_SUPPORTED(lds <= kLdsBytes, "pact_sos_to_delays_adjoint: SOS grid %d x %d does not fit in LDS",
                         sosg.ny, sosg.nx);
    const size_t need = pact_sos_to_delays_adjoint_workspace_size(&sosg, N, &ring);
    if (!ws || ws_bytes < need) {
        set_error("pact_sos_to_delays_adjoint: workspace of %zu bytes needed, %zu given", need, ws_bytes);
        return PACT_EWORKSPACE;
    }
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(rays_adj_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        attr = true;
    }
    const int blocks = adj_blocks();
    float* partial = static_cast<float*>(ws);
    rays_adj_kernel<<<blocks, kThreads, lds, as_stream(stream)>>>(sos, v0, centres, N, ring.n_elem, ring.radius,
                                                                 ring.phi0, n_samples, make_geo(sosg), dL_dw,
                                                                 partial);
    if (int s = launch_status("pact_sos_to_delays_adjoint")) return s;
    const int n = sosg.ny * sosg.nx;
    sum_partials_kernel<<<ceil_div(n, 256), 256, 0, as_stream(stream)>>>(partial, blocks, n, scale, accumulate,
                                                                        dL_dsos);
    return launch_status("pact_sos_to_delays_adjoint (sum)");
}
