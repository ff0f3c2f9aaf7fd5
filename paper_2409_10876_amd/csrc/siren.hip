// The paper's neural-field SOS (Sec. 3.3): one hidden layer of sinusoidal features on the SOS-grid node
// coordinates, v = v0 + s (w2 . sin(omega0 (W1 x + b1)) + b2) + o on the free nodes, v0 on the fixed ones;
// x = node centre / mask radius.  The node grid then feeds the straight-ray kernels like the pixel grid.
//
// Forward: four lanes per node, each summing a quarter of the features (then two shuffles), the
// parameters in LDS.  Adjoint: one workgroup per chunk of 64 nodes with one thread per hidden feature, so
// each thread accumulates its own feature's gradients over the chunk without atomics; per-chunk partials
// are summed in a fixed order by two small kernels.  Small chunks give ~300 workgroups at 140 x 140 nodes,
// enough to spread the 1027-parameter network over the chip.
#include "common.h"

namespace pact {
namespace {

constexpr int kSirenMaxHidden = 1024;
constexpr int kNodesPerChunk = 64;
constexpr int kLanesPerNode = 4;

__device__ __forceinline__ void node_xy(int idx, int Gy, int Gx, float spacing, float inv_rho, float& x, float& y) {
    const int a = idx / Gx, b = idx - a * Gx;
    x = (static_cast<float>(b) - 0.5f * static_cast<float>(Gx - 1)) * spacing * inv_rho;
    y = (static_cast<float>(a) - 0.5f * static_cast<float>(Gy - 1)) * spacing * inv_rho;
}

// Part of w2 . sin(omega0 (W1 (x, y) + b1)) over features k0, k0 + step, ... (parameters in LDS).  The sine
// comes from the hardware unit, which takes revolutions (reduced to [-1/2, 1/2]), as in the adjoint.
__device__ __forceinline__ float siren_part(const float* p, int H, float omega0, float x, float y, int k0, int step) {
    const float* W1 = p;
    const float* b1 = p + 2 * H;
    const float* w2 = p + 3 * H;
    const float rev_per_unit = omega0 * (1.0f / kTwoPi);
    float f = 0.0f;
    for (int k = k0; k < H; k += step) {
        float rev = rev_per_unit * fmaf(W1[2 * k], x, fmaf(W1[2 * k + 1], y, b1[k]));
        rev -= rintf(rev);
        f = fmaf(w2[k], __builtin_amdgcn_sinf(rev), f);
    }
    return f;
}

__global__ __launch_bounds__(256) void siren_fwd_kernel(const float* __restrict__ params, int H, float omega0,
                                                       const unsigned char* __restrict__ mask, int Gy, int Gx,
                                                       float spacing, float inv_rho, float v0,
                                                       float* __restrict__ sos) {
    __shared__ float p[4 * kSirenMaxHidden + 3];
    for (int k = threadIdx.x; k < 4 * H + 3; k += blockDim.x) p[k] = params[k];
    __syncthreads();
    // lanes 4j .. 4j + 3 of the workgroup share node blockIdx.x * 64 + j
    const int idx = blockIdx.x * (blockDim.x / kLanesPerNode) + threadIdx.x / kLanesPerNode;
    const int part = threadIdx.x % kLanesPerNode;
    const bool live = idx < Gy * Gx && mask[idx] != 0;
    float f = 0.0f;
    if (live) {
        float x, y;
        node_xy(idx, Gy, Gx, spacing, inv_rho, x, y);
        f = siren_part(p, H, omega0, x, y, part, kLanesPerNode);
    }
    f += __shfl_xor(f, 1, kLanesPerNode);
    f += __shfl_xor(f, 2, kLanesPerNode);
    if (part == 0 && idx < Gy * Gx) sos[idx] = live ? v0 + fmaf(p[4 * H + 1], f + p[4 * H], p[4 * H + 2]) : v0;
}

// Partial gradients of one chunk of nodes: partial[chunk][4H + 3] in the parameter layout.
__global__ __launch_bounds__(256) void siren_adj_kernel(const float* __restrict__ params, int H, float omega0,
                                                       const unsigned char* __restrict__ mask, int Gy, int Gx,
                                                       float spacing, float inv_rho,
                                                       const float* __restrict__ dL_dsos,
                                                       float* __restrict__ partial) {
    __shared__ float p[4 * kSirenMaxHidden + 3];
    __shared__ float nx_[kNodesPerChunk], ny_[kNodesPerChunk], ng[kNodesPerChunk], nf[kNodesPerChunk];
    __shared__ float red[256 / 64];
    for (int k = threadIdx.x; k < 4 * H + 3; k += blockDim.x) p[k] = params[k];
    __syncthreads();
    const int n0 = blockIdx.x * kNodesPerChunk;
    const int count = min(kNodesPerChunk, Gy * Gx - n0);
    const float s = p[4 * H + 1];
    // per node of the chunk (four lanes per node): coordinates, g = dL/dv on free nodes (0 on fixed ones)
    // and the network output
    float gsum = 0.0f, gfsum = 0.0f;
    {
        const int j = threadIdx.x / kLanesPerNode, part = threadIdx.x % kLanesPerNode;
        float x = 0.0f, y = 0.0f, g = 0.0f, f = 0.0f;
        const bool live = j < count && mask[n0 + j] != 0;
        if (j < count) node_xy(n0 + j, Gy, Gx, spacing, inv_rho, x, y);
        if (live) f = siren_part(p, H, omega0, x, y, part, kLanesPerNode);
        f += __shfl_xor(f, 1, kLanesPerNode);
        f += __shfl_xor(f, 2, kLanesPerNode);
        if (live) {
            g = dL_dsos[n0 + j];
            f += p[4 * H];
        }
        if (part == 0) {
            nx_[j] = x;
            ny_[j] = y;
            ng[j] = g;
            nf[j] = f;
            gsum = g;
            gfsum = g * f;
        }
    }
    gsum = block_sum(gsum, red);
    gfsum = block_sum(gfsum, red);     // its barriers also publish the node tables
    float* out = partial + static_cast<size_t>(blockIdx.x) * (4 * H + 3);
    for (int k = threadIdx.x; k < H; k += blockDim.x) {
        const float wx = p[2 * k], wy = p[2 * k + 1], bk = p[2 * H + k], w2k = p[3 * H + k];
        float gW1x = 0.0f, gW1y = 0.0f, gb1 = 0.0f, gw2 = 0.0f;
        for (int j = 0; j < count; ++j) {
            const float g = ng[j];
            if (g == 0.0f) continue;
            // sin and cos from the hardware units, which take revolutions (reduced to [-1/2, 1/2]); their
            // error, ~1e-6, is far inside the gradient tolerance
            float rev = omega0 * fmaf(wx, nx_[j], fmaf(wy, ny_[j], bk)) * (1.0f / kTwoPi);
            rev -= rintf(rev);
            const float sn = __builtin_amdgcn_sinf(rev), cs = __builtin_amdgcn_cosf(rev);
            const float df = g * s;                        // dL/df at the node
            gw2 = fmaf(df, sn, gw2);
            const float dz = df * w2k * cs * omega0;       // dL/d(W1[k] . x + b1[k])
            gb1 += dz;
            gW1x = fmaf(dz, nx_[j], gW1x);
            gW1y = fmaf(dz, ny_[j], gW1y);
        }
        out[2 * k] = gW1x;
        out[2 * k + 1] = gW1y;
        out[2 * H + k] = gb1;
        out[3 * H + k] = gw2;
    }
    if (threadIdx.x == 0) {
        out[4 * H] = gsum * s;          // b2
        out[4 * H + 1] = gfsum;         // s
        out[4 * H + 2] = gsum;          // o
    }
}

// Fixed-order sum of the per-chunk partials in two levels (kSlices contiguous runs of partials per
// parameter, then the runs), so that ~300 partials of ~1000 parameters are read by many threads at once.
constexpr int kSlices = 16;

__global__ __launch_bounds__(256) void siren_reduce1_kernel(const float* __restrict__ partial, int n_part, int n,
                                                           float* __restrict__ part2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int slice = blockIdx.y;
    if (j >= n) return;
    const int per = (n_part + kSlices - 1) / kSlices;
    const int b1 = min((slice + 1) * per, n_part);
    float s = 0.0f;
    for (int b = slice * per; b < b1; ++b) s += partial[static_cast<size_t>(b) * n + j];
    part2[static_cast<size_t>(slice) * n + j] = s;
}

__global__ __launch_bounds__(256) void siren_reduce2_kernel(const float* __restrict__ part2, int n,
                                                           float* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kSlices; ++k) s += part2[static_cast<size_t>(k) * n + j];
    out[j] = s;
}

int check_siren(const float* params, int hidden, float omega0, const unsigned char* mask, const pact_grid* sosg,
                float mask_radius, const char* what) {
    PACT_CHECK_ARG(params && mask && sosg, "%s: null pointer", what);
    PACT_CHECK_SUPPORTED(hidden > 0 && hidden <= kSirenMaxHidden, "%s: hidden width %d outside 1..%d", what, hidden,
                         kSirenMaxHidden);
    PACT_CHECK_ARG(std::isfinite(omega0) && omega0 > 0.0f, "%s: omega0 must be positive", what);
    PACT_CHECK_ARG(mask_radius > 0.0f && std::isfinite(mask_radius), "%s: mask radius must be positive", what);
    return check_grid(*sosg, what);
}

}  // namespace
}  // namespace pact

extern "C" int pact_siren_sos(const float* params, int hidden, float omega0, const unsigned char* mask,
                              const pact_grid* sosg, float mask_radius, float v0, float* sos, void* stream) {
    using namespace pact;
    clear_error();
    if (int s = check_siren(params, hidden, omega0, mask, sosg, mask_radius, "pact_siren_sos")) return s;
    PACT_CHECK_ARG(sos, "pact_siren_sos: null output");
    const int n = sosg->ny * sosg->nx;
    siren_fwd_kernel<<<ceil_div(n, 256 / kLanesPerNode), 256, 0, as_stream(stream)>>>(
        params, hidden, omega0, mask, sosg->ny, sosg->nx, sosg->spacing, 1.0f / mask_radius, v0, sos);
    return launch_status("pact_siren_sos");
}

extern "C" size_t pact_siren_sos_adjoint_workspace_size(const pact_grid* sosg, int hidden) {
    if (!sosg || sosg->ny <= 0 || sosg->nx <= 0 || hidden <= 0) return 0;
    const size_t chunks = (static_cast<size_t>(sosg->ny) * sosg->nx + pact::kNodesPerChunk - 1) / pact::kNodesPerChunk;
    return (chunks + pact::kSlices) * (4 * static_cast<size_t>(hidden) + 3) * sizeof(float);
}

extern "C" int pact_siren_sos_adjoint(const float* params, int hidden, float omega0, const unsigned char* mask,
                                      const pact_grid* sosg, float mask_radius, const float* dL_dsos,
                                      float* dL_dparams, void* ws, size_t ws_bytes, void* stream) {
    using namespace pact;
    clear_error();
    if (int s = check_siren(params, hidden, omega0, mask, sosg, mask_radius, "pact_siren_sos_adjoint")) return s;
    PACT_CHECK_ARG(dL_dsos && dL_dparams, "pact_siren_sos_adjoint: null pointer");
    const size_t need = pact_siren_sos_adjoint_workspace_size(sosg, hidden);
    if (!ws || ws_bytes < need) {
        set_error("pact_siren_sos_adjoint: workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : 0);
        return PACT_EWORKSPACE;
    }
    const int n = sosg->ny * sosg->nx;
    const int chunks = ceil_div(n, kNodesPerChunk);
    const int np = 4 * hidden + 3;
    float* partial = static_cast<float*>(ws);
    siren_adj_kernel<<<chunks, 256, 0, as_stream(stream)>>>(params, hidden, omega0, mask, sosg->ny, sosg->nx,
                                                           sosg->spacing, 1.0f / mask_radius, dL_dsos, partial);
    if (int s = launch_status("pact_siren_sos_adjoint")) return s;
    float* part2 = partial + static_cast<size_t>(chunks) * np;
    siren_reduce1_kernel<<<dim3(ceil_div(np, 256), kSlices), 256, 0, as_stream(stream)>>>(partial, chunks, np, part2);
    if (int s = launch_status("pact_siren_sos_adjoint")) return s;
    siren_reduce2_kernel<<<ceil_div(np, 256), 256, 0, as_stream(stream)>>>(part2, np, dL_dparams);
    return launch_status("pact_siren_sos_adjoint");
}
