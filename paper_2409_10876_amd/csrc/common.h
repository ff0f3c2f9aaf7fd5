// Internal helpers shared by the libpact translation units: error reporting,
// argument checks and small device functions (ring geometry, reductions).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "../../include/pact.h"

namespace pact {

// ---------------------------------------------------------------- errors ---

void set_error(const char* fmt, ...);
void clear_error();

#define PACT_CHECK_ARG(cond, ...)               \
    do {                                        \
        if (!(cond)) {                          \
            ::pact::set_error(__VA_ARGS__);     \
            return PACT_EINVAL;                 \
        }                                       \
    } while (0)

#define PACT_CHECK_SUPPORTED(cond, ...)         \
    do {                                        \
        if (!(cond)) {                          \
            ::pact::set_error(__VA_ARGS__);     \
            return PACT_EUNSUPPORTED;           \
        }                                       \
    } while (0)

// Checks the launch just enqueued.
int launch_status(const char* what);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr int kMaxPatch = 96;         // largest patch side for the LDS-resident transforms
constexpr int kMaxDelays = 16;        // largest delay count of the fused loss kernel
constexpr size_t kLdsBytes = 160 * 1024;

inline int ceil_div(long long a, long long b) { return static_cast<int>((a + b - 1) / b); }

int check_ring(const pact_ring& r);
int check_grid(const pact_grid& g, const char* what);

// ------------------------------------------------------------- device ---

// Angular wavenumber (rad/mm) of FFT index u on a P-point grid of spacing px.
__device__ __forceinline__ float fft_wavenumber(int u, int P, float two_pi_over_Ppx) {
    return static_cast<float>(u <= (P - 1) / 2 ? u : u - P) * two_pi_over_Ppx;
}

// Fractional element index where the ray from (cx, cy) along unit (ux, uy) meets the ring:
// tau = -(c.u) + sqrt((c.u)^2 - |c|^2 + R^2), q = c + tau u,
// f = ((atan2(q_y, q_x) - phi0) mod 2 pi) * n / (2 pi), in [0, n).
__device__ __forceinline__ float ring_hit_index(float cx, float cy, float ux, float uy, float R2mc2,
                                                float phi0, float n_over_two_pi, float n) {
    const float b = cx * ux + cy * uy;
    const float tau = -b + sqrtf(fmaf(b, b, R2mc2));
    const float qx = fmaf(tau, ux, cx);
    const float qy = fmaf(tau, uy, cy);
    float a = atan2f(qy, qx) - phi0;
    a -= kTwoPi * floorf(a * (1.0f / kTwoPi));
    float f = a * n_over_two_pi;
    return f >= n ? f - n : f;
}

// Split a fractional element index into (n0, n1, alpha) with cyclic wrap.
// The index is clamped to [0, n) first (a NaN maps to 0), so the result always addresses the table.
__device__ __forceinline__ void ring_cell(float f, int n, int& n0, int& n1, float& alpha) {
    const float fc = fminf(fmaxf(f, 0.0f), static_cast<float>(n));
    const float fl = floorf(fc);
    alpha = fc - fl;
    n0 = static_cast<int>(fl);
    n0 = n0 >= n ? 0 : (n0 < 0 ? 0 : n0);
    n1 = n0 + 1 == n ? 0 : n0 + 1;
}

// Sum over a 64-lane wavefront (every lane gets the total).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum; `red` must hold blockDim.x / 64 floats.  Result valid in every thread.
__device__ __forceinline__ float block_sum(float v, float* red) {
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    float t = 0.0f;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}

// ---- Sums of partial results in a fixed order ----

// sum_k p[k * stride] for k = 0 .. n - 1 (n >= 1), added in order; loads are issued B at a time, the last
// partial batch too (its missing entries load element n - 1 and are not added).
template <int B = 8>
__device__ __forceinline__ float ordered_strided_sum(const float* __restrict__ p, int n, size_t stride) {
    float s = 0.0f;
    int k = 0;
    for (; k + B <= n; k += B) {
        float v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = p[static_cast<size_t>(k + u) * stride];
#pragma unroll
        for (int u = 0; u < B; ++u) s += v[u];
    }
    if (k < n) {
        float v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = p[static_cast<size_t>(min(k + u, n - 1)) * stride];
#pragma unroll
        for (int u = 0; u < B; ++u) s = k + u < n ? s + v[u] : s;
    }
    return s;
}

}  // namespace pact
