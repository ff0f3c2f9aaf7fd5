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

// Batched solves (pact_batch_plan / pact_batch_step): each source file plans and launches its own stages of
// the grouped step.  Descriptors are written to host memory by the plan functions and read on the device from
// the table.  A launch covers n scans: starts[q] is the first block of its q-th scan (starts[n] = the launch's
// blocks) and ids[q] that scan's descriptor.
size_t batch_ray_desc_bytes();
int batch_ray_plan(const pact_batch_scan& s, int parity, void* desc, int blocks[3], size_t lds[3], const char* what);
int batch_ray_launch(int stage, const void* descs, const int* starts, const int* ids, int n, int total, size_t lds,
                     int with_loss, hipStream_t st);
size_t batch_loss_desc_bytes();
int batch_loss_plan(const pact_batch_scan& s, void* desc, int* blocks, size_t* lds, const char* what);
int batch_loss_launch(int stage, const void* descs, const int* starts, const int* ids, int n, int total, size_t lds,
                      hipStream_t st);

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

// ---- Short polynomials (coefficients fitted by gen_poly.py beside the sources) ----

// sin2pi: max abs error 1.21e-09 (float64)
constexpr float k_sin2pi[4] = {6.283185005187988f, -41.34162902832031f, 81.58812713623047f, -75.24005889892578f};
// cos2pi: max abs error 4.74e-11 (float64)
constexpr float k_cos2pi[5] = {1.0f, -19.739208221435547f, 64.93931579589844f, -85.4428482055664f, 59.220401763916016f};

// Block maximum (deterministic; every thread gets it); `red` must hold blockDim.x / 64 floats.
__device__ __forceinline__ float block_max(float v, float* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float t = red[0];
    for (int k = 1; k < static_cast<int>(blockDim.x >> 6); ++k) t = fmaxf(t, red[k]);
    __syncthreads();
    return t;
}

template <int K>
__device__ __forceinline__ float horner(const float (&c)[K], float z) {
    float p = c[K - 1];
#pragma unroll
    for (int k = K - 2; k >= 0; --k) p = fmaf(p, z, c[k]);
    return p;
}

// sin and cos of 2 pi r (r in revolutions): remove whole quarter turns, then the polynomials on |f| <= 1/8.
__device__ __forceinline__ void sincos_rev(float r, float& s, float& c) {
    const float q = rintf(4.0f * r);
    const float f = fmaf(q, -0.25f, r);
    const float z = f * f;
    const float sf = f * horner(k_sin2pi, z);
    const float cf = horner(k_cos2pi, z);
    const int iq = static_cast<int>(q);
    const bool swap = (iq & 1) != 0;
    const float ss = swap ? cf : sf, cc = swap ? sf : cf;
    s = __int_as_float(__float_as_int(ss) ^ ((iq & 2) << 30));
    c = __int_as_float(__float_as_int(cc) ^ (((iq + 1) & 2) << 30));
}

// q = n / d for 0 <= n < 2^24 and d >= 1, given inv_d = 1 / d (rounded): the float quotient is off by at most two,
// which the two corrections remove.
__device__ __forceinline__ int div_small(int n, int d, float inv_d) {
    int q = static_cast<int>(static_cast<float>(n) * inv_d);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int r = n - q * d;
        q = r < 0 ? q - 1 : (r >= d ? q + 1 : q);
    }
    return q;
}

// ---- TV subgradient and Adam (Eq. jr, Sec. 3.3), shared by the optimiser kernels ----

__device__ __forceinline__ float sgn(float x) { return x > 0.0f ? 1.0f : (x < 0.0f ? -1.0f : 0.0f); }

// TV pairs of node (a, b): its value share (the pairs it starts) and its subgradient (all four pairs).  The
// neighbours' values and masks are loaded unconditionally (the node itself stands in at the grid edge), so
// that all the loads are in flight together; the pairs that exist are then taken as written.
__device__ __forceinline__ void tv_node(const float* __restrict__ v, const unsigned char* __restrict__ mask, int idx,
                                        int a, int b, int Gy, int Gx, float& tv, float& g) {
    const bool has_d = a + 1 < Gy, has_r = b + 1 < Gx, has_u = a > 0, has_l = b > 0;
    const int id = has_d ? idx + Gx : idx, ir = has_r ? idx + 1 : idx;
    const int iu = has_u ? idx - Gx : idx, il = has_l ? idx - 1 : idx;
    const float x = v[idx], vd = v[id], vr = v[ir], vu = v[iu], vl = v[il];
    const bool m = mask[idx] != 0, md = mask[id] != 0, mr = mask[ir] != 0, mu = mask[iu] != 0, ml = mask[il] != 0;
    tv = 0.0f;
    g = 0.0f;
    // pair (a, b)-(a+1, b) and (a, b)-(a, b+1): counted once, by their first node
    if (has_d && (m || md)) {
        const float dv = vd - x;
        tv += fabsf(dv);
        g -= sgn(dv);
    }
    if (has_r && (m || mr)) {
        const float dv = vr - x;
        tv += fabsf(dv);
        g -= sgn(dv);
    }
    // the same pairs seen from their second node
    if (has_u && (m || mu)) g += sgn(x - vu);
    if (has_l && (m || ml)) g += sgn(x - vl);
}

// One Adam update of p with gradient g at step `step` (PyTorch's rule); returns the new parameter.
__device__ __forceinline__ float adam_node(float p, float g, float& m, float& v, int step, float lr, float b1,
                                           float b2, float eps) {
    const float bc1 = 1.0f - powf(b1, static_cast<float>(step));
    const float bc2 = 1.0f - powf(b2, static_cast<float>(step));
    m = fmaf(b1, m, (1.0f - b1) * g);
    v = fmaf(b2, v, (1.0f - b2) * g * g);
    return p - (lr / bc1) * m / fmaf(sqrtf(v), 1.0f / sqrtf(bc2), eps);
}

// Every workgroup has read t[0] (above its barrier); the last workgroup to arrive advances it.
__device__ __forceinline__ void advance_step(int* t, int step) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = atomicAdd(reinterpret_cast<unsigned*>(t + 1), 1u);
        if (prev == gridDim.x - 1) {
            t[0] = step;
            t[1] = 0;
        }
    }
}

}  // namespace pact
