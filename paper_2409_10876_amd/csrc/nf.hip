// Neural-field SOS queried at every ray sample (coordinate network of Sec. 3.3; Eq. wf), forward and
// adjoint, with the network's dense layers on MFMA (BF16 operands, FP32 accumulation).
//
// Network: gamma(p) = [cos(2 pi B p), sin(2 pi B p)] (128 frequencies), h_l = relu(W_l h_{l-1} + b_l)
// for four layers of width 128, f = w5 . h_4 + b5, and v = v0 + amp tanh(f) inside the mask disc.  A ray
// (patch i, element n) is clipped to the disc and sampled at N_s midpoints; w[i,n] = dl sum (1 - v0/v).
//
// Layout on the chip.  A workgroup is 8 waves; wave k owns output rows 16k .. 16k + 15 of every layer.
// The BF16 weights a wave needs as MFMA A operands (its rows of W1..W4, and in the backward pass its
// rows of the transposed W2..W4) stay in registers for the whole launch, so HBM and L2 see the weights
// once per workgroup.  Points go through in chunks of 32 consecutive samples of one ray; a chunk's
// activations live in LDS, point-major (row = point, 8 features contiguous per MFMA B fragment) and,
// where a weight gradient needs them as the reduction operand, feature-major as well.  Rows are padded
// by 16 bytes so that the 16 lanes reading one fragment column hit distinct banks.
//
// MFMA v_mfma_f32_16x16x32_bf16, lane l, r = l % 16, q = l / 16:
//   A (16 x 32):  a[j] = A[r][8q + j]      B (32 x 16):  b[j] = B[8q + j][r]
//   D (16 x 16):  d[i] = D[4q + i][r]
//
// Adjoint.  The pre-activation gradients delta_l are formed chunk by chunk (delta_4 from the head,
// delta_{l-1} = (W_l^T delta_l) * [h_{l-1} > 0]) and the weight gradients sum delta_l h_{l-1}^T over
// the chunk's 32 points, one MFMA K step.  Each wave accumulates its rows of dL/dW_l in registers over
// all the chunks it processes.  From activations stored by the forward pass the adjoint runs two kernels
// (see below); without them it runs four passes that recompute the forward activations (layers 3-4,
// layer 2, and each half of layer 1's columns), the registers holding the layers of one pass only.
// Each workgroup writes its partial gradient once; two small kernels sum the partials in a fixed order.
#include "common.h"

namespace pact {

int device_cu_count();

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kF = 128;               // Fourier frequencies
constexpr int kK1 = 2 * kF;           // layer-1 inputs
constexpr int kH = 128;               // hidden width
constexpr int kWaves = 8;             // 16 output rows each
constexpr int kNT = 64 * kWaves;      // threads per workgroup
constexpr int kPc = 32;               // points per chunk
constexpr int kLd1 = kK1 + 8;         // point-major row of the features (bf16 elements)
constexpr int kLdH = kH + 8;          // point-major row of a hidden activation
constexpr int kLdT = kPc + 8;         // feature-major row (one feature, the chunk's points)

// packed BF16 weights (elements): W1 [H][2F], W2, W3, W4 [H][H], W2^T, W3^T, W4^T [H][H], w5 [H]
constexpr int kOffW1 = 0;
constexpr int kOffW2 = kOffW1 + kH * kK1;
constexpr int kOffW3 = kOffW2 + kH * kH;
constexpr int kOffW4 = kOffW3 + kH * kH;
constexpr int kOffT2 = kOffW4 + kH * kH;
constexpr int kOffT3 = kOffT2 + kH * kH;
constexpr int kOffT4 = kOffT3 + kH * kH;
constexpr int kOffW5 = kOffT4 + kH * kH;
constexpr int kPacked = kOffW5 + kH;
// FP32 parameter vector: W1, b1, W2, b2, W3, b3, W4, b4, w5, b5
constexpr int kPW1 = 0;
constexpr int kPb1 = kPW1 + kH * kK1;
constexpr int kPW2 = kPb1 + kH;
constexpr int kPb2 = kPW2 + kH * kH;
constexpr int kPW3 = kPb2 + kH;
constexpr int kPb3 = kPW3 + kH * kH;
constexpr int kPW4 = kPb3 + kH;
constexpr int kPb4 = kPW4 + kH * kH;
constexpr int kPw5 = kPb4 + kH;
constexpr int kPb5 = kPw5 + kH;
constexpr int kNParams = kPb5 + 1;

__host__ __device__ constexpr int param_w(int l) { return l == 1 ? kPW1 : l == 2 ? kPW2 : l == 3 ? kPW3 : kPW4; }
__host__ __device__ constexpr int param_b(int l) { return l == 1 ? kPb1 : l == 2 ? kPb2 : l == 3 ? kPb3 : kPb4; }

struct NfArgs {
    const float* B;            // [F][2] cycles per mm
    const float* params;       // FP32 parameter vector (biases and b5 are read from it)
    const unsigned short* packed;  // BF16 weights
    float amp, rho2, v0;
    const float* centres;
    int N, n_elem;
    float R, phi0;
    int Ns;
};

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

// Ray (i, n) clipped to the mask disc: start point, direction, first sample distance and step.
struct NfRay {
    float cx, cy, ux, uy, ta, dl;
};

__device__ __forceinline__ NfRay nf_ray(const NfArgs& a, int ray) {
    const int i = ray / a.n_elem, n = ray - i * a.n_elem;
    NfRay r;
    r.cx = a.centres[2 * i];
    r.cy = a.centres[2 * i + 1];
    float sn, cs;
    sincosf(a.phi0 + kTwoPi * (static_cast<float>(n) / a.n_elem), &sn, &cs);
    const float dx = a.R * cs - r.cx, dy = a.R * sn - r.cy;
    const float L = sqrtf(fmaf(dx, dx, dy * dy));
    r.ux = dx / L;
    r.uy = dy / L;
    const float cu = fmaf(r.cx, r.ux, r.cy * r.uy);
    const float disc = cu * cu - fmaf(r.cx, r.cx, r.cy * r.cy) + a.rho2;
    r.ta = 0.0f;
    r.dl = 0.0f;
    if (disc > 0.0f) {
        const float root = sqrtf(disc);
        const float ta = fmaxf(-cu - root, 0.0f);
        const float tb = fminf(-cu + root, L);
        if (tb > ta) {
            r.ta = ta;
            r.dl = (tb - ta) / static_cast<float>(a.Ns);
        }
    }
    return r;
}

// Fourier features of the chunk's points into LDS, point-major.
// Thread t: point t % 32, frequencies 8 (t / 32) .. + 7.
__device__ __forceinline__ void nf_features(const NfArgs& a, const NfRay& r, int s0, const float* Bs, __bf16* feat) {
    const int p = threadIdx.x & (kPc - 1);
    const int k0 = (threadIdx.x >> 5) * 8;
    const float t = fmaf(static_cast<float>(s0 + p) + 0.5f, r.dl, r.ta);
    const float px = fmaf(t, r.ux, r.cx), py = fmaf(t, r.uy, r.cy);
    bf16x8 c8, s8;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float ph = fmaf(Bs[2 * (k0 + j)], px, Bs[2 * (k0 + j) + 1] * py);
        ph -= rintf(ph);                               // revolutions in [-1/2, 1/2]
        c8[j] = static_cast<__bf16>(__builtin_amdgcn_cosf(ph));
        s8[j] = static_cast<__bf16>(__builtin_amdgcn_sinf(ph));
    }
    *reinterpret_cast<bf16x8*>(feat + p * kLd1 + k0) = c8;
    *reinterpret_cast<bf16x8*>(feat + p * kLd1 + kF + k0) = s8;
}

// Fourier features of a chunk, feature-major only (the layer-1 weight-gradient operand).  Task k of 512:
// frequency k % 128, points 8 (k / 128) .. + 7.  Along a ray the samples are dl apart, so the phase of
// a frequency advances by dl (B . u) revolutions per sample: a task takes cos and sin at its first point and
// the step's cos and sin from the hardware functions, then rotates through the other seven points (four
// FP32 products per point instead of two hardware calls), and writes each row's eight values at once.
__device__ __forceinline__ void nf_features_rot(const NfRay& r, int s0, const float* Bs, __bf16* featT) {
    for (int k = threadIdx.x; k < 4 * kF; k += blockDim.x) {
        const int f = k & (kF - 1), p0 = 8 * (k >> 7);
        const float bx = Bs[2 * f], by = Bs[2 * f + 1];
        float step = r.dl * fmaf(bx, r.ux, by * r.uy);
        step -= rintf(step);
        const float cd = __builtin_amdgcn_cosf(step), sd = __builtin_amdgcn_sinf(step);
        const float t = fmaf(static_cast<float>(s0 + p0) + 0.5f, r.dl, r.ta);
        float ph = fmaf(bx, fmaf(t, r.ux, r.cx), by * fmaf(t, r.uy, r.cy));
        ph -= rintf(ph);
        float c = __builtin_amdgcn_cosf(ph), sn = __builtin_amdgcn_sinf(ph);
        bf16x8 c8, s8;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            c8[j] = static_cast<__bf16>(c);
            s8[j] = static_cast<__bf16>(sn);
            const float cn = fmaf(c, cd, -sn * sd);
            sn = fmaf(sn, cd, c * sd);
            c = cn;
        }
        *reinterpret_cast<bf16x8*>(featT + f * kLdT + p0) = c8;
        *reinterpret_cast<bf16x8*>(featT + (kF + f) * kLdT + p0) = s8;
    }
}

// One dense layer for the wave's 16 rows and the chunk's 32 points: acc[nt] (points 16 nt ..) =
// W rows x input (point-major, row length ld).
template <int KS>
__device__ __forceinline__ void nf_layer(const bf16x8 (&w)[KS], const __bf16* in, int ld, f32x4 (&acc)[2]) {
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    acc[0] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    acc[1] = acc[0];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const bf16x8 b0 = ld8(in + r * ld + 32 * ks + 8 * q);
        const bf16x8 b1 = ld8(in + (16 + r) * ld + 32 * ks + 8 * q);
        acc[0] = mfma(w[ks], b0, acc[0]);
        acc[1] = mfma(w[ks], b1, acc[1]);
    }
}

// bias + relu + BF16, written point-major (and feature-major if outT); h keeps the BF16 values as floats.
__device__ __forceinline__ void nf_activate(const f32x4 (&acc)[2], const float* bias, __bf16* out, __bf16* outT,
                                            float (&h)[2][4]) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const int row0 = 16 * w + 4 * q;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        bf16x4 v;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[i] = static_cast<__bf16>(fmaxf(acc[nt][i] + bias[row0 + i], 0.0f));
            h[nt][i] = static_cast<float>(v[i]);
        }
        const int p = 16 * nt + r;
        *reinterpret_cast<bf16x4*>(out + p * kLdH + row0) = v;
        if (outT) {
#pragma unroll
            for (int i = 0; i < 4; ++i) outT[(row0 + i) * kLdT + p] = v[i];
        }
    }
}

// Head for the chunk: f[p] = b5 + sum over rows of w5 h4 (wave partials, then a fixed-order sum).
__device__ __forceinline__ void nf_head_partial(const float (&h4)[2][4], const float* w5, float* headp) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const int row0 = 16 * w + 4 * q;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) s = fmaf(w5[row0 + i], h4[nt][i], s);
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        if (q == 0) headp[w * kPc + 16 * nt + r] = s;
    }
}

__device__ __forceinline__ float nf_head_sum(const float* headp, int p, float b5) {
    float f = 0.0f;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) f += headp[w * kPc + p];
    return f + b5;
}

template <int KS>
__device__ __forceinline__ void load_rows(const unsigned short* packed, int off, int ld, bf16x8 (&w)[KS]) {
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const __bf16* base = reinterpret_cast<const __bf16*>(packed) + off + (16 * wv + r) * ld + 8 * q;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) w[ks] = ld8(base + 32 * ks);
}

// The same for waves of 32 rows (two row tiles): rows 32 wv + 16 rt + r.
template <int KS>
__device__ __forceinline__ void load_rows32(const unsigned short* packed, int off, int ld, bf16x8 (&w)[2][KS]) {
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const __bf16* base = reinterpret_cast<const __bf16*>(packed) + off + (32 * wv + r) * ld + 8 * q;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) w[rt][ks] = ld8(base + 16 * rt * ld + 32 * ks);
}

// Small per-workgroup tables in LDS: B, biases b1..b4, w5 (the BF16 value), b5.
struct NfTables {
    float B[2 * kF];
    float bias[4][kH];
    float w5[kH];
    float b5;
};

__device__ __forceinline__ void load_tables(const NfArgs& a, NfTables& t) {
    for (int k = threadIdx.x; k < 2 * kF; k += blockDim.x) t.B[k] = a.B[k];
    for (int k = threadIdx.x; k < 4 * kH; k += blockDim.x) t.bias[k / kH][k % kH] = a.params[param_b(k / kH + 1) + k % kH];
    const __bf16* w5 = reinterpret_cast<const __bf16*>(a.packed) + kOffW5;
    for (int k = threadIdx.x; k < kH; k += blockDim.x) t.w5[k] = static_cast<float>(w5[k]);
    if (threadIdx.x == 0) t.b5 = a.params[kPb5];
}

struct NfFwdLds {
    NfTables tab;
    float headp[kWaves * kPc];
    alignas(16) __bf16 feat[kPc * kLd1];
    alignas(16) __bf16 hA[kPc * kLdH];
    alignas(16) __bf16 hB[kPc * kLdH];
    alignas(16) __bf16 hT[2][kH * kLdT];      // feature-major staging of the activations being stored
};

// Stored activations of one chunk: h1..h4 feature-major, [4][128][32] BF16 (32 KB), chunk = ray * n_chunks + ch.
constexpr int kActChunk = 4 * kH * kPc;


// ---- forward pass: 4 waves of 32 rows (two MFMA row tiles per B fragment read from LDS) ----
constexpr int kWF = 4;
constexpr int kNTF = 64 * kWF;

// Fourier features of the chunk's points into LDS, point-major, with 256 threads: thread t takes point
// t % 32 and frequencies 16 (t / 32) .. + 15 (the arithmetic of nf_features).
__device__ __forceinline__ void nf_features_p256(const NfRay& r, int s0, const float* Bs, __bf16* feat) {
    const int p = threadIdx.x & (kPc - 1);
    const int k0 = (threadIdx.x >> 5) * 16;
    const float t = fmaf(static_cast<float>(s0 + p) + 0.5f, r.dl, r.ta);
    const float px = fmaf(t, r.ux, r.cx), py = fmaf(t, r.uy, r.cy);
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        bf16x8 c8, s8;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = k0 + 8 * hh + j;
            float ph = fmaf(Bs[2 * k], px, Bs[2 * k + 1] * py);
            ph -= rintf(ph);
            c8[j] = static_cast<__bf16>(__builtin_amdgcn_cosf(ph));
            s8[j] = static_cast<__bf16>(__builtin_amdgcn_sinf(ph));
        }
        *reinterpret_cast<bf16x8*>(feat + p * kLd1 + k0 + 8 * hh) = c8;
        *reinterpret_cast<bf16x8*>(feat + p * kLd1 + kF + k0 + 8 * hh) = s8;
    }
}

// One dense layer for the wave's 32 rows and the chunk's 32 points: acc[rt][nt] = rows 32 wv + 16 rt ..,
// points 16 nt ..; each B fragment feeds both row tiles.
template <int KS>
__device__ __forceinline__ void nf_layer2(const bf16x8 (&w)[2][KS], const __bf16* in, int ld, f32x4 (&acc)[2][2]) {
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) acc[rt][0] = acc[rt][1] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const bf16x8 b0 = ld8(in + r * ld + 32 * ks + 8 * q);
        const bf16x8 b1 = ld8(in + (16 + r) * ld + 32 * ks + 8 * q);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            acc[rt][0] = mfma(w[rt][ks], b0, acc[rt][0]);
            acc[rt][1] = mfma(w[rt][ks], b1, acc[rt][1]);
        }
    }
}

// bias + relu + BF16, point-major (and feature-major if outT); h keeps the BF16 values as floats.
__device__ __forceinline__ void nf_activate2(const f32x4 (&acc)[2][2], const float* bias, __bf16* out, __bf16* outT,
                                             float (&h)[2][2][4]) {
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        const int row0 = 32 * wv + 16 * rt + 4 * q;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            bf16x4 v;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[i] = static_cast<__bf16>(fmaxf(acc[rt][nt][i] + bias[row0 + i], 0.0f));
                h[rt][nt][i] = static_cast<float>(v[i]);
            }
            const int p = 16 * nt + r;
            *reinterpret_cast<bf16x4*>(out + p * kLdH + row0) = v;
            if (outT) {
#pragma unroll
                for (int i = 0; i < 4; ++i) outT[(row0 + i) * kLdT + p] = v[i];
            }
        }
    }
}

// Head partials per 16-row tile (slot 2 wv + rt, the same slots and sums as 16-row waves).
__device__ __forceinline__ void nf_head_partial2(const float (&h4)[2][2][4], const float* w5, float* headp) {
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        const int row0 = 32 * wv + 16 * rt + 4 * q;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            float s = 0.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i) s = fmaf(w5[row0 + i], h4[rt][nt][i], s);
            s += __shfl_xor(s, 16, 64);
            s += __shfl_xor(s, 32, 64);
            if (q == 0) headp[(2 * wv + rt) * kPc + 16 * nt + r] = s;
        }
    }
}

// Copy a feature-major LDS block [128][kLdT] to its stored block, 256 threads x 2 x 16 bytes.
__device__ __forceinline__ void nf_store_layer256(const __bf16* hT, __bf16* dst) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int idx = threadIdx.x + kNTF * k, feature = idx >> 2, part = idx & 3;
        *reinterpret_cast<bf16x8*>(dst + feature * kPc + 8 * part) = ld8(hT + feature * kLdT + 8 * part);
    }
}

__global__ __launch_bounds__(kNTF, 2) void nf_fwd_kernel(NfArgs a, float* __restrict__ w_out, __bf16* __restrict__ act,
                                                      float* __restrict__ f_out) {
    __shared__ NfFwdLds sm;
    load_tables(a, sm.tab);
    bf16x8 w1[2][8], w2[2][4], w3[2][4], w4[2][4];
    load_rows32<8>(a.packed, kOffW1, kK1, w1);
    load_rows32<4>(a.packed, kOffW2, kH, w2);
    load_rows32<4>(a.packed, kOffW3, kH, w3);
    load_rows32<4>(a.packed, kOffW4, kH, w4);
    __syncthreads();
    const int n_rays = a.N * a.n_elem;
    const int n_chunks = (a.Ns + kPc - 1) / kPc;
    for (int ray = blockIdx.x; ray < n_rays; ray += gridDim.x) {
        const NfRay r = nf_ray(a, ray);
        if (r.dl == 0.0f) {
            if (threadIdx.x == 0) w_out[ray] = 0.0f;
            continue;
        }
        float sum = 0.0f;
        for (int ch = 0; ch < n_chunks; ++ch) {
            const int s0 = ch * kPc;
            const size_t chunk = static_cast<size_t>(ray) * n_chunks + ch;
            __bf16* dst = act ? act + chunk * kActChunk : nullptr;
            nf_features_p256(r, s0, sm.tab.B, sm.feat);
            __syncthreads();
            f32x4 acc[2][2];
            float h[2][2][4];
            nf_layer2<8>(w1, sm.feat, kLd1, acc);
            nf_activate2(acc, sm.tab.bias[0], sm.hA, dst ? sm.hT[0] : nullptr, h);
            __syncthreads();
            if (dst) nf_store_layer256(sm.hT[0], dst);
            nf_layer2<4>(w2, sm.hA, kLdH, acc);
            nf_activate2(acc, sm.tab.bias[1], sm.hB, dst ? sm.hT[1] : nullptr, h);
            __syncthreads();
            if (dst) nf_store_layer256(sm.hT[1], dst + kH * kPc);
            nf_layer2<4>(w3, sm.hB, kLdH, acc);
            nf_activate2(acc, sm.tab.bias[2], sm.hA, dst ? sm.hT[0] : nullptr, h);
            __syncthreads();
            if (dst) nf_store_layer256(sm.hT[0], dst + 2 * kH * kPc);
            nf_layer2<4>(w4, sm.hA, kLdH, acc);
            nf_activate2(acc, sm.tab.bias[3], sm.hB, dst ? sm.hT[1] : nullptr, h);
            nf_head_partial2(h, sm.tab.w5, sm.headp);
            __syncthreads();
            if (dst) nf_store_layer256(sm.hT[1], dst + 3 * kH * kPc);
            if (threadIdx.x < kPc) {
                const float f = nf_head_sum(sm.headp, threadIdx.x, sm.tab.b5);
                if (f_out) f_out[chunk * kPc + threadIdx.x] = f;
                if (s0 + static_cast<int>(threadIdx.x) < a.Ns) {
                    const float th = tanhf(f);
                    sum += a.amp * th / (a.v0 + a.amp * th);      // 1 - v0 / v
                }
            }
        }
        if (threadIdx.x < 64) {
#pragma unroll
            for (int off = 16; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 32);
            if (threadIdx.x == 0) w_out[ray] = sum * r.dl;
        }
    }
}

// Backward pass over the rays with nonzero dL/dw; accumulates the gradients of layers LO..HI (and of the
// head when HI == 4) and writes them into this workgroup's row of `partial` [gridDim.x][n_params].
template <int LO, int HI>
struct NfBwdLds {
    NfTables tab;
    float headp[kWaves * kPc];
    float df[kPc];
    alignas(16) __bf16 feat[kPc * kLd1];
    alignas(16) __bf16 featT[LO == 1 ? kK1 * kLdT : 8];
    alignas(16) __bf16 h[4][kPc * kLdH];      // h1..h4, point-major
    alignas(16) __bf16 hT[HI >= 2 ? 3 : 1][kH * kLdT];  // h1..h3 feature-major (weight gradients of 2..4)
    alignas(16) __bf16 dP[2][kPc * kLdH];     // delta, point-major (dgrad operand), two buffers
    alignas(16) __bf16 dT[2][kH * kLdT];      // delta, feature-major (weight-gradient operand)
};

// Level L of the backward chain for one chunk, delta_L in buffer `cur`: the weight gradient of layer L
// (if L is in this pass) and delta_{L-1} into the other buffer (if L > LO).  Ends with a barrier.
template <int L, int LO, int HI, int NG, int K1C>
__device__ __forceinline__ void nf_level(NfBwdLds<LO, HI>& sm, const bf16x8 (&tw)[4], f32x4 (&gl)[NG],
                                         float (&gb)[4][4], int cur) {
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r16 = l & 15, q = l >> 4;
    const int row0 = 16 * wv + 4 * q;
    if (L >= LO && L <= HI) {
        // rows of delta_L (feature-major) against h_{L-1} (feature-major): one K step of 32 points
        const bf16x8 da = ld8(sm.dT[cur] + (16 * wv + r16) * kLdT + 8 * q);
        const __bf16* hT = L == 1 ? sm.featT : sm.hT[L >= 2 ? L - 2 : 0];
#pragma unroll
        for (int kt = 0; kt < NG; ++kt)
            gl[kt] = mfma(da, ld8(hT + (16 * (kt + (L == 1 ? K1C : 0)) + r16) * kLdT + 8 * q), gl[kt]);
    }
    if (L > LO) {
        // delta_{L-1} = (W_L^T delta_L) [h_{L-1} > 0]
        f32x4 d2[2] = {f32x4{0.0f, 0.0f, 0.0f, 0.0f}, f32x4{0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            d2[0] = mfma(tw[ks], ld8(sm.dP[cur] + r16 * kLdH + 32 * ks + 8 * q), d2[0]);
            d2[1] = mfma(tw[ks], ld8(sm.dP[cur] + (16 + r16) * kLdH + 32 * ks + 8 * q), d2[1]);
        }
        const int nxt = cur ^ 1;
        const __bf16* hprev = sm.h[L >= 2 ? L - 2 : 0];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int p = 16 * nt + r16;
            const bf16x4 hv = *reinterpret_cast<const bf16x4*>(hprev + p * kLdH + row0);
            bf16x4 dv;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                dv[i] = static_cast<__bf16>(static_cast<float>(hv[i]) > 0.0f ? d2[nt][i] : 0.0f);
                gb[L >= 2 ? L - 2 : 0][i] += static_cast<float>(dv[i]);
                sm.dT[nxt][(row0 + i) * kLdT + p] = dv[i];
            }
            *reinterpret_cast<bf16x4*>(sm.dP[nxt] + p * kLdH + row0) = dv;
        }
    }
    __syncthreads();
}

template <int LO, int HI, int K1C, int K1N>
__global__ __launch_bounds__(kNT) void nf_bwd_kernel(NfArgs a, const float* __restrict__ dL_dw,
                                                     const float* __restrict__ scale, float* __restrict__ partial) {
    extern __shared__ __attribute__((aligned(16))) unsigned char nf_dyn[];
    NfBwdLds<LO, HI>& sm = *reinterpret_cast<NfBwdLds<LO, HI>*>(nf_dyn);
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r16 = l & 15, q = l >> 4;
    load_tables(a, sm.tab);
    bf16x8 w1[8], w2[4], w3[4], w4[4], t2[4], t3[4], t4[4];
    load_rows<8>(a.packed, kOffW1, kK1, w1);
    load_rows<4>(a.packed, kOffW2, kH, w2);
    load_rows<4>(a.packed, kOffW3, kH, w3);
    load_rows<4>(a.packed, kOffW4, kH, w4);
    if (LO < 4) load_rows<4>(a.packed, kOffT4, kH, t4);
    if (LO < 3) load_rows<4>(a.packed, kOffT3, kH, t3);
    if (LO < 2) load_rows<4>(a.packed, kOffT2, kH, t2);
    // weight-gradient accumulators of this wave's rows: dW1 [16][256] as 16 tiles, dW2..4 as 8 tiles
    f32x4 g1[LO == 1 ? K1N : 1], g2[LO <= 2 && HI >= 2 ? 8 : 1], g3[LO <= 3 && HI >= 3 ? 8 : 1],
        g4[HI == 4 ? 8 : 1];
    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    for (auto& x : g1) x = zero;
    for (auto& x : g2) x = zero;
    for (auto& x : g3) x = zero;
    for (auto& x : g4) x = zero;
    float gb[4][4] = {};                      // bias gradients of layers 1..4, rows 16 wv + 4 q + i
    float gw5[4] = {}, gb5 = 0.0f;
    const float sc = scale ? *scale : 1.0f;
    __syncthreads();

    const int n_rays = a.N * a.n_elem;
    const int n_chunks = (a.Ns + kPc - 1) / kPc;
    const int row0 = 16 * wv + 4 * q;
    for (int ray = blockIdx.x; ray < n_rays; ray += gridDim.x) {
        const float g = dL_dw[ray] * sc;
        if (g == 0.0f) continue;
        const NfRay r = nf_ray(a, ray);
        if (r.dl == 0.0f) continue;
        for (int ch = 0; ch < n_chunks; ++ch) {
            const int s0 = ch * kPc;
            nf_features(a, r, s0, sm.tab.B, sm.feat);
            if (LO == 1) nf_features_rot(r, s0, sm.tab.B, sm.featT);
            __syncthreads();
            f32x4 acc[2];
            float h[2][4];
            nf_layer<8>(w1, sm.feat, kLd1, acc);
            nf_activate(acc, sm.tab.bias[0], sm.h[0], (LO <= 2 && HI >= 2) ? sm.hT[0] : nullptr, h);
            __syncthreads();
            nf_layer<4>(w2, sm.h[0], kLdH, acc);
            nf_activate(acc, sm.tab.bias[1], sm.h[1], (LO <= 3 && HI >= 3) ? sm.hT[1] : nullptr, h);
            __syncthreads();
            nf_layer<4>(w3, sm.h[1], kLdH, acc);
            nf_activate(acc, sm.tab.bias[2], sm.h[2], HI == 4 ? sm.hT[2] : nullptr, h);
            __syncthreads();
            nf_layer<4>(w4, sm.h[2], kLdH, acc);
            nf_activate(acc, sm.tab.bias[3], sm.h[3], nullptr, h);
            nf_head_partial(h, sm.tab.w5, sm.headp);
            __syncthreads();
            if (threadIdx.x < kPc) {
                float d = 0.0f;
                if (s0 + static_cast<int>(threadIdx.x) < a.Ns) {
                    const float th = tanhf(nf_head_sum(sm.headp, threadIdx.x, sm.tab.b5));
                    const float v = a.v0 + a.amp * th;
                    d = g * r.dl * a.v0 * a.amp * (1.0f - th * th) / (v * v);   // d w / d f, times dL/dw
                }
                sm.df[threadIdx.x] = d;
            }
            __syncthreads();
            // delta_4 = df w5 [h4 > 0], from the registers of layer 4
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const int p = 16 * nt + r16;
                const float dfp = sm.df[p];
                bf16x4 dv;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (HI == 4) gw5[i] = fmaf(dfp, h[nt][i], gw5[i]);
                    dv[i] = static_cast<__bf16>(h[nt][i] > 0.0f ? dfp * sm.tab.w5[row0 + i] : 0.0f);
                    gb[3][i] += static_cast<float>(dv[i]);
                    sm.dT[0][(row0 + i) * kLdT + p] = dv[i];
                }
                *reinterpret_cast<bf16x4*>(sm.dP[0] + p * kLdH + row0) = dv;
            }
            if (HI == 4 && threadIdx.x < kPc) gb5 += sm.df[threadIdx.x];
            __syncthreads();
            nf_level<4, LO, HI, HI == 4 ? 8 : 1, K1C>(sm, t4, g4, gb, 0);
            if (LO <= 3) nf_level<3, LO, HI, (LO <= 3 && HI >= 3) ? 8 : 1, K1C>(sm, t3, g3, gb, 1);
            if (LO <= 2) nf_level<2, LO, HI, (LO <= 2 && HI >= 2) ? 8 : 1, K1C>(sm, t2, g2, gb, 0);
            if (LO <= 1) nf_level<1, LO, HI, LO == 1 ? K1N : 1, K1C>(sm, t2, g1, gb, 1);
        }
    }

    // this workgroup's partial gradients: weight tiles (D layout: rows 4 q + i, column r16 of tile kt)
    float* out = partial + static_cast<size_t>(blockIdx.x) * kNParams;
    auto put_w = [&](int L, const f32x4* gl, int tiles, int ld) {
        for (int kt = 0; kt < tiles; ++kt)
#pragma unroll
            for (int i = 0; i < 4; ++i) out[param_w(L) + (row0 + i) * ld + 16 * kt + r16] = gl[kt][i];
    };
    if (LO == 1) {
        for (int kt = 0; kt < K1N; ++kt)
#pragma unroll
            for (int i = 0; i < 4; ++i) out[kPW1 + (row0 + i) * kK1 + 16 * (K1C + kt) + r16] = g1[kt][i];
    }
    if (LO <= 2 && HI >= 2) put_w(2, g2, 8, kH);
    if (LO <= 3 && HI >= 3) put_w(3, g3, 8, kH);
    if (HI == 4) put_w(4, g4, 8, kH);
    // bias gradients: sum the 16 lanes that share rows (lanes r16 = 0..15 of each q)
#pragma unroll
    for (int L = 1; L <= 4; ++L) {
        if (L < LO || L > HI || (L == 1 && K1C != 0)) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float s = gb[L - 1][i];
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
            if (r16 == 0) out[param_b(L) + row0 + i] = s;
        }
    }
    if (HI == 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float s = gw5[i];
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
            if (r16 == 0) out[kPw5 + row0 + i] = s;
        }
        // b5: the first 32 threads hold per-point sums over the rays
        float s = threadIdx.x < 64 ? gb5 : 0.0f;
        if (threadIdx.x < 64) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
            if (threadIdx.x == 0) out[kPb5] = s;
        }
    }
}

// Backward pass from stored activations (written by the forward pass), in two kernels:
//   A (8 waves, 16 rows each): the head and layers 4, 3, 2 (weight gradients, pre-activation gradients,
//      biases) from the stored h1..h4 and f; it also writes each chunk's layer-1 pre-activation gradient
//      delta_1 (BF16, 8 KB per chunk) into the tail of the activation buffer;
//   B (4 waves, 32 rows each, so that every B fragment read from LDS feeds two MFMAs): the layer-1 weight
//      gradient delta_1 gamma^T from the stored delta_1 and recomputed features.
// So the stored activations are read once, and layer 1's accumulators need no registers in A.  Pass A
// forms the ReLU masks of a chunk as one 32-bit word per feature (bit p: point p is positive) from the
// activations it loads, so that a lane reads the masks of its four rows in one load.
constexpr int kWavesS = 4;
constexpr int kNTS = 64 * kWavesS;
constexpr int kD1Chunk = kH * kPc;     // stored delta_1 of one chunk, feature-major [128][32]
constexpr int kW1 = kH * kK1;          // entries of W1, the first block of the parameter vector


// Value of lane l ^ 1 (l ^ 2) within groups of four lanes, by DPP quad permutes (no LDS traffic).
__device__ __forceinline__ unsigned quad_xor1(unsigned v) {
    return static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ unsigned quad_xor2(unsigned v) {
    return static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x4E, 0xF, 0xF, false));
}
__device__ __forceinline__ float quad_sum(float v) {
    v += __int_as_float(static_cast<int>(quad_xor1(static_cast<unsigned>(__float_as_int(v)))));
    v += __int_as_float(static_cast<int>(quad_xor2(static_cast<unsigned>(__float_as_int(v)))));
    return v;
}

// Bit j: element j of v is positive (v holds ReLU outputs, so positive means a nonzero magnitude).
__device__ __forceinline__ unsigned positive_bits8(const bf16x8& v) {
    const uint4 d = __builtin_bit_cast(uint4, v);
    const auto two = [](unsigned x) { return ((x & 0x7FFFu) ? 1u : 0u) | ((x & 0x7FFF0000u) ? 2u : 0u); };
    return two(d.x) | (two(d.y) << 2) | (two(d.z) << 4) | (two(d.w) << 6);
}

struct NfBwdALds {
    NfTables tab;
    alignas(16) float df[kPc];
    alignas(16) unsigned on[4][kH];           // bit p of on[l][row]: h_{l+1}[row][p] > 0
    alignas(16) __bf16 hT[4][kH * kLdT];      // h1..h4 of the chunk, feature-major
    alignas(16) __bf16 dP[2][kPc * kLdH];     // delta, point-major (input-gradient operand)
    alignas(16) __bf16 dT[2][kH * kLdT];      // delta, feature-major (weight-gradient operand)
};

// Level L (4, 3 or 2) of pass A for one chunk, delta_L in buffer `cur`: dW_L += delta_L h_{L-1}^T over the
// chunk's 32 points, and delta_{L-1} = (W_L^T delta_L) [h_{L-1} > 0] into the other buffer (its bias
// gradient into gb).  Ends with a barrier.
template <int L>
__device__ __forceinline__ void nf_level_a(NfBwdALds& sm, const bf16x8 (&tw)[4], f32x4 (&gl)[2][4], float (&gb)[4],
                                           int cur) {
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r16 = l & 15, q = l >> 4;
    const int row0 = 16 * wv + 4 * q;
    const __bf16* hprev = sm.hT[L - 2];
    // weight gradient: wave wv takes rows 32 (wv / 2) .. + 31 and columns 64 (wv % 2) .. + 63 of dW_L, so
    // that each fragment read feeds two MFMAs
    const int rg = wv >> 1, cg = wv & 1;
    bf16x8 da[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) da[rt] = ld8(sm.dT[cur] + (32 * rg + 16 * rt + r16) * kLdT + 8 * q);
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
        const bf16x8 hb = ld8(hprev + (64 * cg + 16 * kt + r16) * kLdT + 8 * q);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) gl[rt][kt] = mfma(da[rt], hb, gl[rt][kt]);
    }
    const uint4 on = *reinterpret_cast<const uint4*>(&sm.on[L - 2][row0]);
    f32x4 d2[2] = {f32x4{0.0f, 0.0f, 0.0f, 0.0f}, f32x4{0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
            d2[nt] = mfma(tw[ks], ld8(sm.dP[cur] + (16 * nt + r16) * kLdH + 32 * ks + 8 * q), d2[nt]);
    const unsigned onw[4] = {on.x, on.y, on.z, on.w};
    const int nxt = cur ^ 1;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const int p = 16 * nt + r16;
        bf16x4 dv;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            dv[i] = static_cast<__bf16>((onw[i] >> p) & 1u ? d2[nt][i] : 0.0f);
            gb[i] += static_cast<float>(dv[i]);
            sm.dT[nxt][(row0 + i) * kLdT + p] = dv[i];
        }
        if (L > 2) *reinterpret_cast<bf16x4*>(sm.dP[nxt] + p * kLdH + row0) = dv;
    }
    __syncthreads();
}

// Rows 32 wv + 16 rt + 4 q + i of a weight gradient (tiles of 16 columns) into this workgroup's partial.
template <int NT>
__device__ __forceinline__ void put_rows32(float* out, int off, int ld, const f32x4 (&gl)[2][NT]) {
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r16 = l & 15, q = l >> 4;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int kt = 0; kt < NT; ++kt)
#pragma unroll
            for (int i = 0; i < 4; ++i) out[off + (32 * wv + 16 * rt + 4 * q + i) * ld + 16 * kt + r16] = gl[rt][kt][i];
}

__global__ __launch_bounds__(kNT) void nf_bwd_a_kernel(NfArgs a, const __bf16* __restrict__ act,
                                                       const float* __restrict__ f_in,
                                                       __bf16* __restrict__ d1,
                                                       const float* __restrict__ dL_dw,
                                                       const float* __restrict__ scale, float* __restrict__ partial) {
    extern __shared__ __attribute__((aligned(16))) unsigned char nf_dyn[];
    NfBwdALds& sm = *reinterpret_cast<NfBwdALds*>(nf_dyn);
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r16 = l & 15, q = l >> 4;
    const int row0 = 16 * wv + 4 * q;
    load_tables(a, sm.tab);
    bf16x8 t2[4], t3[4], t4[4];
    load_rows<4>(a.packed, kOffT4, kH, t4);
    load_rows<4>(a.packed, kOffT3, kH, t3);
    load_rows<4>(a.packed, kOffT2, kH, t2);
    f32x4 g2[2][4], g3[2][4], g4[2][4];       // weight gradients: rows 32 (wv / 2) + 16 rt, columns 64 (wv % 2) + 16 kt
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            g2[rt][kt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            g3[rt][kt] = g2[rt][kt];
            g4[rt][kt] = g2[rt][kt];
        }
    float gb[4][4] = {};                      // bias gradients of layers 1..4, rows row0 + i
    float gw5 = 0.0f, gb5 = 0.0f;             // w5 gradient of feature t / 4 (partial over its 8 points)
    const float sc = scale ? *scale : 1.0f;
    __syncthreads();

    const int n_rays = a.N * a.n_elem;
    const int n_chunks = (a.Ns + kPc - 1) / kPc;
    // stored blocks move through registers: thread t carries points 8 (t % 4) .. + 7 of feature t / 4 of
    // each layer, 16 bytes; the next chunk's loads are issued before this chunk's work (barriers wait on
    // LDS only)
    const int feature = threadIdx.x >> 2, part = threadIdx.x & 3;
    for (int ray = blockIdx.x; ray < n_rays; ray += gridDim.x) {
        const float g = dL_dw[ray] * sc;
        if (g == 0.0f) continue;
        const NfRay r = nf_ray(a, ray);
        if (r.dl == 0.0f) continue;
        bf16x8 nxt[4];
        float fnxt = 0.0f;
        {
            const size_t chunk0 = static_cast<size_t>(ray) * n_chunks;
            const __bf16* src = act + chunk0 * kActChunk;
#pragma unroll
            for (int L = 0; L < 4; ++L) nxt[L] = ld8(src + (L * kH + feature) * kPc + 8 * part);
            if (threadIdx.x < kPc) fnxt = f_in[chunk0 * kPc + threadIdx.x];
        }
        for (int ch = 0; ch < n_chunks; ++ch) {
            const int s0 = ch * kPc;
            const size_t chunk = static_cast<size_t>(ray) * n_chunks + ch;
#pragma unroll
            for (int L = 0; L < 4; ++L) {
                *reinterpret_cast<bf16x8*>(sm.hT[L] + feature * kLdT + 8 * part) = nxt[L];
                // the ReLU mask word of (L, feature): this lane's 8 points, then the quad's 32
                unsigned m = positive_bits8(nxt[L]) << (8 * part);
                m |= quad_xor1(m);
                m |= quad_xor2(m);
                if (part == L) sm.on[L][feature] = m;
            }
            const float fcur = fnxt;
            if (ch + 1 < n_chunks) {
                const __bf16* src = act + (chunk + 1) * kActChunk;
#pragma unroll
                for (int L = 0; L < 4; ++L) nxt[L] = ld8(src + (L * kH + feature) * kPc + 8 * part);
                if (threadIdx.x < kPc) fnxt = f_in[(chunk + 1) * kPc + threadIdx.x];
            }
            if (threadIdx.x < kPc) {
                float d = 0.0f;
                if (s0 + static_cast<int>(threadIdx.x) < a.Ns) {
                    const float th = tanhf(fcur);
                    const float v = a.v0 + a.amp * th;
                    d = g * r.dl * a.v0 * a.amp * (1.0f - th * th) / (v * v);   // d w / d f, times dL/dw
                }
                sm.df[threadIdx.x] = d;
            }
            __syncthreads();
            // w5 gradient: sum over the chunk's points of df h4, 8 points per thread
            {
                const float4 dA = *reinterpret_cast<const float4*>(sm.df + 8 * part);
                const float4 dB = *reinterpret_cast<const float4*>(sm.df + 8 * part + 4);
                const float dfv[8] = {dA.x, dA.y, dA.z, dA.w, dB.x, dB.y, dB.z, dB.w};
                const bf16x8 hv = ld8(sm.hT[3] + feature * kLdT + 8 * part);
#pragma unroll
                for (int j = 0; j < 8; ++j) gw5 = fmaf(dfv[j], static_cast<float>(hv[j]), gw5);
            }
            // delta_4 = df w5 [h4 > 0]
            {
                const uint4 on = *reinterpret_cast<const uint4*>(&sm.on[3][row0]);
                const unsigned onw[4] = {on.x, on.y, on.z, on.w};
                const float4 w5v = *reinterpret_cast<const float4*>(&sm.tab.w5[row0]);
                const float w5r[4] = {w5v.x, w5v.y, w5v.z, w5v.w};
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const int p = 16 * nt + r16;
                    const float dfp = sm.df[p];
                    bf16x4 dv;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        dv[i] = static_cast<__bf16>((onw[i] >> p) & 1u ? dfp * w5r[i] : 0.0f);
                        gb[3][i] += static_cast<float>(dv[i]);
                        sm.dT[0][(row0 + i) * kLdT + p] = dv[i];
                    }
                    *reinterpret_cast<bf16x4*>(sm.dP[0] + p * kLdH + row0) = dv;
                }
            }
            if (threadIdx.x < kPc) gb5 += sm.df[threadIdx.x];
            __syncthreads();
            nf_level_a<4>(sm, t4, g4, gb[2], 0);
            nf_level_a<3>(sm, t3, g3, gb[1], 1);
            nf_level_a<2>(sm, t2, g2, gb[0], 0);
            // delta_1 (in dT[1]) of the chunk to the buffer; the next chunk rewrites dT[1] only after two
            // barriers
            *reinterpret_cast<bf16x8*>(d1 + chunk * kD1Chunk + feature * kPc + 8 * part) =
                ld8(sm.dT[1] + feature * kLdT + 8 * part);
        }
    }

    float* out = partial + static_cast<size_t>(blockIdx.x) * kNParams;
    auto put_w = [&](int off, const f32x4 (&gl)[2][4]) {
        const int rg = wv >> 1, cg = wv & 1;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int kt = 0; kt < 4; ++kt)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    out[off + (32 * rg + 16 * rt + 4 * q + i) * kH + 64 * cg + 16 * kt + r16] = gl[rt][kt][i];
    };
    put_w(kPW2, g2);
    put_w(kPW3, g3);
    put_w(kPW4, g4);
#pragma unroll
    for (int L = 1; L <= 4; ++L)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float v = gb[L - 1][i];
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
            if (r16 == 0) out[param_b(L) + row0 + i] = v;
        }
    const float w5s = quad_sum(gw5);
    if (part == 0) out[kPw5 + feature] = w5s;
    // b5: the first 32 threads hold per-point sums over the rays
    if (threadIdx.x < 64) {
        float v = gb5;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (threadIdx.x == 0) out[kPb5] = v;
    }
}

struct NfBwdBLds {
    float B[2 * kF];
    alignas(16) __bf16 featT[kK1 * kLdT];     // the chunk's features, feature-major
    alignas(16) __bf16 dT[kH * kLdT];         // the chunk's delta_1, feature-major
};

__global__ __launch_bounds__(kNTS, 2) void nf_bwd_b_kernel(NfArgs a, const __bf16* __restrict__ d1,
                                                           const float* __restrict__ dL_dw,
                                                           const float* __restrict__ scale, float* __restrict__ w1part) {
    extern __shared__ __attribute__((aligned(16))) unsigned char nf_dyn[];
    NfBwdBLds& sm = *reinterpret_cast<NfBwdBLds*>(nf_dyn);
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r16 = l & 15, q = l >> 4;
    for (int k = threadIdx.x; k < 2 * kF; k += blockDim.x) sm.B[k] = a.B[k];
    f32x4 g1[2][16];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int kt = 0; kt < 16; ++kt) g1[rt][kt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const float sc = scale ? *scale : 1.0f;
    const int n_rays = a.N * a.n_elem;
    const int n_chunks = (a.Ns + kPc - 1) / kPc;
    const int feature = threadIdx.x >> 2, part = threadIdx.x & 3;
    for (int ray = blockIdx.x; ray < n_rays; ray += gridDim.x) {
        if (dL_dw[ray] * sc == 0.0f) continue;               // the rays pass A skipped
        const NfRay r = nf_ray(a, ray);
        if (r.dl == 0.0f) continue;
        bf16x8 nxt[2];
        {
            const __bf16* src = d1 + static_cast<size_t>(ray) * n_chunks * kD1Chunk;
#pragma unroll
            for (int h = 0; h < 2; ++h) nxt[h] = ld8(src + (feature + 64 * h) * kPc + 8 * part);
        }
        for (int ch = 0; ch < n_chunks; ++ch) {
            const size_t chunk = static_cast<size_t>(ray) * n_chunks + ch;
            __syncthreads();                                  // the previous chunk's fragments are read
#pragma unroll
            for (int h = 0; h < 2; ++h)
                *reinterpret_cast<bf16x8*>(sm.dT + (feature + 64 * h) * kLdT + 8 * part) = nxt[h];
            if (ch + 1 < n_chunks) {
                const __bf16* src = d1 + (chunk + 1) * kD1Chunk;
#pragma unroll
                for (int h = 0; h < 2; ++h) nxt[h] = ld8(src + (feature + 64 * h) * kPc + 8 * part);
            }
            nf_features_rot(r, ch * kPc, sm.B, sm.featT);
            __syncthreads();
            bf16x8 da[2];
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) da[rt] = ld8(sm.dT + (32 * wv + 16 * rt + r16) * kLdT + 8 * q);
#pragma unroll
            for (int kt = 0; kt < 16; ++kt) {
                const bf16x8 fb = ld8(sm.featT + (16 * kt + r16) * kLdT + 8 * q);
#pragma unroll
                for (int rt = 0; rt < 2; ++rt) g1[rt][kt] = mfma(da[rt], fb, g1[rt][kt]);
            }
        }
    }
    put_rows32<16>(w1part + static_cast<size_t>(blockIdx.x) * kW1, 0, kK1, g1);
}

// dL/dparams[j] = sum over workgroups of partial[b][j] in a fixed order, in two levels (kSlices contiguous
// runs of partials, then the runs) so that many threads read the partials at once.
constexpr int kSlices = 16;

// The W1 entries come from w1part [n_w1][kW1] when it is given (the stored-activation form's pass B).
__global__ __launch_bounds__(256) void nf_reduce1_kernel(const float* __restrict__ partial, int n_part,
                                                        const float* __restrict__ w1part, int n_w1,
                                                        float* __restrict__ part2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int slice = blockIdx.y;
    if (j >= kNParams) return;
    const bool w1 = w1part && j < kW1;
    const float* src = w1 ? w1part + j : partial + j;
    const size_t pitch = w1 ? kW1 : kNParams;
    const int n = w1 ? n_w1 : n_part;
    const int per = (n + kSlices - 1) / kSlices;
    const int b1 = min((slice + 1) * per, n);
    float s = 0.0f;
    for (int b = slice * per; b < b1; ++b) s += src[static_cast<size_t>(b) * pitch];
    part2[static_cast<size_t>(slice) * kNParams + j] = s;
}

__global__ __launch_bounds__(256) void nf_reduce2_kernel(const float* __restrict__ part2, float* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kNParams) return;
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kSlices; ++k) s += part2[static_cast<size_t>(k) * kNParams + j];
    out[j] = s;
}

int launch_nf_reduce(const float* partial, int n_part, const float* w1part, int n_w1, float* out, hipStream_t st) {
    float* part2 = const_cast<float*>(partial) + static_cast<size_t>(n_part) * kNParams;
    nf_reduce1_kernel<<<dim3(ceil_div(kNParams, 256), kSlices), 256, 0, st>>>(partial, n_part, w1part, n_w1,
                                                                              part2);
    if (int s = launch_status("pact_nf_sos_to_delays_adjoint")) return s;
    nf_reduce2_kernel<<<ceil_div(kNParams, 256), 256, 0, st>>>(part2, out);
    return launch_status("pact_nf_sos_to_delays_adjoint");
}

__device__ __forceinline__ unsigned short bf16_rne(float x) {
    const unsigned u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<unsigned short>((u >> 16) | 0x40u);   // NaN
    return static_cast<unsigned short>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__global__ __launch_bounds__(256) void nf_pack_kernel(const float* __restrict__ params,
                                                     unsigned short* __restrict__ packed) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kPacked) return;
    float x;
    if (j < kOffW2) {
        x = params[kPW1 + j];
    } else if (j < kOffT2) {
        const int L = 2 + (j - kOffW2) / (kH * kH), o = (j - kOffW2) % (kH * kH);
        x = params[param_w(L) + o];
    } else if (j < kOffW5) {
        const int L = 2 + (j - kOffT2) / (kH * kH), o = (j - kOffT2) % (kH * kH);
        const int c = o / kH, rr = o % kH;                  // W^T[c][rr] = W[rr][c]
        x = params[param_w(L) + rr * kH + c];
    } else {
        x = params[kPw5 + (j - kOffW5)];
    }
    packed[j] = bf16_rne(x);
}

int check_nf(const float* B, const float* params, const unsigned short* packed, int n_freq, int width, float amp,
             float mask_radius, float v0, const float* centres, int N, const pact_ring* ring, int n_samples,
             const char* what) {
    PACT_CHECK_ARG(B && params && packed && centres && ring, "%s: null pointer", what);
    PACT_CHECK_SUPPORTED(n_freq == kF && width == kH, "%s: only 128 frequencies and width 128 are built (got %d, %d)",
                         what, n_freq, width);
    PACT_CHECK_ARG(N > 0 && n_samples > 0, "%s: N and n_samples must be positive", what);
    PACT_CHECK_ARG(v0 > 0.0f && std::isfinite(v0), "%s: v0 must be positive", what);
    PACT_CHECK_ARG(amp >= 0.0f && amp < v0, "%s: amp must be in [0, v0)", what);
    PACT_CHECK_ARG(mask_radius > 0.0f && std::isfinite(mask_radius), "%s: mask radius must be positive", what);
    if (int s = check_ring(*ring)) return s;
    PACT_CHECK_ARG(mask_radius < ring->radius, "%s: the mask disc must lie inside the ring", what);
    PACT_CHECK_SUPPORTED(static_cast<long long>(N) * ring->n_elem < (1LL << 31), "%s: too many rays", what);
    return PACT_OK;
}

NfArgs nf_args(const float* B, const float* params, const unsigned short* packed, float amp, float mask_radius,
               float v0, const float* centres, int N, const pact_ring& ring, int n_samples) {
    NfArgs a;
    a.B = B;
    a.params = params;
    a.packed = packed;
    a.amp = amp;
    a.rho2 = mask_radius * mask_radius;
    a.v0 = v0;
    a.centres = centres;
    a.N = N;
    a.n_elem = ring.n_elem;
    a.R = ring.radius;
    a.phi0 = ring.phi0;
    a.Ns = n_samples;
    return a;
}

template <int LO, int HI, int K1C, int K1N>
int launch_bwd(const NfArgs& a, const float* dL_dw, const float* scale, float* partial, int blocks, hipStream_t st) {
    static bool attr = false;
    const size_t lds = sizeof(NfBwdLds<LO, HI>);
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(nf_bwd_kernel<LO, HI, K1C, K1N>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        attr = true;
    }
    nf_bwd_kernel<LO, HI, K1C, K1N><<<blocks, kNT, lds, st>>>(a, dL_dw, scale, partial);
    return launch_status("pact_nf_sos_to_delays_adjoint");
}

template <typename K>
void set_lds_attr(K kernel, size_t lds) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(lds));
}

// Pass A on `blocks` workgroups (rows of partial), pass B on 2 blocks (rows of w1part: two per CU fit).
int launch_bwd_stored(const NfArgs& a, const __bf16* act, const float* f_in, __bf16* d1, const float* dL_dw,
                      const float* scale, float* partial, float* w1part, int blocks, hipStream_t st) {
    static bool attr = false;
    if (!attr) {
        set_lds_attr(nf_bwd_a_kernel, sizeof(NfBwdALds));
        set_lds_attr(nf_bwd_b_kernel, sizeof(NfBwdBLds));
        attr = true;
    }
    nf_bwd_a_kernel<<<blocks, kNT, sizeof(NfBwdALds), st>>>(a, act, f_in, d1, dL_dw, scale, partial);
    if (int s = launch_status("pact_nf_sos_to_delays_adjoint")) return s;
    nf_bwd_b_kernel<<<2 * blocks, kNTS, sizeof(NfBwdBLds), st>>>(a, d1, dL_dw, scale, w1part);
    return launch_status("pact_nf_sos_to_delays_adjoint");
}

// Activation buffer: h1..h4 [chunks][4][128][32] BF16, f [chunks][32] FP32, then the adjoint's delta_1
// [chunks][128][32] BF16.
struct NfActView {
    __bf16* h;
    float* f;
    __bf16* d1;
};

NfActView nf_act_view(void* act, long long n_rays, int n_samples) {
    const size_t chunks = static_cast<size_t>(n_rays) * ((n_samples + kPc - 1) / kPc);
    NfActView v;
    v.h = static_cast<__bf16*>(act);
    v.f = reinterpret_cast<float*>(v.h + chunks * kActChunk);
    v.d1 = reinterpret_cast<__bf16*>(v.f + chunks * kPc);
    return v;
}

// Adjoint workspace: one partial gradient per workgroup of pass A (or of the recomputing passes), 16 for the
// second level of the sum, then pass B's W1 partials, two per CU.
size_t nf_adjoint_ws_bytes(int cus) {
    return (static_cast<size_t>(cus + kSlices) * kNParams + static_cast<size_t>(2 * cus) * kW1) * sizeof(float);
}

size_t nf_activation_bytes(long long n_rays, int n_samples) {
    const long long chunks = n_rays * ((n_samples + kPc - 1) / kPc);
    return static_cast<size_t>(chunks) * (kActChunk * sizeof(__bf16) + kPc * sizeof(float) + kD1Chunk * sizeof(__bf16));
}

}  // namespace
}  // namespace pact

extern "C" size_t pact_nf_activation_bytes(int N, const pact_ring* ring, int n_samples) {
    if (!ring || N <= 0 || ring->n_elem <= 0 || n_samples <= 0) return 0;
    return pact::nf_activation_bytes(static_cast<long long>(N) * ring->n_elem, n_samples);
}

extern "C" size_t pact_nf_param_count(int n_freq, int width) {
    if (n_freq <= 0 || width <= 0) return 0;
    return static_cast<size_t>(width) * 2 * n_freq + width + 3 * (static_cast<size_t>(width) * width + width) +
           width + 1;
}

extern "C" size_t pact_nf_packed_count(int n_freq, int width) {
    if (n_freq != pact::kF || width != pact::kH) return 0;
    return pact::kPacked;
}

extern "C" int pact_nf_pack(const float* params, int n_freq, int width, unsigned short* packed, void* stream) {
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(params && packed, "pact_nf_pack: null pointer");
    PACT_CHECK_SUPPORTED(n_freq == kF && width == kH, "pact_nf_pack: only 128 frequencies and width 128 are built");
    nf_pack_kernel<<<ceil_div(kPacked, 256), 256, 0, as_stream(stream)>>>(params, packed);
    return launch_status("pact_nf_pack");
}

extern "C" int pact_nf_sos_to_delays(const float* B, const float* params, const unsigned short* packed, int n_freq,
                                     int width, float amp, float mask_radius, float v0, const float* centres, int N,
                                     const pact_ring* ring, int n_samples, float* w, void* act, size_t act_bytes,
                                     void* stream) {
    using namespace pact;
    clear_error();
    if (int s = check_nf(B, params, packed, n_freq, width, amp, mask_radius, v0, centres, N, ring, n_samples,
                         "pact_nf_sos_to_delays"))
        return s;
    PACT_CHECK_ARG(w, "pact_nf_sos_to_delays: null output");
    const NfArgs a = nf_args(B, params, packed, amp, mask_radius, v0, centres, N, *ring, n_samples);
    const long long n_rays = static_cast<long long>(N) * ring->n_elem;
    NfActView v = {nullptr, nullptr, nullptr};
    if (act) {
        const size_t need = nf_activation_bytes(n_rays, n_samples);
        if (act_bytes < need) {
            set_error("pact_nf_sos_to_delays: activation buffer of %zu bytes needed, %zu given", need, act_bytes);
            return PACT_EWORKSPACE;
        }
        v = nf_act_view(act, n_rays, n_samples);
    }
    const int blocks = static_cast<int>(std::min<long long>(n_rays, 2LL * device_cu_count()));
    nf_fwd_kernel<<<blocks, kNTF, 0, as_stream(stream)>>>(a, w, v.h, v.f);
    return launch_status("pact_nf_sos_to_delays");
}

extern "C" size_t pact_nf_sos_to_delays_adjoint_workspace_size(int n_freq, int width) {
    if (n_freq != pact::kF || width != pact::kH) return 0;
    return pact::nf_adjoint_ws_bytes(pact::device_cu_count());
}

extern "C" int pact_nf_sos_to_delays_adjoint(const float* B, const float* params, const unsigned short* packed,
                                             int n_freq, int width, float amp, float mask_radius, float v0,
                                             const float* centres, int N, const pact_ring* ring, int n_samples,
                                             const float* dL_dw, const float* scale, float* dL_dparams,
                                             void* act, size_t act_bytes, void* ws, size_t ws_bytes,
                                             void* stream) {
    using namespace pact;
    clear_error();
    if (int s = check_nf(B, params, packed, n_freq, width, amp, mask_radius, v0, centres, N, ring, n_samples,
                         "pact_nf_sos_to_delays_adjoint"))
        return s;
    PACT_CHECK_ARG(dL_dw && dL_dparams, "pact_nf_sos_to_delays_adjoint: null pointer");
    const int blocks = device_cu_count();
    const size_t need = nf_adjoint_ws_bytes(blocks);
    if (!ws || ws_bytes < need) {
        set_error("pact_nf_sos_to_delays_adjoint: workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : 0);
        return PACT_EWORKSPACE;
    }
    const NfArgs a = nf_args(B, params, packed, amp, mask_radius, v0, centres, N, *ring, n_samples);
    float* partial = static_cast<float*>(ws);
    hipStream_t st = as_stream(stream);
    if (act) {
        const long long n_rays = static_cast<long long>(N) * ring->n_elem;
        const size_t need = nf_activation_bytes(n_rays, n_samples);
        if (act_bytes < need) {
            set_error("pact_nf_sos_to_delays_adjoint: activation buffer of %zu bytes needed, %zu given", need,
                      act_bytes);
            return PACT_EWORKSPACE;
        }
        const NfActView v = nf_act_view(act, n_rays, n_samples);
        // from the stored activations: the head and layers 4..2 (writing delta_1), then layer 1
        float* w1part = partial + static_cast<size_t>(blocks + kSlices) * kNParams;
        if (int s = launch_bwd_stored(a, v.h, v.f, v.d1, dL_dw, scale, partial, w1part, blocks, st)) return s;
        return launch_nf_reduce(partial, blocks, w1part, 2 * blocks, dL_dparams, st);
    }
    // four passes, each recomputing the forward activations: layers 3-4 (and the head), layer 2, and the
    // two column halves of layer 1, so that each pass's gradient accumulators fit in registers
    if (int s = launch_bwd<3, 4, 0, 0>(a, dL_dw, scale, partial, blocks, st)) return s;
    if (int s = launch_bwd<2, 2, 0, 0>(a, dL_dw, scale, partial, blocks, st)) return s;
    if (int s = launch_bwd<1, 1, 0, 8>(a, dL_dw, scale, partial, blocks, st)) return s;
    if (int s = launch_bwd<1, 1, 8, 8>(a, dL_dw, scale, partial, blocks, st)) return s;
    return launch_nf_reduce(partial, blocks, nullptr, 0, dL_dparams, st);
}
