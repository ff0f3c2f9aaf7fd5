// Windowed patch spectra (Eq. conv / Sec. 3.3) and the inverse transform of patch spectra.
//
// One workgroup per (patch, delay) image.  The P x P patch (P <= 96) is staged in LDS with its Gaussian
// window applied and transformed along rows, then along columns.  When P factors into 2, 3 and 5 (the paper's
// 80 = 4 * 4 * 5, and 64 = 4 * 4 * 4) each pass is a batch of mixed-radix FFTs: Stockham stages of radix 4,
// 2, 3, 5 (self-sorting, out of place between two LDS buffers, one barrier per stage) against an LDS table
// of e^{2 pi i m / P}, O(P^2 log P) per image.  Any other P takes length-P DFTs against the same table
// (P^2 (P/2 + 1) complex multiply-adds per pass for the half spectrum).  The loads of a patch row and the
// stores of a spectrum row are coalesced.
#include "common.h"

namespace pact {
namespace {

// ---- mixed-radix FFT (P = 2^a 3^b 5^c) ----

constexpr int kMaxStages = 8;

// Radices of a length-P transform in stage order (4s, then 2, 3s, 5s); n = 0 if P has another prime factor.
struct FftPlan {
    int n;
    int r[kMaxStages];
};

FftPlan fft_plan(int P) {
    FftPlan f{};
    int m = P;
    for (int radix : {4, 2, 3, 5})
        while (m % radix == 0 && f.n < kMaxStages) {
            f.r[f.n++] = radix;
            m /= radix;
        }
    if (m != 1 || P < 2) f.n = 0;
    return f;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// e^{sign 2 pi i m / P} from the table of e^{2 pi i m / P}
__device__ __forceinline__ float2 twiddle(const float2* tw, int m, float sign) {
    const float2 w = tw[m];
    return make_float2(w.x, sign * w.y);
}

// In-place length-R DFT X[m] = sum_r v[r] e^{sign 2 pi i r m / R}.
template <int R>
__device__ __forceinline__ void small_dft(float2 (&v)[R], const float2* tw, int P, float sign) {
    if constexpr (R == 2) {
        const float2 a = v[0], b = v[1];
        v[0] = make_float2(a.x + b.x, a.y + b.y);
        v[1] = make_float2(a.x - b.x, a.y - b.y);
    } else if constexpr (R == 4) {
        // with W = e^{sign i pi / 2} = sign i: X1 = (v0 - v2) + W (v1 - v3), X3 = (v0 - v2) - W (v1 - v3)
        const float2 s02 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
        const float2 d02 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
        const float2 s13 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
        const float2 d13 = make_float2(v[1].x - v[3].x, v[1].y - v[3].y);
        const float2 wd = make_float2(-sign * d13.y, sign * d13.x);
        v[0] = make_float2(s02.x + s13.x, s02.y + s13.y);
        v[1] = make_float2(d02.x + wd.x, d02.y + wd.y);
        v[2] = make_float2(s02.x - s13.x, s02.y - s13.y);
        v[3] = make_float2(d02.x - wd.x, d02.y - wd.y);
    } else {
        float2 x[R];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            float2 acc = v[0];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const float2 t = cmul(v[r], twiddle(tw, ((r * m) % R) * (P / R), sign));
                acc.x += t.x;
                acc.y += t.y;
            }
            x[m] = acc;
        }
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = x[m];
    }
}

// One radix-R Stockham stage over `count` length-P vectors, element e of vector b at b * ldb + e * lde:
// butterfly j (of P / R) of a vector takes inputs j + r P / R, scales input r by e^{sign 2 pi i k r / (Ns R)}
// (k = j mod Ns, Ns the product of the earlier radices), transforms them and writes output r at
// (j / Ns) Ns R + k + r Ns.  b_fast: consecutive threads take consecutive vectors (columns of a row-major
// image), else consecutive butterflies of one vector.
template <int R>
__device__ __forceinline__ void stockham_stage(const float2* src, float2* dst, int P, int Ns, int count, int ldb,
                                               int lde, bool b_fast, const float2* tw, float sign) {
    const int nb = P / R;
    const int step = P / (Ns * R);
    for (int t = threadIdx.x; t < count * nb; t += blockDim.x) {
        const int b = b_fast ? t % count : t / nb;
        const int j = b_fast ? t / count : t % nb;
        const int k = j % Ns;
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float2 x = src[b * ldb + (j + r * nb) * lde];
            v[r] = r == 0 ? x : cmul(x, twiddle(tw, k * r * step, sign));
        }
        small_dft<R>(v, tw, P, sign);
        const int base = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[b * ldb + (base + r * Ns) * lde] = v[r];
    }
}

// All stages of a batch of transforms; the result ends in *src (the buffers swap after every stage).
__device__ __forceinline__ void fft_batch(float2*& src, float2*& dst, const FftPlan& f, int P, int count, int ldb,
                                          int lde, bool b_fast, const float2* tw, float sign) {
    int Ns = 1;
    for (int s = 0; s < f.n; ++s) {
        const int R = f.r[s];
        if (R == 4) stockham_stage<4>(src, dst, P, Ns, count, ldb, lde, b_fast, tw, sign);
        else if (R == 2) stockham_stage<2>(src, dst, P, Ns, count, ldb, lde, b_fast, tw, sign);
        else if (R == 3) stockham_stage<3>(src, dst, P, Ns, count, ldb, lde, b_fast, tw, sign);
        else stockham_stage<5>(src, dst, P, Ns, count, ldb, lde, b_fast, tw, sign);
        __syncthreads();
        float2* t = src;
        src = dst;
        dst = t;
        Ns *= R;
    }
}

__device__ __forceinline__ void fill_twiddles(float2* tw, int P) {
    for (int m = threadIdx.x; m < P; m += blockDim.x) {
        float sn, cs;
        sincospif(2.0f * m / P, &sn, &cs);
        tw[m] = make_float2(cs, sn);
    }
}

// One image per workgroup; many waves per workgroup keep a CU busy through the stages' barriers.
constexpr int kFftThreads = 512;

// LDS of a transform with two buffers of rows x P values, the twiddle table and the window.
size_t fft_lds_bytes(int P, int rows) {
    return (2 * static_cast<size_t>(rows) * P + P) * sizeof(float2) + P * sizeof(float);
}

// Windowed half (Wout = P / 2 + 1) or full (Wout = P) spectra of one patch image by FFTs.  Rows 2 r and 2 r + 1
// go through one complex transform as its real and imaginary parts (ceil(P / 2) transforms); with Z its result,
// their spectra are X_2r[k] = (Z[k] + conj Z[-k]) / 2 and X_2r+1[k] = (Z[k] - conj Z[-k]) / 2i.  Then the
// Wout columns needed.  Two LDS buffers of max(ceil(P / 2), Wout) x P values (26 KB each at P = 80, half).
__global__ __launch_bounds__(kFftThreads) void patch_fft_kernel(const float* __restrict__ stack, int M, int ny, int nx,
                                                                int P, int stride, int npx, float px,
                                                                float inv_two_sigma2, int Wout, FftPlan f,
                                                                float2* __restrict__ Y) {
    extern __shared__ float2 lds2[];
    const int H = (P + 1) / 2;
    const int cap = max(H, Wout) * P;
    float2* bufA = lds2;
    float2* bufB = bufA + cap;
    float2* tw = bufB + cap;               // [P]
    float* g1 = reinterpret_cast<float*>(tw + P);   // [P] 1-D window factor
    const int img = blockIdx.x;            // = i * M + j
    const int i = img / M, j = img % M;
    const int r0 = (i / npx) * stride, c0 = (i % npx) * stride;
    fill_twiddles(tw, P);
    for (int m = threadIdx.x; m < P; m += blockDim.x) {
        const float u = (m - 0.5f * (P - 1)) * px;
        g1[m] = expf(-u * u * inv_two_sigma2);
    }
    __syncthreads();
    const float* src = stack + (static_cast<size_t>(j) * ny + r0) * nx + c0;
    for (int idx = threadIdx.x; idx < H * P; idx += blockDim.x) {
        const int r = idx / P, v = idx % P;
        const int u = 2 * r;
        const float gv = g1[v];
        const float re = src[static_cast<size_t>(u) * nx + v] * (g1[u] * gv);
        const float im = u + 1 < P ? src[static_cast<size_t>(u + 1) * nx + v] * (g1[u + 1] * gv) : 0.0f;
        bufA[idx] = make_float2(re, im);
    }
    __syncthreads();
    float2* a = bufA;
    float2* b = bufB;
    fft_batch(a, b, f, P, H, P, 1, false, tw, -1.0f);        // row pairs: Z[r][k]
    for (int idx = threadIdx.x; idx < P * Wout; idx += blockDim.x) {
        const int u = idx / Wout, kx = idx % Wout;
        const float2 z = a[(u >> 1) * P + kx];
        const float2 zc = a[(u >> 1) * P + (kx == 0 ? 0 : P - kx)];    // Z[-k], to be conjugated
        b[idx] = (u & 1) ? make_float2(0.5f * (z.y + zc.y), -0.5f * (z.x - zc.x))
                         : make_float2(0.5f * (z.x + zc.x), 0.5f * (z.y - zc.y));
    }
    __syncthreads();
    float2* t = a;
    a = b;
    b = t;
    fft_batch(a, b, f, P, Wout, 1, Wout, true, tw, -1.0f);   // columns kx < Wout: Y[ky][kx]
    float2* dst = Y + static_cast<size_t>(img) * P * Wout;
    for (int idx = threadIdx.x; idx < P * Wout; idx += blockDim.x) dst[idx] = a[idx];
}

// x[b] = Re(IFFT2(X[b])) for full P x P spectra, by FFTs: columns, then rows.
__global__ __launch_bounds__(kFftThreads) void ifft_real_kernel(const float2* __restrict__ X, int P, FftPlan f,
                                                        float* __restrict__ x) {
    extern __shared__ float2 lds2[];
    float2* bufA = lds2;
    float2* bufB = bufA + P * P;
    float2* tw = bufB + P * P;
    const int bimg = blockIdx.x;
    fill_twiddles(tw, P);
    const float2* src = X + static_cast<size_t>(bimg) * P * P;
    for (int idx = threadIdx.x; idx < P * P; idx += blockDim.x) bufA[idx] = src[idx];
    __syncthreads();
    float2* a = bufA;
    float2* b = bufB;
    fft_batch(a, b, f, P, P, 1, P, true, tw, 1.0f);          // columns: z[u][kx] = sum_ky X[ky][kx] e^{+...}
    fft_batch(a, b, f, P, P, P, 1, false, tw, 1.0f);         // rows
    const float scale = 1.0f / (static_cast<float>(P) * P);
    float* dst = x + static_cast<size_t>(bimg) * P * P;
    for (int idx = threadIdx.x; idx < P * P; idx += blockDim.x) dst[idx] = a[idx].x * scale;
}

// ---- length-P DFTs (P with a prime factor above 5) ----

__global__ __launch_bounds__(256) void patch_dft_kernel(const float* __restrict__ stack, int M, int ny, int nx,
                                                        int P, int stride, int npx, float px, float inv_two_sigma2,
                                                        int Wout, float2* __restrict__ Y) {
    extern __shared__ float lds[];
    float* xs = lds;                       // [P][P] windowed patch
    float* zr = xs + P * P;                // [P][Wout] row transforms
    float* zi = zr + P * Wout;
    float* twc = zi + P * Wout;            // [P] cos(2 pi m / P)
    float* tws = twc + P;                  // [P] sin(2 pi m / P)
    float* g1 = tws + P;                   // [P] 1-D window factor

    const int img = blockIdx.x;            // = i * M + j
    const int i = img / M;
    const int j = img % M;
    const int r0 = (i / npx) * stride;
    const int c0 = (i % npx) * stride;
    const int tid = threadIdx.x;

    for (int m = tid; m < P; m += blockDim.x) {
        float s, c;
        sincospif(2.0f * m / P, &s, &c);
        twc[m] = c;
        tws[m] = s;
        const float u = (m - 0.5f * (P - 1)) * px;
        g1[m] = expf(-u * u * inv_two_sigma2);
    }
    __syncthreads();
    const float* src = stack + (static_cast<size_t>(j) * ny + r0) * nx + c0;
    for (int idx = tid; idx < P * P; idx += blockDim.x) {
        const int u = idx / P, v = idx % P;
        xs[idx] = src[static_cast<size_t>(u) * nx + v] * (g1[u] * g1[v]);
    }
    __syncthreads();
    // rows: z[u][kx] = sum_v x[u][v] e^{-2 pi i v kx / P}
    for (int idx = tid; idx < P * Wout; idx += blockDim.x) {
        const int u = idx / Wout, kx = idx % Wout;
        const float* row = xs + u * P;
        float ar = 0.0f, ai = 0.0f;
        int m = 0;
        for (int v = 0; v < P; ++v) {
            const float xv = row[v];
            ar = fmaf(xv, twc[m], ar);
            ai = fmaf(-xv, tws[m], ai);
            m += kx;
            if (m >= P) m -= P;
        }
        zr[idx] = ar;
        zi[idx] = ai;
    }
    __syncthreads();
    // columns: Y[ky][kx] = sum_u z[u][kx] e^{-2 pi i u ky / P}
    float2* dst = Y + static_cast<size_t>(img) * P * Wout;
    for (int idx = tid; idx < P * Wout; idx += blockDim.x) {
        const int ky = idx / Wout, kx = idx % Wout;
        float ar = 0.0f, ai = 0.0f;
        int m = 0;
        for (int u = 0; u < P; ++u) {
            const float a = zr[u * Wout + kx], b = zi[u * Wout + kx];
            const float c = twc[m], s = tws[m];
            ar = fmaf(a, c, fmaf(b, s, ar));
            ai = fmaf(b, c, fmaf(-a, s, ai));
            m += ky;
            if (m >= P) m -= P;
        }
        dst[idx] = make_float2(ar, ai);
    }
}

// x[b] = Re(IFFT2(X[b])) for full P x P spectra.
__global__ __launch_bounds__(256) void idft_real_kernel(const float2* __restrict__ X, int P,
                                                        float* __restrict__ x) {
    extern __shared__ float lds[];
    float* ar_ = lds;                      // [P][P] input re
    float* ai_ = ar_ + P * P;              // [P][P] input im
    float* zr = ai_ + P * P;               // [P][P] after the column pass (re)
    float* zi = zr + P * P;
    float* twc = zi + P * P;
    float* tws = twc + P;
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    for (int m = tid; m < P; m += blockDim.x) {
        float s, c;
        sincospif(2.0f * m / P, &s, &c);
        twc[m] = c;
        tws[m] = s;
    }
    const float2* src = X + static_cast<size_t>(b) * P * P;
    for (int idx = tid; idx < P * P; idx += blockDim.x) {
        const float2 v = src[idx];
        ar_[idx] = v.x;
        ai_[idx] = v.y;
    }
    __syncthreads();
    // z[u][kx] = sum_ky X[ky][kx] e^{+2 pi i ky u / P}
    for (int idx = tid; idx < P * P; idx += blockDim.x) {
        const int u = idx / P, kx = idx % P;
        float sr = 0.0f, si = 0.0f;
        int m = 0;
        for (int ky = 0; ky < P; ++ky) {
            const float a = ar_[ky * P + kx], bb = ai_[ky * P + kx];
            const float c = twc[m], s = tws[m];
            sr = fmaf(a, c, fmaf(-bb, s, sr));
            si = fmaf(a, s, fmaf(bb, c, si));
            m += u;
            if (m >= P) m -= P;
        }
        zr[idx] = sr;
        zi[idx] = si;
    }
    __syncthreads();
    // x[u][v] = Re(sum_kx z[u][kx] e^{+2 pi i kx v / P}) / P^2
    const float scale = 1.0f / (static_cast<float>(P) * P);
    float* dst = x + static_cast<size_t>(b) * P * P;
    for (int idx = tid; idx < P * P; idx += blockDim.x) {
        const int u = idx / P, v = idx % P;
        float sr = 0.0f;
        int m = 0;
        for (int kx = 0; kx < P; ++kx) {
            sr = fmaf(zr[u * P + kx], twc[m], fmaf(-zi[u * P + kx], tws[m], sr));
            m += v;
            if (m >= P) m -= P;
        }
        dst[idx] = sr * scale;
    }
}

}  // namespace

int launch_idft_real(const float* X, int B, int P, float* x, hipStream_t stream) {
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(idft_real_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(ifft_real_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        attr = true;
    }
    const FftPlan f = fft_plan(P);
    if (f.n > 0) {
        ifft_real_kernel<<<B, kFftThreads, fft_lds_bytes(P, P), stream>>>(reinterpret_cast<const float2*>(X), P, f, x);
    } else {
        const size_t lds = (4 * static_cast<size_t>(P) * P + 2 * P) * sizeof(float);
        idft_real_kernel<<<B, 256, lds, stream>>>(reinterpret_cast<const float2*>(X), P, x);
    }
    return launch_status("pact_ifft2_real");
}

}  // namespace pact

extern "C" int pact_patch_fft(const float* stack, int M, const pact_grid* img_, const pact_patches* pp_, int half, float* Y,
                              void* stream) {
    if (!img_ || !pp_) {
        pact::set_error("pact_patch_fft: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_grid img = *img_;
    const pact_patches pp = *pp_;
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(stack && Y, "pact_patch_fft: null pointer");
    PACT_CHECK_ARG(M > 0, "pact_patch_fft: M must be positive");
    PACT_CHECK_ARG(pp.fwhm > 0.0f, "pact_patch_fft: fwhm must be positive");
    int npy = 0, npx = 0;
    if (int s = pact_patch_count(&img, &pp, &npy, &npx)) return s;
    PACT_CHECK_SUPPORTED(pp.P <= kMaxPatch, "pact_patch_fft: P = %d exceeds %d", pp.P, kMaxPatch);
    const int P = pp.P;
    const int Wout = half ? P / 2 + 1 : P;
    const double sigma = pp.fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    const float inv_two_sigma2 = static_cast<float>(1.0 / (2.0 * sigma * sigma));
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(patch_dft_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(patch_fft_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        attr = true;
    }
    const FftPlan f = fft_plan(P);
    if (f.n > 0) {
        patch_fft_kernel<<<npy * npx * M, kFftThreads, fft_lds_bytes(P, std::max((P + 1) / 2, Wout)), as_stream(stream)>>>(
            stack, M, img.ny, img.nx, P, pp.stride, npx, img.spacing, inv_two_sigma2, Wout, f,
            reinterpret_cast<float2*>(Y));
    } else {
        const size_t lds = (static_cast<size_t>(P) * P + 2 * static_cast<size_t>(P) * Wout + 3 * P) * sizeof(float);
        patch_dft_kernel<<<npy * npx * M, 256, lds, as_stream(stream)>>>(stack, M, img.ny, img.nx, P, pp.stride, npx,
                                                                       img.spacing, inv_two_sigma2, Wout,
                                                                       reinterpret_cast<float2*>(Y));
    }
    return launch_status("pact_patch_fft");
}

extern "C" int pact_ifft2_real(const float* X, int B, int P, float* x, void* stream) {
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(X && x, "pact_ifft2_real: null pointer");
    PACT_CHECK_ARG(B > 0 && P > 0, "pact_ifft2_real: B and P must be positive");
    PACT_CHECK_SUPPORTED(P <= kMaxPatch, "pact_ifft2_real: P = %d exceeds %d", P, kMaxPatch);
    return launch_idft_real(X, B, P, x, as_stream(stream));
}
