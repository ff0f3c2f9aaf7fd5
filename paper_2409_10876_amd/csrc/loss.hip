// The fused optimisation-step kernel: Eq. TF + Eq. multi-deconv + data term of Eq. jr and its
// gradient with respect to the wavefront table, in one pass over the half spectra Y.
//
// Algebra used (exact rewriting of the three equations, no approximation).  At a
// bin k of patch i write th = angle(k), Wa = W_i(th), Wb = W_i(th + pi),
// wbar = (Wa + Wb) / 2, psi = -|k| (Wa - Wb) / 2 and, for each delay,
// c_j = cos(|k| (d_j - wbar)).  Then H_j = e^{j psi} c_j: the antisymmetric
// (first-order) part of the wavefront is a phase common to all delays.  With
// N = sum_j c_j Y_j, D = sum_j c_j^2 and Xt = N / (D + eps):
//   X_hat = e^{-j psi} Xt,   Y_j - H_j X_hat = Y_j - c_j Xt =: r_j   (phase-free),
//   loss_k = |k| sum_j |r_j|^2,
//   d loss_k / d c_j = -2 |k| [Re(conj(r_j) Xt) + eps Re(conj(Xt) (Y_j - 2 c_j Xt)) / (D + eps)],
//   d c_j / d wbar = |k| sin(|k| (d_j - wbar)),   d wbar / dWa = d wbar / dWb = 1/2,
// and Wa, Wb scatter to the two neighbouring elements of their ring hits.  The
// residual form keeps the loss and gradient accurate near convergence (no
// difference of two large sums).  No transfer function is stored.
//
// Half spectra: Y of a real patch satisfies Y(-k) = conj(Y(k)); the loss and
// gradient at -k equal those at k because wbar is pi-periodic -- except on the
// Nyquist row of an even P, where the bin (P/2, P - kx) is not the negative of
// (P/2, kx) on the FFT grid.  So interior columns count twice, columns 0 and
// P/2 once, and each Nyquist-row interior bin also evaluates its twin
// (physical k = (-k_x, k_y), data conj(Y)) explicitly.
//
// Layout: workgroup = 256 consecutive bins of one patch's half spectrum, so the
// M channel loads of a wave are M coalesced 512-byte rows.  The patch's
// wavefront row and its gradient accumulator live in LDS.  Per-workgroup
// partials are summed in a fixed order by a second small kernel.
#include "common.h"

namespace pact {
namespace {

constexpr int kBlock = 256;

struct LossArgs {
    const float2* Yh;
    const float* w;
    const float* centres;
    const float* d;
    int n_elem;
    float R, phi0;
    int P, Wh, S;
    float k0, eps;
    float* part_loss;     // [N * S]
    float* part_gw;       // [N * S][n_elem]
    float2* X;            // [N][P][P] or null
};

template <int M>
__device__ __forceinline__ float eval_bin(const LossArgs& a, int i, float kxv, float kyv, const float2 (&Y)[M],
                                          bool conj_y, float weight, float cx, float cy, float R2mc2,
                                          const float* wl, float* gw, const float* ds, float2* xout,
                                          float2* xmirror) {
    const float kabs = sqrtf(kxv * kxv + kyv * kyv);
    const float ys = conj_y ? -1.0f : 1.0f;
    if (kabs == 0.0f) {
        if (xout) {
            float sr = 0.0f, si = 0.0f;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                sr += Y[j].x;
                si += ys * Y[j].y;
            }
            const float inv = 1.0f / (static_cast<float>(M) + a.eps);
            *xout = make_float2(sr * inv, si * inv);
        }
        return 0.0f;
    }
    const float inv = 1.0f / kabs;
    const float ux = kxv * inv, uy = kyv * inv;
    const float nf = static_cast<float>(a.n_elem);
    const float n2pi = nf / kTwoPi;
    int n0a, n1a, n0b, n1b;
    float al_a, al_b;
    ring_cell(ring_hit_index(cx, cy, ux, uy, R2mc2, a.phi0, n2pi, nf), a.n_elem, n0a, n1a, al_a);
    ring_cell(ring_hit_index(cx, cy, -ux, -uy, R2mc2, a.phi0, n2pi, nf), a.n_elem, n0b, n1b, al_b);
    const float Wa = fmaf(al_a, wl[n1a] - wl[n0a], wl[n0a]);
    const float Wb = fmaf(al_b, wl[n1b] - wl[n0b], wl[n0b]);
    const float wbar = 0.5f * (Wa + Wb);

    float c[M], s[M];
    float nr = 0.0f, ni = 0.0f, D = 0.0f;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        sincosf(kabs * (ds[j] - wbar), &s[j], &c[j]);
        nr = fmaf(c[j], Y[j].x, nr);
        ni = fmaf(c[j], ys * Y[j].y, ni);
        D = fmaf(c[j], c[j], D);
    }
    const float De = D + a.eps;
    const float invD = 1.0f / De;
    const float xr = nr * invD, xi = ni * invD;
    float l = 0.0f, gbar = 0.0f;
    const float eps_invD = a.eps * invD;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const float yr = Y[j].x, yi = ys * Y[j].y;
        const float rr = fmaf(-c[j], xr, yr), ri = fmaf(-c[j], xi, yi);
        l = fmaf(rr, rr, fmaf(ri, ri, l));
        // Re(conj(r) Xt) + eps Re(conj(Xt)(Y - 2 c Xt)) / (D + eps)
        const float t1 = rr * xr + ri * xi;
        const float t2 = (yr - 2.0f * c[j] * xr) * xr + (yi - 2.0f * c[j] * xi) * xi;
        const float dl_dc = fmaf(eps_invD, t2, t1);
        gbar = fmaf(dl_dc, s[j], gbar);
    }
    // d loss / d wbar = sum_j (-2 |k| dl_dc_j) (|k| s_j); half of it to each of Wa and Wb
    const float gW = weight * (-kabs * kabs) * gbar;
    atomicAdd(&gw[n0a], gW - al_a * gW);
    atomicAdd(&gw[n1a], al_a * gW);
    atomicAdd(&gw[n0b], gW - al_b * gW);
    atomicAdd(&gw[n1b], al_b * gW);
    if (xout) {
        const float psi = -0.5f * kabs * (Wa - Wb);
        float sp, cp;
        sincosf(psi, &sp, &cp);
        // X_hat = e^{-j psi} Xt
        const float2 xh = make_float2(xr * cp + xi * sp, xi * cp - xr * sp);
        *xout = xh;
        if (xmirror) *xmirror = make_float2(xh.x, -xh.y);
    }
    return weight * kabs * l;
}

template <int M>
__global__ __launch_bounds__(kBlock) void loss_grad_kernel(LossArgs a) {
    extern __shared__ float lds[];
    float* wl = lds;
    float* gw = lds + a.n_elem;
    __shared__ float ds[M];
    __shared__ float red[kBlock / 64];
    const int i = blockIdx.y;
    const int tid = threadIdx.x;
    for (int n = tid; n < a.n_elem; n += kBlock) {
        wl[n] = a.w[static_cast<size_t>(i) * a.n_elem + n];
        gw[n] = 0.0f;
    }
    if (tid < M) ds[tid] = a.d[tid];
    __syncthreads();

    const int P = a.P, Wh = a.Wh;
    const int nbins = P * Wh;
    const int bin = blockIdx.x * kBlock + tid;
    float l = 0.0f;
    if (bin < nbins) {
        const int ky = bin / Wh, kx = bin % Wh;
        const float cx = a.centres[2 * i], cy = a.centres[2 * i + 1];
        const float R2mc2 = a.R * a.R - (cx * cx + cy * cy);
        float2 Y[M];
        const size_t PW = static_cast<size_t>(P) * Wh;
        const float2* src = a.Yh + static_cast<size_t>(i) * M * PW + bin;
#pragma unroll
        for (int j = 0; j < M; ++j) Y[j] = src[j * PW];
        const bool even = (P & 1) == 0;
        const bool self_col = kx == 0 || (even && kx == P / 2);
        const bool nyq_row = even && ky == P / 2;
        const float kxv = fft_wavenumber(kx, P, a.k0);
        const float kyv = fft_wavenumber(ky, P, a.k0);
        float2* X = a.X ? a.X + static_cast<size_t>(i) * P * P : nullptr;
        float2* xout = X ? X + ky * P + kx : nullptr;
        if (self_col) {
            l = eval_bin<M>(a, i, kxv, kyv, Y, false, 1.0f, cx, cy, R2mc2, wl, gw, ds, xout, nullptr);
        } else if (nyq_row) {
            l = eval_bin<M>(a, i, kxv, kyv, Y, false, 1.0f, cx, cy, R2mc2, wl, gw, ds, xout, nullptr);
            l += eval_bin<M>(a, i, -kxv, kyv, Y, true, 1.0f, cx, cy, R2mc2, wl, gw, ds,
                             X ? X + ky * P + (P - kx) : nullptr, nullptr);
        } else {
            float2* xm = X ? X + ((P - ky) % P) * P + (P - kx) : nullptr;
            l = eval_bin<M>(a, i, kxv, kyv, Y, false, 2.0f, cx, cy, R2mc2, wl, gw, ds, xout, xm);
        }
    }
    const float bl = block_sum(l, red);   // ends with the barrier that also orders the LDS atomics
    const int part = i * a.S + blockIdx.x;
    if (tid == 0) a.part_loss[part] = bl;
    float* dst = a.part_gw + static_cast<size_t>(part) * a.n_elem;
    for (int n = tid; n < a.n_elem; n += kBlock) dst[n] = gw[n];
}

// dL_dw[i][n] = sum_s part_gw[i][s][n];  loss = sum over all partial losses (last workgroup).
__global__ __launch_bounds__(256) void loss_finish_kernel(const float* __restrict__ part_loss,
                                                          const float* __restrict__ part_gw, int N, int S,
                                                          int n_elem, float* __restrict__ loss,
                                                          float* __restrict__ dL_dw) {
    __shared__ float red[4];
    if (blockIdx.x == gridDim.x - 1) {
        float s = 0.0f;
        for (int k = threadIdx.x; k < N * S; k += blockDim.x) s += part_loss[k];
        s = block_sum(s, red);
        if (threadIdx.x == 0) *loss = s;
        return;
    }
    if (!dL_dw) return;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * n_elem) return;
    const int i = idx / n_elem, n = idx % n_elem;
    const float* p = part_gw + static_cast<size_t>(i) * S * n_elem + n;
    float s = 0.0f;
    for (int k = 0; k < S; ++k) s += p[static_cast<size_t>(k) * n_elem];
    dL_dw[idx] = s;
}

template <int M>
int launch_loss(const LossArgs& a, int N, hipStream_t stream) {
    dim3 grid(a.S, N);
    loss_grad_kernel<M><<<grid, kBlock, 2 * a.n_elem * sizeof(float), stream>>>(a);
    return launch_status("pact_loss_and_grad");
}

int dispatch_loss(int M, const LossArgs& a, int N, hipStream_t s) {
    switch (M) {
        case 1: return launch_loss<1>(a, N, s);
        case 2: return launch_loss<2>(a, N, s);
        case 3: return launch_loss<3>(a, N, s);
        case 4: return launch_loss<4>(a, N, s);
        case 5: return launch_loss<5>(a, N, s);
        case 6: return launch_loss<6>(a, N, s);
        case 7: return launch_loss<7>(a, N, s);
        case 8: return launch_loss<8>(a, N, s);
        case 9: return launch_loss<9>(a, N, s);
        case 10: return launch_loss<10>(a, N, s);
        case 11: return launch_loss<11>(a, N, s);
        case 12: return launch_loss<12>(a, N, s);
        case 13: return launch_loss<13>(a, N, s);
        case 14: return launch_loss<14>(a, N, s);
        case 15: return launch_loss<15>(a, N, s);
        case 16: return launch_loss<16>(a, N, s);
        default: set_error("pact_loss_and_grad: M = %d exceeds %d", M, kMaxDelays); return PACT_EUNSUPPORTED;
    }
}

int blocks_per_patch(int P) { return ceil_div(static_cast<long long>(P) * (P / 2 + 1), kBlock); }

}  // namespace
}  // namespace pact

extern "C" size_t pact_loss_and_grad_workspace_size(int N, int M, int P, int n_elem) {
    (void)M;
    if (N <= 0 || P <= 0 || n_elem <= 0) return 0;
    const size_t parts = static_cast<size_t>(N) * pact::blocks_per_patch(P);
    return parts * (1 + static_cast<size_t>(n_elem)) * sizeof(float);
}

extern "C" int pact_loss_and_grad(const float* Y_half, const float* w, const float* centres, int N, const pact_ring* ring_,
                                  const float* d, int M, int P, float px, float eps, float* loss, float* dL_dw,
                                  float* X_opt, void* ws, size_t ws_bytes, void* stream) {
    if (!ring_) {
        pact::set_error("pact_loss_and_grad: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_ring ring = *ring_;
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(Y_half && w && centres && d && loss, "pact_loss_and_grad: null pointer");
    PACT_CHECK_ARG(N > 0 && M > 0 && P > 0, "pact_loss_and_grad: N, M and P must be positive");
    PACT_CHECK_ARG(px > 0.0f && std::isfinite(px), "pact_loss_and_grad: px must be positive");
    PACT_CHECK_ARG(eps >= 0.0f && std::isfinite(eps), "pact_loss_and_grad: eps must be >= 0");
    if (int s = check_ring(ring)) return s;
    PACT_CHECK_SUPPORTED(M <= kMaxDelays, "pact_loss_and_grad: M = %d exceeds %d", M, kMaxDelays);
    PACT_CHECK_SUPPORTED(2 * static_cast<size_t>(ring.n_elem) * sizeof(float) <= 64 * 1024,
                         "pact_loss_and_grad: n_elem = %d too large", ring.n_elem);
    const size_t need = pact_loss_and_grad_workspace_size(N, M, P, ring.n_elem);
    if (!ws || ws_bytes < need) {
        set_error("pact_loss_and_grad: workspace of %zu bytes needed, %zu given", need, ws_bytes);
        return PACT_EWORKSPACE;
    }
    LossArgs a;
    a.Yh = reinterpret_cast<const float2*>(Y_half);
    a.w = w;
    a.centres = centres;
    a.d = d;
    a.n_elem = ring.n_elem;
    a.R = ring.radius;
    a.phi0 = ring.phi0;
    a.P = P;
    a.Wh = P / 2 + 1;
    a.S = blocks_per_patch(P);
    a.k0 = static_cast<float>(2.0 * M_PI / (static_cast<double>(P) * px));
    a.eps = eps;
    a.part_loss = static_cast<float*>(ws);
    a.part_gw = a.part_loss + static_cast<size_t>(N) * a.S;
    a.X = reinterpret_cast<float2*>(X_opt);
    if (int s = dispatch_loss(M, a, N, as_stream(stream))) return s;
    const int nb = ceil_div(static_cast<long long>(N) * ring.n_elem, 256) + 1;
    loss_finish_kernel<<<nb, 256, 0, as_stream(stream)>>>(a.part_loss, a.part_gw, N, a.S, ring.n_elem, loss, dL_dw);
    return launch_status("pact_loss_and_grad (finish)");
}
