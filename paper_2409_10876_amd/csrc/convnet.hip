// Learned warm start: the convolutional SOS initialiser's kernels (BF16 operands on MFMA, FP32
// accumulation), its input preparation and loss, and the synthetic channel model of its training scans.
//
// The paper's method needs no training data (Sec. 3.3); this network is an addition that maps the
// delay-and-sum stack (Eq. DAS), averaged down to the SOS node grid, to a starting SOS for the plain
// optimisation of Eq. jr.  Its training scans come from the method's own forward model: arrival times by
// Eq. TOF through the wavefront errors of Eq. wf, then Eq. DAS.
//
// Tensors are NHWC BF16 ([image][row][column][channel], channels contiguous).  A 3 x 3 convolution with
// zero padding 1 is an implicit GEMM: output channels x pixels, reduced over K = (tap, input channel),
// tap-major, K padded with zero weights to a multiple of 32.
//
// MFMA v_mfma_f32_16x16x32_bf16, lane l, r = l % 16, q = l / 16:
//   A (16 x 32):  a[j] = A[r][8q + j]      B (32 x 16):  b[j] = B[8q + j][r]
//   D (16 x 16):  d[i] = D[4q + i][r]
//
// Convolution (and the input gradient, which is the same convolution with the weights transposed in
// channels and flipped in taps): a workgroup of 4 waves loops over output tiles of 8 rows x 16 columns.
// The tile's input halo (10 x 18 pixels, all input channels) sits in LDS with pixels padded by 16 bytes so
// that the 16 lanes of a B fragment read distinct banks; a lane's 8 K values are 8 consecutive channels of
// one tap, one 16-byte read.  Each wave keeps the A fragments of its 16 output channels (all K) in
// registers for the whole launch.
//
// Weight gradient: dW[co][tap][ci] = sum over pixels g[p][co] x[p + tap][ci], a GEMM reduced over pixels.
// Both operands need 8 consecutive pixels of one channel per lane, so the tile (4 rows x 16 columns) is
// transposed into LDS channel-major.  The column shift of a tap is moved onto the output gradient (three
// copies shifted by +1, 0, -1 columns) and the row shift stays on the input (one copy with a halo of one
// row above and below), so that every fragment read is one aligned 16-byte read and every LDS write
// packs two adjacent pixels.  Each workgroup accumulates its share of the pixels in registers and writes
// one partial gradient; two small kernels sum the partials in a fixed order.
#include "common.h"

namespace pact {

int device_cu_count();

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, u32x4{0u, 0u, 0u, 0u}); }

constexpr int kThreads = 256;
constexpr int kTH = 8;                 // output rows of a convolution tile
constexpr int kTW = 16;                // output columns of a tile (one MFMA N tile)
constexpr int kHW = kTW + 2;           // halo columns
constexpr int kWTH = 4;                // output rows of a weight-gradient tile (64 pixels, two K steps)
constexpr int kXB = (kWTH + 2) * kTW + 8;   // one channel of the transposed input tile (16-byte padding)
constexpr int kGL = kWTH * kTW + 8;    // one channel of a transposed output-gradient copy
constexpr int kSlices = 16;

__host__ __device__ constexpr int kpad(int c) { return (9 * c + 31) / 32 * 32; }

bool supported_pair(int ci, int co) {
    return (ci == 16 && co == 64) || (ci == 64 && co == 64) || (ci == 64 && co == 16);
}

template <int CI, int CO>
__global__ __launch_bounds__(kThreads) void conv3x3_kernel(const __bf16* __restrict__ x, int H, int W, int tiles_x,
                                                           int tiles_y, int n_tiles, const __bf16* __restrict__ wpk,
                                                           const float* __restrict__ bias, int relu,
                                                           const __bf16* __restrict__ mask, __bf16* __restrict__ y) {
    constexpr int LDX = CI + 8;            // halo pixel stride (elements)
    constexpr int KP = kpad(CI);
    constexpr int KS = KP / 32;
    constexpr int RT = CO / 16;            // row tiles of the output channels
    constexpr int STEP = 4 / RT;           // waves that share a row tile split the tile's rows
    constexpr int NPW = kTH / STEP;        // output rows per wave
    constexpr int NG = NPW < 4 ? NPW : 4;  // independent accumulators in flight
    __shared__ __attribute__((aligned(16))) __bf16 halo[(kTH + 2) * kHW * LDX];
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const int rt = wv % RT, r0 = wv / RT;
    bf16x8 a[KS];
    int off[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        a[ks] = ld8(wpk + (16 * rt + r) * KP + 32 * ks + 8 * q);
        const int k0 = 32 * ks + 8 * q;
        int tap = k0 / CI, ci0 = k0 - tap * CI;
        if (tap > 8) {                     // K padding: zero weights, any in-bounds read
            tap = 8;
            ci0 = 0;
        }
        off[ks] = ((tap / 3) * kHW + r + tap % 3) * LDX + ci0;
    }
    float bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bv[i] = bias ? bias[16 * rt + 4 * q + i] : 0.0f;
    const int per_img = tiles_x * tiles_y;
    // the halo of the next tile is loaded into registers while this tile is computed (barriers wait on
    // LDS only): chunk c = threadIdx.x + kThreads k of (kTH + 2) x kHW pixels x CI / 8 parts
    constexpr int CH = CI / 8;
    constexpr int NCH = (kTH + 2) * kHW * CH;
    constexpr int NPRE = (NCH + kThreads - 1) / kThreads;
    bf16x8 pre[NPRE];
    auto load_halo = [&](int tile) {
        const int img = tile / per_img, rem = tile - img * per_img;
        const int y0 = (rem / tiles_x) * kTH, x0 = (rem % tiles_x) * kTW;
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {
            const int c = threadIdx.x + kThreads * k;
            const int pix = c / CH, part = c - pix * CH;
            const int hy = pix / kHW, hx = pix - hy * kHW;
            const int gy = y0 - 1 + hy, gx = x0 - 1 + hx;
            pre[k] = zero8();
            if (c < NCH && gy >= 0 && gy < H && gx >= 0 && gx < W)
                pre[k] = ld8(x + ((static_cast<size_t>(img) * H + gy) * W + gx) * CI + 8 * part);
        }
    };
    if (static_cast<int>(blockIdx.x) < n_tiles) load_halo(blockIdx.x);
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int img = tile / per_img, rem = tile - img * per_img;
        const int y0 = (rem / tiles_x) * kTH, x0 = (rem % tiles_x) * kTW;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {
            const int c = threadIdx.x + kThreads * k;
            if (c < NCH) {
                const int pix = c / CH, part = c - pix * CH;
                *reinterpret_cast<bf16x8*>(halo + pix * LDX + 8 * part) = pre[k];
            }
        }
        __syncthreads();
        if (tile + static_cast<int>(gridDim.x) < n_tiles) load_halo(tile + gridDim.x);
#pragma unroll
        for (int g0 = 0; g0 < NPW; g0 += NG) {
            f32x4 acc[NG];
#pragma unroll
            for (int j = 0; j < NG; ++j) acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int j = 0; j < NG; ++j) {
                    const int tr = r0 + (g0 + j) * STEP;
                    acc[j] = mfma(a[ks], ld8(halo + tr * kHW * LDX + off[ks]), acc[j]);
                }
#pragma unroll
            for (int j = 0; j < NG; ++j) {
                const int gy = y0 + r0 + (g0 + j) * STEP, gx = x0 + r;
                if (gy >= H || gx >= W) continue;
                const size_t o = ((static_cast<size_t>(img) * H + gy) * W + gx) * CO + 16 * rt + 4 * q;
                bf16x4 mk;
                if (mask) mk = *reinterpret_cast<const bf16x4*>(mask + o);
                bf16x4 out;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float v = acc[j][i] + bv[i];
                    if (relu) v = fmaxf(v, 0.0f);
                    if (mask && !(static_cast<float>(mk[i]) > 0.0f)) v = 0.0f;
                    out[i] = static_cast<__bf16>(v);
                }
                *reinterpret_cast<bf16x4*>(y + o) = out;
            }
        }
    }
}

// Weight gradient: dW[co][ky][kx][ci] = sum over pixels p of g[p][co] x[p + (ky - 1, kx - 1)][ci].  The tap's
// column shift is put on the operand with fewer channels.  For CI >= CO (conv3x3_wgrad_kernel), with
// p' = p + (0, kx - 1) the sum becomes
//   dW[co][ky][kx][ci] = sum_p' g[p'_y][p'_x + 1 - kx][co] x[p'_y + ky - 1][p'_x][ci],
// so the input needs only row shifts (one transposed copy, rows y0 - 1 .. y0 + 4 of the tile's 16 columns)
// and the output gradient the column shifts (three transposed copies, one per kx).  For CI < CO
// (conv3x3_wgrad_sx_kernel) the input is held in three copies, copy kx holding column j of the tile at
// x0 + j + kx - 1, and the output gradient in one.  Every copy is filled from pairs of adjacent pixels with
// 4-byte LDS writes.
// Threads of a weight-gradient workgroup: 8 waves when there are 16 (output, input) channel-tile pairs, so
// that each wave holds the accumulators of two pairs (4 would take the registers of two waves per SIMD).
template <int CI, int CO>
constexpr int wgrad_threads() { return (CI / 16) * (CO / 16) >= 16 ? 512 : 256; }

template <int CI, int CO>
constexpr bool wgrad_shift_x() { return CI < CO; }

template <int CI, int CO>
__global__ __launch_bounds__((wgrad_threads<CI, CO>())) void conv3x3_wgrad_kernel(const __bf16* __restrict__ x,
                                                                 const __bf16* __restrict__ g, int H, int W,
                                                                 int tiles_x, int tiles_y, int n_tiles,
                                                                 float* __restrict__ partial) {
    extern __shared__ __attribute__((aligned(16))) unsigned char cv_dyn[];
    __bf16* xT = reinterpret_cast<__bf16*>(cv_dyn);      // [CI][kXB]: rows y0 - 1 .. y0 + 4, 16 columns
    __bf16* gT = xT + CI * kXB;                           // [3 (kx)][CO][kGL]: column j holds g at x0 + j + 1 - kx
    constexpr int NT = wgrad_threads<CI, CO>(), CT = CI / 16, OT = CO / 16, PAIRS = CT * OT / (NT / 64);
    constexpr int CHI = CI / 8, CHO = CO / 8;
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    f32x4 acc[PAIRS][9];
#pragma unroll
    for (int p = 0; p < PAIRS; ++p)
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[p][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float db[8] = {};
    const int per_img = tiles_x * tiles_y;
    // the next tile is loaded into registers while this one is computed.  Input item i = threadIdx.x +
    // NT k: halo row, column pair, channel part (pixels x0 + 2 jp, + 1); output-gradient item: tile row,
    // column pair, channel part (pixels x0 + 2 jp - 1 .. x0 + 2 jp + 2)
    constexpr int NXI = (kWTH + 2) * (kTW / 2) * CHI, NXP = (NXI + NT - 1) / NT;
    constexpr int NGI = kWTH * (kTW / 2) * CHO, NGP = (NGI + NT - 1) / NT;
    bf16x8 px[NXP][2], pg[NGP][4];
    auto load_tile = [&](int tile) {
        const int img = tile / per_img, rem = tile - img * per_img;
        const int y0 = (rem / tiles_x) * kWTH, x0 = (rem % tiles_x) * kTW;
#pragma unroll
        for (int k = 0; k < NXP; ++k) {
            const int it = threadIdx.x + NT * k;
            const int part = it % CHI, pr = it / CHI, jp = pr % (kTW / 2), hy = pr / (kTW / 2);
            const int gy = y0 - 1 + hy;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int gx = x0 + 2 * jp + u;
                px[k][u] = zero8();
                if (it < NXI && gy >= 0 && gy < H && gx < W)
                    px[k][u] = ld8(x + ((static_cast<size_t>(img) * H + gy) * W + gx) * CI + 8 * part);
            }
        }
#pragma unroll
        for (int k = 0; k < NGP; ++k) {
            const int it = threadIdx.x + NT * k;
            const int part = it % CHO, pr = it / CHO, jp = pr % (kTW / 2), row = pr / (kTW / 2);
            const int gy = y0 + row;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int gx = x0 + 2 * jp - 1 + u;
                pg[k][u] = zero8();
                if (it < NGI && gy < H && gx >= 0 && gx < W)
                    pg[k][u] = ld8(g + ((static_cast<size_t>(img) * H + gy) * W + gx) * CO + 8 * part);
            }
        }
    };
    auto pair = [](__bf16 lo, __bf16 hi) {
        return static_cast<unsigned>(__builtin_bit_cast(unsigned short, lo)) |
               (static_cast<unsigned>(__builtin_bit_cast(unsigned short, hi)) << 16);
    };
    if (static_cast<int>(blockIdx.x) < n_tiles) load_tile(blockIdx.x);
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NXP; ++k) {
            const int it = threadIdx.x + NT * k;
            if (it >= NXI) continue;
            const int part = it % CHI, pr = it / CHI, jp = pr % (kTW / 2), hy = pr / (kTW / 2);
#pragma unroll
            for (int e = 0; e < 8; ++e)
                *reinterpret_cast<unsigned*>(xT + (8 * part + e) * kXB + hy * kTW + 2 * jp) = pair(px[k][0][e], px[k][1][e]);
        }
#pragma unroll
        for (int k = 0; k < NGP; ++k) {
            const int it = threadIdx.x + NT * k;
            if (it >= NGI) continue;
            const int part = it % CHO, pr = it / CHO, jp = pr % (kTW / 2), row = pr / (kTW / 2);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int o = (8 * part + e) * kGL + row * kTW + 2 * jp;
                *reinterpret_cast<unsigned*>(gT + o) = pair(pg[k][2][e], pg[k][3][e]);                   // kx = 0
                *reinterpret_cast<unsigned*>(gT + CO * kGL + o) = pair(pg[k][1][e], pg[k][2][e]);        // kx = 1
                *reinterpret_cast<unsigned*>(gT + 2 * CO * kGL + o) = pair(pg[k][0][e], pg[k][1][e]);    // kx = 2
                db[e] += static_cast<float>(pg[k][1][e]) + static_cast<float>(pg[k][2][e]);
            }
        }
        __syncthreads();
        if (tile + static_cast<int>(gridDim.x) < n_tiles) load_tile(tile + gridDim.x);
        // K step ks: pixels 32 ks .. 32 ks + 31 of the tile = rows 2 ks, 2 ks + 1; lane q takes row
        // 2 ks + q / 2, columns 8 (q % 2) .. + 7
#pragma unroll
        for (int ks = 0; ks < kWTH / 2; ++ks) {
            const int row = 2 * ks + (q >> 1), col = 8 * (q & 1);
#pragma unroll
            for (int p = 0; p < PAIRS; ++p) {
                const int idx = wv * PAIRS + p, ot = idx / CT, ct = idx - ot * CT;
                bf16x8 av[3], bv[3];
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) av[kx] = ld8(gT + (kx * CO + 16 * ot + r) * kGL + 32 * ks + 8 * q);
#pragma unroll
                for (int ky = 0; ky < 3; ++ky) bv[ky] = ld8(xT + (16 * ct + r) * kXB + (row + ky) * kTW + col);
#pragma unroll
                for (int t = 0; t < 9; ++t) acc[p][t] = mfma(av[t % 3], bv[t / 3], acc[p][t]);
            }
        }
    }
    float* out = partial + static_cast<size_t>(blockIdx.x) * (CO * 9 * CI + CO);
#pragma unroll
    for (int p = 0; p < PAIRS; ++p) {
        const int idx = wv * PAIRS + p, ot = idx / CT, ct = idx - ot * CT;
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) out[((16 * ot + 4 * q + i) * 9 + t) * CI + 16 * ct + r] = acc[p][t][i];
    }
    // bias gradient: thread t always loaded channel part t % CHO
    __syncthreads();
    float* red = reinterpret_cast<float*>(cv_dyn);
#pragma unroll
    for (int e = 0; e < 8; ++e) red[threadIdx.x * 8 + e] = db[e];
    __syncthreads();
    if (threadIdx.x < CO) {
        const int part = threadIdx.x / 8, e = threadIdx.x % 8;
        float s = 0.0f;
        for (int t = part; t < NT; t += CHO) s += red[t * 8 + e];
        out[CO * 9 * CI + threadIdx.x] = s;
    }
}

// The same weight gradient with the column shift on the input (used for CI < CO).
template <int CI, int CO>
__global__ __launch_bounds__((wgrad_threads<CI, CO>())) void conv3x3_wgrad_sx_kernel(const __bf16* __restrict__ x,
                                                                 const __bf16* __restrict__ g, int H, int W,
                                                                 int tiles_x, int tiles_y, int n_tiles,
                                                                 float* __restrict__ partial) {
    extern __shared__ __attribute__((aligned(16))) unsigned char cv_dyn[];
    __bf16* xT = reinterpret_cast<__bf16*>(cv_dyn);      // [3 (kx)][CI][kXB]: rows y0 - 1 .. y0 + 4; column j
                                                          // holds x at x0 + j + kx - 1
    __bf16* gT = xT + 3 * CI * kXB;                       // [CO][kGL]: rows y0 .. y0 + 3, 16 columns
    constexpr int NT = wgrad_threads<CI, CO>(), CT = CI / 16, OT = CO / 16, PAIRS = CT * OT / (NT / 64);
    constexpr int CHI = CI / 8, CHO = CO / 8;
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    f32x4 acc[PAIRS][9];
#pragma unroll
    for (int p = 0; p < PAIRS; ++p)
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[p][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float db[8] = {};
    const int per_img = tiles_x * tiles_y;
    // The next tile is loaded into registers while this one is computed.  Input item i = threadIdx.x +
    // NT k: halo row, column pair jp, channel part (pixels x0 + 2 jp - 1 .. x0 + 2 jp + 2); output-gradient
    // item: tile row, column pair, channel part (pixels x0 + 2 jp, + 1).
    constexpr int XP = 4, GP = 2, XO = 1, GO = 0;
    constexpr int NXI = (kWTH + 2) * (kTW / 2) * CHI, NXP = (NXI + NT - 1) / NT;
    constexpr int NGI = kWTH * (kTW / 2) * CHO, NGP = (NGI + NT - 1) / NT;
    bf16x8 px[NXP][XP], pg[NGP][GP];
    auto load_tile = [&](int tile) {
        const int img = tile / per_img, rem = tile - img * per_img;
        const int y0 = (rem / tiles_x) * kWTH, x0 = (rem % tiles_x) * kTW;
#pragma unroll
        for (int k = 0; k < NXP; ++k) {
            const int it = threadIdx.x + NT * k;
            const int part = it % CHI, pr = it / CHI, jp = pr % (kTW / 2), hy = pr / (kTW / 2);
            const int gy = y0 - 1 + hy;
#pragma unroll
            for (int u = 0; u < XP; ++u) {
                const int gx = x0 + 2 * jp - XO + u;
                px[k][u] = zero8();
                if (it < NXI && gy >= 0 && gy < H && gx >= 0 && gx < W)
                    px[k][u] = ld8(x + ((static_cast<size_t>(img) * H + gy) * W + gx) * CI + 8 * part);
            }
        }
#pragma unroll
        for (int k = 0; k < NGP; ++k) {
            const int it = threadIdx.x + NT * k;
            const int part = it % CHO, pr = it / CHO, jp = pr % (kTW / 2), row = pr / (kTW / 2);
            const int gy = y0 + row;
#pragma unroll
            for (int u = 0; u < GP; ++u) {
                const int gx = x0 + 2 * jp - GO + u;
                pg[k][u] = zero8();
                if (it < NGI && gy < H && gx >= 0 && gx < W)
                    pg[k][u] = ld8(g + ((static_cast<size_t>(img) * H + gy) * W + gx) * CO + 8 * part);
            }
        }
    };
    auto pair = [](__bf16 lo, __bf16 hi) {
        return static_cast<unsigned>(__builtin_bit_cast(unsigned short, lo)) |
               (static_cast<unsigned>(__builtin_bit_cast(unsigned short, hi)) << 16);
    };
    if (static_cast<int>(blockIdx.x) < n_tiles) load_tile(blockIdx.x);
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NXP; ++k) {
            const int it = threadIdx.x + NT * k;
            if (it >= NXI) continue;
            const int part = it % CHI, pr = it / CHI, jp = pr % (kTW / 2), hy = pr / (kTW / 2);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int o = (8 * part + e) * kXB + hy * kTW + 2 * jp;
#pragma unroll
                for (int kx = 0; kx < 3; ++kx)
                    *reinterpret_cast<unsigned*>(xT + kx * CI * kXB + o) = pair(px[k][kx][e], px[k][kx + 1][e]);
            }
        }
#pragma unroll
        for (int k = 0; k < NGP; ++k) {
            const int it = threadIdx.x + NT * k;
            if (it >= NGI) continue;
            const int part = it % CHO, pr = it / CHO, jp = pr % (kTW / 2), row = pr / (kTW / 2);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                *reinterpret_cast<unsigned*>(gT + (8 * part + e) * kGL + row * kTW + 2 * jp) = pair(pg[k][0][e], pg[k][1][e]);
                db[e] += static_cast<float>(pg[k][0][e]) + static_cast<float>(pg[k][1][e]);
            }
        }
        __syncthreads();
        if (tile + static_cast<int>(gridDim.x) < n_tiles) load_tile(tile + gridDim.x);
        // K step ks: pixels 32 ks .. 32 ks + 31 of the tile = rows 2 ks, 2 ks + 1; lane q takes row
        // 2 ks + q / 2, columns 8 (q % 2) .. + 7
#pragma unroll
        for (int ks = 0; ks < kWTH / 2; ++ks) {
            const int row = 2 * ks + (q >> 1), col = 8 * (q & 1);
#pragma unroll
            for (int p = 0; p < PAIRS; ++p) {
                const int idx = wv * PAIRS + p, ot = idx / CT, ct = idx - ot * CT;
                const bf16x8 av = ld8(gT + (16 * ot + r) * kGL + 32 * ks + 8 * q);
                bf16x8 bv[9];
#pragma unroll
                for (int t = 0; t < 9; ++t)
                    bv[t] = ld8(xT + ((t % 3) * CI + 16 * ct + r) * kXB + (row + t / 3) * kTW + col);
#pragma unroll
                for (int t = 0; t < 9; ++t) acc[p][t] = mfma(av, bv[t], acc[p][t]);
            }
        }
    }
    float* out = partial + static_cast<size_t>(blockIdx.x) * (CO * 9 * CI + CO);
#pragma unroll
    for (int p = 0; p < PAIRS; ++p) {
        const int idx = wv * PAIRS + p, ot = idx / CT, ct = idx - ot * CT;
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) out[((16 * ot + 4 * q + i) * 9 + t) * CI + 16 * ct + r] = acc[p][t][i];
    }
    // bias gradient: thread t always loaded channel part t % CHO
    __syncthreads();
    float* red = reinterpret_cast<float*>(cv_dyn);
#pragma unroll
    for (int e = 0; e < 8; ++e) red[threadIdx.x * 8 + e] = db[e];
    __syncthreads();
    if (threadIdx.x < CO) {
        const int part = threadIdx.x / 8, e = threadIdx.x % 8;
        float s = 0.0f;
        for (int t = part; t < NT; t += CHO) s += red[t * 8 + e];
        out[CO * 9 * CI + threadIdx.x] = s;
    }
}

template <int CI, int CO>
constexpr size_t wgrad_lds() {
    constexpr bool SX = wgrad_shift_x<CI, CO>();
    const size_t b = static_cast<size_t>((SX ? 3 : 1) * CI * kXB + (SX ? 1 : 3) * CO * kGL) * sizeof(__bf16);
    const size_t r = static_cast<size_t>(wgrad_threads<CI, CO>()) * 8 * sizeof(float);
    return b > r ? b : r;
}

// out[j] = sum over partials b of partial[b][j], fixed order: kSlices runs, then the runs.
__global__ __launch_bounds__(256) void sum_partials1_kernel(const float* __restrict__ partial, int n_part, int n,
                                                            float* __restrict__ part2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int per = (n_part + kSlices - 1) / kSlices;
    const int b0 = blockIdx.y * per, b1 = min(b0 + per, n_part);
    float s = 0.0f;
    for (int b = b0; b < b1; ++b) s += partial[static_cast<size_t>(b) * n + j];
    part2[static_cast<size_t>(blockIdx.y) * n + j] = s;
}

__global__ __launch_bounds__(256) void sum_partials2_kernel(const float* __restrict__ part2, int n,
                                                            float* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kSlices; ++k) s += part2[static_cast<size_t>(k) * n + j];
    out[j] = s;
}

__device__ __forceinline__ unsigned short bf16_bits(float x) {
    const unsigned u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<unsigned short>((u >> 16) | 0x40u);
    return static_cast<unsigned short>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// W [CO][9][CI] FP32 -> fwd [CO][kpad(CI)] (k = tap CI + ci) and adj [CI][kpad(CO)] (k = tap' CO + co,
// value W[co][8 - tap'][ci]), BF16, zero in the K padding.
__global__ __launch_bounds__(256) void conv_pack_kernel(const float* __restrict__ Wt, int CI, int CO,
                                                        unsigned short* __restrict__ fwd,
                                                        unsigned short* __restrict__ adj) {
    const int kf = kpad(CI), ka = kpad(CO);
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = CO * kf;
    if (j < nf) {
        const int co = j / kf, k = j - co * kf;
        fwd[j] = k < 9 * CI ? bf16_bits(Wt[(co * 9 + k / CI) * CI + k % CI]) : 0;
    } else if (adj && j < nf + CI * ka) {
        const int jj = j - nf, ci = jj / ka, k = jj - ci * ka;
        adj[jj] = k < 9 * CO ? bf16_bits(Wt[(k % CO * 9 + 8 - k / CO) * CI + ci]) : 0;
    }
}

// ---- resampling between resolutions (8 channels per thread) ----

__global__ __launch_bounds__(256) void pool2_kernel(const __bf16* __restrict__ x, int n, int H, int W, int C,
                                                    __bf16* __restrict__ y) {
    const int h = H / 2, w = W / 2, ch = C / 8;
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<long long>(n) * h * w * ch) return;
    const int part = static_cast<int>(idx % ch);
    const long long pix = idx / ch;
    const int xx = static_cast<int>(pix % w), yy = static_cast<int>((pix / w) % h), img = static_cast<int>(pix / (static_cast<long long>(w) * h));
    float s[8] = {};
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            const bf16x8 v = ld8(x + ((static_cast<size_t>(img) * H + 2 * yy + dy) * W + 2 * xx + dx) * C + 8 * part);
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] += static_cast<float>(v[e]);
        }
    bf16x8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = static_cast<__bf16>(0.25f * s[e]);
    *reinterpret_cast<bf16x8*>(y + idx * 8) = o;
}

// y (H x W) = up2(x (H/2 x W/2)) + skip
__global__ __launch_bounds__(256) void up2_add_kernel(const __bf16* __restrict__ x, const __bf16* __restrict__ skip,
                                                      int n, int H, int W, int C, __bf16* __restrict__ y) {
    const int ch = C / 8;
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<long long>(n) * H * W * ch) return;
    const int part = static_cast<int>(idx % ch);
    const long long pix = idx / ch;
    const int xx = static_cast<int>(pix % W), yy = static_cast<int>((pix / W) % H), img = static_cast<int>(pix / (static_cast<long long>(W) * H));
    const bf16x8 lo = ld8(x + ((static_cast<size_t>(img) * (H / 2) + yy / 2) * (W / 2) + xx / 2) * C + 8 * part);
    const bf16x8 sk = ld8(skip + idx * 8);
    bf16x8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = static_cast<__bf16>(static_cast<float>(lo[e]) + static_cast<float>(sk[e]));
    *reinterpret_cast<bf16x8*>(y + idx * 8) = o;
}

// g_low (H/2 x W/2) = (2 x 2 sum of g_high) [mask_low > 0]
__global__ __launch_bounds__(256) void up2_add_adjoint_kernel(const __bf16* __restrict__ gh,
                                                              const __bf16* __restrict__ mask, int n, int H, int W,
                                                              int C, __bf16* __restrict__ gl) {
    const int h = H / 2, w = W / 2, ch = C / 8;
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<long long>(n) * h * w * ch) return;
    const int part = static_cast<int>(idx % ch);
    const long long pix = idx / ch;
    const int xx = static_cast<int>(pix % w), yy = static_cast<int>((pix / w) % h), img = static_cast<int>(pix / (static_cast<long long>(w) * h));
    float s[8] = {};
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            const bf16x8 v = ld8(gh + ((static_cast<size_t>(img) * H + 2 * yy + dy) * W + 2 * xx + dx) * C + 8 * part);
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] += static_cast<float>(v[e]);
        }
    bf16x8 mk;
    if (mask) mk = ld8(mask + idx * 8);
    bf16x8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = static_cast<__bf16>(mask && !(static_cast<float>(mk[e]) > 0.0f) ? 0.0f : s[e]);
    *reinterpret_cast<bf16x8*>(gl + idx * 8) = o;
}

// g_high (H x W) = (g_low / 4 at the parent pixel + skip) [mask > 0]
__global__ __launch_bounds__(256) void pool2_adjoint_kernel(const __bf16* __restrict__ glo,
                                                            const __bf16* __restrict__ skip,
                                                            const __bf16* __restrict__ mask, int n, int H, int W,
                                                            int C, __bf16* __restrict__ gh) {
    const int ch = C / 8;
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<long long>(n) * H * W * ch) return;
    const int part = static_cast<int>(idx % ch);
    const long long pix = idx / ch;
    const int xx = static_cast<int>(pix % W), yy = static_cast<int>((pix / W) % H), img = static_cast<int>(pix / (static_cast<long long>(W) * H));
    const bf16x8 lo = ld8(glo + ((static_cast<size_t>(img) * (H / 2) + yy / 2) * (W / 2) + xx / 2) * C + 8 * part);
    bf16x8 sk = zero8(), mk;
    if (skip) sk = ld8(skip + idx * 8);
    if (mask) mk = ld8(mask + idx * 8);
    bf16x8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float v = 0.25f * static_cast<float>(lo[e]) + static_cast<float>(sk[e]);
        o[e] = static_cast<__bf16>(mask && !(static_cast<float>(mk[e]) > 0.0f) ? 0.0f : v);
    }
    *reinterpret_cast<bf16x8*>(gh + idx * 8) = o;
}

// ---- input, output, loss ----

// x[r][c][m] = scale * mean of stack[m] over the f x f block (r, c); zero for m >= M
__global__ __launch_bounds__(256) void warm_input_kernel(const float* __restrict__ stack, int M, int H, int W, int f,
                                                         float scale, int C, __bf16* __restrict__ x) {
    const int h = H / f, w = W / f;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= h * w) return;
    const int rr = idx / w, cc = idx - rr * w;
    const float inv = scale / static_cast<float>(f * f);
    for (int m = 0; m < C; ++m) {
        float s = 0.0f;
        if (m < M)
            for (int dy = 0; dy < f; ++dy)
                for (int dx = 0; dx < f; ++dx) s += stack[(static_cast<size_t>(m) * H + rr * f + dy) * W + cc * f + dx];
        x[static_cast<size_t>(idx) * C + m] = static_cast<__bf16>(s * inv);
    }
}

// g = d loss / d z (channel 0 only) and per-block partial sums of the masked squared error
__global__ __launch_bounds__(256) void warm_loss_kernel(const __bf16* __restrict__ z, int n, int HW, int C,
                                                        const float* __restrict__ t,
                                                        const unsigned char* __restrict__ mask, float norm,
                                                        __bf16* __restrict__ g, float* __restrict__ partial) {
    __shared__ float red[kThreads / 64];
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    float e = 0.0f;
    if (idx < n * HW) {
        const int node = idx % HW;
        const float d = static_cast<float>(z[static_cast<size_t>(idx) * C]) - t[idx];
        const bool free_node = mask[node] != 0;
        e = free_node ? d * d : 0.0f;
        __bf16* gp = g + static_cast<size_t>(idx) * C;
        gp[0] = static_cast<__bf16>(free_node ? 2.0f * norm * d : 0.0f);
        for (int c = 1; c < C; ++c) gp[c] = static_cast<__bf16>(0.0f);
    }
    const float s = block_sum(e, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void warm_loss_finish_kernel(const float* __restrict__ partial, int n_part,
                                                               float norm, float* __restrict__ loss) {
    __shared__ float red[kThreads / 64];
    float s = 0.0f;
    for (int b = threadIdx.x; b < n_part; b += blockDim.x) s += partial[b];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *loss = norm * s;
}

__global__ __launch_bounds__(256) void warm_sos_kernel(const __bf16* __restrict__ z, int n, int HW, int C,
                                                       const unsigned char* __restrict__ mask, float v0, float s,
                                                       float* __restrict__ sos) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * HW) return;
    sos[idx] = mask[idx % HW] ? v0 + s * static_cast<float>(z[static_cast<size_t>(idx) * C]) : v0;
}

// ---- synthetic channel data of the training scans ----

// S[n][t] = sum_b A_b (1 - u^2) exp(-u^2 / 2) over |u| <= 8, u = (t0 + t / fs - T_bn) v0 / sigma_b,
// T_bn = (|r_n - c_b| - w[b][n]) / v0.  Block: one element, 256 samples; sources staged in LDS.
__global__ __launch_bounds__(256) void ricker_kernel(const float* __restrict__ w, const float* __restrict__ src,
                                                     const float* __restrict__ amp,
                                                     const float* __restrict__ sigma, int n_src, int n_elem,
                                                     float R, float phi0, float v0, int n_t, float fs, float t0,
                                                     float* __restrict__ S) {
    __shared__ float sT[256], sA[256], sK[256];
    const int n = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    float sn, cs;
    sincosf(phi0 + kTwoPi * (static_cast<float>(n) / n_elem), &sn, &cs);
    const float ex = R * cs, ey = R * sn;
    const float time = t0 + static_cast<float>(t) / fs;
    float acc = 0.0f;
    for (int b0 = 0; b0 < n_src; b0 += 256) {
        __syncthreads();
        const int b = b0 + threadIdx.x;
        if (b < n_src) {
            const float dx = ex - src[2 * b], dy = ey - src[2 * b + 1];
            sT[threadIdx.x] = (sqrtf(fmaf(dx, dx, dy * dy)) - w[static_cast<size_t>(b) * n_elem + n]) / v0;
            sA[threadIdx.x] = amp[b];
            sK[threadIdx.x] = v0 / sigma[b];
        }
        __syncthreads();
        const int nb = min(256, n_src - b0);
        for (int j = 0; j < nb; ++j) {
            const float u = (time - sT[j]) * sK[j];
            if (fabsf(u) <= 8.0f) {
                const float u2 = u * u;
                acc = fmaf(sA[j] * (1.0f - u2), expf(-0.5f * u2), acc);
            }
        }
    }
    if (t < n_t) S[static_cast<size_t>(n) * n_t + t] = acc;
}

// ---- host side ----

template <int CI, int CO>
int launch_conv(const __bf16* x, int n, int H, int W, const __bf16* wpk, const float* bias, int relu,
                const __bf16* mask, __bf16* y, hipStream_t st) {
    const int tx = ceil_div(W, kTW), ty = ceil_div(H, kTH);
    const long long tiles = static_cast<long long>(n) * tx * ty;
    PACT_CHECK_SUPPORTED(tiles < (1LL << 31), "pact_conv3x3_bf16: too many tiles");
    const int blocks = static_cast<int>(std::min<long long>(tiles, 8LL * device_cu_count()));
    conv3x3_kernel<CI, CO><<<blocks, kThreads, 0, st>>>(x, H, W, tx, ty, static_cast<int>(tiles), wpk, bias, relu,
                                                        mask, y);
    return launch_status("pact_conv3x3_bf16");
}

int wgrad_blocks(long long tiles) { return static_cast<int>(std::min<long long>(tiles, device_cu_count())); }

template <int CI, int CO>
int launch_wgrad(const __bf16* x, const __bf16* g, int n, int H, int W, float* grad, float* ws, hipStream_t st) {
    const int tx = ceil_div(W, kTW), ty = ceil_div(H, kWTH);
    const long long tiles = static_cast<long long>(n) * tx * ty;
    const int blocks = wgrad_blocks(tiles);
    const int nout = CO * 9 * CI + CO;
    static bool attr = false;
    const size_t lds = wgrad_lds<CI, CO>();
    auto kern = [] {
        if constexpr (wgrad_shift_x<CI, CO>()) return conv3x3_wgrad_sx_kernel<CI, CO>;
        else return conv3x3_wgrad_kernel<CI, CO>;
    }();
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  static_cast<int>(lds));
        attr = true;
    }
    kern<<<blocks, wgrad_threads<CI, CO>(), lds, st>>>(x, g, H, W, tx, ty, static_cast<int>(tiles), ws);
    if (int s = launch_status("pact_conv3x3_wgrad_bf16")) return s;
    float* part2 = ws + static_cast<size_t>(blocks) * nout;
    sum_partials1_kernel<<<dim3(ceil_div(nout, 256), kSlices), 256, 0, st>>>(ws, blocks, nout, part2);
    if (int s = launch_status("pact_conv3x3_wgrad_bf16")) return s;
    sum_partials2_kernel<<<ceil_div(nout, 256), 256, 0, st>>>(part2, nout, grad);
    return launch_status("pact_conv3x3_wgrad_bf16");
}

int check_conv_shape(int n, int H, int W, int ci, int co, const char* what) {
    PACT_CHECK_ARG(n > 0 && H > 0 && W > 0, "%s: n, H and W must be positive", what);
    PACT_CHECK_SUPPORTED(supported_pair(ci, co), "%s: channel counts (%d, %d) are not built ((16, 64), (64, 64), (64, 16))", what,
                         ci, co);
    PACT_CHECK_SUPPORTED(static_cast<long long>(n) * H * W * std::max(ci, co) < (1LL << 40), "%s: tensor too large",
                         what);
    return PACT_OK;
}

long long elementwise_count(long long pixels, int C) { return pixels * (C / 8); }

}  // namespace
}  // namespace pact

extern "C" size_t pact_conv3x3_packed_count(int ci, int co) {
    if (ci <= 0 || co <= 0) return 0;
    return static_cast<size_t>(co) * pact::kpad(ci);
}

extern "C" int pact_conv3x3_pack(const float* weights, int ci, int co, void* packed, void* packed_adjoint,
                                 void* stream) {
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(weights && packed, "pact_conv3x3_pack: null pointer");
    PACT_CHECK_SUPPORTED(supported_pair(ci, co), "pact_conv3x3_pack: channel counts (%d, %d) are not built", ci, co);
    const int total = co * kpad(ci) + ci * kpad(co);
    conv_pack_kernel<<<ceil_div(total, 256), 256, 0, as_stream(stream)>>>(
        weights, ci, co, static_cast<unsigned short*>(packed), static_cast<unsigned short*>(packed_adjoint));
    return launch_status("pact_conv3x3_pack");
}

extern "C" int pact_conv3x3_bf16(const void* x, int n, int H, int W, int ci, const void* packed, const float* bias,
                                 int co, int relu, const void* mask, void* y, void* stream) {
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(x && packed && y, "pact_conv3x3_bf16: null pointer");
    if (int s = check_conv_shape(n, H, W, ci, co, "pact_conv3x3_bf16")) return s;
    const __bf16* xp = static_cast<const __bf16*>(x);
    const __bf16* wp = static_cast<const __bf16*>(packed);
    const __bf16* mp = static_cast<const __bf16*>(mask);
    __bf16* yp = static_cast<__bf16*>(y);
    hipStream_t st = as_stream(stream);
    if (ci == 16 && co == 64) return launch_conv<16, 64>(xp, n, H, W, wp, bias, relu, mp, yp, st);
    if (ci == 64 && co == 64) return launch_conv<64, 64>(xp, n, H, W, wp, bias, relu, mp, yp, st);
    return launch_conv<64, 16>(xp, n, H, W, wp, bias, relu, mp, yp, st);
}

extern "C" size_t pact_conv3x3_wgrad_workspace_size(int n, int H, int W, int ci, int co) {
    using namespace pact;
    if (n <= 0 || H <= 0 || W <= 0 || !supported_pair(ci, co)) return 0;
    const long long tiles = static_cast<long long>(n) * ceil_div(W, kTW) * ceil_div(H, kWTH);
    return static_cast<size_t>(wgrad_blocks(tiles) + kSlices) * (co * 9 * ci + co) * sizeof(float);
}

extern "C" int pact_conv3x3_wgrad_bf16(const void* x, const void* g, int n, int H, int W, int ci, int co,
                                       float* grad, void* ws, size_t ws_bytes, void* stream) {
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(x && g && grad, "pact_conv3x3_wgrad_bf16: null pointer");
    if (int s = check_conv_shape(n, H, W, ci, co, "pact_conv3x3_wgrad_bf16")) return s;
    const size_t need = pact_conv3x3_wgrad_workspace_size(n, H, W, ci, co);
    if (!ws || ws_bytes < need) {
        set_error("pact_conv3x3_wgrad_bf16: workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : 0);
        return PACT_EWORKSPACE;
    }
    const __bf16* xp = static_cast<const __bf16*>(x);
    const __bf16* gp = static_cast<const __bf16*>(g);
    float* wsp = static_cast<float*>(ws);
    hipStream_t st = as_stream(stream);
    if (ci == 16 && co == 64) return launch_wgrad<16, 64>(xp, gp, n, H, W, grad, wsp, st);
    if (ci == 64 && co == 64) return launch_wgrad<64, 64>(xp, gp, n, H, W, grad, wsp, st);
    return launch_wgrad<64, 16>(xp, gp, n, H, W, grad, wsp, st);
}

namespace {
int check_resample(const void* a, const void* b, int n, int H, int W, int C, const char* what) {
    PACT_CHECK_ARG(a && b, "%s: null pointer", what);
    PACT_CHECK_ARG(n > 0 && H > 0 && W > 0 && H % 2 == 0 && W % 2 == 0, "%s: n > 0 and even H, W required", what);
    PACT_CHECK_ARG(C > 0 && C % 8 == 0, "%s: the channel count must be a multiple of 8", what);
    return PACT_OK;
}
}  // namespace

extern "C" int pact_pool2_bf16(const void* x, int n, int H, int W, int C, void* y, void* stream) {
    using namespace pact;
    clear_error();
    if (int s = check_resample(x, y, n, H, W, C, "pact_pool2_bf16")) return s;
    const long long cnt = elementwise_count(static_cast<long long>(n) * (H / 2) * (W / 2), C);
    pool2_kernel<<<ceil_div(cnt, 256), 256, 0, as_stream(stream)>>>(static_cast<const __bf16*>(x), n, H, W, C,
                                                                   static_cast<__bf16*>(y));
    return launch_status("pact_pool2_bf16");
}

extern "C" int pact_up2_add_bf16(const void* x, const void* skip, int n, int H, int W, int C, void* y,
                                 void* stream) {
    using namespace pact;
    clear_error();
    if (int s = check_resample(x, y, n, H, W, C, "pact_up2_add_bf16")) return s;
    PACT_CHECK_ARG(skip, "pact_up2_add_bf16: null skip");
    const long long cnt = elementwise_count(static_cast<long long>(n) * H * W, C);
    up2_add_kernel<<<ceil_div(cnt, 256), 256, 0, as_stream(stream)>>>(
        static_cast<const __bf16*>(x), static_cast<const __bf16*>(skip), n, H, W, C, static_cast<__bf16*>(y));
    return launch_status("pact_up2_add_bf16");
}

extern "C" int pact_up2_add_adjoint_bf16(const void* g_high, const void* mask_low, int n, int H, int W, int C,
                                         void* g_low, void* stream) {
    using namespace pact;
    clear_error();
    if (int s = check_resample(g_high, g_low, n, H, W, C, "pact_up2_add_adjoint_bf16")) return s;
    const long long cnt = elementwise_count(static_cast<long long>(n) * (H / 2) * (W / 2), C);
    up2_add_adjoint_kernel<<<ceil_div(cnt, 256), 256, 0, as_stream(stream)>>>(
        static_cast<const __bf16*>(g_high), static_cast<const __bf16*>(mask_low), n, H, W, C,
        static_cast<__bf16*>(g_low));
    return launch_status("pact_up2_add_adjoint_bf16");
}

extern "C" int pact_pool2_adjoint_bf16(const void* g_low, const void* skip, const void* mask, int n, int H, int W,
                                       int C, void* g_high, void* stream) {
    using namespace pact;
    clear_error();
    if (int s = check_resample(g_low, g_high, n, H, W, C, "pact_pool2_adjoint_bf16")) return s;
    const long long cnt = elementwise_count(static_cast<long long>(n) * H * W, C);
    pool2_adjoint_kernel<<<ceil_div(cnt, 256), 256, 0, as_stream(stream)>>>(
        static_cast<const __bf16*>(g_low), static_cast<const __bf16*>(skip), static_cast<const __bf16*>(mask), n, H,
        W, C, static_cast<__bf16*>(g_high));
    return launch_status("pact_pool2_adjoint_bf16");
}

extern "C" int pact_warm_input(const float* stack, int M, int H, int W, int factor, float scale, int C, void* x,
                               void* stream) {
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(stack && x, "pact_warm_input: null pointer");
    PACT_CHECK_ARG(M > 0 && M <= C && factor > 0 && H > 0 && W > 0 && H % factor == 0 && W % factor == 0,
                   "pact_warm_input: need 0 < M <= C and H, W multiples of the factor");
    PACT_CHECK_ARG(C % 8 == 0, "pact_warm_input: the channel count must be a multiple of 8");
    const int cnt = (H / factor) * (W / factor);
    warm_input_kernel<<<ceil_div(cnt, 256), 256, 0, as_stream(stream)>>>(stack, M, H, W, factor, scale, C,
                                                                        static_cast<__bf16*>(x));
    return launch_status("pact_warm_input");
}

extern "C" size_t pact_warm_loss_workspace_size(int n, int H, int W) {
    if (n <= 0 || H <= 0 || W <= 0) return 0;
    return static_cast<size_t>(pact::ceil_div(static_cast<long long>(n) * H * W, 256)) * sizeof(float);
}

extern "C" int pact_warm_loss(const void* z, int n, int H, int W, int C, const float* target,
                              const unsigned char* mask, float norm, float* loss, void* g, void* ws, size_t ws_bytes,
                              void* stream) {
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(z && target && mask && loss && g, "pact_warm_loss: null pointer");
    PACT_CHECK_ARG(n > 0 && H > 0 && W > 0 && C > 0, "pact_warm_loss: sizes must be positive");
    PACT_CHECK_SUPPORTED(static_cast<long long>(n) * H * W < (1LL << 31), "pact_warm_loss: too many nodes");
    const size_t need = pact_warm_loss_workspace_size(n, H, W);
    if (!ws || ws_bytes < need) {
        set_error("pact_warm_loss: workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : 0);
        return PACT_EWORKSPACE;
    }
    const int nodes = n * H * W, blocks = ceil_div(nodes, 256);
    hipStream_t st = as_stream(stream);
    warm_loss_kernel<<<blocks, 256, 0, st>>>(static_cast<const __bf16*>(z), n, H * W, C, target, mask, norm,
                                            static_cast<__bf16*>(g), static_cast<float*>(ws));
    if (int s = launch_status("pact_warm_loss")) return s;
    warm_loss_finish_kernel<<<1, 256, 0, st>>>(static_cast<const float*>(ws), blocks, norm, loss);
    return launch_status("pact_warm_loss");
}

extern "C" int pact_warm_sos(const void* z, int n, int H, int W, int C, const unsigned char* mask, float v0,
                             float scale, float* sos, void* stream) {
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(z && mask && sos, "pact_warm_sos: null pointer");
    PACT_CHECK_ARG(n > 0 && H > 0 && W > 0 && C > 0, "pact_warm_sos: sizes must be positive");
    PACT_CHECK_SUPPORTED(static_cast<long long>(n) * H * W < (1LL << 31), "pact_warm_sos: too many nodes");
    const int nodes = n * H * W;
    warm_sos_kernel<<<ceil_div(nodes, 256), 256, 0, as_stream(stream)>>>(static_cast<const __bf16*>(z), n, H * W, C,
                                                                        mask, v0, scale, sos);
    return launch_status("pact_warm_sos");
}

extern "C" int pact_ricker_channels(const float* w, const float* sources, const float* amp, const float* sigma,
                                    int n_src, const pact_ring* ring, float v0, int n_t, float fs, float t0, float* S,
                                    void* stream) {
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(w && sources && amp && sigma && ring && S, "pact_ricker_channels: null pointer");
    PACT_CHECK_ARG(n_src > 0 && n_t > 0 && fs > 0.0f && v0 > 0.0f, "pact_ricker_channels: sizes and rates must be positive");
    if (int s = check_ring(*ring)) return s;
    dim3 grid(ceil_div(n_t, 256), ring->n_elem);
    ricker_kernel<<<grid, 256, 0, as_stream(stream)>>>(w, sources, amp, sigma, n_src, ring->n_elem, ring->radius,
                                                      ring->phi0, v0, n_t, fs, t0, S);
    return launch_status("pact_ricker_channels");
}
