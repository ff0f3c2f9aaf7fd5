// Straight-ray wavefront errors, Eq. TOF / Eq. wf (Sec. 3.1), and their adjoint.
//
// Forward.  The node grid of SOS contrasts delta = v - v0 is staged in LDS with a
// one-node ring of zeros (the fixed background), so that every midpoint sample
// inside the clipped ray reads its four bilinear neighbours without a bounds
// test: (G + 2)^2 floats, 80.6 KB at G = 140, so that two workgroups of 1024
// threads share a CU.  A ray (patch i, element n) is cut into K segments of
// consecutive samples (K a power of two chosen on the host to fill the chip),
// one per lane, so the K lanes of a ray are adjacent in a wave and combine their
// sums with K-wide shuffles; each lane sets up its ray once (element position
// included) and walks its samples two at a time so that two LDS gathers are in
// flight.  Rays are numbered patch-major: the lanes of a wave fan out from one
// centre and their gathers often hit the same words (LDS broadcasts).  The
// integrand is evaluated as delta / (v0 + delta) = 1 - v0 / v, which keeps the
// contrast exact instead of cancelling 1 against v0 / v.
//
// Adjoint.  dL/dv at a node collects dL/dw * dl * v0 / v^2 * (bilinear weight)
// from every sample whose cell touches the node.  The main form scatters over
// the whole grid, or over bands of its rows, held in one CU's LDS
// (rays_adj_grid_kernel, described there).  The tiled form below gathers by
// node tile and is used only where even a band of 8 rows does not fit.  One
// workgroup owns a kTile x kTile tile of nodes: it stages the contrast of the
// tile and its one-node halo, and for every patch it enumerates only the
// elements whose ray direction falls in the angular sector the tile's cell
// region subtends from the patch centre (found by the same ring-hit mapping as
// the wavefront interpolation); each such ray is clipped to the region.  Lane
// t takes rays t, t + 256, ...: the lanes of a wave hold adjacent elements of
// one patch, set up their rays together and run similar sample counts.  LDS
// float atomics are slow on this GPU, so none are used: every
// lane owns a private copy of the tile's accumulator (tile plus halo, so that
// no corner needs a test), laid out node-major with the lane index fastest so
// that a wave's read-modify-writes hit distinct banks; samples of the margin
// that fall outside the region add zero.  The private copies of the interior
// nodes are reduced in a fixed order and the tile is written once
// (deterministic, no grid-sized partials).  The sample positions are computed
// by the same code as in the forward pass, so the adjoint is the transpose of
// the forward sum.
#include "common.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace pact {

int device_cu_count();

namespace {

constexpr int kThreads = 1024;    // forward workgroup
constexpr int kTile = 4;              // tile side (nodes) of the tiled adjoint
constexpr int kAdjThreads = 256;      // adjoint workgroup
// padded rows a wave loads before storing them while a workgroup stages the contrast grid (1, 2 and 3
// time the same at 140^2 nodes)
constexpr int kStageRows = 2;

struct RayGeo {
    float inv_ds;       // 1 / node spacing
    float off_x;        // (Gx + 1) / 2: padded node coordinate of x = 0
    float off_y;
    float hx, hy;       // half-extent of the box where v differs from v0
    float inv_ns;       // 1 / n_samples
    int Gx, Gy, W;      // W = Gx + 2 (padded row length)
};

// Element positions, computed by the same code in every kernel that traces rays.
__device__ __forceinline__ void element_position(int n, int n_elem, float R, float phi0, float& ex, float& ey) {
    float sn, cs;
    sincosf(phi0 + kTwoPi * (static_cast<float>(n) / n_elem), &sn, &cs);
    ex = R * cs;
    ey = R * sn;
}

__device__ __forceinline__ void load_elements(float* ex, float* ey, int n_elem, float R, float phi0) {
    for (int n = threadIdx.x; n < n_elem; n += blockDim.x) element_position(n, n_elem, R, phi0, ex[n], ey[n]);
}

// Block maximum (deterministic); `red` must hold blockDim.x / 64 floats.  Result valid in every thread.
__device__ __forceinline__ float block_max(float v, float* red) {
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    float t = red[0];
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 1; i < nw; ++i) t = fmaxf(t, red[i]);
    return t;
}

// Stage the contrast sos - v0 of padded rows R0 .. R0 + H - 1 of the Gy x Gx node grid with a one-node ring
// of zeros (padded node (r, c) is grid node (r - 1, c - 1)) into vs [H][W] (all rows: R0 = 0,
// H = Gy + 2).  Wave w takes rows w, w + waves, ... and lane l
// the columns l, l + 64, ... of each, kStageChunks chunks of 64 columns at a time, so that rows and chunks
// are wave-uniform and no node needs a division.  kRows rows are loaded before any is stored, so each
// lane has up to kRows * kStageChunks loads in flight (a load and its wait per node would serialise some
// twenty round trips to L2 in every workgroup).  A lane's column offsets and column tests are formed once
// per pass of chunks and its loads address the grid by 32-bit byte offsets from the base pointer (every grid
// staged here has far fewer than 2^30 nodes: it, or each band of it, fits in LDS, and there are at most 64
// bands).  With acc, the same nodes of acc are cleared; vmin and nan_check receive the smallest v and
// 0 * (every contrast) (NaN if any node is not finite).
constexpr int kStageChunks = 3;   // one pass covers W <= 192 (140^2 nodes: W = 142)

template <int kRows>
__device__ __forceinline__ void stage_contrast(const float* __restrict__ sos, float v0, const RayGeo& g, float* vs,
                                               int* acc, int R0, int H, float& vmin, float& nan_check) {
    const int W = g.W;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int nw = static_cast<int>(blockDim.x >> 6);
    const char* base = reinterpret_cast<const char*>(sos);
    for (int cb = 0; cb < W; cb += 64 * kStageChunks) {
        unsigned colb[kStageChunks];     // byte offset of the lane's grid column in a row (column 0 outside)
        bool cin[kStageChunks];          // the column lies in the grid (not the ring, not beyond)
#pragma unroll
        for (int q = 0; q < kStageChunks; ++q) {
            const int b = cb + 64 * q + lane - 1;
            cin[q] = static_cast<unsigned>(b) < static_cast<unsigned>(g.Gx);
            colb[q] = cin[q] ? static_cast<unsigned>(b) * 4u : 0u;
        }
        for (int r0 = wave; r0 < H; r0 += kRows * nw) {
            // every load is unconditional and in the grid (row 0 stands in for ring rows, column 0 for ring and
            // outside columns, whose values are not used), and its value is used only after all are issued
            float x[kRows][kStageChunks];
#pragma unroll
            for (int k = 0; k < kRows; ++k) {
                const int a = R0 + r0 + k * nw - 1;
                const bool row_in = a >= 0 && a < g.Gy;
                const unsigned rowb = row_in ? static_cast<unsigned>(a * g.Gx) * 4u : 0u;
#pragma unroll
                for (int q = 0; q < kStageChunks; ++q)
                    x[k][q] = *reinterpret_cast<const float*>(base + (rowb + colb[q]));
            }
#pragma unroll
            for (int k = 0; k < kRows; ++k) {
                const int r = r0 + k * nw, a = R0 + r - 1;
                if (r < H) {
                    const bool row_in = a >= 0 && a < g.Gy;
#pragma unroll
                    for (int q = 0; q < kStageChunks; ++q) {
                        const int c = cb + 64 * q + lane;
                        if (c < W) {
                            const float d = (row_in && cin[q]) ? x[k][q] - v0 : 0.0f;
                            vs[r * W + c] = d;
                            if (acc) acc[r * W + c] = 0;
                            vmin = fminf(vmin, v0 + d);
                            nan_check += 0.0f * d;
                        }
                    }
                }
            }
        }
    }
}

// Geometry of ray (centre c, element e): padded node coordinates of the start point and their
// increment per sample step, and the step length dl = L / n_samples.
__device__ __forceinline__ void ray_setup(float cx, float cy, float ex, float ey, const RayGeo& g, float& gx0,
                                          float& gy0, float& dgx, float& dgy, float& dl) {
    const float dx = ex - cx, dy = ey - cy;
    const float d2 = fmaf(dx, dx, dy * dy);
    const float inv = rsqrtf(d2);
    const float ux = dx * inv, uy = dy * inv;
    float L = d2 * inv;
    if (ux != 0.0f) L = fminf(L, ((ux > 0.0f ? g.hx : -g.hx) - cx) * __builtin_amdgcn_rcpf(ux));
    if (uy != 0.0f) L = fminf(L, ((uy > 0.0f ? g.hy : -g.hy) - cy) * __builtin_amdgcn_rcpf(uy));
    L = fmaxf(L, 0.0f);
    dl = L * g.inv_ns;
    gx0 = fmaf(cx, g.inv_ds, g.off_x);
    gy0 = fmaf(cy, g.inv_ds, g.off_y);
    dgx = dl * ux * g.inv_ds;
    dgy = dl * uy * g.inv_ds;
}

// Cell of sample sf of a ray: flat padded index c of its lower-left node and the fractions (fx, fy) inside
// it.  With kClamp the cell is clamped into the padded grid whatever the input; without, the caller has
// checked that it lies there (segment_inside).  The flat index is formed in float (exact: the padded grid
// has far fewer than 2^24 nodes).
template <bool kClamp>
__device__ __forceinline__ int sample_cell(float sf, float gx0, float gy0, float dgx, float dgy, const RayGeo& g,
                                           float& fx, float& fy) {
    const float gx = fmaf(sf, dgx, gx0), gy = fmaf(sf, dgy, gy0);
    const float bf = floorf(gx), af = floorf(gy);
    fx = gx - bf;
    fy = gy - af;
    const float bc = kClamp ? __builtin_amdgcn_fmed3f(bf, 0.0f, static_cast<float>(g.Gx)) : bf;
    const float ac = kClamp ? __builtin_amdgcn_fmed3f(af, 0.0f, static_cast<float>(g.Gy)) : af;
    return static_cast<int>(fmaf(ac, static_cast<float>(g.W), bc));
}

// True when every sample s0 .. s1 - 1 (s1 > s0) has its cell inside the padded grid, so that clamping
// would change nothing: the positions fma(sf, d, g0) are monotone in sf (fma rounds monotonically), so the
// two end samples bound them all.  False for non-finite positions.
__device__ __forceinline__ bool segment_inside(int s0, int s1, float gx0, float gy0, float dgx, float dgy,
                                               const RayGeo& g) {
    const float xmax = static_cast<float>(g.Gx + 1), ymax = static_cast<float>(g.Gy + 1);
    bool in = true;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float sf = static_cast<float>(e ? s1 - 1 : s0) + 0.5f;
        const float gx = fmaf(sf, dgx, gx0), gy = fmaf(sf, dgy, gy0);
        in = in && gx >= 0.0f && gx < xmax && gy >= 0.0f && gy < ymax;
    }
    return in;
}

// The staged grid seen as an LDS pointer: a gather's address is then one shift-and-add of the cell index
// (through a generic pointer the array's base is added by an instruction of its own).
using LdsFloat = __attribute__((address_space(3))) const float;
__device__ __forceinline__ LdsFloat* lds_view(const float* vs) { return (LdsFloat*)(vs); }

template <bool kClamp>
__device__ __forceinline__ float contrast_sample(const float* vs, float sf, float gx0, float gy0, float dgx, float dgy,
                                                 const RayGeo& g) {
    float fx, fy;
    const int c = sample_cell<kClamp>(sf, gx0, gy0, dgx, dgy, g, fx, fy);
    LdsFloat* p = lds_view(vs) + c;
    const float v00 = p[0], v01 = p[1], v10 = p[g.W], v11 = p[g.W + 1];
    const float top = fmaf(fx, v01 - v00, v00);
    const float bot = fmaf(fx, v11 - v10, v10);
    return fmaf(fy, bot - top, top);
}

// Sum of the integrand delta / (v0 + delta) over samples s0 .. s1 - 1, two at a time (two gathers in flight).
template <bool kClamp>
__device__ __forceinline__ float fwd_segment(const float* vs, int s0, int s1, float v0, float gx0, float gy0,
                                             float dgx, float dgy, const RayGeo& g) {
    float acc0 = 0.0f, acc1 = 0.0f;
    // the loop runs on the sample's float coordinate alone (exact: sample counts are far below 2^24)
    float sf = static_cast<float>(s0) + 0.5f;
    const float sf_pair_end = static_cast<float>(s1) - 0.5f;     // a pair starting at sf fits while sf < this
    for (; sf < sf_pair_end; sf += 2.0f) {
        const float d0 = contrast_sample<kClamp>(vs, sf, gx0, gy0, dgx, dgy, g);
        const float d1 = contrast_sample<kClamp>(vs, sf + 1.0f, gx0, gy0, dgx, dgy, g);
        acc0 = fmaf(d0, __builtin_amdgcn_rcpf(v0 + d0), acc0);
        acc1 = fmaf(d1, __builtin_amdgcn_rcpf(v0 + d1), acc1);
    }
    if (sf < static_cast<float>(s1)) {
        const float d0 = contrast_sample<kClamp>(vs, sf, gx0, gy0, dgx, dgy, g);
        acc0 = fmaf(d0, __builtin_amdgcn_rcpf(v0 + d0), acc0);
    }
    return acc0 + acc1;
}

__global__ __launch_bounds__(kThreads) void rays_fwd_kernel(const float* __restrict__ sos, float v0,
                                                            const float* __restrict__ centres, int N, int n_elem,
                                                            float R, float phi0, int Ns, RayGeo g, int K,
                                                            int n_items, float* __restrict__ w) {
    extern __shared__ float vs[];
    {
        float vmin = v0, nan_check = 0.0f;   // not used by the forward
        stage_contrast<kStageRows>(sos, v0, g, vs, nullptr, 0, g.Gy + 2, vmin, nan_check);
    }
    __syncthreads();
    // K divides the workgroup size and n_items = rays * K, so the K lanes of a ray enter and leave the
    // loop together
    for (int item = blockIdx.x * blockDim.x + threadIdx.x; item < n_items; item += gridDim.x * blockDim.x) {
        const int ray = item / K, k = item - ray * K;
        const int i = ray / n_elem, n = ray - i * n_elem;
        float ex, ey;
        element_position(n, n_elem, R, phi0, ex, ey);
        float gx0, gy0, dgx, dgy, dl;
        ray_setup(centres[2 * i], centres[2 * i + 1], ex, ey, g, gx0, gy0, dgx, dgy, dl);
        const int s0 = (k * Ns) / K, s1 = ((k + 1) * Ns) / K;
        float acc = 0.0f;
        if (s1 > s0) {
            // the clamp-free loop where the whole segment is inside the grid (the same bits)
            acc = segment_inside(s0, s1, gx0, gy0, dgx, dgy, g)
                      ? fwd_segment<false>(vs, s0, s1, v0, gx0, gy0, dgx, dgy, g)
                      : fwd_segment<true>(vs, s0, s1, v0, gx0, gy0, dgx, dgy, g);
        }
        for (int off = K >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, K);
        if (k == 0) w[ray] = acc * dl;
    }
}

// Sector of the elements whose rays from (cx, cy) can cross the rectangle [x0, x1] x [y0, y1]:
// a first element and a count (cyclic), with one element of margin on each side.
__device__ __forceinline__ void sector(float cx, float cy, float x0, float x1, float y0, float y1, float R,
                                       float phi0, int n_elem, int& first, int& count) {
    if (cx >= x0 && cx <= x1 && cy >= y0 && cy <= y1) {
        first = 0;
        count = n_elem;
        return;
    }
    const float ref = atan2f(0.5f * (y0 + y1) - cy, 0.5f * (x0 + x1) - cx);
    float lo = 0.0f, hi = 0.0f;
    const float xs[4] = {x0, x1, x0, x1}, ys[4] = {y0, y0, y1, y1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float d = atan2f(ys[k] - cy, xs[k] - cx) - ref;
        d -= kTwoPi * rintf(d * (1.0f / kTwoPi));           // wrap to [-pi, pi]
        lo = fminf(lo, d);
        hi = fmaxf(hi, d);
    }
    const float R2mc2 = R * R - (cx * cx + cy * cy);
    const float nf = static_cast<float>(n_elem);
    float sl, cl, sh, ch;
    sincosf(ref + lo, &sl, &cl);
    sincosf(ref + hi, &sh, &ch);
    const float flo = ring_hit_index(cx, cy, cl, sl, R2mc2, phi0, nf / kTwoPi, nf);
    float fhi = ring_hit_index(cx, cy, ch, sh, R2mc2, phi0, nf / kTwoPi, nf);
    if (fhi < flo) fhi += nf;
    const int a = static_cast<int>(floorf(flo)) - 1;
    const int b = static_cast<int>(floorf(fhi)) + 2;
    count = min(max(b - a, 0), n_elem);
    first = ((a % n_elem) + n_elem) % n_elem;
}

// Clipped sample range [s0, s1] of a ray inside the tile region (padded node coordinates gx in
// [b_lo, b_hi + 1), gy in [a_lo, a_hi + 1)), one sample of margin on each side; empty if s1 < s0.
__device__ __forceinline__ void clip_samples(float gx0, float gy0, float dgx, float dgy, int a_lo, int a_hi, int b_lo,
                                             int b_hi, int Ns, int& s0, int& s1) {
    float slo = 0.0f, shi = static_cast<float>(Ns);
    bool empty = false;
    if (dgx != 0.0f) {
        const float r = __builtin_amdgcn_rcpf(dgx);
        const float t0 = (b_lo - gx0) * r, t1 = (b_hi + 1 - gx0) * r;
        slo = fmaxf(slo, fminf(t0, t1));
        shi = fminf(shi, fmaxf(t0, t1));
    } else {
        empty = gx0 < b_lo || gx0 >= b_hi + 1;
    }
    if (dgy != 0.0f) {
        const float r = __builtin_amdgcn_rcpf(dgy);
        const float t0 = (a_lo - gy0) * r, t1 = (a_hi + 1 - gy0) * r;
        slo = fmaxf(slo, fminf(t0, t1));
        shi = fminf(shi, fmaxf(t0, t1));
    } else {
        empty = empty || gy0 < a_lo || gy0 >= a_hi + 1;
    }
    if (empty || !(shi >= slo)) {
        s0 = 0;
        s1 = -1;
        return;
    }
    s0 = max(static_cast<int>(ceilf(slo - 0.5f)) - 1, 0);
    s1 = min(static_cast<int>(floorf(shi - 0.5f)) + 1, Ns - 1);
}

__global__ __launch_bounds__(kAdjThreads) void rays_adj_tile_kernel(
    const float* __restrict__ sos, float v0, const float* __restrict__ centres, int N, int n_elem, float R, float phi0,
    int Ns, RayGeo g, int tiles_x, const float* __restrict__ dL_dw, const float* __restrict__ scale, int accumulate,
    float* __restrict__ out) {
    constexpr int L = kTile + 2;                      // local nodes per side, including the halo
    constexpr int NN = L * L;                         // accumulator nodes per lane
    __shared__ float dv[NN];                          // contrast on the tile's nodes and halo
    __shared__ int scan_a[kAdjThreads], scan_b[kAdjThreads];
    extern __shared__ float lds[];
    float* acc = lds;                                 // per-lane accumulators, [node][thread]
    float* ex = acc + NN * kAdjThreads;
    float* ey = ex + n_elem;
    int* first = reinterpret_cast<int*>(ey + n_elem);  // [N] first element of each patch's sector
    int* cnt = first + N;                              // [N] elements in the sector
    int* offs = cnt + N;                               // [N + 1] exclusive prefix sum of cnt

    const int tid = threadIdx.x;
    const int ty = blockIdx.x / tiles_x, tx = blockIdx.x % tiles_x;
    const int a_lo = ty * kTile, a_hi = min(a_lo + kTile, g.Gy);
    const int b_lo = tx * kTile, b_hi = min(b_lo + kTile, g.Gx);
    const int th = a_hi - a_lo, tw = b_hi - b_lo;      // interior extent (ragged at the grid edge)
    // local node (la, lb) is grid node (a_lo - 1 + la, b_lo - 1 + lb); interior nodes have la, lb in 1..kTile
    for (int idx = tid; idx < NN; idx += blockDim.x) {
        const int a = a_lo - 1 + idx / L, b = b_lo - 1 + idx % L;
        dv[idx] = (a >= 0 && a < g.Gy && b >= 0 && b < g.Gx) ? sos[a * g.Gx + b] - v0 : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < NN; ++j) acc[j * kAdjThreads + tid] = 0.0f;
    load_elements(ex, ey, n_elem, R, phi0);
    // Samples that touch the tile have their cell in rows a_lo-1 .. a_hi-1 and columns b_lo-1 .. b_hi-1,
    // i.e. padded node coordinates gy in [a_lo, a_hi + 1), gx in [b_lo, b_hi + 1).
    const float ds = 1.0f / g.inv_ds;
    const float x0 = (b_lo - g.off_x) * ds, x1 = (b_hi + 1 - g.off_x) * ds;
    const float y0 = (a_lo - g.off_y) * ds, y1 = (a_hi + 1 - g.off_y) * ds;
    const float margin = 1e-3f * ds;
    // 1. per-patch element sectors; thread t owns the contiguous run of patches t * per .. t * per + per - 1
    const int per = (N + kAdjThreads - 1) / kAdjThreads;
    int run = 0;
    for (int k = 0; k < per; ++k) {
        const int i = tid * per + k;
        if (i < N) {
            int f, c;
            sector(centres[2 * i], centres[2 * i + 1], x0 - margin, x1 + margin, y0 - margin, y1 + margin, R, phi0,
                   n_elem, f, c);
            first[i] = f;
            cnt[i] = c;
            run += c;
        }
    }
    // inclusive scan of per-thread values (Hillis-Steele, double-buffered); returns the inclusive prefix
    auto block_scan = [&](int v) -> int {
        scan_a[tid] = v;
        __syncthreads();
        int* src = scan_a;
        int* dst = scan_b;
        for (int off = 1; off < kAdjThreads; off <<= 1) {
            dst[tid] = src[tid] + (tid >= off ? src[tid - off] : 0);
            __syncthreads();
            int* t = src;
            src = dst;
            dst = t;
        }
        const int r = src[tid];
        __syncthreads();
        return r;
    };
    {
        int s0 = block_scan(run) - run;
        for (int k = 0; k < per; ++k) {
            const int i = tid * per + k;
            if (i < N) {
                offs[i] = s0;
                s0 += cnt[i];
            }
        }
        if (tid == kAdjThreads - 1) offs[N] = s0;
    }
    __syncthreads();
    const int total = offs[N];
    const float sc = (scale ? *scale : 1.0f) * v0;

    // 2. lane t takes items t, t + 256, ...: the 64 lanes of a wave hold 64 adjacent elements of one or
    // two patches, so they set up their rays together and have similar sample counts
    float* my = acc + tid;
    for (int k = tid; k < total; k += kAdjThreads) {
        int lo = 0, hi = N - 1;                        // patch of item k: the last i with offs[i] <= k
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (offs[mid] <= k) lo = mid; else hi = mid - 1;
        }
        const int i = lo;
        const int n = (first[i] + (k - offs[i])) % n_elem;
        float gx0, gy0, dgx, dgy, dl;
        ray_setup(centres[2 * i], centres[2 * i + 1], ex[n], ey[n], g, gx0, gy0, dgx, dgy, dl);
        int s0, s1;
        clip_samples(gx0, gy0, dgx, dgy, a_lo, a_hi, b_lo, b_hi, Ns, s0, s1);
        const float q0 = dL_dw[static_cast<size_t>(i) * n_elem + n] * dl * sc;
        // every sample is tested: margin samples, and samples of rays grazing an edge of the region, can
        // fall outside it; they add zero to node 0
        float sf = static_cast<float>(s0) + 0.5f;
        for (int s = s0; s <= s1; ++s, sf += 1.0f) {
            const float gx = fmaf(sf, dgx, gx0), gy = fmaf(sf, dgy, gy0);
            const float bf = floorf(gx), af = floorf(gy);
            int lb = static_cast<int>(bf) - b_lo;         // local column of the cell's first node
            int la = static_cast<int>(af) - a_lo;
            const bool inside = static_cast<unsigned>(lb) <= static_cast<unsigned>(tw) &&
                                static_cast<unsigned>(la) <= static_cast<unsigned>(th);
            const float qs = inside ? q0 : 0.0f;
            lb = inside ? lb : 0;
            la = inside ? la : 0;
            const int c = la * L + lb;
            const float fx = gx - bf, fy = gy - af;
            const float v00 = dv[c], v01 = dv[c + 1], v10 = dv[c + L], v11 = dv[c + L + 1];
            const float top = fmaf(fx, v01 - v00, v00);
            const float bot = fmaf(fx, v11 - v10, v10);
            const float r = __builtin_amdgcn_rcpf(v0 + fmaf(fy, bot - top, top));
            const float qv = qs * r * r;                  // dL/dw * dl * v0 / v^2
            const float qy1 = qv * fy, qy0 = qv - qy1;
            float* p = my + c * kAdjThreads;
            p[0] += qy0 - qy0 * fx;
            p[kAdjThreads] += qy0 * fx;
            p[L * kAdjThreads] += qy1 - qy1 * fx;
            p[(L + 1) * kAdjThreads] += qy1 * fx;
        }
    }
    __syncthreads();
    // 3. fixed-order reduction of the interior nodes' columns: each 16-lane group sums the 256 columns of
    // one node (16 strided columns per lane, then shuffles)
    const int part = tid & 15;
    for (int j = tid >> 4; j < kTile * kTile; j += kAdjThreads / 16) {
        const int la = j / kTile, lb = j % kTile;
        const float* col = acc + ((la + 1) * L + (lb + 1)) * kAdjThreads;
        float sum = 0.0f;
#pragma unroll
        for (int q = 0; q < kAdjThreads / 16; ++q) sum += col[part + 16 * q];
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 16);
        if (part == 0 && la < th && lb < tw) {
            const size_t o = static_cast<size_t>(a_lo + la) * g.Gx + (b_lo + lb);
            out[o] = accumulate ? out[o] + sum : sum;
        }
    }
}

// Adjoint (scatter over the whole grid, when the contrast grid and an integer accumulator of the same shape
// both fit in one CU's LDS, G <= 141; else over bands of its rows, below).  One 1024-thread workgroup per
// CU; the rays are cut into K segments of consecutive samples (K chosen on the host so that the work is
// about one segment per lane) and work item (ray, segment) goes to one lane, which walks its samples with the same
// position formula as the forward pass.  Rays are numbered element-major, so that the lanes of a wave
// hold parallel rays from neighbouring patch centres and rarely hit the same node at once.  A lane sums
// the four bilinear shares of consecutive samples in the same cell in registers and adds them to the
// accumulator with integer LDS atomics when its walk leaves the cell, in fixed point at a power-of-two
// scale F chosen per workgroup from a bound on any node's sum:
//   |sum| <= sum over the workgroup's rays of |dL/dw * sc| * v0 / vmin^2 * (2 sqrt(2) ds + dl),
// since a ray meets a node's bilinear support over at most 2 sqrt(2) ds and every weight is <= 1.
// F = 2^30 / bound (rounded down to a power of two) keeps every partial sum inside int32 with room for
// the truncation of each flushed term.  Integer sums do not depend on the order of the atomics, so the result is
// deterministic.  The interior nodes are written, scaled back, to one partial grid per workgroup, and
// a reduce kernel adds the partial grids in a fixed order.
constexpr int kGridThreads = 1024;

// Adjoint shares of samples s0 .. s1 - 1 (s1 > s0) of one ray, added into the fixed-point accumulator acc
// (same layout as vs).  Consecutive samples in the same cell add into registers; a cell's four shares go to
// LDS once, when the walk leaves it (truncation toward zero: at most one unit of 2^-30 of the bound per
// flush).  q0 = dL/dw * dl * v0 * F.
// Banded (kBanded): vs and acc hold padded rows R0 .. R0 + band_cells / W of the grid, and only samples whose
// cell's lower row lies in R0 .. R0 + band_cells / W - 1 are taken (cbase = R0 W); the others belong to
// another band.
template <bool kClamp, bool kBanded>
__device__ __forceinline__ void adj_segment(const float* vs, int* acc, int s0, int s1, float v0, float q0, float gx0,
                                            float gy0, float dgx, float dgy, const RayGeo& g, int cbase,
                                            int band_cells) {
    const int W = g.W;
    float sf = static_cast<float>(s0) + 0.5f;
    float fx, fy;
    // the first sample's cell (banded: none yet, so that the first taken sample opens its cell) and the
    // contrast at its corners, loaded again only when a sample enters another cell (about every second
    // sample at half a node per step)
    LdsFloat* lv = lds_view(vs);
    int cprev = kBanded ? -1 : sample_cell<kClamp>(sf, gx0, gy0, dgx, dgy, g, fx, fy);
    float v00 = 0.0f, v01 = 0.0f, v10 = 0.0f, v11 = 0.0f;
    if (!kBanded) v00 = lv[cprev], v01 = lv[cprev + 1], v10 = lv[cprev + W], v11 = lv[cprev + W + 1];
    float a00 = 0.0f, a01 = 0.0f, a10 = 0.0f, a11 = 0.0f;
    const float sf1 = static_cast<float>(s1);    // the loop runs on sf alone (exact: counts far below 2^24)
    for (; sf < sf1; sf += 1.0f) {
        int c = sample_cell<kClamp>(sf, gx0, gy0, dgx, dgy, g, fx, fy);
        if (kBanded) {
            c -= cbase;
            if (c < 0 || c >= band_cells) continue;
            if (cprev < 0) {
                cprev = c;
                v00 = lv[c], v01 = lv[c + 1], v10 = lv[c + W], v11 = lv[c + W + 1];
            }
        }
        if (c != cprev) {
            atomicAdd(acc + cprev, static_cast<int>(a00));
            atomicAdd(acc + cprev + 1, static_cast<int>(a01));
            atomicAdd(acc + cprev + W, static_cast<int>(a10));
            atomicAdd(acc + cprev + W + 1, static_cast<int>(a11));
            cprev = c;
            a00 = a01 = a10 = a11 = 0.0f;
            v00 = lv[c], v01 = lv[c + 1], v10 = lv[c + W], v11 = lv[c + W + 1];
        }
        const float top = fmaf(fx, v01 - v00, v00);
        const float bot = fmaf(fx, v11 - v10, v10);
        const float r = __builtin_amdgcn_rcpf(v0 + fmaf(fy, bot - top, top));
        const float qv = q0 * r * r;                     // dL/dw * dl * v0 / v^2, times F
        const float qy1 = qv * fy, qy0 = qv - qy1;
        a00 += qy0 - qy0 * fx;
        a01 += qy0 * fx;
        a10 += qy1 - qy1 * fx;
        a11 += qy1 * fx;
    }
    if (kBanded && cprev < 0) return;
    atomicAdd(acc + cprev, static_cast<int>(a00));
    atomicAdd(acc + cprev + 1, static_cast<int>(a01));
    atomicAdd(acc + cprev + W, static_cast<int>(a10));
    atomicAdd(acc + cprev + W + 1, static_cast<int>(a11));
}

// Samples of s0 .. s1 - 1 whose position row gy may lie in [R0, R1): a conservative range (one sample of
// margin each side) from gy = gy0 + (s + 1/2) dgy; the per-sample test in adj_segment is exact.
__device__ __forceinline__ void band_samples(int s0, int s1, float gy0, float dgy, int R0, int R1, int& sa, int& sb) {
    sa = s0;
    sb = s1;
    if (!(dgy != 0.0f) || !isfinite(gy0) || !isfinite(dgy)) return;
    const float t0 = (static_cast<float>(R0) - gy0) / dgy - 0.5f, t1 = (static_cast<float>(R1) - gy0) / dgy - 0.5f;
    const float lo = fmaxf(fminf(t0, t1), static_cast<float>(s0) - 2.0f);
    const float hi = fminf(fmaxf(t0, t1), static_cast<float>(s1) + 2.0f);
    if (!(lo <= hi)) {
        sb = sa;
        return;
    }
    sa = max(s0, static_cast<int>(floorf(lo)) - 1);
    sb = min(s1, static_cast<int>(ceilf(hi)) + 2);
}


// Banded form (kBanded), for grids whose contrast fits in LDS but not twice: workgroup b takes band
// b % n_bands, cell rows R0 .. R1 - 1 (padded coordinates, R0 = band band_rows), stages padded rows
// R0 .. R1 and accumulates the samples whose cells lie in its band; the workgroups of a band share out
// every ray segment.  Bands overlap in one row of nodes, which both accumulate; the partial grids (zero
// outside a workgroup's rows) are summed as before.
template <bool kBanded>
__global__ __launch_bounds__(kGridThreads) void rays_adj_grid_kernel(
    const float* __restrict__ sos, float v0, const float* __restrict__ centres, int N, int n_elem, float R, float phi0,
    int Ns, RayGeo g, int K, int n_items, int per_block, int n_bands, int band_rows, const float* __restrict__ dL_dw,
    const float* __restrict__ scale, float* __restrict__ partial) {
    extern __shared__ float lds[];
    const int W = g.W;
    const int band = kBanded ? static_cast<int>(blockIdx.x) % n_bands : 0;
    const int bblock = kBanded ? static_cast<int>(blockIdx.x) / n_bands : static_cast<int>(blockIdx.x);
    const int R0 = kBanded ? band * band_rows : 0;                        // cell rows R0 .. R1 - 1
    const int R1 = kBanded ? min(R0 + band_rows, g.Gy + 1) : g.Gy + 1;
    const int total = (R1 - R0 + 1) * W;                                  // staged padded rows R0 .. R1
    float* vs = lds;                                        // contrast with a ring of zeros
    int* acc = reinterpret_cast<int*>(vs + total);          // fixed-point sums, same layout
    float* red = reinterpret_cast<float*>(acc + total);     // kGridThreads / 64 floats
    const int tid = threadIdx.x;
    float vmin = v0, nan_check = 0.0f;                     // nan_check turns NaN if any node is not finite
    stage_contrast<kStageRows>(sos, v0, g, vs, acc, R0, R1 - R0 + 1, vmin, nan_check);
    vmin = -block_max(-vmin, red);
    const int it0 = bblock * per_block;
    const int it1 = min(it0 + per_block, n_items);
    const float sc = (scale ? *scale : 1.0f) * v0;
    const float ds = 1.0f / g.inv_ds;
    // bound on any node's sum over this workgroup's rays
    float bnd = 0.0f;
    if (it1 > it0) {
        for (int ray = it0 / K + tid; ray <= (it1 - 1) / K; ray += blockDim.x) {
            const int n = ray / N, i = ray - n * N;
            float ex, ey;
            element_position(n, n_elem, R, phi0, ex, ey);
            float gx0, gy0, dgx, dgy, dl;
            ray_setup(centres[2 * i], centres[2 * i + 1], ex, ey, g, gx0, gy0, dgx, dgy, dl);
            bnd += fabsf(dL_dw[static_cast<size_t>(i) * n_elem + n] * sc) * (2.8285f * ds + dl);
        }
    }
    bnd = block_sum(bnd + nan_check, red) / (vmin * vmin);
    const bool ok = vmin > 0.0f && bnd <= 3.0e38f;        // false for NaN or infinite bounds too
    const float F = (ok && bnd > 0.0f) ? ldexpf(1.0f, min(30 - (ilogbf(bnd) + 1), 126)) : 1.0f;
    __syncthreads();

    const int cbase = R0 * W, band_cells = (R1 - R0) * W;
    for (int item = it0 + tid; item < it1; item += blockDim.x) {
        const int ray = item / K, k = item - ray * K;
        const int n = ray / N, i = ray - n * N;
        float ex, ey;
        element_position(n, n_elem, R, phi0, ex, ey);
        float gx0, gy0, dgx, dgy, dl;
        ray_setup(centres[2 * i], centres[2 * i + 1], ex, ey, g, gx0, gy0, dgx, dgy, dl);
        const float q0 = ok ? dL_dw[static_cast<size_t>(i) * n_elem + n] * dl * sc * F : 0.0f;
        int s0 = (k * Ns) / K, s1 = ((k + 1) * Ns) / K;
        if (kBanded) band_samples(s0, s1, gy0, dgy, R0, R1, s0, s1);
        if (s1 > s0) {
            // the clamp-free loop where the whole segment is inside the grid (the same bits)
            if (segment_inside(s0, s1, gx0, gy0, dgx, dgy, g))
                adj_segment<false, kBanded>(vs, acc, s0, s1, v0, q0, gx0, gy0, dgx, dgy, g, cbase, band_cells);
            else
                adj_segment<true, kBanded>(vs, acc, s0, s1, v0, q0, gx0, gy0, dgx, dgy, g, cbase, band_cells);
        }
    }
    __syncthreads();
    const float invF = 1.0f / F;
    const float bad = __builtin_nanf("");
    float* part = partial + static_cast<size_t>(blockIdx.x) * g.Gy * g.Gx;
    // rows per wave and columns per lane, as in the staging; grid row a is padded row a + 1, held in this
    // workgroup's rows when R0 <= a + 1 <= R1 (zero otherwise)
    {
        const int lane = tid & 63;
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        for (int a = wave; a < g.Gy; a += kGridThreads / 64) {
            const bool mine = !kBanded || (a + 1 >= R0 && a + 1 <= R1);
            for (int b = lane; b < g.Gx; b += 64)
                part[a * g.Gx + b] = !ok ? bad : (mine ? static_cast<float>(acc[(a + 1 - R0) * W + b + 1]) * invF : 0.0f);
        }
    }
}

// Sum of the per-workgroup partial grids in a fixed order.  A workgroup owns 64 consecutive nodes; its
// wave s sums, for those nodes, the s-th of kAdjSlices contiguous runs of partials (in order), so that
// every load of a wave is one 256-byte row and each lane has 16 loads in flight; the run sums then meet in
// LDS and are added in order (= or += into out).
constexpr int kAdjSlices = 16;

// Run `slice` of the kAdjSlices contiguous runs of the n_part partials at one node, added in order.
__device__ __forceinline__ float adj_run_sum(const float* __restrict__ partial, int n_part, int n_nodes, int node,
                                             int slice) {
    const int per = (n_part + kAdjSlices - 1) / kAdjSlices;
    const int p0 = slice * per, p1 = min(p0 + per, n_part);
    return p1 > p0 ? ordered_strided_sum<16>(partial + static_cast<size_t>(p0) * n_nodes + node, p1 - p0,
                                                   n_nodes)
                   : 0.0f;
}

constexpr int kReduceNodes = 64;

__global__ __launch_bounds__(kAdjSlices * kReduceNodes) void rays_adj_reduce_kernel(
    const float* __restrict__ partial, int n_part, int n_nodes, int accumulate, float* __restrict__ out) {
    __shared__ float run[kAdjSlices][kReduceNodes];
    const int j = threadIdx.x % kReduceNodes, slice = threadIdx.x / kReduceNodes;
    const int node = blockIdx.x * kReduceNodes + j;
    run[slice][j] = node < n_nodes ? adj_run_sum(partial, n_part, n_nodes, node, slice) : 0.0f;
    __syncthreads();
    if (slice == 0 && node < n_nodes) {
        float t = 0.0f;
#pragma unroll
        for (int k = 0; k < kAdjSlices; ++k) t += run[k][j];
        out[node] = accumulate ? out[node] + t : t;
    }
}

RayGeo make_geo(const pact_grid& sosg, int n_samples) {
    RayGeo g;
    g.inv_ds = 1.0f / sosg.spacing;
    g.off_x = 0.5f * (sosg.nx + 1);
    g.off_y = 0.5f * (sosg.ny + 1);
    g.hx = 0.5f * (sosg.nx + 1) * sosg.spacing;
    g.hy = 0.5f * (sosg.ny + 1) * sosg.spacing;
    g.inv_ns = 1.0f / static_cast<float>(n_samples);
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
    PACT_CHECK_SUPPORTED(static_cast<long long>(N) * ring.n_elem < (1LL << 31), "%s: too many rays", what);
    return PACT_OK;
}

// Ray tilings chosen by pact_rays_autotune, per device and geometry: lanes per ray of the forward kernel
// and segments per ray of the adjoint (0 = the built-in rule).
using TuneKey = std::tuple<int, int, int, int, int, int>;     // device, N, n_elem, n_samples, ny, nx
struct RayTiling {
    int fwd = 0, adj = 0;
};
std::mutex g_tune_mu;
std::map<TuneKey, RayTiling> g_tuned;

TuneKey tune_key(int N, const pact_ring& ring, int n_samples, const pact_grid& sosg) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    return TuneKey(dev, N, ring.n_elem, n_samples, sosg.ny, sosg.nx);
}

RayTiling tuned_tiling(int N, const pact_ring& ring, int n_samples, const pact_grid& sosg) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tuned.find(tune_key(N, ring, n_samples, sosg));
    return it == g_tuned.end() ? RayTiling() : it->second;
}

// Lanes per ray of the forward kernel by the built-in rule: the smallest power of two (at most 64, at
// least 16 samples a segment) whose work items fill about two rounds of two workgroups per CU (measured
// at 86,528 rays x 256 samples: K = 8 is 10% faster than one round with K = 4).
int fwd_lanes_rule(long long n_rays, int n_samples) {
    const long long lanes = 2LL * device_cu_count() * kThreads;
    int K = 1;
    while (K < 64 && n_rays * K < lanes && n_samples / (2 * K) >= 16) K *= 2;
    return K;
}

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
    // lanes per ray: the autotuned value for this geometry, else the built-in rule
    const long long n_rays = static_cast<long long>(N) * ring.n_elem;
    const int tuned = tuned_tiling(N, ring, n_samples, sosg).fwd;
    const int K = tuned > 0 ? tuned : fwd_lanes_rule(n_rays, n_samples);
    PACT_CHECK_SUPPORTED(n_rays * K < (1LL << 31), "pact_sos_to_delays: too many rays");
    const int n_items = static_cast<int>(n_rays * K);
    const int blocks = static_cast<int>(std::min<long long>(ceil_div(n_items, kThreads), 2LL * device_cu_count()));
    rays_fwd_kernel<<<blocks, kThreads, lds, as_stream(stream)>>>(sos, v0, centres, N, ring.n_elem, ring.radius,
                                                                 ring.phi0, n_samples, make_geo(sosg, n_samples), K,
                                                                 n_items, w);
    return launch_status("pact_sos_to_delays");
}

namespace pact {
namespace {

// Layout of rays_adj_grid_kernel for a grid: bands of band_rows cell rows (1 band: the whole grid) and the
// LDS bytes of one band; bands == 0 if even bands of 8 rows do not fit (the tile kernel is used instead).
struct AdjPlan {
    int bands, band_rows;
    size_t lds;
};

AdjPlan adj_plan(const pact_grid& sosg) {
    const size_t W = static_cast<size_t>(sosg.nx) + 2, H = static_cast<size_t>(sosg.ny) + 2;
    const size_t red = (kGridThreads / 64) * sizeof(float);
    if (2 * H * W * sizeof(float) + red <= kLdsBytes) return {1, sosg.ny + 1, 2 * H * W * sizeof(float) + red};
    const long long max_rows = static_cast<long long>((kLdsBytes - red) / (2 * W * sizeof(float))) - 1;
    if (max_rows < 8) return {0, 0, 0};
    const int bands = ceil_div(sosg.ny + 1, max_rows);
    if (bands > 64) return {0, 0, 0};
    const int rows = ceil_div(sosg.ny + 1, bands);             // balanced bands
    return {bands, rows, 2 * (static_cast<size_t>(rows) + 1) * W * sizeof(float) + red};
}

size_t adj_grid_lds(const pact_grid& sosg) { return adj_plan(sosg).bands ? adj_plan(sosg).lds : 0; }

// Segments per ray for rays_adj_grid_kernel: the K that minimises the critical path of one lane, rounds of
// items times (segment length + a ray set-up worth about two samples), with at least 8 samples a segment.
int adj_segments(long long n_rays, int n_samples, long long lanes) {
    int best = 1;
    long long best_cost = -1;
    const int kmax = std::max(1, std::min(n_samples / 8, 256));
    for (int K = 1; K <= kmax; ++K) {
        const long long rounds = (n_rays * K + lanes - 1) / lanes;
        const long long cost = rounds * ((n_samples + K - 1) / K + 2);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = K;
        }
    }
    return best;
}

// The grid adjoint into one partial node grid per workgroup (the caller sums them); *n_part = their count.
int launch_adj_grid(const float* sos, const pact_grid& sosg, float v0, const float* centres, int N,
                    const pact_ring& ring, int n_samples, const float* dL_dw, const float* scale, float* partial,
                    size_t ws_bytes, hipStream_t st, int* n_part, const char* what) {
    const AdjPlan plan = adj_plan(sosg);
    const int cus = device_cu_count();
    const int per_band = std::max(1, cus / plan.bands);           // workgroups per band
    const int blocks = plan.bands * per_band;
    const size_t need = static_cast<size_t>(blocks) * sosg.ny * sosg.nx * sizeof(float);
    if (!partial || ws_bytes < need) {
        set_error("%s: workspace of %zu bytes needed, %zu given", what, need, partial ? ws_bytes : 0);
        return PACT_EWORKSPACE;
    }
    static bool gattr = false;
    if (!gattr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(rays_adj_grid_kernel<false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(rays_adj_grid_kernel<true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        gattr = true;
    }
    const long long n_rays = static_cast<long long>(N) * ring.n_elem;
    const int tuned = tuned_tiling(N, ring, n_samples, sosg).adj;
    const int K = tuned > 0 ? tuned : adj_segments(n_rays, n_samples, static_cast<long long>(per_band) * kGridThreads);
    PACT_CHECK_SUPPORTED(n_rays * K < (1LL << 31), "%s: too many ray segments", what);
    const int n_items = static_cast<int>(n_rays * K);
    const int per_block = ceil_div(n_items, per_band);
    if (plan.bands == 1)
        rays_adj_grid_kernel<false><<<blocks, kGridThreads, plan.lds, st>>>(
            sos, v0, centres, N, ring.n_elem, ring.radius, ring.phi0, n_samples, make_geo(sosg, n_samples), K, n_items,
            per_block, 1, sosg.ny + 1, dL_dw, scale, partial);
    else
        rays_adj_grid_kernel<true><<<blocks, kGridThreads, plan.lds, st>>>(
            sos, v0, centres, N, ring.n_elem, ring.radius, ring.phi0, n_samples, make_geo(sosg, n_samples), K, n_items,
            per_block, plan.bands, plan.band_rows, dL_dw, scale, partial);
    *n_part = blocks;
    return launch_status(what);
}

}  // namespace
}  // namespace pact

extern "C" size_t pact_sos_to_delays_adjoint_workspace_size(const pact_grid* sosg_, int N, const pact_ring* ring_) {
    (void)N;
    (void)ring_;
    if (!sosg_ || sosg_->ny <= 0 || sosg_->nx <= 0) return 0;
    const pact::AdjPlan plan = pact::adj_plan(*sosg_);
    if (!plan.bands) return 0;
    const int blocks = plan.bands * std::max(1, pact::device_cu_count() / plan.bands);
    return static_cast<size_t>(blocks) * sosg_->ny * sosg_->nx * sizeof(float);
}

extern "C" int pact_sos_to_delays_adjoint(const float* sos, const pact_grid* sosg_, float v0, const float* centres,
                                          int N, const pact_ring* ring_, int n_samples, const float* dL_dw,
                                          const float* scale, float* dL_dsos, int accumulate, void* ws,
                                          size_t ws_bytes, void* stream) {
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
    if (adj_grid_lds(sosg)) {
        float* partial = static_cast<float*>(ws);
        int n_part = 0;
        if (int st = launch_adj_grid(sos, sosg, v0, centres, N, ring, n_samples, dL_dw, scale, partial, ws_bytes,
                                     as_stream(stream), &n_part, "pact_sos_to_delays_adjoint"))
            return st;
        const int n_nodes = sosg.ny * sosg.nx;
        rays_adj_reduce_kernel<<<ceil_div(n_nodes, kReduceNodes), kAdjSlices * kReduceNodes, 0, as_stream(stream)>>>(
            partial, n_part, n_nodes, accumulate, dL_dsos);
        return launch_status("pact_sos_to_delays_adjoint");
    }
    const size_t lds = static_cast<size_t>(kTile + 2) * (kTile + 2) * kAdjThreads * sizeof(float) +
                       2 * static_cast<size_t>(ring.n_elem) * sizeof(float) +
                       (3 * static_cast<size_t>(N) + 1) * sizeof(int);
    PACT_CHECK_SUPPORTED(lds + 4 * 1024 <= kLdsBytes,
                         "pact_sos_to_delays_adjoint: %d patches x %d elements exceed the LDS work tables", N,
                         ring.n_elem);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(rays_adj_tile_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes - 8 * 1024));
        attr = true;
    }
    const int tiles_x = ceil_div(sosg.nx, kTile), tiles_y = ceil_div(sosg.ny, kTile);
    rays_adj_tile_kernel<<<tiles_x * tiles_y, kAdjThreads, lds, as_stream(stream)>>>(
        sos, v0, centres, N, ring.n_elem, ring.radius, ring.phi0, n_samples, make_geo(sosg, n_samples), tiles_x,
        dL_dw, scale, accumulate, dL_dsos);
    return launch_status("pact_sos_to_delays_adjoint");
}

namespace pact {
namespace {

void set_tiling(int N, const pact_ring& ring, int n_samples, const pact_grid& sosg, RayTiling t) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuned[tune_key(N, ring, n_samples, sosg)] = t;
}

// Median time (ms) of `reps` runs of fn on the stream, by HIP events; negative on an error, with the
// call's own status in `status` (PACT_EHIP for an event failure).
template <typename F>
float time_ms(F fn, hipStream_t st, int reps, int& status) {
    status = PACT_EHIP;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1.0f;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -1.0f;
    }
    std::vector<float> t;
    float out = -1.0f;
    for (int r = 0; r <= reps; ++r) {                    // the first run warms up
        if (hipEventRecord(a, st) != hipSuccess) break;
        const int s = fn();
        if (s != PACT_OK) {
            status = s;
            break;
        }
        if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess) break;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, a, b) != hipSuccess) break;
        if (r > 0) t.push_back(ms);
    }
    if (static_cast<int>(t.size()) == reps) {
        std::sort(t.begin(), t.end());
        out = t[t.size() / 2];
        status = PACT_OK;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return out;
}

}  // namespace
}  // namespace pact

extern "C" int pact_rays_autotune(const float* sos, const pact_grid* sosg_, float v0, const float* centres, int N,
                                  const pact_ring* ring_, int n_samples, const float* dL_dw, float* w,
                                  float* dL_dsos, void* ws, size_t ws_bytes, int* tiling, void* stream) {
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(sosg_ && ring_ && dL_dw && w && dL_dsos, "pact_rays_autotune: null pointer");
    const pact_grid sosg = *sosg_;
    const pact_ring ring = *ring_;
    if (int s = check_rays(sos, sosg, v0, centres, N, ring, n_samples, "pact_rays_autotune")) return s;
    hipStream_t st = as_stream(stream);
    const long long n_rays = static_cast<long long>(N) * ring.n_elem;
    const int reps = 5;
    set_tiling(N, ring, n_samples, sosg, RayTiling());   // time every candidate from a clean table
    // forward: powers of two from 1 to 64 lanes per ray with at least 8 samples a lane
    RayTiling best;
    float best_ms = -1.0f;
    for (int K = 1; K <= 64 && n_samples / K >= 8; K *= 2) {
        if (n_rays * K >= (1LL << 31)) break;
        set_tiling(N, ring, n_samples, sosg, RayTiling{K, 0});
        int status = PACT_OK;
        const float ms = time_ms([&] { return pact_sos_to_delays(sos, &sosg, v0, centres, N, &ring, n_samples, w,
                                                                 stream); }, st, reps, status);
        if (ms < 0.0f) {
            set_tiling(N, ring, n_samples, sosg, RayTiling());
            if (status == PACT_EHIP) set_error("pact_rays_autotune: timing events failed");
            return status;
        }
        if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            best.fwd = K;
        }
    }
    // adjoint (grid form only): segments per ray around the built-in rule
    if (const AdjPlan plan = adj_plan(sosg); plan.bands) {
        const long long per_band = std::max(1, device_cu_count() / plan.bands);
        const int rule = adj_segments(n_rays, n_samples, per_band * kGridThreads);
        std::vector<int> cand = {rule, rule - 1, rule + 1, rule / 2, rule * 2, 1, 2, 4, 8, 16};
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        best_ms = -1.0f;
        for (int K : cand) {
            if (K < 1 || K > std::max(1, n_samples / 4) || n_rays * K >= (1LL << 31)) continue;
            set_tiling(N, ring, n_samples, sosg, RayTiling{best.fwd, K});
            int status = PACT_OK;
            const float ms = time_ms([&] { return pact_sos_to_delays_adjoint(sos, &sosg, v0, centres, N, &ring,
                                                                             n_samples, dL_dw, nullptr, dL_dsos, 0,
                                                                             ws, ws_bytes, stream); }, st, reps,
                                     status);
            if (ms < 0.0f) {
                set_tiling(N, ring, n_samples, sosg, RayTiling());
                if (status == PACT_EHIP) set_error("pact_rays_autotune: timing events failed");
                return status;
            }
            if (best_ms < 0.0f || ms < best_ms) {
                best_ms = ms;
                best.adj = K;
            }
        }
    }
    set_tiling(N, ring, n_samples, sosg, best);
    if (tiling) {
        tiling[0] = best.fwd;
        tiling[1] = best.adj;
    }
    return PACT_OK;
}
