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
#include <cstring>
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
    // support disc (0: none): nodes whose centre lies farther than sqrt(rho2) (mm) from the origin are taken
    // as v0 and get no gradient; samples farther than sqrt(rc2) touch no node of the disc
    float rho2, rc2;
    float ds;           // node spacing (mm)
};

// Node (padded row r, padded column c) lies in the support disc.  y2 is the squared y coordinate of row r.
__device__ __forceinline__ bool node_in_support(int c, float y2, const RayGeo& g) {
    const float x = (static_cast<float>(c) - g.off_x) * g.ds;
    return !(g.rho2 > 0.0f) || fmaf(x, x, y2) <= g.rho2;
}

__device__ __forceinline__ float row_y2(int r, const RayGeo& g) {
    const float y = (static_cast<float>(r) - g.off_y) * g.ds;
    return y * y;
}

// Element positions, computed by the same code in every kernel that traces rays: the angle in revolutions,
// n / n_elem + phi0 / (2 pi), through the short sin / cos polynomials.
__device__ __forceinline__ void element_position(int n, int n_elem, float R, float phi0, float& ex, float& ey) {
    float sn, cs;
    sincos_rev(fmaf(phi0, 0.159154943091895335769f, static_cast<float>(n) / static_cast<float>(n_elem)), sn, cs);
    ex = R * cs;
    ey = R * sn;
}

__device__ __forceinline__ void load_elements(float* ex, float* ey, int n_elem, float R, float phi0) {
    for (int n = threadIdx.x; n < n_elem; n += blockDim.x) element_position(n, n_elem, R, phi0, ex[n], ey[n]);
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
                    const float y2 = row_y2(R0 + r, g);
#pragma unroll
                    for (int q = 0; q < kStageChunks; ++q) {
                        const int c = cb + 64 * q + lane;
                        if (c < W) {
                            const bool in = row_in && cin[q] && node_in_support(c, y2, g);
                            const float d = in ? x[k][q] - v0 : 0.0f;
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
// increment per sample step, and the step length dl = L / n_samples.  With a support disc, [sa, sb) are the
// samples that can touch one of its nodes: those within sqrt(rc2) of the origin, found from the ray's chord
// through that disc with one sample of margin at each end (empty if the ray misses it); else all samples.
// The samples outside add exactly zero to the forward sum (every node of their cell is v0) and their adjoint
// shares would land on nodes outside the support only.
__device__ __forceinline__ void ray_setup(float cx, float cy, float ex, float ey, const RayGeo& g, int Ns, float& gx0,
                                          float& gy0, float& dgx, float& dgy, float& dl, int& sa, int& sb) {
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
    sa = 0;
    sb = Ns;
    if (g.rc2 > 0.0f) {
        const float b = fmaf(cx, ux, cy * uy);
        const float disc = fmaf(b, b, g.rc2 - fmaf(cx, cx, cy * cy));
        if (disc > 0.0f && dl > 0.0f) {
            // sample s sits at (s + 1/2) dl from the centre: inside for ta <= s <= tb (the one-sample margins
            // cover the rounding of the hardware square root and reciprocal)
            const float root = __builtin_amdgcn_sqrtf(disc);
            const float idl = __builtin_amdgcn_rcpf(dl);
            const float ta = fmaf(-b - root, idl, -0.5f), tb = fmaf(-b + root, idl, -0.5f);
            const float nsf = static_cast<float>(Ns);
            sa = static_cast<int>(floorf(fminf(fmaxf(ta, -2.0f), nsf + 2.0f)));
            sb = static_cast<int>(floorf(fminf(fmaxf(tb, -2.0f), nsf + 2.0f))) + 2;
            sa = max(sa, 0);
            sb = min(sb, Ns);
            if (sb < sa) sb = sa;
        } else {
            sb = 0;
        }
    }
}

// The same rows from a staged contrast grid (what stage_kernel writes, [Gy + 2][W]): a plain copy of padded rows
// R0 .. R0 + H - 1 into vs, four floats a load where the rows start on a 16-byte boundary, each lane's loads all
// issued before it stores any; acc (if given) cleared; vmin and nan_check as in stage_contrast.
constexpr int kCopyBatch = 8;     // float4 loads in flight per lane (one pass covers 32768 floats at 1024 lanes)

__device__ __forceinline__ void copy_staged(const float* __restrict__ staged, float v0, const RayGeo& g, float* vs,
                                            int* acc, int R0, int H, float& vmin, float& nan_check) {
    const int n = H * g.W;
    const float* src = staged + static_cast<size_t>(R0) * g.W;
    const int nt = static_cast<int>(blockDim.x);
    float dmin = 0.0f;
    int head = 0;                 // floats copied by the vector loop
    if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
        const int n4 = n >> 2;
        const float4* s4 = reinterpret_cast<const float4*>(src);
        float4* d4 = reinterpret_cast<float4*>(vs);
        for (int j0 = threadIdx.x; j0 < n4; j0 += kCopyBatch * nt) {
            float4 x[kCopyBatch];
#pragma unroll
            for (int k = 0; k < kCopyBatch; ++k) {
                const int j = j0 + k * nt;
                x[k] = j < n4 ? s4[j] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
#pragma unroll
            for (int k = 0; k < kCopyBatch; ++k) {
                const int j = j0 + k * nt;
                if (j < n4) d4[j] = x[k];
                dmin = fminf(dmin, fminf(fminf(x[k].x, x[k].y), fminf(x[k].z, x[k].w)));
                nan_check += 0.0f * ((x[k].x + x[k].y) + (x[k].z + x[k].w));
            }
        }
        head = n4 << 2;
    }
    for (int j = head + static_cast<int>(threadIdx.x); j < n; j += nt) {
        const float d = src[j];
        vs[j] = d;
        dmin = fminf(dmin, d);
        nan_check += 0.0f * d;
    }
    vmin = fminf(vmin, v0 + dmin);
    if (acc) {
        if ((reinterpret_cast<uintptr_t>(acc) & 15) == 0) {
            int4* a4 = reinterpret_cast<int4*>(acc);
            for (int j = threadIdx.x; j < (n >> 2); j += nt) a4[j] = make_int4(0, 0, 0, 0);
            for (int j = ((n >> 2) << 2) + static_cast<int>(threadIdx.x); j < n; j += nt) acc[j] = 0;
        } else {
            for (int j = threadIdx.x; j < n; j += nt) acc[j] = 0;
        }
    }
}

// The staged contrast grid of sos: padded node (r, c) (grid node (r - 1, c - 1)) holds sos - v0 where that node
// lies in the grid and in the support disc, 0 elsewhere, exactly as stage_contrast forms it.
__global__ __launch_bounds__(256) void stage_kernel(const float* __restrict__ sos, float v0, RayGeo g,
                                                    float* __restrict__ staged) {
    const int H = g.Gy + 2;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= H * g.W) return;
    const int r = j / g.W, c = j - r * g.W;
    const int a = r - 1, b = c - 1;
    const bool in = a >= 0 && a < g.Gy && b >= 0 && b < g.Gx && node_in_support(c, row_y2(r, g), g);
    staged[j] = in ? sos[a * g.Gx + b] - v0 : 0.0f;
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

// Sum of the integrand delta / (v0 + delta) over the samples first, first + stride, ... below end, two at a time
// (two gathers in flight).
template <bool kClamp>
__device__ __forceinline__ float fwd_samples(const float* vs, int first, int stride, int end, float v0, float gx0,
                                             float gy0, float dgx, float dgy, const RayGeo& g) {
    float acc0 = 0.0f, acc1 = 0.0f;
    // the loop runs on the sample's float coordinate alone (exact: sample counts are far below 2^24)
    const float st = static_cast<float>(stride);
    float sf = static_cast<float>(first) + 0.5f;
    const float sf_end = static_cast<float>(end);
    for (; sf + st < sf_end; sf += 2.0f * st) {
        const float d0 = contrast_sample<kClamp>(vs, sf, gx0, gy0, dgx, dgy, g);
        const float d1 = contrast_sample<kClamp>(vs, sf + st, gx0, gy0, dgx, dgy, g);
        acc0 = fmaf(d0, __builtin_amdgcn_rcpf(v0 + d0), acc0);
        acc1 = fmaf(d1, __builtin_amdgcn_rcpf(v0 + d1), acc1);
    }
    if (sf < sf_end) {
        const float d0 = contrast_sample<kClamp>(vs, sf, gx0, gy0, dgx, dgy, g);
        acc0 = fmaf(d0, __builtin_amdgcn_rcpf(v0 + d0), acc0);
    }
    return acc0 + acc1;
}

// Workgroups are dealt to the 8 XCDs of the GPU in turn (workgroup b to XCD b mod 8), each with its own L2.  The
// ray kernels take their share of rays by this index instead of blockIdx.x, so that the workgroups of one XCD hold
// consecutive elements: their reads of dL/dw and writes of w (one float per ray, n_elem apart) then share cache
// lines within one L2 instead of writing parts of a line back from eight.  A bijection of 0 .. G - 1 for block b
// of G (a batched launch passes the scan's own block and count; its scans start on multiples of 8); correct for
// any XCD count.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int G) {
    const int q = G / kXcds, r = G - q * kXcds;
    const int x = b % kXcds;
    return x * q + min(x, r) + b / kXcds;
}

// Ray-length classes used to order a workgroup's rays (counting sort by the number of samples inside the support).
constexpr int kLenBuckets = 33;

// Bucket counts hist[0 .. kLenBuckets) -> the first slot of each bucket in the longest-first order (bucket b starts
// after every longer bucket: an exclusive suffix sum), by the first wave with shuffles; ends with a barrier.
__device__ __forceinline__ void bucket_starts(int* hist) {
    const int lane = threadIdx.x;
    if (lane < 64) {
        const int c = lane < kLenBuckets ? hist[lane] : 0;
        int s = c;                                    // inclusive suffix sum over the lanes
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_down(s, off, 64);
            if (lane + off < 64) s += t;
        }
        if (lane < kLenBuckets) hist[lane] = s - c;
    }
    __syncthreads();
}

// Workgroup b takes rays b * per_block .. (element-major: ray = n * N + i, so every workgroup holds the rays of
// about one element from every patch, and all workgroups carry about the same work).  Its rays are ordered by
// their sample counts inside the support (longest first, when the order fits in LDS) and each goes to K adjacent
// lanes (K a power of two) that take its samples in turn: the lanes of a wave then walk rays of similar length,
// and the lanes of a ray read neighbouring cells.
struct FwdArgs {
    const float* sos;
    const float* staged;
    float v0;
    const float* centres;
    int N, n_elem;
    float R, phi0;
    int Ns;
    RayGeo g;
    int log2K, n_rays, per_block, sorted;
    float* w;
};

// The forward pass of block blk of nblk (the scan's own numbering) with its LDS at vs.
__device__ __forceinline__ void rays_fwd_body(const FwdArgs& A, int blk, int nblk, float* vs) {
    const float* __restrict__ sos = A.sos;
    const float* __restrict__ staged = A.staged;
    const float v0 = A.v0;
    const float* __restrict__ centres = A.centres;
    const int N = A.N, n_elem = A.n_elem, Ns = A.Ns, log2K = A.log2K, n_rays = A.n_rays, per_block = A.per_block,
              sorted = A.sorted;
    const float R = A.R, phi0 = A.phi0;
    const RayGeo& g = A.g;
    float* __restrict__ w = A.w;
    const int K = 1 << log2K;
    const int total = (g.Gy + 2) * g.W;
    int* hist = reinterpret_cast<int*>(vs + total);        // [kLenBuckets]
    int* order = hist + kLenBuckets;                       // [n_loc] when sorted
    const int tid = threadIdx.x;
    for (int k = tid; k < kLenBuckets; k += blockDim.x) hist[k] = 0;
    {
        float vmin = v0, nan_check = 0.0f;   // not used by the forward
        if (staged)
            copy_staged(staged, v0, g, vs, nullptr, 0, g.Gy + 2, vmin, nan_check);
        else
            stage_contrast<kStageRows>(sos, v0, g, vs, nullptr, 0, g.Gy + 2, vmin, nan_check);
    }
    const int r0 = xcd_block(blk, nblk) * per_block;
    const int n_loc = max(min(per_block, n_rays - r0), 0);
    const float inv_N = 1.0f / static_cast<float>(N);
    auto setup = [&](int ray, int& i, int& n, float& gx0, float& gy0, float& dgx, float& dgy, float& dl, int& sa,
                     int& sb) {
        n = div_small(ray, N, inv_N);
        i = ray - n * N;
        float ex, ey;
        element_position(n, n_elem, R, phi0, ex, ey);
        ray_setup(centres[2 * i], centres[2 * i + 1], ex, ey, g, Ns, gx0, gy0, dgx, dgy, dl, sa, sb);
    };
    auto bucket_of = [&](int cnt) { return min(cnt * kLenBuckets / (Ns + 1), kLenBuckets - 1); };
    if (sorted) {
        __syncthreads();
        // a ray's bucket stays in its thread's register between the two passes when every ray has a thread
        const bool one_each = n_loc <= static_cast<int>(blockDim.x);
        auto bucket_of_ray = [&](int lr) {
            int i, n, sa, sb;
            float gx0, gy0, dgx, dgy, dl;
            setup(r0 + lr, i, n, gx0, gy0, dgx, dgy, dl, sa, sb);
            return bucket_of(max(sb - sa, 0));
        };
        int my_b = 0;
        for (int lr = tid; lr < n_loc; lr += blockDim.x) {
            my_b = bucket_of_ray(lr);
            atomicAdd(&hist[my_b], 1);
        }
        __syncthreads();
        bucket_starts(hist);
        for (int lr = tid; lr < n_loc; lr += blockDim.x)
            order[atomicAdd(&hist[one_each ? my_b : bucket_of_ray(lr)], 1)] = r0 + lr;
    }
    __syncthreads();
    // the K lanes of a ray are adjacent and aligned, so they enter and leave the loop together and add their
    // sums with K-wide shuffles
    const int n_items = n_loc * K;
    for (int base = 0; base < n_items; base += blockDim.x) {
        const int it = base + tid;
        const int lr = it >> log2K, k = it & (K - 1);
        float acc = 0.0f, dl = 0.0f;
        int i = 0, n = 0;
        if (it < n_items) {
            const int ray = sorted ? order[lr] : r0 + lr;
            int sa, sb;
            float gx0, gy0, dgx, dgy;
            setup(ray, i, n, gx0, gy0, dgx, dgy, dl, sa, sb);
            // lane k of the ray takes samples sa + k, sa + k + K, ...: the K lanes of a ray read neighbouring
            // cells at the same time (shared LDS words are broadcast)
            if (sa + k < sb) {
                // the clamp-free loop where the whole ray is inside the grid (the same bits)
                acc = segment_inside(sa, sb, gx0, gy0, dgx, dgy, g)
                          ? fwd_samples<false>(vs, sa + k, K, sb, v0, gx0, gy0, dgx, dgy, g)
                          : fwd_samples<true>(vs, sa + k, K, sb, v0, gx0, gy0, dgx, dgy, g);
            }
        }
        for (int off = K >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, K);
        if (it < n_items && k == 0) w[static_cast<size_t>(i) * n_elem + n] = acc * dl;
    }
}

__global__ __launch_bounds__(kThreads) void rays_fwd_kernel(FwdArgs A) {
    extern __shared__ float vs[];
    rays_fwd_body(A, blockIdx.x, gridDim.x, vs);
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
        const bool in = a >= 0 && a < g.Gy && b >= 0 && b < g.Gx && node_in_support(b + 1, row_y2(a + 1, g), g);
        dv[idx] = in ? sos[a * g.Gx + b] - v0 : 0.0f;
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
        int sa, sb;
        ray_setup(centres[2 * i], centres[2 * i + 1], ex[n], ey[n], g, Ns, gx0, gy0, dgx, dgy, dl, sa, sb);
        int s0, s1;
        clip_samples(gx0, gy0, dgx, dgy, a_lo, a_hi, b_lo, b_hi, Ns, s0, s1);
        s0 = max(s0, sa);
        s1 = min(s1, sb - 1);
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
            if (!node_in_support(b_lo + lb + 1, row_y2(a_lo + la + 1, g), g)) sum = 0.0f;
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

constexpr bool kPartialNt = true;

// Floats per partial grid: the node count rounded up to 64, so that every partial, and every run of 64 nodes in
// it, starts on a 256-byte boundary (a wave's row of loads is then two whole cache lines).
__host__ __device__ inline int partial_pitch(int ny, int nx) { return (ny * nx + 63) & ~63; }

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


// Banded form (kBanded): workgroup vb (the XCD-aware index) takes band vb % n_bands, cell rows R0 .. R1 - 1
// (padded coordinates, R0 = band band_rows), stages padded rows R0 .. R1 and accumulates the samples whose cells
// lie in its band; the workgroups of a band share out every ray segment.  Bands overlap in one row of nodes,
// which both accumulate.  Partial grid vb holds the workgroup's own rows only (the reduction reads, for each
// node, the partials of the one or two bands that hold it).
struct AdjArgs {
    const float* sos;
    const float* staged;
    float v0;
    const float* centres;
    int N, n_elem;
    float R, phi0;
    int Ns;
    RayGeo g;
    int n_rays, per_block, K, sorted, n_bands, band_rows;
    const float* dL_dw;
    const float* scale;
    float* partial;
    int* step_counter;
};

// The grid adjoint of block blk of nblk (the scan's own numbering) with its LDS at lds.
template <bool kBanded>
__device__ __forceinline__ void rays_adj_grid_body(const AdjArgs& A, int blk, int nblk, float* lds) {
    const float* __restrict__ sos = A.sos;
    const float* __restrict__ staged = A.staged;
    const float v0 = A.v0;
    const float* __restrict__ centres = A.centres;
    const int N = A.N, n_elem = A.n_elem, Ns = A.Ns, n_rays = A.n_rays, per_block = A.per_block, K = A.K,
              sorted = A.sorted, n_bands = A.n_bands, band_rows = A.band_rows;
    const float R = A.R, phi0 = A.phi0;
    const RayGeo& g = A.g;
    const float* __restrict__ dL_dw = A.dL_dw;
    const float* __restrict__ scale = A.scale;
    float* __restrict__ partial = A.partial;
    int* __restrict__ step_counter = A.step_counter;
    const int W = g.W;
    const int vb = xcd_block(blk, nblk);
    const int band = kBanded ? vb % n_bands : 0;
    const int bblock = kBanded ? vb / n_bands : vb;
    const int R0 = kBanded ? band * band_rows : 0;                        // cell rows R0 .. R1 - 1
    const int R1 = kBanded ? min(R0 + band_rows, g.Gy + 1) : g.Gy + 1;
    const int total = (R1 - R0 + 1) * W;                                  // staged padded rows R0 .. R1
    float* vs = lds;                                        // contrast with a ring of zeros
    int* acc = reinterpret_cast<int*>(vs + total);          // fixed-point sums, same layout
    float* red = reinterpret_cast<float*>(acc + total);     // kGridThreads / 64 floats
    const int tid = threadIdx.x;
    float vmin = v0, nan_check = 0.0f;                     // nan_check turns NaN if any node is not finite
    if (staged)
        copy_staged(staged, v0, g, vs, acc, R0, R1 - R0 + 1, vmin, nan_check);
    else
        stage_contrast<kStageRows>(sos, v0, g, vs, acc, R0, R1 - R0 + 1, vmin, nan_check);
    vmin = -block_max(-vmin, red);
    const int r0 = bblock * per_block;                      // this workgroup's rays r0 .. r1 - 1 (element-major)
    const int r1 = min(r0 + per_block, n_rays);
    const int n_loc = max(r1 - r0, 0);
    const float inv_N = 1.0f / static_cast<float>(N), inv_K = 1.0f / static_cast<float>(K);
    const float sc = (scale ? *scale : 1.0f) * v0;
    const float ds = 1.0f / g.inv_ds;
    // LDS after the grid arrays: the bucket counters and, if they fit, this workgroup's rays in order of length
    int* hist = reinterpret_cast<int*>(red + kGridThreads / 64);     // [kLenBuckets]
    int* order = hist + kLenBuckets;                                   // [n_loc] when sorted
    for (int k = tid; k < kLenBuckets; k += blockDim.x) hist[k] = 0;
    __syncthreads();
    // bound on any node's sum over this workgroup's rays, and a histogram of the rays' sample counts inside the
    // support (and band)
    auto ray_count = [&](int ray, float& contrib) {
        const int n = div_small(ray, N, inv_N), i = ray - n * N;
        float ex, ey;
        element_position(n, n_elem, R, phi0, ex, ey);
        float gx0, gy0, dgx, dgy, dl;
        int sa, sb;
        ray_setup(centres[2 * i], centres[2 * i + 1], ex, ey, g, Ns, gx0, gy0, dgx, dgy, dl, sa, sb);
        contrib = fabsf(dL_dw[static_cast<size_t>(i) * n_elem + n] * sc) * (2.8285f * ds + dl);
        if (kBanded) band_samples(sa, sb, gy0, dgy, R0, R1, sa, sb);
        return max(sb - sa, 0);
    };
    auto bucket_of = [&](int cnt) { return min(cnt * kLenBuckets / (Ns + 1), kLenBuckets - 1); };
    float bnd = 0.0f;
    const bool one_each = n_loc <= static_cast<int>(blockDim.x);   // then a ray's bucket stays in a register
    int my_b = 0;
    for (int lr = tid; lr < n_loc; lr += blockDim.x) {
        float c;
        const int cnt = ray_count(r0 + lr, c);
        bnd += c;
        my_b = bucket_of(cnt);
        if (sorted) atomicAdd(&hist[my_b], 1);
    }
    bnd = block_sum(bnd + nan_check, red) / (vmin * vmin);
    const bool ok = vmin > 0.0f && bnd <= 3.0e38f;        // false for NaN or infinite bounds too
    const float F = (ok && bnd > 0.0f) ? ldexpf(1.0f, min(30 - (ilogbf(bnd) + 1), 126)) : 1.0f;
    if (sorted) {
        bucket_starts(hist);     // the barriers of block_sum above ordered the counts
        for (int lr = tid; lr < n_loc; lr += blockDim.x) {
            int b = my_b;
            if (!one_each) {
                float c;
                b = bucket_of(ray_count(r0 + lr, c));
            }
            order[atomicAdd(&hist[b], 1)] = r0 + lr;
        }
    }
    __syncthreads();

    // Work items: K segments of each ray's samples inside the support (and band), dealt to the lanes in the order
    // of the rays' lengths (with the order not stored, in element-major order), so that the lanes of a wave walk
    // segments of similar length; neighbouring lanes still walk parallel rays from different patch centres, which
    // rarely meet at one node.  The order within a bucket varies between runs; the integer sums do not depend on it.
    const int cbase = R0 * W, band_cells = (R1 - R0) * W;
    for (int it = tid; it < n_loc * K; it += blockDim.x) {
        const int lr = div_small(it, K, inv_K), k = it - lr * K;
        const int ray = sorted ? order[lr] : r0 + lr;
        const int n = div_small(ray, N, inv_N), i = ray - n * N;
        float ex, ey;
        element_position(n, n_elem, R, phi0, ex, ey);
        float gx0, gy0, dgx, dgy, dl;
        int sa, sb;
        ray_setup(centres[2 * i], centres[2 * i + 1], ex, ey, g, Ns, gx0, gy0, dgx, dgy, dl, sa, sb);
        const float q0 = ok ? dL_dw[static_cast<size_t>(i) * n_elem + n] * dl * sc * F : 0.0f;
        if (kBanded) band_samples(sa, sb, gy0, dgy, R0, R1, sa, sb);
        const int cnt = max(sb - sa, 0);
        const int s0 = sa + div_small(k * cnt, K, inv_K), s1 = sa + div_small((k + 1) * cnt, K, inv_K);
        if (s1 > s0) {
            // the clamp-free loop where the whole segment is inside the grid (the same bits)
            if (segment_inside(s0, s1, gx0, gy0, dgx, dgy, g))
                adj_segment<false, kBanded>(vs, acc, s0, s1, v0, q0, gx0, gy0, dgx, dgy, g, cbase, band_cells);
            else
                adj_segment<true, kBanded>(vs, acc, s0, s1, v0, q0, gx0, gy0, dgx, dgy, g, cbase, band_cells);
        }
    }
    __syncthreads();
    // the optimisation step's counter (no other workgroup of this launch touches it; the update kernel that
    // follows reads the new value)
    if (step_counter && blk == 0 && tid == 0) step_counter[0] += 1;
    const float invF = 1.0f / F;
    const float bad = __builtin_nanf("");
    float* part = partial + static_cast<size_t>(vb) * partial_pitch(g.Gy, g.Gx);
    // rows per wave and columns per lane, as in the staging; grid row a is padded row a + 1, held in this
    // workgroup's rows when R0 <= a + 1 <= R1 (the only rows it writes)
    {
        const int lane = tid & 63;
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int a0 = kBanded ? max(R0 - 1, 0) : 0, a1 = kBanded ? min(R1 - 1, g.Gy - 1) : g.Gy - 1;
        for (int a = a0 + wave; a <= a1; a += kGridThreads / 64) {
            const float y2 = row_y2(a + 1, g);
            for (int b = lane; b < g.Gx; b += 64) {
                // nodes outside the support are not written: the readers of the partials take them as zero
                if (!node_in_support(b + 1, y2, g)) continue;
                const float val = !ok ? bad : static_cast<float>(acc[(a + 1 - R0) * W + b + 1]) * invF;
                if (kPartialNt)
                    __builtin_nontemporal_store(val, part + a * g.Gx + b);
                else
                    part[a * g.Gx + b] = val;
            }
        }
    }
}

template <bool kBanded>
__global__ __launch_bounds__(kGridThreads) void rays_adj_grid_kernel(AdjArgs A) {
    extern __shared__ float lds[];
    rays_adj_grid_body<kBanded>(A, blockIdx.x, gridDim.x, lds);
}

// Sum of the per-workgroup partial grids in a fixed order.  A workgroup owns 64 consecutive nodes; its
// wave s sums, for those nodes, the s-th of kAdjSlices contiguous runs of partials (in order), so that
// every load of a wave is one 256-byte row and each lane has 16 loads in flight; the run sums then meet in
// LDS and are added in order (= or += into out).
constexpr int kAdjSlices = 16;

// Partials of the grid adjoint as the reduction sees them: n_bands bands of band_rows padded cell rows, per_band
// partials each; partial vb belongs to band vb % n_bands (one band: every partial).
struct PartialSet {
    const float* base;
    int pitch, n_bands, band_rows, per_band;
};

// The sum, in order, of `count` partials at one node, from partial index first in steps of `stride`, 16 loads
// in flight.  The loads address the partials by 32-bit byte offsets from their base (the host keeps the buffer
// below 4 GiB), one register per address.
__device__ __forceinline__ float strided_partial_sum(const PartialSet& ps, int first, int count, int stride,
                                                     int node, float s) {
    constexpr int B = 16;
    const char* base = reinterpret_cast<const char*>(ps.base);
    const unsigned step = static_cast<unsigned>(stride) * static_cast<unsigned>(ps.pitch) * 4u;
    unsigned off = static_cast<unsigned>(first) * static_cast<unsigned>(ps.pitch) * 4u + static_cast<unsigned>(node) * 4u;
    for (int k = 0; k < count; k += B) {
        float v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const unsigned o = k + u < count ? off + u * step : off;    // past the run: a load that is not used
            v[u] = *reinterpret_cast<const float*>(base + o);
        }
#pragma unroll
        for (int u = 0; u < B; ++u) s = k + u < count ? s + v[u] : s;
        off += B * step;
    }
    return s;
}

// Run `slice` of the kAdjSlices contiguous runs of the list of partials that hold grid node `node` (row a), added
// in order: the partials of the band above (when the node's padded row a + 1 is the first row of a band, the
// previous band's last row), then those of the node's band.
__device__ __forceinline__ float adj_run_sum(const PartialSet& ps, int node, int a, int slice) {
    const int r = a + 1;
    const int k1 = min(r / ps.band_rows, ps.n_bands - 1);
    const int k0 = (k1 > 0 && r == k1 * ps.band_rows) ? k1 - 1 : -1;
    const int m = ps.per_band * (k0 >= 0 ? 2 : 1);
    const int per = (m + kAdjSlices - 1) / kAdjSlices;
    const int q0 = min(slice * per, m), q1 = min(q0 + per, m);
    float s = 0.0f;
    if (k0 >= 0) {
        const int e = min(q1, ps.per_band);               // list entries q0 .. e - 1 are band k0's
        if (e > q0) s = strided_partial_sum(ps, k0 + ps.n_bands * q0, e - q0, ps.n_bands, node, s);
        const int b0 = max(q0, ps.per_band) - ps.per_band, b1 = q1 - ps.per_band;
        if (b1 > b0) s = strided_partial_sum(ps, k1 + ps.n_bands * b0, b1 - b0, ps.n_bands, node, s);
    } else if (q1 > q0) {
        s = strided_partial_sum(ps, k1 + ps.n_bands * q0, q1 - q0, ps.n_bands, node, s);
    }
    return s;
}

constexpr int kReduceNodes = 64;

// Node `node` of the Gy x Gx grid lies in the support disc.
__device__ __forceinline__ bool grid_node_in_support(int node, const RayGeo& g) {
    const int a = node / g.Gx;
    return node_in_support(node - a * g.Gx + 1, row_y2(a + 1, g), g);
}

__global__ __launch_bounds__(kAdjSlices * kReduceNodes) void rays_adj_reduce_kernel(PartialSet ps, RayGeo g,
                                                                                   int accumulate,
                                                                                   float* __restrict__ out) {
    __shared__ float run[kAdjSlices][kReduceNodes];
    const int n_nodes = g.Gy * g.Gx;
    const int j = threadIdx.x % kReduceNodes, slice = threadIdx.x / kReduceNodes;
    const int node = blockIdx.x * kReduceNodes + j;
    run[slice][j] = node < n_nodes && grid_node_in_support(node, g) ? adj_run_sum(ps, node, node / g.Gx, slice)
                                                                    : 0.0f;
    __syncthreads();
    if (slice == 0 && node < n_nodes) {
        float t = 0.0f;
#pragma unroll
        for (int k = 0; k < kAdjSlices; ++k) t += run[k][j];
        out[node] = accumulate ? out[node] + t : t;
    }
}

// The end of an optimisation step in one launch: the partial grids of the ray adjoint summed in the fixed order
// of rays_adj_reduce_kernel (the data gradient), plus the TV subgradient at sos_in, then Adam from sos_in into
// sos_out, as tv_adam_kernel does.  Only the free nodes inside the support read their partials (fixed nodes keep
// their value, and the partials of nodes outside the support are not written).  The TV value is added to the
// loss with one float atomic per workgroup (loss may be null).  The step counter t[0] was advanced by the grid
// adjoint launched just before (so no workgroup here writes it, and none needs an arrival counter).  Two
// workgroups fit on a CU (eight waves per SIMD: at most 64 VGPRs), so that every workgroup of the 140^2 grid
// is resident at once.
struct UpdArgs {
    PartialSet ps;
    RayGeo g;
    const float* sos_in;
    float* sos_out;
    float *m, *v;
    int* t;
    const unsigned char* mask;
    float lambda;
    float* loss;
    float lr, b1, b2, eps;
    float* grad_out;
    float v0;
    float* staged_out;
};

// The update of nodes blk * 64 .. with the LDS arrays run and red.
__device__ __forceinline__ void adj_reduce_tv_adam_body(const UpdArgs& A, int blk, float (&run)[kAdjSlices][kReduceNodes],
                                                        float* red) {
    const PartialSet& ps = A.ps;
    const RayGeo& g = A.g;
    const float* __restrict__ sos_in = A.sos_in;
    float* __restrict__ sos_out = A.sos_out;
    float* __restrict__ m = A.m;
    float* __restrict__ v = A.v;
    const int* __restrict__ t = A.t;
    const unsigned char* __restrict__ mask = A.mask;
    const float lambda = A.lambda, lr = A.lr, b1 = A.b1, b2 = A.b2, eps = A.eps, v0 = A.v0;
    float* __restrict__ loss = A.loss;
    float* __restrict__ grad_out = A.grad_out;
    float* __restrict__ staged_out = A.staged_out;
    const int step = t[0];          // already advanced by the adjoint launch before this one
    const int n_nodes = g.Gy * g.Gx;
    const int j = threadIdx.x % kReduceNodes, slice = threadIdx.x / kReduceNodes;
    const int node = blk * kReduceNodes + j;
    const bool valid = node < n_nodes;
    const bool is_free = valid && mask[node] != 0;
    // the update's own loads go out before the partial sums, so that their latency is hidden behind them
    const int nd = valid ? node : 0;
    const int a = nd / g.Gx, b = nd - a * g.Gx;
    float tv = 0.0f, g_tv = 0.0f, mm = 0.0f, vv = 0.0f, p = 0.0f;
    if (slice == 0) {
        mm = m[nd];
        vv = v[nd];
        p = sos_in[nd];
        if (lambda != 0.0f) tv_node(sos_in, mask, nd, a, b, g.Gy, g.Gx, tv, g_tv);
        if (!valid) tv = 0.0f;
    }
    run[slice][j] = is_free && grid_node_in_support(node, g) ? adj_run_sum(ps, node, a, slice) : 0.0f;
    __syncthreads();
    if (slice == 0 && valid) {
        float gd = 0.0f;
#pragma unroll
        for (int k = 0; k < kAdjSlices; ++k) gd += run[k][j];
        if (grad_out) grad_out[node] = gd;
        if (is_free) {
            p = adam_node(p, fmaf(lambda, g_tv, gd), mm, vv, step, lr, b1, b2, eps);
            m[node] = mm;
            v[node] = vv;
        }
        sos_out[node] = p;
        if (staged_out) {
            // the staged contrast of sos_out (as stage_kernel forms it), with the ring of zeros next to the
            // grid's edge nodes
            const int W = g.W;
            float* row = staged_out + static_cast<size_t>(a + 1) * W;
            row[b + 1] = node_in_support(b + 1, row_y2(a + 1, g), g) ? p - v0 : 0.0f;
            if (b == 0) row[0] = 0.0f;
            if (b == g.Gx - 1) row[W - 1] = 0.0f;
            if (a == 0) {
                staged_out[b + 1] = 0.0f;
                if (b == 0) staged_out[0] = 0.0f;
                if (b == g.Gx - 1) staged_out[W - 1] = 0.0f;
            }
            if (a == g.Gy - 1) {
                float* last = staged_out + static_cast<size_t>(g.Gy + 1) * W;
                last[b + 1] = 0.0f;
                if (b == 0) last[0] = 0.0f;
                if (b == g.Gx - 1) last[W - 1] = 0.0f;
            }
        }
    }
    if (loss) {
        tv = block_sum(tv, red);
        if (threadIdx.x == 0 && tv != 0.0f) atomicAdd(loss, lambda * tv);
    }
}

__global__ __launch_bounds__(kAdjSlices * kReduceNodes, 8) void adj_reduce_tv_adam_kernel(UpdArgs A) {
    __shared__ float run[kAdjSlices][kReduceNodes];
    __shared__ float red[kAdjSlices * kReduceNodes / 64];
    adj_reduce_tv_adam_body(A, blockIdx.x, run, red);
}

RayGeo make_geo(const pact_grid& sosg, int n_samples, float support) {
    RayGeo g;
    // support disc: a node counts as inside within a relative margin of 1e-6 (so that a node the caller places
    // exactly on the radius is inside whatever the rounding); a sample can touch an inside node when it lies
    // within the disc grown by the cell diagonal (and a margin for rounding)
    const double rho = support > 0.0f ? static_cast<double>(support) * (1.0 + 1e-6) : 0.0;
    g.rho2 = static_cast<float>(rho * rho);
    const double rc = rho > 0.0 ? rho + std::sqrt(2.0) * sosg.spacing * 1.001 : 0.0;
    g.rc2 = static_cast<float>(rc * rc);
    g.ds = sosg.spacing;
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
               int n_samples, float support, const char* what) {
    PACT_CHECK_ARG(support >= 0.0f && std::isfinite(support), "%s: support_radius must be finite and >= 0", what);
    PACT_CHECK_ARG(sos && centres, "%s: null pointer", what);
    PACT_CHECK_ARG(N > 0 && n_samples > 0, "%s: N and n_samples must be positive", what);
    PACT_CHECK_ARG(v0 > 0.0f && std::isfinite(v0), "%s: v0 must be positive", what);
    if (int s = check_ring(ring)) return s;
    if (int s = check_grid(sosg, what)) return s;
    PACT_CHECK_SUPPORTED(static_cast<long long>(N) * ring.n_elem < (1LL << 31), "%s: too many rays", what);
    return PACT_OK;
}

// Ray tilings chosen by pact_rays_autotune, per device and geometry: lanes per ray of the forward kernel (0 = the
// built-in rule).  The adjoint's work items have a fixed length and need no tuning.
// device, N, n_elem, n_samples, ny, nx, support radius (bits)
using TuneKey = std::tuple<int, int, int, int, int, int, unsigned>;
struct RayTiling {
    int fwd = 0;
};
std::mutex g_tune_mu;
std::map<TuneKey, RayTiling> g_tuned;

TuneKey tune_key(int N, const pact_ring& ring, int n_samples, const pact_grid& sosg, float support) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    unsigned bits = 0;
    std::memcpy(&bits, &support, sizeof(bits));
    return TuneKey(dev, N, ring.n_elem, n_samples, sosg.ny, sosg.nx, bits);
}

RayTiling tuned_tiling(int N, const pact_ring& ring, int n_samples, const pact_grid& sosg, float support) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tuned.find(tune_key(N, ring, n_samples, sosg, support));
    return it == g_tuned.end() ? RayTiling() : it->second;
}

// Lanes per ray of the forward kernel by the built-in rule: the largest power of two (at most 64, at least 8
// samples a segment) with which a workgroup's rays fill its lanes in one round.
int fwd_lanes_rule(int per_block, int n_samples) {
    int K = 1;
    while (K < 64 && 2 * K * per_block <= kThreads && n_samples / (2 * K) >= 8) K *= 2;
    return K;
}

}  // namespace
}  // namespace pact

namespace pact {
namespace {

// The forward launch of one scan (arguments already checked): its kernel arguments, workgroups and LDS bytes.
// Two workgroups per CU, each with about the same number of rays (element-major, so about one element's rays
// from every patch); lanes per ray: the autotuned value for this geometry, else the built-in rule; the rays'
// order by length when it fits beside the staged grid.
int plan_fwd(const float* sos, const float* staged, const pact_grid& sosg, float v0, const float* centres, int N,
             const pact_ring& ring, int n_samples, float support_radius, float* w, FwdArgs* A, int* blocks,
             size_t* lds, const char* what) {
    const size_t grid_lds = static_cast<size_t>(sosg.ny + 2) * (sosg.nx + 2) * sizeof(float);
    PACT_CHECK_SUPPORTED(grid_lds + kLenBuckets * sizeof(int) <= kLdsBytes, "%s: SOS grid %d x %d does not fit in LDS",
                         what, sosg.ny, sosg.nx);
    const long long n_rays = static_cast<long long>(N) * ring.n_elem;
    // ray indices are split by float quotients, exact below 2^24
    PACT_CHECK_SUPPORTED(n_rays < (1LL << 24), "%s: too many rays", what);
    *blocks = static_cast<int>(std::min<long long>(2LL * device_cu_count(), n_rays));
    const int per_block = ceil_div(n_rays, *blocks);
    const int tuned = tuned_tiling(N, ring, n_samples, sosg, support_radius).fwd;
    const int K = tuned > 0 ? tuned : fwd_lanes_rule(per_block, n_samples);
    int log2K = 0;
    while ((1 << log2K) < K) ++log2K;
    PACT_CHECK_ARG((1 << log2K) == K, "%s: lanes per ray must be a power of two", what);
    const size_t base = grid_lds + kLenBuckets * sizeof(int);
    const size_t with_order = base + static_cast<size_t>(per_block) * sizeof(int);
    const int sorted = with_order <= kLdsBytes ? 1 : 0;
    *lds = sorted ? with_order : base;
    *A = FwdArgs{sos, staged, v0, centres, N, ring.n_elem, ring.radius, ring.phi0, n_samples,
                 make_geo(sosg, n_samples, support_radius), log2K, static_cast<int>(n_rays), per_block, sorted, w};
    return PACT_OK;
}

void fwd_lds_attribute() {
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(rays_fwd_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        attr = true;
    }
}

}  // namespace
}  // namespace pact

extern "C" int pact_sos_to_delays(const float* sos, const pact_grid* sosg_, float v0, const float* centres, int N,
                                  const pact_ring* ring_, int n_samples, float support_radius, const float* staged,
                                  float* w, void* stream) {
    if (!sosg_ || !ring_) {
        pact::set_error("pact_sos_to_delays: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_grid sosg = *sosg_;
    const pact_ring ring = *ring_;
    using namespace pact;
    clear_error();
    if (int s = check_rays(sos, sosg, v0, centres, N, ring, n_samples, support_radius, "pact_sos_to_delays"))
        return s;
    PACT_CHECK_ARG(w, "pact_sos_to_delays: null output");
    FwdArgs A;
    int blocks = 0;
    size_t lds = 0;
    if (int s = plan_fwd(sos, staged, sosg, v0, centres, N, ring, n_samples, support_radius, w, &A, &blocks, &lds,
                         "pact_sos_to_delays"))
        return s;
    fwd_lds_attribute();
    rays_fwd_kernel<<<blocks, kThreads, lds, as_stream(stream)>>>(A);
    return launch_status("pact_sos_to_delays");
}

namespace pact {
namespace {

// Layout of rays_adj_grid_kernel for a grid: bands of band_rows cell rows (1 band: the whole grid) and the
// LDS bytes of one band; bands == 0 if even bands of 8 rows do not fit (the tile kernel is used instead).
// Bands of the grid adjoint.  A workgroup holds its band's contrast and accumulator in LDS (padded rows R0 .. R1,
// one row shared with the next band) and writes a partial grid of those rows only, so with more bands fewer
// partial bytes are written and read back (each band's workgroups walk only the samples inside the band, and set
// up every ray).  Grids are cut into kAdjBands bands of at least kAdjMinBandRows rows where they have the rows
// (one band below 2 kAdjMinBandRows), more where a band would not fit in LDS; kAdjWgsPerCu workgroups share a
// CU where their LDS allows.
constexpr int kAdjBands = 1;
constexpr int kAdjMinBandRows = 16;
constexpr int kAdjWgsPerCu = 1;

struct AdjPlan {
    int bands, band_rows;
    size_t lds;        // without the ray order list
};

AdjPlan adj_plan(const pact_grid& sosg) {
    const size_t W = static_cast<size_t>(sosg.nx) + 2;
    // after the grid arrays: the block reduction's slots and the ray-length buckets
    const size_t red = (kGridThreads / 64) * sizeof(float) + kLenBuckets * sizeof(int);
    const long long max_rows = static_cast<long long>((kLdsBytes - red) / (2 * W * sizeof(float))) - 1;
    if (max_rows < 8) return {0, 0, 0};
    const int cell_rows = sosg.ny + 1;
    const int fit = ceil_div(cell_rows, static_cast<int>(std::min<long long>(max_rows, cell_rows)));
    const int bands = std::max(fit, std::min(kAdjBands, std::max(1, cell_rows / kAdjMinBandRows)));
    if (bands > 64) return {0, 0, 0};
    const int rows = ceil_div(cell_rows, bands);                 // balanced bands
    return {bands, rows, 2 * (static_cast<size_t>(rows) + 1) * W * sizeof(float) + red};
}

// Workgroups of the grid adjoint: per band, and in all.
int adj_per_band(const AdjPlan& plan, int cus) {
    const int per_cu = std::max<int>(1, std::min<size_t>(kAdjWgsPerCu, kLdsBytes / (plan.lds + 4096)));
    return std::max(1, ceil_div(cus * per_cu, plan.bands));
}

size_t adj_grid_lds(const pact_grid& sosg) { return adj_plan(sosg).bands ? adj_plan(sosg).lds : 0; }

// The grid adjoint of one scan (arguments already checked): its kernel arguments, workgroups, LDS bytes and the
// partial grids it leaves for the reduction (one per workgroup, rows of its band only).
int plan_adj_grid(const float* sos, const float* staged, const pact_grid& sosg, float v0, const float* centres,
                  int N, const pact_ring& ring, int n_samples, float support, const float* dL_dw, const float* scale,
                  float* partial, size_t ws_bytes, int* step_counter, AdjArgs* A, int* blocks, size_t* lds,
                  PartialSet* ps, const char* what) {
    const AdjPlan plan = adj_plan(sosg);
    const int per_band = adj_per_band(plan, device_cu_count());
    *blocks = plan.bands * per_band;
    const size_t need = static_cast<size_t>(*blocks) * partial_pitch(sosg.ny, sosg.nx) * sizeof(float);
    PACT_CHECK_SUPPORTED(need < (size_t{1} << 32), "%s: the adjoint's partial grids exceed 4 GiB", what);
    if (!partial || ws_bytes < need) {
        set_error("%s: workspace of %zu bytes needed, %zu given", what, need, partial ? ws_bytes : 0);
        return PACT_EWORKSPACE;
    }
    const long long n_rays = static_cast<long long>(N) * ring.n_elem;
    // ray and item indices are split by float quotients, exact below 2^24
    PACT_CHECK_SUPPORTED(n_rays < (1LL << 24), "%s: too many rays", what);
    const int per_block = ceil_div(n_rays, per_band);
    // segments per ray: as many as fill the workgroup's lanes in one round with one band's rays (at least 8
    // samples a segment); a band's segments are about 1 / bands of a ray, but its longest are whole rays, so
    // with several bands each lane takes several short segments instead of one long one
    const int K = std::max(1, std::min(kGridThreads * plan.bands / std::max(per_block, 1), std::max(1, n_samples / 8)));
    // the rays in order of length, if the workgroup's list fits beside the grid arrays
    const size_t order_bytes = static_cast<size_t>(per_block) * sizeof(int);
    const int sorted = plan.lds + order_bytes <= kLdsBytes ? 1 : 0;
    *lds = plan.lds + (sorted ? order_bytes : 0);
    *A = AdjArgs{sos, staged, v0, centres, N, ring.n_elem, ring.radius, ring.phi0, n_samples,
                 make_geo(sosg, n_samples, support), static_cast<int>(n_rays), per_block, K, sorted, plan.bands,
                 plan.bands == 1 ? sosg.ny + 1 : plan.band_rows, dL_dw, scale, partial, step_counter};
    *ps = PartialSet{partial, partial_pitch(sosg.ny, sosg.nx), plan.bands, plan.band_rows, per_band};
    return PACT_OK;
}

void adj_lds_attribute() {
    static bool gattr = false;
    if (!gattr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(rays_adj_grid_kernel<false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(rays_adj_grid_kernel<true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        gattr = true;
    }
}

int launch_adj_grid(const float* sos, const float* staged, const pact_grid& sosg, float v0, const float* centres, int N,
                    const pact_ring& ring, int n_samples, float support, const float* dL_dw, const float* scale,
                    float* partial, size_t ws_bytes, hipStream_t st, PartialSet* ps, const char* what,
                    int* step_counter = nullptr) {
    AdjArgs A;
    int blocks = 0;
    size_t lds = 0;
    if (int s = plan_adj_grid(sos, staged, sosg, v0, centres, N, ring, n_samples, support, dL_dw, scale, partial,
                              ws_bytes, step_counter, &A, &blocks, &lds, ps, what))
        return s;
    adj_lds_attribute();
    if (A.n_bands == 1)
        rays_adj_grid_kernel<false><<<blocks, kGridThreads, lds, st>>>(A);
    else
        rays_adj_grid_kernel<true><<<blocks, kGridThreads, lds, st>>>(A);
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
    const int blocks = plan.bands * pact::adj_per_band(plan, pact::device_cu_count());
    return static_cast<size_t>(blocks) * pact::partial_pitch(sosg_->ny, sosg_->nx) * sizeof(float);
}

extern "C" int pact_sos_to_delays_adjoint(const float* sos, const pact_grid* sosg_, float v0, const float* centres,
                                          int N, const pact_ring* ring_, int n_samples, float support_radius,
                                          const float* staged, const float* dL_dw, const float* scale, float* dL_dsos, int accumulate,
                                          void* ws, size_t ws_bytes, void* stream) {
    if (!sosg_ || !ring_) {
        pact::set_error("pact_sos_to_delays_adjoint: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_grid sosg = *sosg_;
    const pact_ring ring = *ring_;
    using namespace pact;
    clear_error();
    if (int s = check_rays(sos, sosg, v0, centres, N, ring, n_samples, support_radius, "pact_sos_to_delays_adjoint"))
        return s;
    PACT_CHECK_ARG(dL_dw && dL_dsos, "pact_sos_to_delays_adjoint: null pointer");
    if (adj_grid_lds(sosg)) {
        float* partial = static_cast<float*>(ws);
        PartialSet ps;
        if (int st = launch_adj_grid(sos, staged, sosg, v0, centres, N, ring, n_samples, support_radius, dL_dw, scale,
                                     partial, ws_bytes, as_stream(stream), &ps, "pact_sos_to_delays_adjoint"))
            return st;
        const int n_nodes = sosg.ny * sosg.nx;
        rays_adj_reduce_kernel<<<ceil_div(n_nodes, kReduceNodes), kAdjSlices * kReduceNodes, 0, as_stream(stream)>>>(
            ps, make_geo(sosg, n_samples, support_radius), accumulate, dL_dsos);
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
        sos, v0, centres, N, ring.n_elem, ring.radius, ring.phi0, n_samples, make_geo(sosg, n_samples, support_radius),
        tiles_x,
        dL_dw, scale, accumulate, dL_dsos);
    return launch_status("pact_sos_to_delays_adjoint");
}

extern "C" int pact_sos_adjoint_tv_adam_step(const float* sos_in, float* sos_out, float* m, float* v, int* t,
                                             const unsigned char* mask, const pact_grid* sosg_, float v0,
                                             const float* centres, int N, const pact_ring* ring_, int n_samples,
                                             float support_radius, const float* staged_in, float* staged_out,
                                             const float* dL_dw, float lambda, float* loss, float lr, float b1,
                                             float b2, float eps, float* grad, void* ws, size_t ws_bytes,
                                             void* stream) {
    if (!sosg_ || !ring_) {
        pact::set_error("pact_sos_adjoint_tv_adam_step: null geometry pointer");
        return PACT_EINVAL;
    }
    const pact_grid sosg = *sosg_;
    const pact_ring ring = *ring_;
    using namespace pact;
    clear_error();
    const char* what = "pact_sos_adjoint_tv_adam_step";
    if (int s = check_rays(sos_in, sosg, v0, centres, N, ring, n_samples, support_radius, what)) return s;
    PACT_CHECK_ARG(sos_out && m && v && t && mask && dL_dw, "%s: null pointer", what);
    PACT_CHECK_ARG(sos_in != sos_out, "%s: sos_out must not be sos_in", what);
    PACT_CHECK_ARG(std::isfinite(lambda), "%s: lambda must be finite", what);
    PACT_CHECK_ARG(b1 >= 0.0f && b1 < 1.0f && b2 >= 0.0f && b2 < 1.0f, "%s: betas must be in [0, 1)", what);
    PACT_CHECK_ARG(eps > 0.0f && std::isfinite(lr), "%s: eps must be positive and lr finite", what);
    PACT_CHECK_SUPPORTED(adj_grid_lds(sosg) > 0, "%s: the %d x %d grid takes the tiled adjoint; use "
                         "pact_sos_to_delays_adjoint and pact_tv_adam_step", what, sosg.ny, sosg.nx);
    float* partial = static_cast<float*>(ws);
    PartialSet ps;
    PACT_CHECK_ARG(!staged_out || (staged_out != staged_in && static_cast<const float*>(staged_out) != sos_in),
                   "%s: staged_out must not alias staged_in or sos_in", what);
    if (int st = launch_adj_grid(sos_in, staged_in, sosg, v0, centres, N, ring, n_samples, support_radius, dL_dw, nullptr,
                                 partial, ws_bytes, as_stream(stream), &ps, what, t))
        return st;
    const int n_nodes = sosg.ny * sosg.nx;
    const UpdArgs U{ps, make_geo(sosg, n_samples, support_radius), sos_in, sos_out, m, v, t, mask, lambda, loss, lr,
                    b1, b2, eps, grad, v0, staged_out};
    adj_reduce_tv_adam_kernel<<<ceil_div(n_nodes, kReduceNodes), kAdjSlices * kReduceNodes, 0, as_stream(stream)>>>(U);
    return launch_status(what);
}

namespace pact {
namespace {

void set_tiling(int N, const pact_ring& ring, int n_samples, const pact_grid& sosg, float support, RayTiling t) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuned[tune_key(N, ring, n_samples, sosg, support)] = t;
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
                                  const pact_ring* ring_, int n_samples, float support_radius, const float* dL_dw,
                                  float* w,
                                  float* dL_dsos, void* ws, size_t ws_bytes, int* tiling, void* stream) {
    using namespace pact;
    clear_error();
    (void)dL_dw;
    (void)dL_dsos;
    (void)ws;
    (void)ws_bytes;
    PACT_CHECK_ARG(sosg_ && ring_ && w, "pact_rays_autotune: null pointer");
    const pact_grid sosg = *sosg_;
    const pact_ring ring = *ring_;
    if (int s = check_rays(sos, sosg, v0, centres, N, ring, n_samples, support_radius, "pact_rays_autotune"))
        return s;
    hipStream_t st = as_stream(stream);
    const long long n_rays = static_cast<long long>(N) * ring.n_elem;
    const int reps = 5;
    set_tiling(N, ring, n_samples, sosg, support_radius, RayTiling());   // time every candidate from a clean table
    // forward: powers of two from 1 to 64 lanes per ray with at least 8 samples a lane
    RayTiling best;
    float best_ms = -1.0f;
    for (int K = 1; K <= 64 && n_samples / K >= 8; K *= 2) {
        if (n_rays * K >= (1LL << 24)) break;
        set_tiling(N, ring, n_samples, sosg, support_radius, RayTiling{K});
        int status = PACT_OK;
        const float ms = time_ms([&] { return pact_sos_to_delays(sos, &sosg, v0, centres, N, &ring, n_samples,
                                                                 support_radius, nullptr, w, stream); }, st, reps, status);
        if (ms < 0.0f) {
            set_tiling(N, ring, n_samples, sosg, support_radius, RayTiling());
            if (status == PACT_EHIP) set_error("pact_rays_autotune: timing events failed");
            return status;
        }
        if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            best.fwd = K;
        }
    }
    set_tiling(N, ring, n_samples, sosg, support_radius, best);
    if (tiling) {
        tiling[0] = best.fwd;
        tiling[1] = 0;
    }
    return PACT_OK;
}

extern "C" size_t pact_staged_contrast_floats(const pact_grid* sosg) {
    if (!sosg || sosg->ny <= 0 || sosg->nx <= 0) return 0;
    return static_cast<size_t>(sosg->ny + 2) * (sosg->nx + 2);
}

extern "C" int pact_stage_contrast(const float* sos, const pact_grid* sosg_, float v0, float support_radius,
                                   float* staged, void* stream) {
    using namespace pact;
    clear_error();
    PACT_CHECK_ARG(sosg_, "pact_stage_contrast: null geometry pointer");
    const pact_grid sosg = *sosg_;
    PACT_CHECK_ARG(sos && staged, "pact_stage_contrast: null pointer");
    if (int s = check_grid(sosg, "pact_stage_contrast")) return s;
    PACT_CHECK_ARG(v0 > 0.0f && std::isfinite(v0), "pact_stage_contrast: v0 must be positive");
    PACT_CHECK_ARG(support_radius >= 0.0f && std::isfinite(support_radius),
                   "pact_stage_contrast: support_radius must be >= 0");
    const long long n = static_cast<long long>(sosg.ny + 2) * (sosg.nx + 2);
    stage_kernel<<<ceil_div(n, 256), 256, 0, as_stream(stream)>>>(sos, v0, make_geo(sosg, 1, support_radius), staged);
    return launch_status("pact_stage_contrast");
}

// ---- Batched step: the ray stages of many scans, one launch each ----
//
// Every workgroup finds its scan in the launch's block ranges and runs that scan's block with the scan's own
// block number and count, so each scan's work is split exactly as in its own launch (the same rays per
// workgroup, lanes per ray, length order, fixed-point scales and partial grids) and its results are the same.
// A launch's dynamic LDS is the largest any of its scans needs.  Forward and adjoint ranges start on multiples
// of 8 blocks, so that the XCD-aware numbering of each scan sees the hardware's dealing of blocks to XCDs.

namespace pact {
namespace {

struct RayBatchDesc {
    FwdArgs fwd;
    AdjArgs adj;
    UpdArgs upd;
    int blocks[3];      // forward, adjoint, update
};

// Position of this workgroup's scan in a launch: the last s with starts[s] <= blockIdx.x (uniform across the
// workgroup); ids[s] is that scan's descriptor.
__device__ __forceinline__ int batch_scan_of(const int* __restrict__ starts, int n) {
    const int b = static_cast<int>(blockIdx.x);
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kThreads) void rays_fwd_batch_kernel(const RayBatchDesc* __restrict__ d,
                                                                  const int* __restrict__ starts,
                                                                  const int* __restrict__ ids, int n) {
    extern __shared__ float vs[];
    const int q = batch_scan_of(starts, n), s = ids[q];
    const int b = static_cast<int>(blockIdx.x) - starts[q];
    if (b >= d[s].blocks[0]) return;            // padding to the next multiple of 8
    rays_fwd_body(d[s].fwd, b, d[s].blocks[0], vs);
}

__global__ __launch_bounds__(kGridThreads) void rays_adj_batch_kernel(const RayBatchDesc* __restrict__ d,
                                                                      const int* __restrict__ starts,
                                                                      const int* __restrict__ ids, int n) {
    extern __shared__ float lds[];
    const int q = batch_scan_of(starts, n), s = ids[q];
    const int b = static_cast<int>(blockIdx.x) - starts[q];
    if (b >= d[s].blocks[1]) return;
    if (d[s].adj.n_bands == 1)
        rays_adj_grid_body<false>(d[s].adj, b, d[s].blocks[1], lds);
    else
        rays_adj_grid_body<true>(d[s].adj, b, d[s].blocks[1], lds);
}

__global__ __launch_bounds__(kAdjSlices * kReduceNodes, 8) void adj_update_batch_kernel(
    const RayBatchDesc* __restrict__ d, const int* __restrict__ starts, const int* __restrict__ ids, int n,
    int with_loss) {
    __shared__ float run[kAdjSlices][kReduceNodes];
    __shared__ float red[kAdjSlices * kReduceNodes / 64];
    const int q = batch_scan_of(starts, n), s = ids[q];
    const int b = static_cast<int>(blockIdx.x) - starts[q];
    if (b >= d[s].blocks[2]) return;
    UpdArgs A = d[s].upd;
    if (!with_loss) A.loss = nullptr;
    adj_reduce_tv_adam_body(A, b, run, red);
}

void batch_lds_attributes() {
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(rays_fwd_batch_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(rays_adj_batch_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        attr = true;
    }
}

}  // namespace

size_t batch_ray_desc_bytes() { return sizeof(RayBatchDesc); }

int batch_ray_plan(const pact_batch_scan& s, int parity, void* desc, int blocks[3], size_t lds[3], const char* what) {
    const float* sos_in = s.sos[parity];
    float* sos_out = s.sos[1 - parity];
    const float* st_in = s.staged[parity];
    float* st_out = s.staged[1 - parity];
    if (int e = check_rays(sos_in, s.sosg, s.v0, s.centres, s.N, s.ring, s.n_samples, s.support_radius, what))
        return e;
    PACT_CHECK_ARG(sos_out && st_in && st_out && s.m && s.v && s.t && s.mask && s.w && s.dL_dw,
                   "%s: null pointer", what);
    PACT_CHECK_ARG(sos_in != sos_out && st_in != st_out, "%s: the two SOS (and staged) buffers must differ", what);
    PACT_CHECK_ARG(std::isfinite(s.lambda), "%s: lambda must be finite", what);
    PACT_CHECK_ARG(s.b1 >= 0.0f && s.b1 < 1.0f && s.b2 >= 0.0f && s.b2 < 1.0f, "%s: betas must be in [0, 1)", what);
    PACT_CHECK_ARG(s.adam_eps > 0.0f && std::isfinite(s.lr), "%s: adam_eps must be positive and lr finite", what);
    PACT_CHECK_SUPPORTED(adj_grid_lds(s.sosg) > 0, "%s: the %d x %d grid takes the tiled adjoint", what, s.sosg.ny,
                         s.sosg.nx);
    RayBatchDesc D;
    if (int e = plan_fwd(sos_in, st_in, s.sosg, s.v0, s.centres, s.N, s.ring, s.n_samples, s.support_radius, s.w,
                         &D.fwd, &blocks[0], &lds[0], what))
        return e;
    PartialSet ps;
    if (int e = plan_adj_grid(sos_in, st_in, s.sosg, s.v0, s.centres, s.N, s.ring, s.n_samples, s.support_radius,
                              s.dL_dw, nullptr, s.partial, s.partial_bytes, s.t, &D.adj, &blocks[1], &lds[1], &ps,
                              what))
        return e;
    D.upd = UpdArgs{ps, make_geo(s.sosg, s.n_samples, s.support_radius), sos_in, sos_out, s.m, s.v, s.t, s.mask,
                    s.lambda, s.loss, s.lr, s.b1, s.b2, s.adam_eps, s.grad, s.v0, st_out};
    blocks[2] = ceil_div(s.sosg.ny * s.sosg.nx, kReduceNodes);
    lds[2] = 0;
    for (int k = 0; k < 3; ++k) D.blocks[k] = blocks[k];
    std::memcpy(desc, &D, sizeof D);
    return PACT_OK;
}

int batch_ray_launch(int stage, const void* descs, const int* starts, const int* ids, int n, int total, size_t lds,
                     int with_loss, hipStream_t st) {
    const auto* d = static_cast<const RayBatchDesc*>(descs);
    batch_lds_attributes();
    if (stage == 0)
        rays_fwd_batch_kernel<<<total, kThreads, lds, st>>>(d, starts, ids, n);
    else if (stage == 1)
        rays_adj_batch_kernel<<<total, kGridThreads, lds, st>>>(d, starts, ids, n);
    else
        adj_update_batch_kernel<<<total, kAdjSlices * kReduceNodes, 0, st>>>(d, starts, ids, n, with_loss);
    return launch_status("pact_batch_step (rays)");
}

}  // namespace pact
