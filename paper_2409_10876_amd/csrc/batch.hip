// Batched solves: one launch per stage of the pixel-grid step over many independent scans (the batched
// reconstructions of many scans), or the whole step in one persistent launch.  The stages themselves live beside
// their single-scan kernels (rays.hip, loss.hip, compiled here as part of this translation unit so that the
// persistent kernel can run the bodies of both); this file keeps the plan: per-scan launch arguments for both
// step parities, each stage's block ranges, the largest LDS each launch needs, and the persistent form's task
// queue.
#include "rays.hip"
#include "loss.hip"

#include <algorithm>
#include <cstring>
#include <vector>

namespace pact {
namespace {

constexpr unsigned kPlanMagic = 0x50424154u;     // "PBAT"
constexpr int kMaxBatch = 256;

// ---- The persistent step ----
//
// The stages of one scan's step in dependency order: the loss reads the forward's w, the scalar sum and the
// adjoint read the loss's patch losses and dL/dw, the update reads the adjoint's partial grids and step counter
// and adds its TV term to the sum.  The queue holds, per stage, every scan's blocks (a segment per scan and
// stage), stages in this order and the scans of every stage in the same order; a task's inputs are therefore
// produced by tasks earlier in the queue.  A workgroup takes the next task, waits until its scan's counters
// show those inputs complete, runs the stage body with the task's block number, and counts the task done.
// Every task it waits on was taken before it by a workgroup that is running, and that task waits only on
// earlier tasks still, so every wait ends whatever the number of resident workgroups.  A wait is also bounded in
// time (the GPU's wall clock): past the bound the task is skipped, so a fault in this reasoning would give wrong
// results, not a kernel that does not end.
//
// Memory ordering: a task's writes are complete (every wave waits for its stores) before one thread writes the
// L2 back and counts the task (a device-scope release); a waiting thread polls the counter with device-scope
// loads that leave the caches alone, sleeping about a microsecond between polls, and invalidates its L2 once, when
// the count is reached (the acquire), before the workgroup reads the task's inputs.
enum Stage { kSFwd = 0, kSLoss, kSSum, kSAdj, kSUpd, kStages };
constexpr int kPersistThreads = 1024;       // the workgroup size of every stage body
constexpr int kWaitMs = 50;                 // the longest a wait may take
constexpr bool kPersistEnabled = false;     // the entry point refuses to launch (see pact_batch_step_persistent)

struct PersistArgs {
    const RayBatchDesc* rays;     // the ray descriptors of the step's parity
    const LossBatchDesc* loss;
    const int* seg_start;         // [n_seg + 1]: the first task of each segment
    const int* seg_code;          // [n_seg]: stage << 16 | scan
    const int* loss_red;          // [n_scans]: byte offset of the loss body's reduction array in LDS
    int n_seg, n_scans, with_loss;
    int* ctr;                     // [n_scans * kStages] tasks done per scan and stage, then the queue head and
                                  // the count of workgroups that have left
    long long wait_ticks;         // kWaitMs in wall-clock ticks
    int ctl_off;                  // float offset of the kernel's two control words, after every stage's LDS
};

// Polls counter c until it reaches need (true), or until wait_ticks of the wall clock have passed (false).
__device__ __forceinline__ bool wait_count(const int* c, int need, long long wait_ticks) {
    const long long t0 = wall_clock64();
    while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (wall_clock64() - t0 > wait_ticks) return false;
        __builtin_amdgcn_s_sleep(32);
    }
    return true;
}

// A scan's loss: its patch losses added in the order of loss_sum_batch_kernel (256 threads, then the four wave
// sums in order), with the workgroup's first four waves.
__device__ __forceinline__ void scan_loss_sum(const LossBatchDesc& D, float* red) {
    const int t = threadIdx.x, N = D.a.N;
    float s = t < 256 && t < N ? ordered_strided_sum<8>(D.a.patch_loss + t, (N - t + 255) / 256, 256) : 0.0f;
    s = wave_sum(s);
    if ((t & 63) == 0 && t < 256) red[t >> 6] = s;
    __syncthreads();
    if (t == 0) {
        float tot = 0.0f;
        for (int k = 0; k < 4; ++k) tot += red[k];
        *D.loss = tot;
    }
}

__global__ __launch_bounds__(kPersistThreads) void batch_persist_kernel(PersistArgs A) {
    // the stage bodies' LDS starts at 0, as in their own kernels (no static LDS here), and the two control words
    // (the task taken; whether its inputs are complete) follow the largest of them
    extern __shared__ float lds[];
    int* ctl = reinterpret_cast<int*>(lds + A.ctl_off);
    const int tid = threadIdx.x, lane = tid & 63;
    // The queue and counter work is done by the whole first wave under wave-uniform branches (one lane's share
    // of each atomic is 1, the others' 0), never under a one-thread branch: a one-thread branch at the loop's
    // head and end let the compiler run the task body as an inner loop that the other lanes repeat while the
    // one thread waits to rejoin them, so the next task was never taken.
    const bool wave0 = __builtin_amdgcn_readfirstlane(tid >> 6) == 0;
    const int total = A.seg_start[A.n_seg];
    int* head = A.ctr + A.n_scans * kStages;
    for (;;) {
        if (wave0) {
            const int t = __hip_atomic_fetch_add(head, lane == 0 ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ctl[0] = __builtin_amdgcn_readfirstlane(t);
        }
        __syncthreads();
        const int task = __builtin_amdgcn_readfirstlane(ctl[0]);
        if (task >= total) break;
        int lo = 0, hi = A.n_seg - 1;            // the task's segment: the last one starting at or before it
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.seg_start[mid] <= task)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int code = A.seg_code[lo], stage = code >> 16, s = code & 0xffff, b = task - A.seg_start[lo];
        const RayBatchDesc& R = A.rays[s];
        const LossBatchDesc& L = A.loss[s];
        int* done = A.ctr + s * kStages;
        if (wave0) {
            const long long wt = A.wait_ticks;
            bool ok = true;
            switch (stage) {
                case kSLoss: ok = wait_count(done + kSFwd, R.blocks[0], wt); break;
                case kSSum:
                case kSAdj: ok = wait_count(done + kSLoss, L.blocks, wt); break;
                case kSUpd: ok = wait_count(done + kSAdj, R.blocks[1], wt) && wait_count(done + kSSum, 1, wt); break;
                default: break;
            }
            if (stage != kSFwd) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            ctl[1] = __builtin_amdgcn_readfirstlane(ok ? 1 : 0);
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(ctl[1])) {
            switch (stage) {
                case kSFwd: rays_fwd_body(R.fwd, b, R.blocks[0], lds); break;
                case kSLoss: {
                    float* red = reinterpret_cast<float*>(reinterpret_cast<char*>(lds) + A.loss_red[s]);
                    loss_proj_body(L.a, b, reinterpret_cast<unsigned long long*>(lds),
                                   *reinterpret_cast<float(*)[kBlock / 64]>(red));
                    break;
                }
                case kSSum:
                    if (A.with_loss) scan_loss_sum(L, lds);
                    break;
                case kSAdj:
                    if (R.adj.n_bands == 1)
                        rays_adj_grid_body<false>(R.adj, b, R.blocks[1], lds);
                    else
                        rays_adj_grid_body<true>(R.adj, b, R.blocks[1], lds);
                    break;
                default: {
                    UpdArgs U = R.upd;
                    if (!A.with_loss) U.loss = nullptr;
                    adj_reduce_tv_adam_body(U, b, *reinterpret_cast<float(*)[kAdjSlices][kReduceNodes]>(lds),
                                            lds + kAdjSlices * kReduceNodes);
                    break;
                }
            }
        }
        // every wave's stores are complete before the first wave writes the L2 back and counts the task
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (wave0) __hip_atomic_fetch_add(done + stage, lane == 0 ? 1 : 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the last workgroup to leave returns the counters to zero for the next step (no other workgroup reads them
    // any more)
    if (tid == 0) {
        const int prev = __hip_atomic_fetch_add(head + 1, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == static_cast<int>(gridDim.x) - 1)
            for (int k = 0; k < A.n_scans * kStages + 2; ++k) A.ctr[k] = 0;
    }
}

// LDS of the persistent kernel for one scan's stages (the loss keeps its reduction array after its own LDS, the
// update its two arrays at the start).
size_t persist_lds(const size_t lds[3], size_t loss_lds) {
    const size_t loss_need = ((loss_lds + 15) & ~static_cast<size_t>(15)) + (kBlock / 64) * sizeof(float);
    const size_t upd_need = (kAdjSlices * kReduceNodes + kAdjSlices * kReduceNodes / 64) * sizeof(float);
    return std::max({lds[0], lds[1], loss_need, upd_need, static_cast<size_t>(64 * sizeof(float))});
}

// The launches of one batched step, in order.  The two ray stages are split by the LDS their scans' workgroups
// need: scans whose workgroups fit twice in a CU's LDS (smaller SOS grids) run in a launch of their own, whose
// LDS then lets two workgroups share a CU; one launch has one LDS size, so mixed with the large grids they would
// run one per CU.  The large-grid launch goes first.  Within a launch, scans come in order of decreasing work per
// workgroup, so the longest workgroups are dispatched first.
enum Launch { kFwdLarge = 0, kFwdSmall, kLoss, kSum, kAdjLarge, kAdjSmall, kUpd, kLaunches };

// The host part of a plan (the caller's HOST buffer).
struct BatchPlan {
    unsigned magic;
    int n;
    const char* table;              // DEVICE
    size_t off_ray[2];              // ray descriptors of parity 0 and 1
    size_t off_loss;                // loss descriptors
    size_t off_starts[kLaunches];   // each launch's block ranges: count + 1 ints
    size_t off_ids[kLaunches];      // each launch's scans: count ints
    int count[kLaunches];           // scans in each launch
    int total[kLaunches];           // blocks of each launch
    size_t lds[kLaunches];          // dynamic LDS of each launch
    size_t off_seg_start, off_seg_code, off_ctr, off_loss_red;   // the persistent form's queue and counters
    int n_seg;
    int persist_grid;               // workgroups of the persistent launch (0: not supported for these scans)
    size_t persist_lds;
    int persist_ctl;                // float offset of the persistent kernel's control words in its LDS
    long long wait_ticks;           // the persistent kernel's bound on a wait, in wall-clock ticks
};

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct TableLayout {
    size_t off_ray[2], off_loss, off_starts[kLaunches], off_ids[kLaunches], off_seg_start, off_seg_code, off_ctr,
        off_loss_red, bytes;
};

TableLayout layout(int n) {
    TableLayout L;
    size_t o = 0;
    for (int p = 0; p < 2; ++p) {
        L.off_ray[p] = o;
        o = align256(o + static_cast<size_t>(n) * batch_ray_desc_bytes());
    }
    L.off_loss = o;
    o = align256(o + static_cast<size_t>(n) * batch_loss_desc_bytes());
    for (int k = 0; k < kLaunches; ++k) {
        L.off_starts[k] = o;
        o = align256(o + static_cast<size_t>(n + 1) * sizeof(int));
        L.off_ids[k] = o;
        o = align256(o + static_cast<size_t>(n) * sizeof(int));
    }
    L.off_seg_start = o;
    o = align256(o + static_cast<size_t>(n * kStages + 1) * sizeof(int));
    L.off_seg_code = o;
    o = align256(o + static_cast<size_t>(n * kStages) * sizeof(int));
    L.off_ctr = o;
    o = align256(o + static_cast<size_t>(n * kStages + 2) * sizeof(int));
    L.off_loss_red = o;
    o = align256(o + static_cast<size_t>(n) * sizeof(int));
    L.bytes = o;
    return L;
}

struct ScanStages {
    int blocks[3];          // forward, adjoint, update
    size_t lds[3];
    int loss_blocks;
    size_t loss_lds;
    double work[2];         // forward and adjoint work per workgroup (ray samples)
};

}  // namespace
}  // namespace pact

extern "C" size_t pact_batch_plan_bytes(int n_scans) {
    (void)n_scans;
    return sizeof(pact::BatchPlan);
}

extern "C" size_t pact_batch_table_bytes(int n_scans) {
    if (n_scans <= 0 || n_scans > pact::kMaxBatch) return 0;
    return pact::layout(n_scans).bytes;
}

extern "C" int pact_batch_plan(const pact_batch_scan* scans, int n_scans, void* plan, size_t plan_bytes, void* table,
                               size_t table_bytes, void* stream) {
    using namespace pact;
    clear_error();
    const char* what = "pact_batch_plan";
    PACT_CHECK_ARG(scans && plan && table, "%s: null pointer", what);
    PACT_CHECK_ARG(n_scans > 0, "%s: n_scans must be positive", what);
    PACT_CHECK_SUPPORTED(n_scans <= kMaxBatch, "%s: n_scans = %d exceeds %d", what, n_scans, kMaxBatch);
    PACT_CHECK_ARG(plan_bytes >= sizeof(BatchPlan), "%s: plan buffer of %zu bytes, %zu needed", what, plan_bytes,
                   sizeof(BatchPlan));
    const TableLayout L = layout(n_scans);
    if (table_bytes < L.bytes) {
        set_error("%s: table of %zu bytes needed, %zu given", what, L.bytes, table_bytes);
        return PACT_EWORKSPACE;
    }
    std::vector<char> host(L.bytes, 0);
    BatchPlan P{};
    P.magic = kPlanMagic;
    P.n = n_scans;
    P.table = static_cast<const char*>(table);
    for (int p = 0; p < 2; ++p) P.off_ray[p] = L.off_ray[p];
    P.off_loss = L.off_loss;
    std::vector<ScanStages> st(n_scans);
    for (int s = 0; s < n_scans; ++s) {
        ScanStages& S = st[s];
        for (int p = 0; p < 2; ++p) {
            void* d = host.data() + L.off_ray[p] + static_cast<size_t>(s) * batch_ray_desc_bytes();
            if (int e = batch_ray_plan(scans[s], p, d, S.blocks, S.lds, what)) return e;
        }
        if (int e = batch_loss_plan(scans[s], host.data() + L.off_loss + static_cast<size_t>(s) * batch_loss_desc_bytes(),
                                    &S.loss_blocks, &S.loss_lds, what))
            return e;
        const double samples = static_cast<double>(scans[s].N) * scans[s].ring.n_elem * scans[s].n_samples;
        S.work[0] = samples / S.blocks[0];
        S.work[1] = samples / S.blocks[1];
    }
    // the scans of each launch, in order of decreasing work per workgroup
    std::vector<int> members[kLaunches];
    for (int s = 0; s < n_scans; ++s) {
        const bool fwd_small = 2 * st[s].lds[0] <= kLdsBytes, adj_small = 2 * st[s].lds[1] <= kLdsBytes;
        members[fwd_small ? kFwdSmall : kFwdLarge].push_back(s);
        members[adj_small ? kAdjSmall : kAdjLarge].push_back(s);
        members[kLoss].push_back(s);
        members[kSum].push_back(s);
        members[kUpd].push_back(s);
    }
    for (int k : {kFwdLarge, kFwdSmall, kAdjLarge, kAdjSmall}) {
        const int w = (k == kFwdLarge || k == kFwdSmall) ? 0 : 1;
        std::stable_sort(members[k].begin(), members[k].end(),
                         [&](int a, int b) { return st[a].work[w] > st[b].work[w]; });
    }
    for (int k = 0; k < kLaunches; ++k) {
        P.off_starts[k] = L.off_starts[k];
        P.off_ids[k] = L.off_ids[k];
        int* starts = reinterpret_cast<int*>(host.data() + L.off_starts[k]);
        int* ids = reinterpret_cast<int*>(host.data() + L.off_ids[k]);
        starts[0] = 0;
        size_t lds = 0;
        for (size_t q = 0; q < members[k].size(); ++q) {
            const int s = members[k][q];
            ids[q] = s;
            int blocks = 0;
            switch (k) {
                case kFwdLarge: case kFwdSmall:   // ray ranges start on multiples of 8 (XCD-aware numbering)
                    blocks = ceil_div(st[s].blocks[0], 8) * 8;
                    lds = std::max(lds, st[s].lds[0]);
                    break;
                case kAdjLarge: case kAdjSmall:
                    blocks = ceil_div(st[s].blocks[1], 8) * 8;
                    lds = std::max(lds, st[s].lds[1]);
                    break;
                case kLoss:
                    blocks = st[s].loss_blocks;
                    lds = std::max(lds, st[s].loss_lds);
                    break;
                case kSum: blocks = 1; break;
                default: blocks = st[s].blocks[2]; break;
            }
            starts[q + 1] = starts[q] + blocks;
        }
        P.count[k] = static_cast<int>(members[k].size());
        P.total[k] = starts[P.count[k]];
        P.lds[k] = lds;
    }
    // The persistent form's queue: for each stage in order, a segment per scan, the scans in the order of their
    // forward blocks (large-LDS launch, then the small one), so that a scan whose forward blocks were taken first
    // comes first in every later stage too.  Its counters start at zero (the table is zeroed here).
    {
        std::vector<int> order(members[kFwdLarge]);
        order.insert(order.end(), members[kFwdSmall].begin(), members[kFwdSmall].end());
        int* seg_start = reinterpret_cast<int*>(host.data() + L.off_seg_start);
        int* seg_code = reinterpret_cast<int*>(host.data() + L.off_seg_code);
        int* loss_red = reinterpret_cast<int*>(host.data() + L.off_loss_red);
        for (int s = 0; s < n_scans; ++s) loss_red[s] = static_cast<int>((st[s].loss_lds + 15) & ~size_t{15});
        int q = 0;
        long long next = 0;
        size_t plds = 0;
        for (int stage = 0; stage < kStages; ++stage)
            for (int s : order) {
                const ScanStages& S = st[s];
                const int count = stage == kSFwd ? S.blocks[0]
                                  : stage == kSLoss ? S.loss_blocks
                                  : stage == kSSum ? 1
                                  : stage == kSAdj ? S.blocks[1]
                                                   : S.blocks[2];
                seg_start[q] = static_cast<int>(next);
                seg_code[q] = (stage << 16) | s;
                next += count;
                ++q;
                if (stage == 0) plds = std::max(plds, persist_lds(S.lds, S.loss_lds));
            }
        seg_start[q] = static_cast<int>(next);
        PACT_CHECK_SUPPORTED(next < (1LL << 30), "%s: %lld tasks in the persistent queue", what, next);
        P.off_seg_start = L.off_seg_start;
        P.off_seg_code = L.off_seg_code;
        P.off_ctr = L.off_ctr;
        P.off_loss_red = L.off_loss_red;
        P.n_seg = q;
        P.persist_ctl = static_cast<int>((plds + 15) / 16 * 4);   // floats, 16-byte aligned
        plds = static_cast<size_t>(P.persist_ctl) * sizeof(float) + 16;
        P.persist_lds = plds;
        P.persist_grid = 0;
        hipFuncAttributes fa{};
        int dev = 0, cus = 0, per_cu = 0, clock_khz = 0;
        if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(batch_persist_kernel)) == hipSuccess &&
            plds + fa.sharedSizeBytes <= kLdsBytes &&
            hipFuncSetAttribute(reinterpret_cast<const void*>(batch_persist_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(plds)) == hipSuccess &&
            hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(batch_persist_kernel),
                                                         kPersistThreads, plds) == hipSuccess &&
            hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && clock_khz > 0) {
            P.persist_grid = static_cast<int>(std::min<long long>(static_cast<long long>(cus) * per_cu, next));
            P.wait_ticks = static_cast<long long>(clock_khz) * kWaitMs;
        }
        (void)hipGetLastError();
    }
    // the table is small (a few hundred bytes per scan): a synchronous copy, after the stream's earlier work
    if (hipStreamSynchronize(as_stream(stream)) != hipSuccess ||
        hipMemcpy(table, host.data(), L.bytes, hipMemcpyHostToDevice) != hipSuccess) {
        set_error("%s: copying the plan table failed", what);
        return PACT_EHIP;
    }
    std::memcpy(plan, &P, sizeof P);
    return PACT_OK;
}

extern "C" int pact_batch_step(const void* plan, int parity, int with_loss, void* stream) {
    using namespace pact;
    clear_error();
    const char* what = "pact_batch_step";
    PACT_CHECK_ARG(plan, "%s: null plan", what);
    BatchPlan P;
    std::memcpy(&P, plan, sizeof P);
    PACT_CHECK_ARG(P.magic == kPlanMagic && P.n > 0, "%s: not a plan made by pact_batch_plan", what);
    PACT_CHECK_ARG(parity == 0 || parity == 1, "%s: parity must be 0 or 1", what);
    const hipStream_t st = as_stream(stream);
    const auto starts = [&](int k) { return reinterpret_cast<const int*>(P.table + P.off_starts[k]); };
    const auto ids = [&](int k) { return reinterpret_cast<const int*>(P.table + P.off_ids[k]); };
    const void* rays = P.table + P.off_ray[parity];
    const void* loss = P.table + P.off_loss;
    for (int k : {kFwdLarge, kFwdSmall})
        if (P.count[k] > 0)
            if (int e = batch_ray_launch(0, rays, starts(k), ids(k), P.count[k], P.total[k], P.lds[k], 0, st)) return e;
    if (int e = batch_loss_launch(0, loss, starts(kLoss), ids(kLoss), P.count[kLoss], P.total[kLoss], P.lds[kLoss], st))
        return e;
    if (with_loss)
        if (int e = batch_loss_launch(1, loss, starts(kSum), ids(kSum), P.count[kSum], P.total[kSum], 0, st)) return e;
    for (int k : {kAdjLarge, kAdjSmall})
        if (P.count[k] > 0)
            if (int e = batch_ray_launch(1, rays, starts(k), ids(k), P.count[k], P.total[k], P.lds[k], 0, st)) return e;
    return batch_ray_launch(2, rays, starts(kUpd), ids(kUpd), P.count[kUpd], P.total[kUpd], 0, with_loss, st);
}

extern "C" int pact_batch_step_persistent(const void* plan, int parity, int with_loss, void* stream) {
    using namespace pact;
    clear_error();
    const char* what = "pact_batch_step_persistent";
    PACT_CHECK_ARG(plan, "%s: null plan", what);
    BatchPlan P;
    std::memcpy(&P, plan, sizeof P);
    PACT_CHECK_ARG(P.magic == kPlanMagic && P.n > 0, "%s: not a plan made by pact_batch_plan", what);
    PACT_CHECK_ARG(parity == 0 || parity == 1, "%s: parity must be 0 or 1", what);
    // Switched off: an earlier form of the kernel did not finish on the GPU (one-thread branches around the task
    // queue, which the compiler turned into an inner loop that the other lanes repeated on the same task); the
    // rewritten kernel has not run on the GPU, so it is not launched.
    PACT_CHECK_SUPPORTED(kPersistEnabled, "%s: the persistent step is switched off (an earlier form did not finish "
                         "on the GPU; the rewritten kernel is untested there); use pact_batch_step", what);
    PACT_CHECK_SUPPORTED(P.persist_grid > 0, "%s: the scans' stages need %zu bytes of LDS, too many for one launch",
                         what, P.persist_lds);
    PersistArgs A;
    A.rays = reinterpret_cast<const RayBatchDesc*>(P.table + P.off_ray[parity]);
    A.loss = reinterpret_cast<const LossBatchDesc*>(P.table + P.off_loss);
    A.seg_start = reinterpret_cast<const int*>(P.table + P.off_seg_start);
    A.seg_code = reinterpret_cast<const int*>(P.table + P.off_seg_code);
    A.loss_red = reinterpret_cast<const int*>(P.table + P.off_loss_red);
    A.n_seg = P.n_seg;
    A.n_scans = P.n;
    A.with_loss = with_loss != 0;
    A.ctr = reinterpret_cast<int*>(const_cast<char*>(P.table) + P.off_ctr);
    A.wait_ticks = P.wait_ticks;
    A.ctl_off = P.persist_ctl;
    batch_persist_kernel<<<P.persist_grid, kPersistThreads, P.persist_lds, as_stream(stream)>>>(A);
    return launch_status(what);
}
