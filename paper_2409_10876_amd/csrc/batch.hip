// Batched solves: one launch per stage of the pixel-grid step over many independent scans (the batched
// reconstructions of many scans).  The stages themselves live beside their single-scan kernels (rays.hip,
// loss.hip); this file keeps the plan: per-scan launch arguments for both step parities, each stage's block
// ranges, and the largest LDS each launch needs.
#include "common.h"

#include <algorithm>
#include <cstring>
#include <vector>

namespace pact {
namespace {

constexpr unsigned kPlanMagic = 0x50424154u;     // "PBAT"
constexpr int kMaxBatch = 256;

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
};

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct TableLayout {
    size_t off_ray[2], off_loss, off_starts[kLaunches], off_ids[kLaunches], bytes;
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
