// Batched solves: one launch per stage of the pixel-grid step over many independent scans (the batched
// reconstructions of many scans).  The stages themselves live beside their single-scan kernels (rays.hip,
// loss.hip); this file keeps the plan: per-scan launch arguments for both step parities, each stage's block
// ranges, and the largest LDS each launch needs.
#include "common.h"

#include <cstring>
#include <vector>

namespace pact {
namespace {

constexpr unsigned kPlanMagic = 0x50424154u;     // "PBAT"
constexpr int kMaxBatch = 256;

enum Stage { kFwd = 0, kLoss, kSum, kAdj, kUpd, kStages };

// The host part of a plan (the caller's HOST buffer).
struct BatchPlan {
    unsigned magic;
    int n;
    const char* table;          // DEVICE
    size_t off_ray[2];          // ray descriptors of parity 0 and 1
    size_t off_loss;            // loss descriptors
    size_t off_starts[kStages]; // block ranges of each stage: n + 1 ints
    int total[kStages];         // blocks of each launch
    size_t lds[kStages];        // dynamic LDS of each launch
};

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct TableLayout {
    size_t off_ray[2], off_loss, off_starts[kStages], bytes;
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
    for (int k = 0; k < kStages; ++k) {
        L.off_starts[k] = o;
        o = align256(o + static_cast<size_t>(n + 1) * sizeof(int));
    }
    L.bytes = o;
    return L;
}

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
    int* starts[kStages];
    for (int k = 0; k < kStages; ++k) {
        P.off_starts[k] = L.off_starts[k];
        starts[k] = reinterpret_cast<int*>(host.data() + L.off_starts[k]);
        starts[k][0] = 0;
    }
    for (int p = 0; p < 2; ++p) P.off_ray[p] = L.off_ray[p];
    P.off_loss = L.off_loss;
    for (int s = 0; s < n_scans; ++s) {
        int rb[3] = {0, 0, 0};
        size_t rl[3] = {0, 0, 0};
        for (int p = 0; p < 2; ++p) {
            void* d = host.data() + L.off_ray[p] + static_cast<size_t>(s) * batch_ray_desc_bytes();
            if (int e = batch_ray_plan(scans[s], p, d, rb, rl, what)) return e;
        }
        int lb = 0;
        size_t ll = 0;
        if (int e = batch_loss_plan(scans[s], host.data() + L.off_loss + static_cast<size_t>(s) * batch_loss_desc_bytes(),
                                    &lb, &ll, what))
            return e;
        // forward and adjoint ranges start on multiples of 8 blocks (the XCD-aware numbering of each scan)
        starts[kFwd][s + 1] = starts[kFwd][s] + ceil_div(rb[0], 8) * 8;
        starts[kAdj][s + 1] = starts[kAdj][s] + ceil_div(rb[1], 8) * 8;
        starts[kUpd][s + 1] = starts[kUpd][s] + rb[2];
        starts[kLoss][s + 1] = starts[kLoss][s] + lb;
        starts[kSum][s + 1] = s + 1;
        P.lds[kFwd] = std::max(P.lds[kFwd], rl[0]);
        P.lds[kAdj] = std::max(P.lds[kAdj], rl[1]);
        P.lds[kLoss] = std::max(P.lds[kLoss], ll);
    }
    for (int k = 0; k < kStages; ++k) P.total[k] = starts[k][n_scans];
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
    const auto start = [&](int k) { return reinterpret_cast<const int*>(P.table + P.off_starts[k]); };
    const void* rays = P.table + P.off_ray[parity];
    const void* loss = P.table + P.off_loss;
    if (int e = batch_ray_launch(0, rays, start(kFwd), P.n, P.total[kFwd], P.lds[kFwd], 0, st)) return e;
    if (int e = batch_loss_launch(0, loss, start(kLoss), P.n, P.total[kLoss], P.lds[kLoss], st)) return e;
    if (with_loss)
        if (int e = batch_loss_launch(1, loss, start(kSum), P.n, P.n, 0, st)) return e;
    if (int e = batch_ray_launch(1, rays, start(kAdj), P.n, P.total[kAdj], P.lds[kAdj], 0, st)) return e;
    return batch_ray_launch(2, rays, start(kUpd), P.n, P.total[kUpd], 0, with_loss, st);
}
