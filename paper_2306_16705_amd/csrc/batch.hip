// Batched sample-aware local energy over many systems (uneven N and sample
// counts) in one persistent launch, optionally captured in a hipGraph, with
// launch schedules chosen by timing (the autotuner below).
//
// One step of a batch, all on the caller's stream:
//   1. for each system with a model: log|psi| and phase of its samples from
//      the BF16 network (Section 3.1 ansatz; the sample-aware method takes the
//      samples' own amplitudes, Section 3.4 item 4);
//   2. for each system: the sorted sample table;
//   3. one persistent k_eloc_sa_batch launch over every (system, sample)
//      tile: blocks pull tiles from a device counter;
//   4. for each system: the weighted energy of Eq. 6.
// Nothing in a step synchronises the host or allocates, so the step can be
// captured into a graph and replayed.
#include <algorithm>
#include <vector>

#include "model.hpp"

struct nnqs_batch {
    std::vector<nnqs_batch_item> items;
    nnqs_tune tune{};
    int W = 1;
    int waves = 12;
    size_t lds = 0;
    unsigned grid = 0;
    int ntiles = 0;
    nnqs::SaBatchItem *d_items = nullptr;
    nnqs::SaTile *d_tiles = nullptr;
    int *d_counter = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
    int cu_count = 0;
    int max_lds = 0;
};

namespace nnqs {

static void batch_drop_graph(nnqs_batch *b) {
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Apply b->tune: table tunes, per-system views, the tile list and the launch
// shape.  Synchronous (uploads the device descriptors).
static nnqs_status batch_plan(nnqs_batch *b) {
    batch_drop_graph(b);
    const int n_items = (int)b->items.size();
    std::vector<SaBatchItem> hi(n_items);
    std::vector<SaTile> tiles;
    int fl_min = b->tune.filter_log2_bits;
    b->W = 1;
    for (const auto &it : b->items)
        if (it.system->view.N > 64) b->W = 2;
    b->waves = std::min(b->tune.waves_per_block, 12);
    // LDS of the largest system; filters fold to fit
    int max_sl = 1;
    for (int k = 0; k < n_items; k++) {
        nnqs_tune tt = b->items[k].table->tune;
        tt.filter_log2_bits = b->tune.filter_log2_bits;
        tt.splitter_levels = b->tune.splitter_levels;
        tt.search = b->tune.search;
        b->items[k].table->tune = tt;
        const TableView tv = table_view_planned(b->items[k].table, b->items[k].n);
        max_sl = std::max(max_sl, tv.split_levels);
    }
    const int budget = b->max_lds - 16;  // the kernel's next-tile slot follows the layout
    while (fl_min > 10 && sa_lds_bytes(fl_min, max_sl, b->W, b->waves) > (size_t)budget) fl_min--;
    const size_t layout = sa_lds_bytes(fl_min, max_sl, b->W, b->waves);
    if (layout > (size_t)budget) return fail(NNQS_EINVAL, "LDS budget exceeded (%zu bytes)", layout);
    b->lds = ((layout + 15) & ~(size_t)15) + 16;
    for (int k = 0; k < n_items; k++) {
        const nnqs_batch_item &it = b->items[k];
        SaBatchItem &d = hi[k];
        d.S = it.system->view;
        d.T = table_view_planned(it.table, it.n);
        d.lds_filter_log2 = std::min(fl_min, d.T.filter_log2);
        d.keys = it.keys;
        d.logabs = it.logabs;
        d.phase = it.phase;
        d.eloc = it.eloc;
        d.status = it.table->status;
        for (int64_t s0 = 0; s0 < it.n; s0 += b->tune.tile_samples) {
            SaTile t;
            t.item = k;
            t.begin = s0;
            t.count = (int32_t)std::min<int64_t>(b->tune.tile_samples, it.n - s0);
            tiles.push_back(t);
        }
    }
    if (tiles.size() > (size_t)INT32_MAX) return fail(NNQS_EINVAL, "too many tiles");
    b->ntiles = (int)tiles.size();
    hipFree(b->d_items);
    hipFree(b->d_tiles);
    b->d_items = nullptr;
    b->d_tiles = nullptr;
    if (hipMalloc(&b->d_items, sizeof(SaBatchItem) * n_items) != hipSuccess ||
        hipMalloc(&b->d_tiles, sizeof(SaTile) * tiles.size()) != hipSuccess)
        return fail(NNQS_ENOMEM, "batch descriptor allocation failed");
    NNQS_HIP_CHECK(hipMemcpy(b->d_items, hi.data(), sizeof(SaBatchItem) * n_items, hipMemcpyHostToDevice));
    NNQS_HIP_CHECK(hipMemcpy(b->d_tiles, tiles.data(), sizeof(SaTile) * tiles.size(), hipMemcpyHostToDevice));
    for (bool exact : {false, true}) {
        const void *fn = sa_batch_kernel_ptr(b->W, b->tune.search, exact);
        nnqs_status s = sa_check_no_spill(fn);
        if (s != NNQS_OK) return s;
        NNQS_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds));
    }
    b->grid = (unsigned)(b->cu_count * b->tune.blocks_per_cu);
    return NNQS_OK;
}

// Enqueue one step (see the file comment).  No host synchronisation.
static nnqs_status batch_step(nnqs_batch *b, hipStream_t st) {
    for (const auto &it : b->items) {
        if (it.model) {
            nnqs_status s = enqueue_logpsi(it.model, it.keys, it.n, NNQS_BF16, it.logabs, it.phase, st);
            if (s != NNQS_OK) return s;
        }
        nnqs_status s = nnqs_table_build(it.table, it.keys, it.logabs, it.phase, it.n, 0, st);
        if (s != NNQS_OK) return s;
    }
    sa_launch_batch(b->W, b->tune.search, b->grid, b->waves, b->lds, st, b->d_items, b->d_tiles, b->ntiles,
                    b->d_counter);
    NNQS_HIP_CHECK(hipGetLastError());
    for (const auto &it : b->items) {
        if (!it.energy) continue;
        nnqs_status s = enqueue_energy(it.table, it.counts, it.eloc, it.n, it.energy, st);
        if (s != NNQS_OK) return s;
    }
    return NNQS_OK;
}

}  // namespace nnqs

using namespace nnqs;

extern "C" {

nnqs_status nnqs_batch_create(nnqs_batch **out, const nnqs_batch_item *items, int32_t n_items) {
    clear_error();
    if (!out || !items) return fail(NNQS_EINVAL, "null pointer argument");
    *out = nullptr;
    if (n_items < 1) return fail(NNQS_EINVAL, "a batch needs at least one system");
    for (int k = 0; k < n_items; k++) {
        const nnqs_batch_item &it = items[k];
        if (!it.system || !it.table || !it.keys || !it.logabs || !it.phase || !it.eloc)
            return fail(NNQS_EINVAL, "item %d: null pointer", k);
        if (it.energy && !it.counts) return fail(NNQS_EINVAL, "item %d: energy requested without counts", k);
        if (it.n <= 0 || it.n > it.table->capacity)
            return fail(NNQS_EINVAL, "item %d: n=%lld outside 1..table capacity", k, (long long)it.n);
        if (it.table->sys != it.system) return fail(NNQS_EINVAL, "item %d: table belongs to another system", k);
        if (it.model && (it.model->desc.n_orb != it.system->view.K || it.model->desc.n_up != it.system->view.n_up ||
                         it.model->desc.n_dn != it.system->view.n_dn || !it.model->bf16_ok))
            return fail(NNQS_EINVAL, "item %d: model does not fit the system or has no BF16 path", k);
        if (it.system->device != items[0].system->device)
            return fail(NNQS_EINVAL, "item %d: all systems of a batch must live on one device", k);
    }
    nnqs_batch *b = new nnqs_batch();
    b->items.assign(items, items + n_items);
    b->device = items[0].system->device;
    b->cu_count = items[0].system->cu_count;
    b->max_lds = items[0].system->max_lds;
    nnqs_table_get_tune(items[0].table, &b->tune);
    if (hipMalloc(&b->d_counter, sizeof(int)) != hipSuccess) {
        delete b;
        return fail(NNQS_ENOMEM, "batch counter allocation failed");
    }
    nnqs_status s = batch_plan(b);
    if (s != NNQS_OK) {
        nnqs_batch_destroy(b);
        return s;
    }
    *out = b;
    return NNQS_OK;
}

nnqs_status nnqs_batch_destroy(nnqs_batch *b) {
    if (!b) return NNQS_OK;
    batch_drop_graph(b);
    hipFree(b->d_items);
    hipFree(b->d_tiles);
    hipFree(b->d_counter);
    delete b;
    return NNQS_OK;
}

nnqs_status nnqs_batch_run(nnqs_batch *b, void *stream) {
    clear_error();
    if (!b) return fail(NNQS_EINVAL, "null batch");
    return batch_step(b, as_stream(stream));
}

nnqs_status nnqs_batch_capture(nnqs_batch *b, void *stream) {
    clear_error();
    if (!b) return fail(NNQS_EINVAL, "null batch");
    if (!stream) return fail(NNQS_EINVAL, "graph capture needs a created (non-null) stream");
    hipStream_t st = as_stream(stream);
    batch_drop_graph(b);
    NNQS_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    nnqs_status s = batch_step(b, st);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (s != NNQS_OK) {
        if (g) hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return fail(NNQS_EHIP, "stream capture failed: %s", hipGetErrorString(e));
    b->graph = g;
    const hipError_t e2 = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e2 != hipSuccess) {
        batch_drop_graph(b);
        return fail(NNQS_EHIP, "graph instantiation failed: %s", hipGetErrorString(e2));
    }
    return NNQS_OK;
}

nnqs_status nnqs_batch_launch(nnqs_batch *b, void *stream) {
    clear_error();
    if (!b) return fail(NNQS_EINVAL, "null batch");
    if (!b->exec) return fail(NNQS_EINVAL, "no captured graph (call nnqs_batch_capture first)");
    NNQS_HIP_CHECK(hipGraphLaunch(b->exec, as_stream(stream)));
    return NNQS_OK;
}

nnqs_status nnqs_batch_set_tune(nnqs_batch *b, const nnqs_tune *tune) {
    clear_error();
    if (!b || !tune) return fail(NNQS_EINVAL, "null pointer argument");
    nnqs_tune d = b->tune;
    if (tune->waves_per_block) d.waves_per_block = tune->waves_per_block;
    if (tune->blocks_per_cu) d.blocks_per_cu = tune->blocks_per_cu;
    if (tune->filter_log2_bits) d.filter_log2_bits = tune->filter_log2_bits;
    if (tune->splitter_levels) d.splitter_levels = tune->splitter_levels;
    if (tune->search) d.search = tune->search;
    if (tune->tile_samples) d.tile_samples = tune->tile_samples;
    if (!tune_valid(d)) return fail(NNQS_EINVAL, "tuning parameters out of range");
    b->tune = d;
    return batch_plan(b);
}

nnqs_status nnqs_batch_get_tune(const nnqs_batch *b, nnqs_tune *tune) {
    if (!b || !tune) return fail(NNQS_EINVAL, "null pointer argument");
    *tune = b->tune;
    return NNQS_OK;
}

// Times every candidate schedule on the batch itself (one untimed warm-up
// step, then the best of `reps` timed steps each) and keeps the fastest.
// Candidates: waves per block {8, 12} x splitter levels {8, 10, 12} x search
// variant {1, 2} x tile size {64, 256, 1024}.  Results are identical for
// every candidate (one wave per sample, fixed order), so only time decides.
nnqs_status nnqs_batch_autotune(nnqs_batch *b, int32_t reps, nnqs_tune *best_out, double *best_ms, void *stream) {
    clear_error();
    if (!b) return fail(NNQS_EINVAL, "null batch");
    if (reps < 1) reps = 1;
    hipStream_t st = as_stream(stream);
    hipEvent_t e0, e1;
    NNQS_HIP_CHECK(hipEventCreate(&e0));
    NNQS_HIP_CHECK(hipEventCreate(&e1));
    const nnqs_tune start = b->tune;
    nnqs_tune best = start;
    float best_t = 1e30f;
    nnqs_status s = NNQS_OK;
    for (int waves : {8, 12})
        for (int sl : {8, 10, 12})
            for (int search : {1, 2})
                for (int tile : {64, 256, 1024}) {
                    nnqs_tune c = start;
                    c.waves_per_block = waves;
                    c.splitter_levels = sl;
                    c.search = search;
                    c.tile_samples = tile;
                    b->tune = c;
                    s = batch_plan(b);
                    if (s != NNQS_OK) continue;  // e.g. does not fit the LDS: skip the candidate
                    s = batch_step(b, st);
                    if (s != NNQS_OK) goto done;
                    float tmin = 1e30f;
                    for (int r = 0; r < reps; r++) {
                        if (hipEventRecord(e0, st) != hipSuccess) { s = fail(NNQS_EHIP, "event record failed"); goto done; }
                        s = batch_step(b, st);
                        if (s != NNQS_OK) goto done;
                        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                            s = fail(NNQS_EHIP, "event timing failed");
                            goto done;
                        }
                        float ms = 0.f;
                        hipEventElapsedTime(&ms, e0, e1);
                        tmin = std::min(tmin, ms);
                    }
                    if (tmin < best_t) {
                        best_t = tmin;
                        best = c;
                    }
                }
    s = NNQS_OK;
done:
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    b->tune = best;
    nnqs_status s2 = batch_plan(b);
    if (s == NNQS_OK) s = s2;
    if (s == NNQS_OK) {
        if (best_out) *best_out = best;
        if (best_ms) *best_ms = best_t;
    }
    return s;
}

}  // extern "C"
