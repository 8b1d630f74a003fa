// Mixed-code batches: segment table, launch plans, HIP graph capture and the
// plan autotuner.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <numeric>

#include "internal.h"

namespace sagms {

constexpr int kDefaultQueues = 8;  // one per XCD: a block starts on queue blockIdx mod 8

int mixed_tier_of_shape(int idx) {
    for (int t = 0; t < kNumMixedTiers; ++t)
        if (idx >= 0 && idx <= kMixedTiers[t]) return t;
    return -1;
}

int mixed_budget_of(int tier, int requested) { return requested == 1 && mixed_has_budget(tier, 1) ? 1 : 0; }

int mixed_waves_of(int tier, int requested) {
    int w = requested;
    while (w > 1 && (size_t)w * mixed_words(tier) * sizeof(float) > 65536) w /= 2;
    return w;
}

OccupancyCache::OccupancyCache() {
    for (auto& a : blocks)
        for (auto& b : a)
            for (auto& c : b)
                for (auto& d : c)
                    for (int& e : d) e = -1;
}

int OccupancyCache::get(int tier, int budget, int mt, int unroll, int wpb, int* out) {
    if (tier < 0 || tier >= kNumMixedTiers || budget < 0 || budget > 1 || mt < 0 || mt > 2 || unroll < 1 ||
        unroll > 2 || wpb < 1 || wpb > 4)
        return fail(SAGMS_EINVAL, "occupancy key out of range (internal)");
    int& slot = blocks[tier][budget][mt][unroll - 1][wpb];
    if (slot < 0) {
        int n = 0;
        int rc = mixed_max_blocks(tier, budget, mt, unroll, wpb, &n);
        if (rc) return rc;
        slot = n;
    }
    *out = slot;
    return SAGMS_OK;
}

int launch_segments(const MixedSegment* segs, int nseg, int tier, const MixedLaunch& p, int num_cu, int mt,
                    uint32_t* queues, OccupancyCache* occ, hipStream_t st) {
    if (nseg < 1 || nseg > kMaxSegments) return fail(SAGMS_EINVAL, "segment count out of range (internal)");
    MixedArgs m{};
    for (int s = 0; s < nseg; ++s) m.segs[s] = segs[s];
    m.queues = queues;
    m.nseg = nseg;
    m.tile_frames = p.tile_frames;
    m.words = mixed_words(tier);
    int64_t tiles = 0;
    for (int s = 0; s < nseg; ++s) {
        if (mixed_tier_of_shape(segs[s].shape) > tier) return fail(SAGMS_EINVAL, "segment above the kernel's tier (internal)");
        tiles += (segs[s].a.nframes + p.tile_frames - 1) / p.tile_frames;
        m.tile_end[s] = tiles;
    }
    if (tiles == 0) return SAGMS_OK;
    if (tiles > 0x7fffffffLL) return fail(SAGMS_EINVAL, "too many tiles for one launch: raise tile_frames");
    m.ntiles = tiles;
    m.nq = (int)std::min<int64_t>(kDefaultQueues, tiles);
    const int budget = mixed_budget_of(tier, p.reg_budget);
    const int wpb = mixed_waves_of(tier, p.waves_per_block);
    int per_cu = 0;
    int rc = occ->get(tier, budget, mt, p.unroll, wpb, &per_cu);
    if (rc) return rc;
    if (per_cu < 1) return fail(SAGMS_EUNSUPPORTED, "mixed kernel of tier %d does not fit a compute unit", tier);
    if (p.blocks_per_cu > 0) per_cu = std::min(per_cu, p.blocks_per_cu);
    int64_t blocks = (int64_t)per_cu * num_cu;
    blocks = std::min<int64_t>(blocks, (tiles + wpb - 1) / wpb);
    return launch_mixed(tier, budget, mt, p.unroll, m, (int)blocks, wpb, st);
}

int prepare_segments(const sagms_segment* segs, int nseg, const sagms_decoder_cfg* cfg, bool upload,
                     SegmentSet* out) {
    if (!segs) return fail(SAGMS_EINVAL, "segs is null");
    if (nseg < 1 || nseg > kMaxSegments) return fail(SAGMS_EINVAL, "nseg must lie in [1, %d]", kMaxSegments);
    int rc = check_cfg(cfg);
    if (rc) return rc;
    if (cfg->kind == SAGMS_BP) return fail(SAGMS_EUNSUPPORTED, "batches run MS, SMS and SAGMS only");
    if (cfg->schedule != SAGMS_FLOODING) return fail(SAGMS_EUNSUPPORTED, "batches run the flooding schedule only");
    for (int s = 0; s < nseg; ++s) {
        const sagms_segment& x = segs[s];
        Graph* g = reinterpret_cast<Graph*>(x.graph);
        if (!g) return fail(SAGMS_EINVAL, "segment %d: null graph", s);
        if (g->joint) return fail(SAGMS_EUNSUPPORTED, "segment %d: joint graphs decode through sagms_decode only", s);
        if (!g->shape_ok) return fail(SAGMS_EUNSUPPORTED, "segment %d: no decode kernel fits the code", s);
        if (shape_index(g->shape) < 0) return fail(SAGMS_EUNSUPPORTED, "segment %d: shape not compiled", s);
        if (x.nframes < 0 || x.nframes > kMaxFramesPerCall)
            return fail(SAGMS_EINVAL, "segment %d: nframes must lie in [0, 2^31 - 1]", s);
        if (x.nframes > 0 && (!x.synd || !x.llr0 || !x.ehat || !x.iters || !x.converged))
            return fail(SAGMS_EINVAL, "segment %d: null buffer", s);
    }
    // launch order: largest register tier first, then the most lane slots per
    // round (the most expensive frames first), then the caller's order
    // (insertion sort on a fixed array: stable, no allocation)
    int order[kMaxSegments];
    auto cost = [&](int s) {
        const DecodeShape& sh = reinterpret_cast<Graph*>(segs[s].graph)->shape;
        return sh.cpl * sh.dc + sh.vpl * sh.dv;
    };
    auto tier = [&](int s) { return mixed_tier_of_shape(shape_index(reinterpret_cast<Graph*>(segs[s].graph)->shape)); };
    auto before = [&](int x, int y) { return tier(x) != tier(y) ? tier(x) > tier(y) : cost(x) > cost(y); };
    for (int s = 0; s < nseg; ++s) {
        int i = s;
        while (i > 0 && before(s, order[i - 1])) {
            order[i] = order[i - 1];
            --i;
        }
        order[i] = s;
    }
    out->nseg = nseg;
    for (int i = 0; i < nseg; ++i) {
        const int s = order[i];
        const sagms_segment& x = segs[s];
        Graph* g = reinterpret_cast<Graph*>(x.graph);
        DeviceTables* t = nullptr;
        rc = upload ? upload_tables(g, &t) : device_tables(g, &t);
        if (rc) return rc;
        MixedSegment ms{};
        ms.a = decode_args(g, t, gain_law(cfg), x.synd, x.llr0, x.nframes, x.ehat, x.iters, x.converged, x.posterior,
                           cfg->lmax, 0);
        ms.shape = shape_index(g->shape);
        out->segs[i] = ms;
        out->tier[i] = tier(s);
        out->shape[i] = g->shape;
    }
    return SAGMS_OK;
}

int check_plan(const sagms_plan* p) {
    if (!p) return fail(SAGMS_EINVAL, "plan is null");
    if (p->kind < SAGMS_PLAN_SINGLE || p->kind > SAGMS_PLAN_PER_CODE) return fail(SAGMS_EINVAL, "unknown plan kind %d", p->kind);
    if (p->tile_frames < 1 || p->tile_frames > 1024) return fail(SAGMS_EINVAL, "tile_frames must lie in [1, 1024]");
    if (p->unroll < 0 || p->unroll > 2) return fail(SAGMS_EINVAL, "unroll must be 0, 1 or 2");
    if (p->kind == SAGMS_PLAN_PER_CODE) return SAGMS_OK;
    if (p->waves_per_block != 1 && p->waves_per_block != 2 && p->waves_per_block != 4)
        return fail(SAGMS_EINVAL, "waves_per_block must be 1, 2 or 4");
    if (p->blocks_per_cu < 0 || p->blocks_per_cu > 64) return fail(SAGMS_EINVAL, "blocks_per_cu must lie in [0, 64]");
    if (p->reg_budget != 0 && p->reg_budget != 1) return fail(SAGMS_EINVAL, "reg_budget must be 0 or 1");
    return SAGMS_OK;
}

int enqueue_segments(const SegmentSet& set, const sagms_plan& p, int mt, int num_cu, uint32_t* queues,
                     OccupancyCache* occ, hipStream_t st) {
    if (p.kind == SAGMS_PLAN_PER_CODE) {
        for (int s = 0; s < set.nseg; ++s) {
            if (set.segs[s].a.nframes == 0) continue;
            DecodeArgs a = set.segs[s].a;
            a.frames_per_wave = p.tile_frames;
            int rc = launch_decode(set.shape[s], false, mt, a, st);
            if (rc) return rc;
        }
        return SAGMS_OK;
    }
    const MixedLaunch L{p.tile_frames, p.waves_per_block, p.blocks_per_cu, p.reg_budget, p.unroll == 2 ? 2 : 1};
    // SINGLE: one launch with the largest tier's kernel; TIERED: one per tier
    for (int s0 = 0; s0 < set.nseg;) {
        int s1 = s0;
        while (s1 < set.nseg && (p.kind == SAGMS_PLAN_SINGLE || set.tier[s1] == set.tier[s0])) ++s1;
        const int tier = set.tier[s0];
        int rc = launch_segments(set.segs + s0, s1 - s0, tier, L, num_cu, mt,
                                 queues + (size_t)tier * kMaxQueues * kQueueStride, occ, st);
        if (rc) return rc;
        s0 = s1;
    }
    return SAGMS_OK;
}

}  // namespace sagms

using namespace sagms;

namespace {

struct Batch {
    int device = 0;
    sagms_decoder_cfg cfg{};
    int mt = SAGMS_MSG_FP32;
    int num_cu = 0;
    SegmentSet set;                // segments in launch order
    uint32_t* d_queues = nullptr;  // kNumMixedTiers blocks of kMaxQueues counters
    sagms_plan plan{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    OccupancyCache occupancy;
};

void drop_graph(Batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

int blocks_per_cu(Batch* b, int tier, int* out) {
    const int budget = mixed_budget_of(tier, b->plan.reg_budget);
    const int wpb = mixed_waves_of(tier, b->plan.waves_per_block);
    return b->occupancy.get(tier, budget, b->mt, b->plan.unroll == 2 ? 2 : 1, wpb, out);
}

int enqueue(Batch* b, hipStream_t st) {
    return enqueue_segments(b->set, b->plan, b->mt, b->num_cu, b->d_queues, &b->occupancy, st);
}

int check_device(const Batch* b) {
    int dev = -1;
    SAGMS_HIP(hipGetDevice(&dev));
    if (dev != b->device) return fail(SAGMS_EINVAL, "batch was created on device %d, current device is %d", b->device, dev);
    return SAGMS_OK;
}

void destroy(Batch* b) {
    drop_graph(b);
    if (b->d_queues) (void)hipFree(b->d_queues);
    delete b;
}

}  // namespace

extern "C" {

int sagms_batch_create(const sagms_segment* segs, int32_t nseg, const sagms_decoder_cfg* cfg, sagms_batch* out) {
    if (!out) return fail(SAGMS_EINVAL, "out is null");
    *out = nullptr;
    Batch* b = new Batch();
    int rc = prepare_segments(segs, nseg, cfg, true, &b->set);
    if (rc) {
        destroy(b);
        return rc;
    }
    b->cfg = *cfg;
    b->mt = cfg->msg_precision;
    b->plan = sagms_plan{SAGMS_PLAN_SINGLE, kMixedTileFrames, 4, 0, 0, 1};
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e == hipSuccess) e = hipMalloc(&b->d_queues, sizeof(uint32_t) * kScratchWords);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        destroy(b);
        return hip_fail(e, "batch set-up");
    }
    *out = reinterpret_cast<sagms_batch>(b);
    return SAGMS_OK;
}

int sagms_batch_set_plan(sagms_batch bh, const sagms_plan* plan) {
    Batch* b = reinterpret_cast<Batch*>(bh);
    if (!b) return fail(SAGMS_EINVAL, "null batch");
    int rc = check_plan(plan);
    if (rc) return rc;
    drop_graph(b);
    b->plan = *plan;
    return SAGMS_OK;
}

int sagms_batch_get_plan(sagms_batch bh, sagms_plan* plan) {
    Batch* b = reinterpret_cast<Batch*>(bh);
    if (!b || !plan) return fail(SAGMS_EINVAL, "null argument");
    *plan = b->plan;
    return SAGMS_OK;
}

int sagms_batch_run(sagms_batch bh, void* stream) {
    Batch* b = reinterpret_cast<Batch*>(bh);
    if (!b) return fail(SAGMS_EINVAL, "null batch");
    int rc = check_device(b);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (b->exec) {
        SAGMS_HIP(hipGraphLaunch(b->exec, st));
        return SAGMS_OK;
    }
    return enqueue(b, st);
}

int sagms_batch_instantiate(sagms_batch bh) {
    Batch* b = reinterpret_cast<Batch*>(bh);
    if (!b) return fail(SAGMS_EINVAL, "null batch");
    int rc = check_device(b);
    if (rc) return rc;
    drop_graph(b);
    if (b->plan.kind != SAGMS_PLAN_PER_CODE)
        for (int i = 0; i < b->set.nseg; ++i) {  // occupancy queries stay outside the capture
            const int t = b->set.tier[i];
            int n = 0;
            rc = blocks_per_cu(b, t, &n);
            if (rc) return rc;
        }
    hipStream_t cs = nullptr;
    SAGMS_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    rc = enqueue(b, cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    b->graph = graph;
    b->exec = exec;
    return SAGMS_OK;
}

int sagms_batch_tune(sagms_batch bh, void* stream, int32_t reps, sagms_tune_result* results, int32_t cap,
                     int32_t* count, sagms_plan* best) {
    Batch* b = reinterpret_cast<Batch*>(bh);
    if (!b) return fail(SAGMS_EINVAL, "null batch");
    if (reps < 1 || reps > 100) return fail(SAGMS_EINVAL, "reps must lie in [1, 100]");
    if (cap < 0 || (cap > 0 && !results)) return fail(SAGMS_EINVAL, "results is null");
    int rc = check_device(b);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    std::vector<sagms_plan> cands;
    const int tiles[] = {4, 8, 16, 32};
    const int* tiers = b->set.tier;
    const int nseg = b->set.nseg;
    const int multi_tier = std::count(tiers, tiers + nseg, tiers[0]) != nseg;
    bool tight = false;  // a tight budget exists for some tier of the batch
    for (int i = 0; i < nseg; ++i) tight = tight || mixed_has_budget(tiers[i], 1);
    for (int kind : {SAGMS_PLAN_SINGLE, SAGMS_PLAN_TIERED}) {
        if (kind == SAGMS_PLAN_TIERED && !multi_tier) continue;
        for (int budget : {0, 1}) {
            if (budget == 1 && (kind == SAGMS_PLAN_SINGLE ? !mixed_has_budget(tiers[0], 1) : !tight))
                continue;
            for (int unroll : {1, 2})
                for (int wpb : {1, 2, 4})
                    for (int tf : tiles) {
                        // a waves-per-block value that every launched tier halves is a duplicate
                        bool dup = true;
                        for (int i = 0; i < nseg; ++i)
                            if ((kind == SAGMS_PLAN_TIERED || tiers[i] == tiers[0]) &&
                                mixed_waves_of(tiers[i], wpb) == wpb)
                                dup = false;
                        if (dup) continue;
                        sagms_plan p{kind, tf, wpb, 0, budget, unroll};
                        if (check_plan(&p) == SAGMS_OK) cands.push_back(p);
                    }
        }
    }
    for (int tf : tiles) cands.push_back(sagms_plan{SAGMS_PLAN_PER_CODE, tf, 4, 0, 0, 1});
    const sagms_plan saved = b->plan;
    hipGraphExec_t saved_exec = b->exec;
    hipGraph_t saved_graph = b->graph;
    b->exec = nullptr;  // time the eager launches
    b->graph = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    float best_ms = INFINITY;
    sagms_plan best_plan = saved;
    int n = 0;
    for (const sagms_plan& p : cands) {
        if (he != hipSuccess || rc) break;
        b->plan = p;
        rc = enqueue(b, st);  // warm-up
        std::vector<float> ms;
        for (int r = 0; r < reps && !rc && he == hipSuccess; ++r) {
            he = hipEventRecord(e0, st);
            if (he == hipSuccess) rc = enqueue(b, st);
            if (he == hipSuccess && !rc) he = hipEventRecord(e1, st);
            if (he == hipSuccess && !rc) he = hipEventSynchronize(e1);
            float t = 0.0f;
            if (he == hipSuccess && !rc) he = hipEventElapsedTime(&t, e0, e1);
            ms.push_back(t);
        }
        if (he != hipSuccess || rc) break;
        std::sort(ms.begin(), ms.end());
        const float med = ms[ms.size() / 2];
        if (n < cap) results[n] = sagms_tune_result{p, med};
        ++n;
        if (med < best_ms) {
            best_ms = med;
            best_plan = p;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (he == hipSuccess && !rc) he = hipStreamSynchronize(st);
    if (he != hipSuccess || rc) {
        b->plan = saved;
        b->exec = saved_exec;
        b->graph = saved_graph;
        return rc ? rc : hip_fail(he, "autotuner timing");
    }
    b->exec = saved_exec;
    b->graph = saved_graph;
    if (best_plan.kind != saved.kind || best_plan.tile_frames != saved.tile_frames ||
        best_plan.waves_per_block != saved.waves_per_block || best_plan.blocks_per_cu != saved.blocks_per_cu ||
        best_plan.reg_budget != saved.reg_budget || best_plan.unroll != saved.unroll)
        drop_graph(b);
    b->plan = best_plan;
    if (count) *count = std::min(n, cap);
    if (best) *best = best_plan;
    return SAGMS_OK;
}

int sagms_decode_segments(const sagms_segment* segs, int32_t nseg, const sagms_decoder_cfg* cfg,
                          const sagms_plan* plan, void* stream) {
    SegmentSet set;
    int rc = prepare_segments(segs, nseg, cfg, false, &set);
    if (rc) return rc;
    const sagms_plan p = plan ? *plan : sagms_plan{SAGMS_PLAN_SINGLE, kMixedTileFrames, 4, 0, 0, 1};
    rc = check_plan(&p);
    if (rc) return rc;
    uint32_t* queues = nullptr;
    rc = scratch_queues(&queues);
    if (rc) return rc;
    int dev = 0, num_cu = 0;
    SAGMS_HIP(hipGetDevice(&dev));
    SAGMS_HIP(hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    // resident blocks per CU, queried once per key and process (fixed table)
    static std::mutex mu;
    static OccupancyCache occ[kMaxDevices];
    std::lock_guard<std::mutex> lock(mu);
    return enqueue_segments(set, p, cfg->msg_precision, num_cu, queues, &occ[dev], reinterpret_cast<hipStream_t>(stream));
}

int sagms_batch_destroy(sagms_batch bh) {
    Batch* b = reinterpret_cast<Batch*>(bh);
    if (!b) return fail(SAGMS_EINVAL, "null batch");
    destroy(b);
    return SAGMS_OK;
}

}  // extern "C"
