// Serving runtime: continuous batching of decode requests over several codes.
//
// Requests (syndromes of one code, in host memory) wait in one FIFO per
// register class of the codes.  A progress step retires finished launches
// (copying their outputs to the requests' host buffers) and then, while a
// stream is free and the frame budget allows, takes the class whose oldest
// request is oldest, admits requests from its FIFO up to the per-launch frame
// limit, stages their syndromes in pinned memory and enqueues on that stream
// one host-to-device copy, one persistent mixed-code launch over the admitted
// frames (one segment per code), one device-to-host copy and an event.
// Launches on different streams run concurrently, so work admitted while
// other launches are on the GPU fills the compute units their finished waves
// free.  Every frame is decoded by the same per-frame code as sagms_decode.
#include <chrono>
#include <cstring>
#include <deque>

#include "internal.h"

using namespace sagms;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kMaxServerStreams = 8;

struct Code {
    Graph* g = nullptr;
    DeviceTables* t = nullptr;
    float* llr0 = nullptr;  // device copy
    int tier = 0, shape = 0;
};

struct Req {
    int64_t id;
    sagms_request r;
    double submit_us;
};

struct Seg {  // one code's frames in a launch
    int code;
    int64_t frames, in_word, ehat_word, iters_off, conv_off;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    uint64_t* h_in = nullptr;
    unsigned char* h_out = nullptr;
    uint64_t* d_in = nullptr;
    unsigned char* d_out = nullptr;
    uint32_t* d_queues = nullptr;
    std::vector<Req> reqs;
    std::vector<int64_t> first;  // per request: its first frame in its segment
    std::vector<Seg> segs;
    int64_t frames = 0;
    double admit_us = 0.0;
};

struct Server {
    int device = 0, num_cu = 0, mt = 0;
    sagms_decoder_cfg cfg{};
    sagms_server_cfg scfg{};
    std::vector<Code> codes;
    int max_wm = 1, max_wn = 1;
    std::deque<Req> lane[kNumMixedTiers];
    std::vector<Slot> slots;
    std::deque<sagms_completion> completed;
    int64_t next_id = 0, in_flight = 0, queued = 0, with_deadline = 0;
    int64_t lane_frames[kNumMixedTiers] = {};  // frames waiting per class
    OccupancyCache occ;
    Clock::time_point t0;
    size_t in_bytes = 0, out_bytes = 0;

    double now_us() const { return std::chrono::duration<double, std::micro>(Clock::now() - t0).count(); }
};

void destroy(Server* s) {
    for (Slot& x : s->slots) {
        if (x.st) (void)hipStreamSynchronize(x.st);
        if (x.done) (void)hipEventDestroy(x.done);
        if (x.st) (void)hipStreamDestroy(x.st);
        if (x.h_in) (void)hipHostFree(x.h_in);
        if (x.h_out) (void)hipHostFree(x.h_out);
        if (x.d_in) (void)hipFree(x.d_in);
        if (x.d_out) (void)hipFree(x.d_out);
        if (x.d_queues) (void)hipFree(x.d_queues);
    }
    for (Code& c : s->codes)
        if (c.llr0) (void)hipFree(c.llr0);
    delete s;
}

int64_t align64(int64_t x) { return (x + 63) & ~int64_t(63); }

// Copies the outputs of a finished launch to its requests and records them.
void retire(Server* s, Slot& x, double t) {
    for (size_t i = 0; i < x.reqs.size(); ++i) {
        const Req& q = x.reqs[i];
        const Seg* sg = nullptr;
        for (const Seg& g : x.segs)
            if (g.code == q.r.code) sg = &g;
        const Code& c = s->codes[q.r.code];
        const int64_t f0 = x.first[i], nf = q.r.nframes;
        std::memcpy(q.r.ehat, reinterpret_cast<uint64_t*>(x.h_out) + sg->ehat_word + f0 * c.g->wn,
                    (size_t)nf * c.g->wn * sizeof(uint64_t));
        std::memcpy(q.r.iters, reinterpret_cast<int32_t*>(x.h_out + sg->iters_off) + f0, (size_t)nf * sizeof(int32_t));
        std::memcpy(q.r.converged, x.h_out + sg->conv_off + f0, (size_t)nf);
        s->completed.push_back(sagms_completion{q.id, SAGMS_REQ_DONE, 0, q.submit_us, x.admit_us, t});
    }
    s->in_flight -= x.frames;
    x.reqs.clear();
    x.busy = false;
}

// Returns the requests admitted into slot x to the head of their FIFO, in
// their order, after a launch could not be enqueued.
void unadmit(Server* s, Slot& x, int tier) {
    std::deque<Req>& q = s->lane[tier];
    for (size_t i = x.reqs.size(); i-- > 0;) {
        const Req& r = x.reqs[i];
        s->lane_frames[tier] += r.r.nframes;
        if (r.r.deadline_us > 0.0) ++s->with_deadline;
        q.push_front(r);
    }
    s->queued += (int64_t)x.reqs.size();
    x.reqs.clear();
    x.first.clear();
    x.segs.clear();
}

int enqueue(Server* s, Slot& x, int tier, int64_t frames, double t);

// Admits requests of one class into slot x and enqueues its launch.  If the
// launch cannot be enqueued the requests stay queued and the error returns.
int launch(Server* s, Slot& x, int tier, double t) {
    std::deque<Req>& q = s->lane[tier];
    const int64_t cap = std::min<int64_t>(s->scfg.max_frames_per_launch, s->scfg.max_frames_in_flight - s->in_flight);
    x.reqs.clear();
    x.first.clear();
    x.segs.clear();
    int64_t frames = 0;
    while (!q.empty() && frames + q.front().r.nframes <= cap) {
        frames += q.front().r.nframes;
        s->lane_frames[tier] -= q.front().r.nframes;
        if (q.front().r.deadline_us > 0.0) --s->with_deadline;
        x.reqs.push_back(q.front());
        q.pop_front();
    }
    if (x.reqs.empty()) return SAGMS_OK;
    s->queued -= (int64_t)x.reqs.size();
    const int rc = enqueue(s, x, tier, frames, t);
    if (rc) {
        // the copy in may have been enqueued: let it finish reading the
        // staging buffer before a later launch refills it
        (void)hipStreamSynchronize(x.st);
        unadmit(s, x, tier);
    }
    return rc;
}

// Lays out the admitted requests of slot x as one segment per code, stages
// their syndromes and enqueues the copy in, the launch and the copy out.
int enqueue(Server* s, Slot& x, int tier, int64_t frames, double t) {
    // one segment per code, requests in admission order within it
    std::vector<int64_t> seg_of(s->codes.size(), -1);
    for (const Req& r : x.reqs)
        if (seg_of[r.r.code] < 0) {
            seg_of[r.r.code] = (int64_t)x.segs.size();
            x.segs.push_back(Seg{r.r.code, 0, 0, 0, 0, 0});
        }
    for (const Req& r : x.reqs) {
        Seg& g = x.segs[seg_of[r.r.code]];
        x.first.push_back(g.frames);
        g.frames += r.r.nframes;
    }
    int64_t in_w = 0, ehat_w = 0;
    for (Seg& g : x.segs) {
        g.in_word = in_w;
        g.ehat_word = ehat_w;
        in_w += g.frames * s->codes[g.code].g->wm;
        ehat_w += g.frames * s->codes[g.code].g->wn;
    }
    int64_t off = align64(ehat_w * 8);
    for (Seg& g : x.segs) {
        g.iters_off = off;
        off += align64(g.frames * 4);
    }
    for (Seg& g : x.segs) {
        g.conv_off = off;
        off += align64(g.frames);
    }
    if ((size_t)(in_w * 8) > s->in_bytes || (size_t)off > s->out_bytes)
        return fail(SAGMS_EINVAL, "launch exceeds the staging buffers (internal)");
    for (size_t i = 0; i < x.reqs.size(); ++i) {
        const Req& r = x.reqs[i];
        const Seg& g = x.segs[seg_of[r.r.code]];
        const int wm = s->codes[r.r.code].g->wm;
        std::memcpy(x.h_in + g.in_word + x.first[i] * wm, r.r.synd, (size_t)r.r.nframes * wm * sizeof(uint64_t));
    }
    std::vector<MixedSegment> ms;
    for (const Seg& g : x.segs) {
        const Code& c = s->codes[g.code];
        MixedSegment m{};
        m.a = decode_args(c.g, c.t, gain_law(&s->cfg), x.d_in + g.in_word, c.llr0, g.frames,
                          reinterpret_cast<uint64_t*>(x.d_out) + g.ehat_word,
                          reinterpret_cast<int32_t*>(x.d_out + g.iters_off), x.d_out + g.conv_off, nullptr,
                          s->cfg.lmax, 0);
        m.shape = c.shape;
        ms.push_back(m);
    }
    SAGMS_HIP(hipMemcpyAsync(x.d_in, x.h_in, (size_t)in_w * 8, hipMemcpyHostToDevice, x.st));
    MixedLaunch L{s->scfg.tile_frames, s->scfg.waves_per_block, 0, s->scfg.reg_budget, 1};
    int rc = launch_segments(ms.data(), (int)ms.size(), tier, L, s->num_cu, s->mt, x.d_queues, &s->occ, x.st);
    if (rc) return rc;
    SAGMS_HIP(hipMemcpyAsync(x.h_out, x.d_out, (size_t)off, hipMemcpyDeviceToHost, x.st));
    SAGMS_HIP(hipEventRecord(x.done, x.st));
    x.busy = true;
    x.frames = frames;
    x.admit_us = t;
    s->in_flight += frames;
    return SAGMS_OK;
}

int progress(Server* s, int* retired) {
    *retired = 0;
    double t = s->now_us();
    for (Slot& x : s->slots) {
        if (!x.busy) continue;
        hipError_t e = hipEventQuery(x.done);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return hip_fail(e, "hipEventQuery");
        retire(s, x, t);
        ++*retired;
    }
    // cancel waiting requests whose admission deadline has passed
    if (s->with_deadline > 0)
        for (int k = 0; k < kNumMixedTiers; ++k) {
            std::deque<Req>& q = s->lane[k];
            for (auto it = q.begin(); it != q.end();) {
                if (it->r.deadline_us > 0.0 && t - it->submit_us > it->r.deadline_us) {
                    s->completed.push_back(sagms_completion{it->id, SAGMS_REQ_CANCELLED, 0, it->submit_us, -1.0, t});
                    s->lane_frames[k] -= it->r.nframes;
                    it = q.erase(it);
                    --s->queued;
                    --s->with_deadline;
                } else {
                    ++it;
                }
            }
        }
    // a class launches on its waiting time only while fewer than half of the
    // streams (rounded up) are busy: under light load fewer launches share
    // the GPU and each finishes sooner; under load the frame count starts
    // the others
    int busy = 0;
    for (const Slot& x : s->slots) busy += x.busy ? 1 : 0;
    const int eager = (s->scfg.streams + 1) / 2;
    for (Slot& x : s->slots) {
        if (x.busy) continue;
        int tier = -1;
        for (int k = 0; k < kNumMixedTiers; ++k) {
            if (s->lane[k].empty()) continue;
            const bool ready = s->in_flight == 0 || s->lane_frames[k] >= s->scfg.min_launch_frames ||
                               (busy < eager && t - s->lane[k].front().submit_us >= s->scfg.max_wait_us);
            if (ready && (tier < 0 || s->lane[k].front().submit_us < s->lane[tier].front().submit_us)) tier = k;
        }
        if (tier < 0) break;
        if (s->lane[tier].front().r.nframes > s->scfg.max_frames_in_flight - s->in_flight) break;  // budget full
        int rc = launch(s, x, tier, t);
        if (rc) return rc;
        busy += x.busy ? 1 : 0;
    }
    return SAGMS_OK;
}

int check_request(const Server* s, const sagms_request* r) {
    if (!r) return fail(SAGMS_EINVAL, "request is null");
    if (r->code < 0 || r->code >= (int)s->codes.size()) return fail(SAGMS_EINVAL, "request code %d out of range", r->code);
    if (r->nframes < 1 || r->nframes > s->scfg.max_frames_per_launch)
        return fail(SAGMS_EINVAL, "request of %d frames: need 1 .. max_frames_per_launch (%d)", r->nframes,
                    s->scfg.max_frames_per_launch);
    if (!r->synd || !r->ehat || !r->iters || !r->converged) return fail(SAGMS_EINVAL, "request with a null buffer");
    if (!(r->deadline_us >= 0.0)) return fail(SAGMS_EINVAL, "deadline must be >= 0");
    return SAGMS_OK;
}

void push(Server* s, const sagms_request* r, double submit_us, int64_t* id) {
    Req q{s->next_id++, *r, submit_us};
    s->lane[s->codes[r->code].tier].push_back(q);
    s->lane_frames[s->codes[r->code].tier] += r->nframes;
    ++s->queued;
    if (r->deadline_us > 0.0) ++s->with_deadline;
    if (id) *id = q.id;
}

}  // namespace

extern "C" {

int sagms_server_create(const sagms_graph* graphs, const float* const* llr0_host, int32_t ncodes,
                        const sagms_decoder_cfg* cfg, const sagms_server_cfg* scfg, sagms_server* out) {
    if (!out) return fail(SAGMS_EINVAL, "out is null");
    *out = nullptr;
    if (!graphs || !llr0_host) return fail(SAGMS_EINVAL, "graphs and llr0_host must not be null");
    if (ncodes < 1 || ncodes > kMaxSegments) return fail(SAGMS_EINVAL, "ncodes must lie in [1, %d]", kMaxSegments);
    int rc = check_cfg(cfg);
    if (rc) return rc;
    if (cfg->kind == SAGMS_BP) return fail(SAGMS_EUNSUPPORTED, "the server runs MS, SMS and SAGMS only");
    if (cfg->schedule != SAGMS_FLOODING) return fail(SAGMS_EUNSUPPORTED, "the server runs the flooding schedule only");
    if (!scfg) return fail(SAGMS_EINVAL, "server configuration is null");
    if (scfg->max_frames_per_launch < 1 || scfg->max_frames_per_launch > (1 << 24))
        return fail(SAGMS_EINVAL, "max_frames_per_launch must lie in [1, 2^24]");
    if (scfg->max_frames_in_flight < scfg->max_frames_per_launch)
        return fail(SAGMS_EINVAL, "max_frames_in_flight must be >= max_frames_per_launch");
    if (scfg->streams < 1 || scfg->streams > kMaxServerStreams)
        return fail(SAGMS_EINVAL, "streams must lie in [1, %d]", kMaxServerStreams);
    if (scfg->tile_frames < 1 || scfg->tile_frames > 1024) return fail(SAGMS_EINVAL, "tile_frames must lie in [1, 1024]");
    if (scfg->waves_per_block != 1 && scfg->waves_per_block != 2 && scfg->waves_per_block != 4)
        return fail(SAGMS_EINVAL, "waves_per_block must be 1, 2 or 4");
    if (scfg->reg_budget != 0 && scfg->reg_budget != 1) return fail(SAGMS_EINVAL, "reg_budget must be 0 or 1");
    if (scfg->min_launch_frames < 0 || scfg->min_launch_frames > scfg->max_frames_per_launch)
        return fail(SAGMS_EINVAL, "min_launch_frames must lie in [0, max_frames_per_launch]");
    if (!(scfg->max_wait_us >= 0.0)) return fail(SAGMS_EINVAL, "max_wait_us must be >= 0");
    for (int c = 0; c < ncodes; ++c) {
        Graph* g = reinterpret_cast<Graph*>(graphs[c]);
        if (!g) return fail(SAGMS_EINVAL, "code %d: null graph", c);
        if (!llr0_host[c]) return fail(SAGMS_EINVAL, "code %d: null prior", c);
        if (g->joint) return fail(SAGMS_EUNSUPPORTED, "code %d: joint graphs decode through sagms_decode only", c);
        if (!g->shape_ok || mixed_tier_of_shape(shape_index(g->shape)) < 0)
            return fail(SAGMS_EUNSUPPORTED, "code %d: no decode kernel fits it", c);
    }
    Server* s = new Server();
    s->cfg = *cfg;
    s->scfg = *scfg;
    s->mt = cfg->msg_precision;
    s->t0 = Clock::now();
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&s->num_cu, hipDeviceAttributeMultiprocessorCount, s->device);
    if (e != hipSuccess) {
        destroy(s);
        return hip_fail(e, "hipGetDevice / hipDeviceGetAttribute");
    }
    for (int c = 0; c < ncodes; ++c) {
        Code k;
        k.g = reinterpret_cast<Graph*>(graphs[c]);
        k.shape = shape_index(k.g->shape);
        k.tier = mixed_tier_of_shape(k.shape);
        rc = upload_tables(k.g, &k.t);
        if (!rc) {
            e = hipMalloc(&k.llr0, sizeof(float) * k.g->n);
            if (e == hipSuccess) e = hipMemcpy(k.llr0, llr0_host[c], sizeof(float) * k.g->n, hipMemcpyHostToDevice);
            if (e != hipSuccess) rc = hip_fail(e, "prior upload");
        }
        s->codes.push_back(k);
        if (rc) {
            destroy(s);
            return rc;
        }
        s->max_wm = std::max(s->max_wm, k.g->wm);
        s->max_wn = std::max(s->max_wn, k.g->wn);
    }
    const int64_t F = scfg->max_frames_per_launch;
    s->in_bytes = (size_t)F * s->max_wm * 8;
    // ehat block, then per-segment iters and flags, each 64-byte aligned
    s->out_bytes = (size_t)align64(F * s->max_wn * 8) + 2 * kMaxSegments * 64 + (size_t)align64(F * 4) + align64(F);
    s->slots.resize(scfg->streams);
    for (Slot& x : s->slots) {
        e = hipStreamCreateWithFlags(&x.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&x.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc(&x.h_in, s->in_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(&x.h_out, s->out_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(&x.d_in, s->in_bytes);
        if (e == hipSuccess) e = hipMalloc(&x.d_out, s->out_bytes);
        if (e == hipSuccess) e = hipMalloc(&x.d_queues, sizeof(uint32_t) * kMaxQueues * kQueueStride);
        if (e != hipSuccess) {
            destroy(s);
            return hip_fail(e, "server buffers");
        }
    }
    e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        destroy(s);
        return hip_fail(e, "server set-up");
    }
    *out = reinterpret_cast<sagms_server>(s);
    return SAGMS_OK;
}

int sagms_server_submit(sagms_server sh, const sagms_request* req, int64_t* id) {
    Server* s = reinterpret_cast<Server*>(sh);
    if (!s) return fail(SAGMS_EINVAL, "null server");
    int rc = check_request(s, req);
    if (rc) return rc;
    push(s, req, s->now_us(), id);
    return SAGMS_OK;
}

int sagms_server_progress(sagms_server sh, sagms_completion* done, int32_t cap, int32_t* ndone) {
    Server* s = reinterpret_cast<Server*>(sh);
    if (!s) return fail(SAGMS_EINVAL, "null server");
    if (cap < 0 || (cap > 0 && !done)) return fail(SAGMS_EINVAL, "done is null");
    int retired = 0;
    int rc = progress(s, &retired);
    int n = 0;
    while (n < cap && !s->completed.empty()) {
        done[n++] = s->completed.front();
        s->completed.pop_front();
    }
    if (ndone) *ndone = n;
    return rc;
}

int sagms_server_pending(sagms_server sh, int64_t* queued, int64_t* frames_in_flight, int64_t* completions) {
    Server* s = reinterpret_cast<Server*>(sh);
    if (!s) return fail(SAGMS_EINVAL, "null server");
    if (queued) *queued = s->queued;
    if (frames_in_flight) *frames_in_flight = s->in_flight;
    if (completions) *completions = (int64_t)s->completed.size();
    return SAGMS_OK;
}

int sagms_server_replay(sagms_server sh, const sagms_request* reqs, const double* arrival_us, int64_t n,
                        double timeout_s, sagms_completion* out) {
    Server* s = reinterpret_cast<Server*>(sh);
    if (!s) return fail(SAGMS_EINVAL, "null server");
    if (n < 0 || (n > 0 && (!reqs || !arrival_us || !out))) return fail(SAGMS_EINVAL, "null trace buffers");
    if (!(timeout_s > 0.0)) return fail(SAGMS_EINVAL, "timeout_s must be > 0");
    if (s->queued || s->in_flight || !s->completed.empty())
        return fail(SAGMS_EINVAL, "replay needs an idle server (no queued, running or unread requests)");
    for (int64_t i = 0; i < n; ++i) {
        int rc = check_request(s, &reqs[i]);
        if (rc) return rc;
        if (!(arrival_us[i] >= 0.0) || (i > 0 && arrival_us[i] < arrival_us[i - 1]))
            return fail(SAGMS_EINVAL, "arrival times must be >= 0 and non-decreasing");
    }
    const int64_t first_id = s->next_id;
    const double start = s->now_us();
    double last_event = start;
    int64_t next = 0, finished = 0;
    while (finished < n) {
        const double t = s->now_us();
        while (next < n && start + arrival_us[next] <= t) {
            // the scheduled arrival time is the submission time: host lag counts as latency
            push(s, &reqs[next], start + arrival_us[next], nullptr);
            ++next;
        }
        int retired = 0;
        int rc = progress(s, &retired);
        if (rc) return rc;
        while (!s->completed.empty()) {
            sagms_completion c = s->completed.front();
            s->completed.pop_front();
            out[c.id - first_id] = c;
            ++finished;
            last_event = t;
        }
        if (s->in_flight == 0) last_event = t;
        if ((t - last_event) * 1e-6 > timeout_s)
            return fail(SAGMS_EHIP, "no launch finished for %.1f s", timeout_s);
    }
    return SAGMS_OK;
}

int sagms_server_destroy(sagms_server sh) {
    Server* s = reinterpret_cast<Server*>(sh);
    if (!s) return fail(SAGMS_EINVAL, "null server");
    destroy(s);
    return SAGMS_OK;
}

}  // extern "C"
