// Device entry points of libsagms: argument checks and kernel launches.
#include <cmath>

#include "internal.h"

using namespace sagms;

namespace {

constexpr int kSampleFramesPerWave = 4;

}  // namespace

namespace sagms {

int check_frames(int64_t nframes) {
    if (nframes < 0) return fail(SAGMS_EINVAL, "nframes must be >= 0");
    if (nframes > kMaxFramesPerCall)
        return fail(SAGMS_EINVAL, "too many frames for one call: %lld (at most 2^31 - 1)", (long long)nframes);
    return SAGMS_OK;
}

int check_cfg(const sagms_decoder_cfg* c) {
    if (!c) return fail(SAGMS_EINVAL, "cfg is null");
    if (c->kind < SAGMS_MS || c->kind > SAGMS_BP) return fail(SAGMS_EINVAL, "unknown decoder kind %d", c->kind);
    if (c->schedule != SAGMS_FLOODING && c->schedule != SAGMS_LAYERED)
        return fail(SAGMS_EINVAL, "unknown schedule %d", c->schedule);
    if (c->schedule == SAGMS_LAYERED && (c->kind == SAGMS_BP || c->msg_precision != SAGMS_MSG_FP32))
        return fail(SAGMS_EUNSUPPORTED, "the layered schedule runs MS, SMS and SAGMS with FP32 messages");
    if (c->msg_precision < SAGMS_MSG_FP32 || c->msg_precision > SAGMS_MSG_INT6)
        return fail(SAGMS_EUNSUPPORTED, "message precision %d not available", c->msg_precision);
    if (c->kind == SAGMS_BP && c->msg_precision != SAGMS_MSG_FP32)
        return fail(SAGMS_EUNSUPPORTED, "BP runs with FP32 messages only");
    if (c->lmax < 1) return fail(SAGMS_EINVAL, "lmax must be >= 1 (got %d)", c->lmax);
    if (c->frames_per_wave < 0 || c->frames_per_wave > 1024)
        return fail(SAGMS_EINVAL, "frames_per_wave must lie in [0, 1024]");
    if (c->reserved != 0) return fail(SAGMS_EINVAL, "reserved field must be 0");
    if (c->kind == SAGMS_SMS && !(c->alpha > 0.0 && c->alpha <= 1.0))
        return fail(SAGMS_EINVAL, "SMS alpha must lie in (0, 1]");
    if (c->kind == SAGMS_SAGMS) {
        if (!(c->alpha_min > 0.0 && c->alpha_min <= 1.0 && c->alpha_max > 0.0 && c->alpha_max <= 1.0))
            return fail(SAGMS_EINVAL, "alpha_min and alpha_max must lie in (0, 1]");
        if (!(c->eta >= 1.0)) return fail(SAGMS_EINVAL, "eta must be >= 1");
        // stability constraint of Section III: alpha_max * eta <= 1
        if (!(c->alpha_max * c->eta <= 1.0)) return fail(SAGMS_EINVAL, "alpha_max * eta = %g exceeds 1", c->alpha_max * c->eta);
    }
    return SAGMS_OK;
}

GainLaw gain_law(const sagms_decoder_cfg* cfg) {
    GainLaw law{cfg->kind, 0, 0.0, 0.0, 0.0, 0.0};
    if (cfg->kind == SAGMS_SMS) law.a = cfg->alpha;
    if (cfg->kind == SAGMS_SAGMS) {
        law.amin = cfg->alpha_min;
        law.amax = cfg->alpha_max;
        law.eta = cfg->eta;
    }
    if (cfg->kind == SAGMS_BP) law.kind = SAGMS_MS;  // BP ignores the gains
    return law;
}

DecodeArgs decode_args(const Graph* g, const DeviceTables* t, const GainLaw& gains, const uint64_t* synd,
                       const float* llr0, int64_t nframes, uint64_t* ehat, int32_t* iters, uint8_t* converged,
                       float* posterior, int lmax, int frames_per_wave) {
    DecodeArgs a{};
    a.synd = synd;
    a.llr0 = llr0;
    a.gains = gains;
    a.cn_addr = t->cn_addr;
    a.vn_addr = t->vn_addr;
    a.ehat = ehat;
    a.iters = iters;
    a.conv = converged;
    a.post = posterior;
    a.nframes = nframes;
    a.m = g->m;
    a.n = g->n;
    a.wm = g->wm;
    a.wn = g->wn;
    a.lmax = lmax;
    a.frames_per_wave = frames_per_wave;  // 0: the decode launcher's tapered schedule
    a.L = g->layout;
    return a;
}

}  // namespace sagms

extern "C" {

int sagms_gen_errors(sagms_graph gh, uint64_t seed, uint32_t stream_id, uint64_t frame0, int64_t nframes, double p,
                     uint64_t* ex, uint64_t* ez, uint64_t* synd, void* stream) {
    Graph* g = reinterpret_cast<Graph*>(gh);
    if (!g) return fail(SAGMS_EINVAL, "null graph");
    int rc = check_frames(nframes);
    if (rc) return rc;
    if (!(p >= 0.0 && p < 1.0)) return fail(SAGMS_EINVAL, "p must lie in [0, 1)");
    if (nframes == 0) return SAGMS_OK;
    if (!ex || !synd) return fail(SAGMS_EINVAL, "ex and synd must not be null");
    if (g->joint && !ez) return fail(SAGMS_EINVAL, "joint graphs need the ez plane (the X-type checks read it)");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    DeviceTables* t = nullptr;
    rc = device_tables(g, &t);
    if (rc) return rc;
    SampleArgs a{};
    a.cols = t->cols;
    a.rows = t->rows;
    a.ex = ex;
    a.ez = ez;
    a.synd = synd;
    a.seed = seed;
    a.frame0 = frame0;
    a.nframes = nframes;
    a.stream_id = stream_id;
    const double two32 = 4294967296.0;
    a.tx = (uint32_t)std::floor((p / 3.0) * two32);
    a.ty = (uint32_t)std::floor(((2.0 * p) / 3.0) * two32);
    a.tz = (uint32_t)std::floor(p * two32);
    a.m = g->m;
    a.n = g->n;
    a.dc = std::max(g->dc_max, 1);
    a.wn = g->wn;
    a.wm = g->wm;
    a.frames_per_wave = kSampleFramesPerWave;
    a.joint = g->joint ? 1 : 0;
    return launch_sample(a, st);
}

int sagms_decode(sagms_graph gh, const uint64_t* synd, const float* llr0, const sagms_decoder_cfg* cfg,
                 int64_t nframes, uint64_t* ehat, int32_t* iters, uint8_t* converged, void* stream) {
    return sagms_decode_soft(gh, synd, llr0, cfg, nframes, ehat, iters, converged, nullptr, stream);
}

int sagms_decode_soft(sagms_graph gh, const uint64_t* synd, const float* llr0, const sagms_decoder_cfg* cfg,
                      int64_t nframes, uint64_t* ehat, int32_t* iters, uint8_t* converged, float* posterior,
                      void* stream) {
    Graph* g = reinterpret_cast<Graph*>(gh);
    if (!g) return fail(SAGMS_EINVAL, "null graph");
    int rc = check_cfg(cfg);
    if (rc) return rc;
    rc = check_frames(nframes);
    if (rc) return rc;
    if (!g->shape_ok)
        return fail(SAGMS_EUNSUPPORTED, "no decode kernel fits m=%d n=%d dc=%d dv=%d", g->m, g->n, g->dc_max, g->dv_max);
    if (nframes == 0) return SAGMS_OK;
    if (!synd || !llr0 || !ehat || !iters || !converged) return fail(SAGMS_EINVAL, "null buffer");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (cfg->schedule == SAGMS_LAYERED && g->layered.status != SAGMS_OK)
        return fail(g->layered.status, "%s", g->layered.why.c_str());
    if (g->joint && (cfg->kind == SAGMS_BP || cfg->msg_precision != SAGMS_MSG_FP32))
        return fail(SAGMS_EUNSUPPORTED, "joint graphs decode MS, SMS and SAGMS with FP32 messages");
    DeviceTables* t = nullptr;
    rc = device_tables(g, &t);
    if (rc) return rc;
    if (g->joint) {
        JointArgs ja{};
        ja.synd = synd;
        ja.llr0 = llr0;
        ja.gains = gain_law(cfg);
        ja.cn_addr = t->cn_addr;
        ja.vn_addr = t->vn_addr;
        ja.ehat = ehat;
        ja.iters = iters;
        ja.conv = converged;
        ja.gamma = posterior;
        ja.nframes = nframes;
        ja.m = g->m;
        ja.n = g->n;
        ja.wm = g->wm;
        ja.wn = g->wn;
        ja.lmax = cfg->lmax;
        ja.frames_per_wave = cfg->frames_per_wave;
        ja.L = g->jlayout;
        return launch_joint(g->shape, ja, st);
    }
    const DecodeArgs a = decode_args(g, t, gain_law(cfg), synd, llr0, nframes, ehat, iters, converged, posterior,
                                     cfg->lmax, cfg->frames_per_wave);
    if (cfg->schedule == SAGMS_LAYERED) return launch_layered(t->layered, a, st);
    return launch_decode(g->shape, cfg->kind == SAGMS_BP, cfg->msg_precision, a, st);
}

int sagms_judge(sagms_graph gh, const uint64_t* ex, const uint64_t* ehat, const uint8_t* converged,
                const int32_t* iters, int64_t nframes, uint8_t* failv, uint64_t* counters, void* stream) {
    Graph* g = reinterpret_cast<Graph*>(gh);
    if (!g) return fail(SAGMS_EINVAL, "null graph");
    if (!g->have_other) return fail(SAGMS_EINVAL, "the judge needs a graph built with the other check matrix");
    if (g->joint) return fail(SAGMS_EINVAL, "joint graphs are judged by sagms_judge_joint (both error planes)");
    int rc = check_frames(nframes);
    if (rc) return rc;
    if (nframes == 0) return SAGMS_OK;
    if (!ex || !ehat || !converged || !iters || !counters) return fail(SAGMS_EINVAL, "null buffer");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    DeviceTables* t = nullptr;
    rc = device_tables(g, &t);
    if (rc) return rc;
    JudgeArgs a{};
    a.ex = ex;
    a.ehat = ehat;
    a.conv = converged;
    a.iters = iters;
    a.logicals = t->logicals;
    a.fail = failv;
    a.counters = counters;
    a.nframes = nframes;
    a.k = g->k;
    a.wn = g->wn;
    a.wplane = g->wn;
    return launch_judge(a, st);
}

int sagms_judge_joint(sagms_graph gh, const uint64_t* ex, const uint64_t* ez, const uint64_t* ehat,
                      const uint8_t* converged, const int32_t* iters, int64_t nframes, uint8_t* failv,
                      uint64_t* counters, void* stream) {
    Graph* g = reinterpret_cast<Graph*>(gh);
    if (!g) return fail(SAGMS_EINVAL, "null graph");
    if (!g->joint) return fail(SAGMS_EINVAL, "sagms_judge_joint needs a joint graph (sagms_build_gb_joint)");
    int rc = check_frames(nframes);
    if (rc) return rc;
    if (nframes == 0) return SAGMS_OK;
    if (!ex || !ez || !ehat || !converged || !iters || !counters) return fail(SAGMS_EINVAL, "null buffer");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    DeviceTables* t = nullptr;
    rc = device_tables(g, &t);
    if (rc) return rc;
    JudgeArgs a{};
    a.ex = ex;
    a.ez = ez;
    a.ehat = ehat;
    a.conv = converged;
    a.iters = iters;
    a.logicals = t->logicals;
    a.fail = failv;
    a.counters = counters;
    a.nframes = nframes;
    a.k = 2 * g->k;
    a.wn = g->we;
    a.wplane = g->wn;
    return launch_judge(a, st);
}

}  // extern "C"
