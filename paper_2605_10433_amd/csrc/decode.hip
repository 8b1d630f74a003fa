// Decode kernel with a static frame assignment (schedule.h): each wave
// decodes a run of consecutive frames.  The default launch tapers: most
// frames go in runs of kDecodeFramesPerWave, which amortise a wave's set-up,
// and the last ones in runs of halving length, so that the waves still
// running after the whole grid has been dispatched hold little work.  The
// per-frame algorithm (Algorithm 1 of the paper) is in decode_core.h.
#include <mutex>
#include <unordered_map>

#include "decode_core.h"
#include "schedule.h"

namespace sagms {

constexpr int kWavesPerBlock = 4;  // the kernel's bound
// Waves per block at launch.  A block's LDS is released only when its last
// wave ends, and the waves of a block finish their runs at different times.
// One-block codes (CPL = 1) use blocks of 2: 4 % shorter decodes than blocks
// of 4 on the l = 63 code, and more room for the pipelined step's sampler
// than blocks of 1.  Larger codes, whose waves hold 4-8 times the LDS, use
// blocks of 1 (l = 127 / 255 / 511: 1 / 2.5 / 4.5 % shorter than blocks of 2).
constexpr int kLaunchWavesPerBlock = 2;
constexpr int kTaperLevels = 2;  // waves per tail level of the tapered schedule, in resident waves

// kg: the gain pairs of one-block codes (CPL == 1); unused otherwise.
template <int DC, int DV, int CPL, int VPL, bool BP, int MT>
__global__ void __launch_bounds__(64 * kWavesPerBlock) decode_kernel(DecodeArgs a, WaveSchedule ws, KernelGains kg) {
    using LY = Lay<DC, CPL, VPL>;
    extern __shared__ float lds_all[];
    const int lane = threadIdx.x & 63;
    // wave-uniform, so that the frame index and the output addresses are
    // scalar values (the syndrome loads are kept vector loads: scalar loads
    // of them fetched twice their bytes from HBM)
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float* lds = lds_all + wib * LY::WORDS;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + wib;
    if (wave >= ws.wave0[ws.levels]) return;
    int k = 0;
    while (k + 1 < ws.levels && wave >= ws.wave0[k + 1]) ++k;
    const int64_t f_begin = ws.frame0[k] + (wave - ws.wave0[k]) * ws.chunk[k];
    const int64_t f_end = min(f_begin + (int64_t)ws.chunk[k], ws.frame0[k + 1]);
    if (f_begin >= f_end) return;
    using WD = WaveDecoder<DC, DV, CPL, VPL, BP, MT, CPL == 1>;
    WD d;
    d.load(a, lds, lane);
    uint64_t word[CPL];
    uint32_t sb[CPL];
    WD::load_syndrome(a, f_begin, word);
    WD::syndrome_bits(a, lane, word, sb);
    for (int64_t f = f_begin; f < f_end; ++f) d.frame(a, lds, lane, f, sb, f + 1 < f_end ? f + 1 : f, &kg);
}

// Waves per block: for one-block codes up to kLaunchWavesPerBlock, as many as
// fit in 64 KiB of LDS; 1 for larger codes.
static int waves_per_block(const DecodeLayout& L, int cpl) {
    if (cpl > 1) return 1;
    int w = (int)(65536 / ((size_t)L.words * sizeof(float)));
    return w < 1 ? 1 : (w > kLaunchWavesPerBlock ? kLaunchWavesPerBlock : w);
}

// Host evaluation of the gain law, operation for operation as gain_pair.
static float2 host_gain_pair(const GainLaw& law, int w, int m) {
    double gs = 1.0, gu = 1.0;
    if (law.kind == SAGMS_SMS) {
        gs = gu = law.a;
    } else if (law.kind == SAGMS_SAGMS) {
        const double gamma = (double)w / (double)m;
        const double g = law.amax - (law.amax - law.amin) * gamma;
        gs = g;
        gu = g * law.eta;
    }
    return make_float2((float)gs, (float)gu);
}

template <int DC, int DV, int CPL, int VPL, bool BP, int MT>
static void launch_one(dim3 grid, dim3 block, size_t lds, hipStream_t st, const DecodeArgs& a, const WaveSchedule& ws) {
    KernelGains kg{};
    if constexpr (CPL == 1)
        for (int w = 0; w <= 64; ++w) kg.g[w] = host_gain_pair(a.gains, w, a.m);
    hipLaunchKernelGGL((decode_kernel<DC, DV, CPL, VPL, BP, MT>), grid, block, lds, st, a, ws, kg);
}

// Waves of one kernel resident on the current device at once (occupancy of
// registers and LDS times compute units), queried once per kernel and device.
int resident_waves(const void* kernel, int wpb, size_t lds, int64_t* out) {
    static std::mutex mu;
    static std::unordered_map<uint64_t, int64_t> cache;
    int dev = 0;
    SAGMS_HIP(hipGetDevice(&dev));
    const uint64_t key = reinterpret_cast<uintptr_t>(kernel) * 64 + (uint64_t)dev;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            *out = it->second;
            return SAGMS_OK;
        }
    }
    int blocks = 0, cus = 0;
    SAGMS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, 64 * wpb, lds));
    SAGMS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t r = std::max<int64_t>(1, (int64_t)blocks * wpb * cus);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = r;
    *out = r;
    return SAGMS_OK;
}

template <int DC, int DV, int CPL, int VPL, bool BP, int MT>
static int launch_kernel(const DecodeArgs& a, int wpb, size_t lds, hipStream_t st) {
    int64_t resident = 0;
    if (a.frames_per_wave == 0) {
        const int rc = resident_waves(reinterpret_cast<const void*>(&decode_kernel<DC, DV, CPL, VPL, BP, MT>), wpb,
                                      lds, &resident);
        if (rc) return rc;
    }
    const WaveSchedule ws = make_schedule(a.nframes, a.frames_per_wave, resident * kTaperLevels, kDecodeFramesPerWave);
    const int64_t blocks = (ws.wave0[ws.levels] + wpb - 1) / wpb;
    if (blocks > 0x7fffffff) return fail(SAGMS_EINVAL, "too many frames for one launch");
    launch_one<DC, DV, CPL, VPL, BP, MT>(dim3((unsigned)blocks), dim3(64 * wpb), lds, st, a, ws);
    return SAGMS_OK;
}

template <int DC, int DV, int CPL, int VPL>
static int launch_shape(bool bp, int mt, const DecodeArgs& a, hipStream_t st) {
    using LY = Lay<DC, CPL, VPL>;
    if (a.L.cw != LY::CW || a.L.zero != LY::ZERO || a.L.post0 != LY::POST0 || a.L.padpost != LY::PADPOST ||
        a.L.gain0 != LY::GAIN0 || a.L.words != LY::WORDS)
        return fail(SAGMS_EUNSUPPORTED, "decode layout mismatch (internal)");
    if ((size_t)a.L.words * sizeof(float) > 65536) return fail(SAGMS_EUNSUPPORTED, "graph too large for one wave's LDS");
    const int wpb = waves_per_block(a.L, CPL);
    const size_t lds = (size_t)wpb * a.L.words * sizeof(float);
    int rc;
    if (bp)
        rc = launch_kernel<DC, DV, CPL, VPL, true, SAGMS_MSG_FP32>(a, wpb, lds, st);
    else if (mt == SAGMS_MSG_FP16)
        rc = launch_kernel<DC, DV, CPL, VPL, false, SAGMS_MSG_FP16>(a, wpb, lds, st);
    else if (mt == SAGMS_MSG_INT6)
        rc = launch_kernel<DC, DV, CPL, VPL, false, SAGMS_MSG_INT6>(a, wpb, lds, st);
    else
        rc = launch_kernel<DC, DV, CPL, VPL, false, SAGMS_MSG_FP32>(a, wpb, lds, st);
    if (rc) return rc;
    SAGMS_HIP(hipGetLastError());
    return SAGMS_OK;
}

int launch_decode(const DecodeShape& s, bool bp, int mt, const DecodeArgs& a, hipStream_t st) {
#define SHAPE(I, DC, DV, CPL, VPL) \
    if (s.dc == DC && s.dv == DV && s.cpl == CPL && s.vpl == VPL) return launch_shape<DC, DV, CPL, VPL>(bp, mt, a, st);
    SAGMS_DECODE_SHAPES(SHAPE)
#undef SHAPE
    return fail(SAGMS_EUNSUPPORTED, "no decode kernel for shape dc=%d dv=%d cpl=%d vpl=%d", s.dc, s.dv, s.cpl, s.vpl);
}

}  // namespace sagms
