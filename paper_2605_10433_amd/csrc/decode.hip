// Decode kernel with a static frame assignment: wave w of the grid decodes
// frames [w * frames_per_wave, (w + 1) * frames_per_wave).  The per-frame
// algorithm (Algorithm 1 of the paper) is in decode_core.h.
#include "decode_core.h"

namespace sagms {

constexpr int kWavesPerBlock = 4;

template <int DC, int DV, int CPL, int VPL, bool BP, int MT>
__global__ void __launch_bounds__(64 * kWavesPerBlock) decode_kernel(DecodeArgs a) {
    using LY = Lay<DC, CPL, VPL>;
    extern __shared__ float lds_all[];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    float* lds = lds_all + wib * LY::WORDS;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + wib;
    const int64_t f_begin = wave * a.frames_per_wave;
    if (f_begin >= a.nframes) return;
    const int64_t f_end = min(f_begin + (int64_t)a.frames_per_wave, a.nframes);
    using WD = WaveDecoder<DC, DV, CPL, VPL, BP, MT>;
    WD d;
    d.load(a, lds, lane);
    uint64_t word[CPL];
    uint32_t sb[CPL];
    WD::load_syndrome(a, f_begin, word);
    WD::syndrome_bits(a, lane, word, sb);
    for (int64_t f = f_begin; f < f_end; ++f) d.frame(a, lds, lane, f, sb, f + 1 < f_end ? f + 1 : f);
}

// Waves per block: up to kWavesPerBlock, as many as fit in 64 KiB of LDS.
static int waves_per_block(const DecodeLayout& L) {
    int w = (int)(65536 / ((size_t)L.words * sizeof(float)));
    return w < 1 ? 1 : (w > kWavesPerBlock ? kWavesPerBlock : w);
}

template <int DC, int DV, int CPL, int VPL, bool BP, int MT>
static void launch_one(dim3 grid, dim3 block, size_t lds, hipStream_t st, const DecodeArgs& a) {
    hipLaunchKernelGGL((decode_kernel<DC, DV, CPL, VPL, BP, MT>), grid, block, lds, st, a);
}

template <int DC, int DV, int CPL, int VPL>
static int launch_shape(bool bp, int mt, const DecodeArgs& a, hipStream_t st) {
    using LY = Lay<DC, CPL, VPL>;
    if (a.L.cw != LY::CW || a.L.zero != LY::ZERO || a.L.post0 != LY::POST0 || a.L.padpost != LY::PADPOST ||
        a.L.gain0 != LY::GAIN0 || a.L.words != LY::WORDS)
        return fail(SAGMS_EUNSUPPORTED, "decode layout mismatch (internal)");
    if ((size_t)a.L.words * sizeof(float) > 65536) return fail(SAGMS_EUNSUPPORTED, "graph too large for one wave's LDS");
    const int wpb = waves_per_block(a.L);
    int64_t waves = (a.nframes + a.frames_per_wave - 1) / a.frames_per_wave;
    int64_t blocks = (waves + wpb - 1) / wpb;
    if (blocks > 0x7fffffff) return fail(SAGMS_EINVAL, "too many frames for one launch");
    size_t lds = (size_t)wpb * a.L.words * sizeof(float);
    const dim3 grid((unsigned)blocks), block(64 * wpb);
    if (bp)
        launch_one<DC, DV, CPL, VPL, true, SAGMS_MSG_FP32>(grid, block, lds, st, a);
    else if (mt == SAGMS_MSG_FP16)
        launch_one<DC, DV, CPL, VPL, false, SAGMS_MSG_FP16>(grid, block, lds, st, a);
    else if (mt == SAGMS_MSG_INT6)
        launch_one<DC, DV, CPL, VPL, false, SAGMS_MSG_INT6>(grid, block, lds, st, a);
    else
        launch_one<DC, DV, CPL, VPL, false, SAGMS_MSG_FP32>(grid, block, lds, st, a);
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
