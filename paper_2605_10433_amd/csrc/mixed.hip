// Mixed-code persistent decode: one launch decodes the frames of several
// codes (segments), each with its own graph tables, shape and outputs.
//
// The grid is sized to the resident capacity of the device.  Waves take
// tiles of frames from work queues (one atomic increment per tile) until
// every queue is empty, so a wave that draws fast-converging frames simply
// takes more tiles; segments are ordered by the host from the most to the
// least expensive per frame, so the last tiles are the cheapest.  A wave
// keeps the graph tables of its current segment in registers and reloads
// them only when its next tile belongs to another segment.  Each frame is
// decoded by the same per-frame code as the single-code kernel, so results
// do not depend on the mix, the tiling or the order in which tiles run.
#include <mutex>

#include "decode_core.h"

namespace sagms {

// Queue counters of sagms_decode_segments, the entry point that allocates
// nothing: kNumMixedTiers blocks of kMaxQueues counters (16 KiB), one copy on
// every device the library runs on, held until the process ends.  Host code
// never uses the array's name as an address: it uses the device address that
// hipGetSymbolAddress returned for the current device (scratch_queues).
static __device__ __align__(256) uint32_t scratch[kScratchWords];

static std::mutex g_scratch_mu;
static uint32_t* g_scratch_ptr[kMaxDevices];

int scratch_setup() {
    int dev = 0;
    SAGMS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SAGMS_EUNSUPPORTED, "device index %d too large", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return SAGMS_OK;
    void* ptr = nullptr;
    SAGMS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(SAGMS_EHIP, "hipGetSymbolAddress returned a null address for the queue counters");
    g_scratch_ptr[dev] = static_cast<uint32_t*>(ptr);
    return SAGMS_OK;
}

int scratch_queues(uint32_t** out) {
    int dev = 0;
    SAGMS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SAGMS_EUNSUPPORTED, "device index %d too large", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev])
        return fail(SAGMS_EINVAL, "no graph has been uploaded to device %d (sagms_graph_upload sets it up)", dev);
    *out = g_scratch_ptr[dev];
    return SAGMS_OK;
}

constexpr int kMixedMaxWavesPerBlock = 4;

__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// The wave's position in the queue walk: queue q, and the number of queues
// found empty so far.
struct TileQueue {
    int q, tries;

    // Next tile index, or -1 once every queue has been found empty.
    __device__ __forceinline__ int64_t next(const MixedArgs& m, int lane) {
        while (tries < m.nq) {
            uint32_t i = 0;
            if (lane == 0) i = atomicAdd(&m.queues[q * kQueueStride], 1u);
            i = uniform(i);
            const int64_t t = (int64_t)q + (int64_t)i * m.nq;
            if (t < m.ntiles) return t;
            q = q + 1 == m.nq ? 0 : q + 1;
            ++tries;
        }
        return -1;
    }
};

__device__ __forceinline__ int segment_of(const MixedArgs& m, int64_t t) {
    int s = 0;
    while (s + 1 < m.nseg && t >= m.tile_end[s]) ++s;
    return s;
}

// Decodes tile t of segment s and every following tile the wave draws from
// the same segment; returns the first tile of another segment (or -1).
// UR: rounds per iteration of the round loop.
template <int DC, int DV, int CPL, int VPL, bool BP, int MT, int UR>
__device__ __forceinline__ int64_t run_segment(const MixedArgs& m, int s, int64_t t, TileQueue& q, float* lds,
                                               int lane) {
    const DecodeArgs a = m.segs[s].a;  // private copy: the output stores cannot alias it
    const int64_t tb = s == 0 ? 0 : m.tile_end[s - 1], te = m.tile_end[s];
    using WD = WaveDecoder<DC, DV, CPL, VPL, BP, MT>;
    WD d;
    d.load(a, lds, lane);
    do {
        const int64_t f0 = (t - tb) * m.tile_frames;
        const int64_t f1 = min(f0 + (int64_t)m.tile_frames, a.nframes);
        uint64_t word[CPL];
        uint32_t sb[CPL];
        WD::load_syndrome(a, f0, word);
        WD::syndrome_bits(a, lane, word, sb);
        for (int64_t f = f0; f < f1; ++f) d.template frame<UR>(a, lds, lane, f, sb, f + 1 < f1 ? f + 1 : f);
        t = q.next(m, lane);
    } while (t >= tb && t < te);
    return t;
}

// HI: highest shape index compiled in (the tier); WPE: waves per SIMD the
// register allocator must allow (1 = no constraint beyond the hardware's);
// UR: decoding rounds per iteration of the round loop (1 or 2).
template <int HI, int WPE, int MT, int UR>
__global__ void __launch_bounds__(64 * kMixedMaxWavesPerBlock) __attribute__((amdgpu_waves_per_eu(WPE)))
mixed_kernel(MixedArgs m) {
    extern __shared__ float lds_all[];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    float* lds = lds_all + wib * m.words;
    TileQueue q{(int)(blockIdx.x % (unsigned)m.nq), 0};
    int64_t t = q.next(m, lane);
    while (t >= 0) {
        const int s = segment_of(m, t);
        switch (m.segs[s].shape) {
#define MIXED_CASE(I, DC, DV, CPL, VPL)                                                 \
    case I:                                                                            \
        if constexpr (I <= HI) t = run_segment<DC, DV, CPL, VPL, false, MT, UR>(m, s, t, q, lds, lane); \
        else t = -1;                                                                   \
        break;
            SAGMS_DECODE_SHAPES(MIXED_CASE)
#undef MIXED_CASE
            default:
                t = -1;  // unreachable: the host admits only shapes of the tier
        }
    }
}

__global__ void queue_reset_kernel(uint32_t* queues, int nq) {
    const int i = threadIdx.x;
    if (i < nq) __hip_atomic_store(&queues[i * kQueueStride], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int HI>
static constexpr int tier_words() {
    int w = 0;
#define MIXED_WORDS(I, DC, DV, CPL, VPL) \
    if (I <= HI && Lay<DC, CPL, VPL>::WORDS > w) w = Lay<DC, CPL, VPL>::WORDS;
    SAGMS_DECODE_SHAPES(MIXED_WORDS)
#undef MIXED_WORDS
    return w;
}

int mixed_words(int tier) {
    switch (tier) {
        case 0: return tier_words<kMixedTiers[0]>();
        case 1: return tier_words<kMixedTiers[1]>();
        case 2: return tier_words<kMixedTiers[2]>();
        case 3: return tier_words<kMixedTiers[3]>();
    }
    return -1;
}

using MixedFn = void (*)(MixedArgs);

template <int HI, int WPE, int UR>
static MixedFn pick_format(int mt) {
    if (mt == SAGMS_MSG_FP16) return mixed_kernel<HI, WPE, SAGMS_MSG_FP16, UR>;
    if (mt == SAGMS_MSG_INT6) return mixed_kernel<HI, WPE, SAGMS_MSG_INT6, UR>;
    return mixed_kernel<HI, WPE, SAGMS_MSG_FP32, UR>;
}

template <int HI, int WPE>
static MixedFn pick_kernel(int mt, int unroll) {
    return unroll == 2 ? pick_format<HI, WPE, 2>(mt) : pick_format<HI, WPE, 1>(mt);
}

// Register budgets: 0 = the compiler's allocation; 1 = a tighter budget that
// buys one more resident wave per SIMD (tiers 1 and 2 only; it may spill).
// Unroll: 1 or 2 rounds per iteration of the round loop.
static MixedFn mixed_fn(int tier, int budget, int mt, int unroll) {
    if (unroll != 1 && unroll != 2) return nullptr;
    if (budget == 0) {
        switch (tier) {
            case 0: return pick_kernel<kMixedTiers[0], 1>(mt, unroll);
            case 1: return pick_kernel<kMixedTiers[1], 1>(mt, unroll);
            case 2: return pick_kernel<kMixedTiers[2], 1>(mt, unroll);
            case 3: return pick_kernel<kMixedTiers[3], 1>(mt, unroll);
        }
    } else if (budget == 1) {
        switch (tier) {
            case 1: return pick_kernel<kMixedTiers[1], 5>(mt, unroll);
            case 2: return pick_kernel<kMixedTiers[2], 3>(mt, unroll);
        }
    }
    return nullptr;
}

bool mixed_has_budget(int tier, int budget) { return mixed_fn(tier, budget, SAGMS_MSG_FP32, 1) != nullptr; }

int mixed_max_blocks(int tier, int budget, int mt, int unroll, int waves_per_block, int* out) {
    MixedFn fn = mixed_fn(tier, budget, mt, unroll);
    if (!fn)
        return fail(SAGMS_EINVAL, "no mixed kernel for tier %d, register budget %d, unroll %d", tier, budget, unroll);
    if (waves_per_block < 1 || waves_per_block > kMixedMaxWavesPerBlock)
        return fail(SAGMS_EINVAL, "waves_per_block must lie in [1, %d]", kMixedMaxWavesPerBlock);
    const size_t lds = (size_t)waves_per_block * mixed_words(tier) * sizeof(float);
    int blocks = 0;
    SAGMS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(fn),
                                                           64 * waves_per_block, lds));
    *out = blocks;
    return SAGMS_OK;
}

int launch_mixed(int tier, int budget, int mt, int unroll, const MixedArgs& m, int blocks, int waves_per_block,
                 hipStream_t st) {
    MixedFn fn = mixed_fn(tier, budget, mt, unroll);
    if (!fn)
        return fail(SAGMS_EINVAL, "no mixed kernel for tier %d, register budget %d, unroll %d", tier, budget, unroll);
    if (m.nq < 1 || m.nq > kMaxQueues || m.nseg < 1 || m.nseg > kMaxSegments || m.tile_frames < 1 ||
        m.words != mixed_words(tier) || blocks < 1 || waves_per_block < 1 ||
        waves_per_block > kMixedMaxWavesPerBlock)
        return fail(SAGMS_EINVAL, "mixed launch arguments out of range (internal)");
    const size_t lds = (size_t)waves_per_block * m.words * sizeof(float);
    if (lds > 65536) return fail(SAGMS_EUNSUPPORTED, "mixed tier %d needs more than 64 KiB of LDS per block", tier);
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, st, m.queues, m.nq);
    SAGMS_HIP(hipGetLastError());
    static_assert(sizeof(MixedArgs) <= 4096, "kernel arguments");
    MixedArgs args = m;
    void* params[] = {&args};
    SAGMS_HIP(hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)blocks), dim3(64 * waves_per_block),
                              params, lds, st));
    return SAGMS_OK;
}

}  // namespace sagms
