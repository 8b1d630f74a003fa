// Layered-schedule decoder with one frame per lane, for the code compiled
// into lane_code.h (the l = 63 generalized-bicycle code).
//
// The layered schedule updates the checks one after another; the general
// kernel (layered.hip) spreads a frame over a group of lanes, which leaves
// lanes idle when a pass holds fewer checks than the group has lanes, and
// reads its posteriors and tables from LDS.  Here each lane decodes its own
// frame from start to finish and updates all 63 checks of a round itself, in
// the order of lane_code.h.  Its 126 posteriors and the three words of each
// check's outputs are registers whose names are fixed at compile time, so a
// round is straight-line arithmetic: no idle lane, no table read, no LDS
// access.  The check update does the general kernel's arithmetic operation
// for operation and keeps its S1 and S1 xor S2 words; the third word holds
// edge k's v2c sign at bit 2k and its minimum bit at bit 2k + 1.  Output k
// is rebuilt from them bit for bit, so the results are the same.
//
// A workgroup of four wavefronts (one per SIMD of a compute unit: a lane's
// state takes the registers of a whole SIMD lane) owns a contiguous run of
// frames.  A lane that has no frame takes the next unclaimed frame of the run
// from a counter in LDS that the four wavefronts share, and loads its
// syndrome word then.  Frames take from one round to l_max rounds: a lane
// that held a claimed next frame while decoding the current one could leave
// two long frames for the end, and a wavefront with a run of its own would
// finish far from the others.
#include <utility>

#include "decode_core.h"
#include "lane_code.h"

namespace sagms {

namespace {

using lane::kDC;
using lane::kL;
using lane::kN;

// variable of edge k of check c, as a constant expression
template <int C, int K>
constexpr int kVar = lane::kRows.var[C][K];

template <int C, int... K>
__device__ __forceinline__ void gather(const float (&post)[kN], float (&x)[kDC], std::integer_sequence<int, K...>) {
    ((x[K] = post[kVar<C, K>]), ...);
}

template <int C, int... K>
__device__ __forceinline__ void scatter(float (&post)[kN], const float (&x)[kDC], std::integer_sequence<int, K...>) {
    ((post[kVar<C, K>] = x[K]), ...);
}

// Check update of check C in place: posteriors of its variables and its
// compressed outputs (s1 = S1, dd = S1 xor S2, mk = for edge k the v2c sign
// at bit 2k and "|v2c_k| was the minimum" at bit 2k + 1).  sb, rb: syndrome
// and residual bits of the frame.
template <int C>
__device__ __forceinline__ void check_update(float (&post)[kN], uint32_t (&s1)[kL], uint32_t (&dd)[kL],
                                             uint32_t (&mk)[kL], uint32_t sb0, uint32_t sb1, uint32_t rb0,
                                             uint32_t rb1, float gs, float gu) {
    constexpr int b = C & 31;
    float pj[kDC];
    gather<C>(post, pj, std::make_integer_sequence<int, kDC>{});
    const uint32_t S1o = s1[C], Do = dd[C], Mo = mk[C];
    float v[kDC];
#pragma unroll
    for (int k = 0; k < kDC; ++k) {
        const uint32_t minmask = (uint32_t)__builtin_amdgcn_sbfe(Mo, 2 * k + 1, 1);
        const uint32_t prev = xor_and(S1o, Do, minmask) ^ ((Mo << (31 - 2 * k)) & kSign);
        v[k] = pj[k] - __uint_as_float(prev);
    }
    const uint32_t sword = C < 32 ? sb0 : sb1, rword = C < 32 ? rb0 : rb1;
    const uint32_t par = xor_signs<kDC>(v, ((sword >> b) & 1u) << 31);
    const bool unsat = (rword >> b) & 1u;
    const float alpha = unsat ? gu : gs;
    float m1 = fabsf(v[0]), m2 = __builtin_inff();
#pragma unroll
    for (int k = 1; k < kDC; ++k) {
        const float x = fabsf(v[k]);
        m2 = __builtin_amdgcn_fmed3f(m1, x, m2);
        m1 = fminf(m1, x);
    }
    const uint32_t S1 = or_and(bits(alpha * m1), par, kSign);
    const uint32_t S2 = or_and(bits(alpha * m2), par, kSign);
    uint32_t mask = 0;
    float out[kDC];
#pragma unroll
    for (int k = kDC - 1; k >= 0; --k) {
        const bool is_min = fabsf(v[k]) == m1;
        const uint32_t o = xor_and(is_min ? S2 : S1, bits(v[k]), kSign);
        mask = mask + mask + (is_min ? 1u : 0u);                   // bit 2k + 1
        mask = __builtin_amdgcn_alignbit(mask, bits(v[k]), 31);  // bit 2k: the sign of v2c_k
        out[k] = v[k] + __uint_as_float(o);
    }
    scatter<C>(post, out, std::make_integer_sequence<int, kDC>{});
    s1[C] = S1;
    dd[C] = S1 ^ S2;
    mk[C] = mask;
    // keep the checks apart: interleaving them only lengthens the live ranges
    __builtin_amdgcn_sched_barrier(0);
}

template <int... I>
__device__ __forceinline__ void round_checks(float (&post)[kN], uint32_t (&s1)[kL], uint32_t (&dd)[kL],
                                             uint32_t (&mk)[kL], uint32_t sb0, uint32_t sb1, uint32_t rb0,
                                             uint32_t rb1, float gs, float gu, std::integer_sequence<int, I...>) {
    (check_update<lane::kOrder.check[I]>(post, s1, dd, mk, sb0, sb1, rb0, rb1, gs, gu), ...);
}

// XOR of the bit patterns of check C's posteriors: its sign bit is the
// parity of the check's hard decisions.
template <int C, int... K>
__device__ __forceinline__ uint32_t sign_parity(const float (&post)[kN], std::integer_sequence<int, K...>) {
    float x[kDC] = {post[kVar<C, K>]...};
    return xor_signs<kDC>(x, 0u);
}

// Parity bits of checks C0 .. C0 + 31 (those below kL): checks are shifted in
// from the highest, so check C0 + i lands on bit i.
template <int C0, int... I>
__device__ __forceinline__ uint32_t parity_word(const float (&post)[kN], std::integer_sequence<int, I...>) {
    uint32_t w = 0;
    constexpr int top = (kL - C0 < 32 ? kL - C0 : 32) - 1;
    ((w = __builtin_amdgcn_alignbit(w, sign_parity<C0 + top - I>(post, std::make_integer_sequence<int, kDC>{}), 31)),
     ...);
    return w;
}

__device__ __forceinline__ void hard_parity(const float (&post)[kN], uint32_t& p0, uint32_t& p1) {
    p0 = parity_word<0>(post, std::make_integer_sequence<int, 32>{});
    p1 = parity_word<32>(post, std::make_integer_sequence<int, kL - 32>{});
}

}  // namespace

constexpr int kLaneBlock = 256;  // four wavefronts

__global__ void __launch_bounds__(kLaneBlock) __attribute__((amdgpu_waves_per_eu(1, 1)))
layered_lane_kernel(DecodeArgs a, int64_t frames_per_block) {
    __shared__ float t_l0[kN];
    __shared__ float2 t_gain[kL + 1];
    __shared__ uint32_t claimed;  // frames of the run handed out so far
    const int tid = threadIdx.x, lane = tid & 63;
    for (int j = tid; j < kN; j += kLaneBlock) t_l0[j] = a.llr0[j] + 0.0f;  // -0 reads as +0
    if (tid < 64) write_gains(a.gains, kL, kL + 1, reinterpret_cast<float*>(t_gain), tid);
    if (tid == 0) claimed = 0;
    __syncthreads();

    const int64_t f_begin = (int64_t)blockIdx.x * frames_per_block;
    const int64_t f_end = min(f_begin + frames_per_block, a.nframes);
    if (f_begin >= f_end) return;

    float post[kN];
    uint32_t s1[kL], dd[kL], mk[kL];
    // residual bits of H [L0 < 0]: a frame's first residual is its syndrome xor these
#pragma unroll
    for (int j = 0; j < kN; ++j) post[j] = t_l0[j];
    uint32_t r0_0, r0_1;
    hard_parity(post, r0_0, r0_1);

    constexpr uint64_t kKeep = (1ull << kL) - 1;  // bits at or above m are not syndrome bits
    int64_t f = -1;
    uint32_t sb0 = 0, sb1 = 0, rb0 = 0, rb1 = 0;
    int it = 0, w = 0;
    bool active = false, more = true;  // more: the run may still hold a frame for this lane

    // outputs of the lane's frame: hard decisions, rounds, flag and, when
    // asked for, the posteriors
    auto finish = [&](bool on, int rounds, bool conv) {
        if (ballot(on) == 0) return;
        if (on) {
            uint32_t e[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int j = kN - 1; j >= 0; --j) e[j >> 5] = (e[j >> 5] << 1) | (post[j] < 0.0f ? 1u : 0u);
            a.ehat[f * 2] = (uint64_t)e[0] | ((uint64_t)e[1] << 32);
            a.ehat[f * 2 + 1] = (uint64_t)e[2] | ((uint64_t)e[3] << 32);
            a.iters[f] = rounds;
            a.conv[f] = conv ? 1 : 0;
            if (a.post) {
#pragma unroll
                for (int j = 0; j < kN; ++j) a.post[f * kN + j] = post[j];
            }
        }
    };

    while (true) {
        // idle lanes take the next frames of the run (in lane order) and
        // finish those that need no round, until every lane decodes a frame
        // or the run is used up
        while (true) {
            const bool want = !active && more;
            const uint64_t takers = ballot(want);
            if (takers == 0) break;
            const int leader = __ffsll((long long)takers) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&claimed, (uint32_t)__popcll(takers));
            base = __builtin_amdgcn_readlane(base, leader);
            bool start = false;
            if (want) {
                f = f_begin + base + __popcll(takers & ((1ull << lane) - 1));
                more = f < f_end;
                start = more;
            }
            if (start) {
                const uint64_t word = a.synd[f] & kKeep;
#pragma unroll
                for (int j = 0; j < kN; ++j) post[j] = t_l0[j];
#pragma unroll
                for (int c = 0; c < kL; ++c) s1[c] = dd[c] = mk[c] = 0u;
                sb0 = (uint32_t)word;
                sb1 = (uint32_t)(word >> 32);
                rb0 = sb0 ^ r0_0;
                rb1 = sb1 ^ r0_1;
                w = __popc(rb0) + __popc(rb1);
                it = 0;
                active = w != 0;
            }
            finish(start && !active, 0, true);
        }
        if (ballot(active) == 0) break;

        // one round: every check in layer order, then the residual
        const float2 g = t_gain[w];
        bool done = false;
        if (active) {
            round_checks(post, s1, dd, mk, sb0, sb1, rb0, rb1, g.x, g.y, std::make_integer_sequence<int, kL>{});
            uint32_t p0, p1;
            hard_parity(post, p0, p1);
            rb0 = p0 ^ sb0;
            rb1 = p1 ^ sb1;
            w = __popc(rb0) + __popc(rb1);
            ++it;
            done = w == 0 || it >= a.lmax;
        }
        finish(done, it, w == 0);
        if (done) active = false;
    }
}

// Launches the kernel over a.nframes frames of the compiled code.
int launch_layered_lane(const DecodeArgs& a, hipStream_t st) {
    if (a.nframes <= 0) return SAGMS_OK;
    if (a.m != kL || a.n != kN || a.wm != 1 || a.wn != 2)
        return fail(SAGMS_EINVAL, "one-lane layered kernel: graph is not the compiled code (internal)");
    int dev = 0, num_cu = 0, per_cu = 0;
    SAGMS_HIP(hipGetDevice(&dev));
    SAGMS_HIP(hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    SAGMS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&layered_lane_kernel),
                                                           kLaneBlock, 0));
    if (per_cu < 1) return fail(SAGMS_EUNSUPPORTED, "one-lane layered kernel does not fit a compute unit");
    int64_t blocks = std::min<int64_t>((int64_t)per_cu * num_cu, (a.nframes + kLaneBlock - 1) / kLaneBlock);
    const int64_t fpb = (a.nframes + blocks - 1) / blocks;
    blocks = (a.nframes + fpb - 1) / fpb;
    hipLaunchKernelGGL(layered_lane_kernel, dim3((unsigned)blocks), dim3(kLaneBlock), 0, st, a, fpb);
    SAGMS_HIP(hipGetLastError());
    return SAGMS_OK;
}

}  // namespace sagms
