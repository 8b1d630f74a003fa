// Joint (quaternary) decoding of X and Z errors with scalar messages, on the
// Pauli-row Tanner graph of a CSS code: checks 0 .. m/2 - 1 are X-type rows
// (Pauli X on their support), the rest Z-type rows (Section II notation; the
// paper's Section V setup decodes the [[126,28]] code on the overcomplete
// m = 126 matrix of both types, d_c = d_v = 10).
//
// Quaternary beliefs of variable j (W = X, Y, Z; L0 the prior log-ratio of
// I against each W):
//   S_X = sum of the check outputs of j's X-type checks, S_Z likewise
//   Gamma^X = L0 + S_Z,  Gamma^Z = L0 + S_X,  Gamma^Y = L0 + (S_X + S_Z)
// since a check's output moves exactly the hypotheses that anticommute with
// its Pauli.  The scalar message to a check of Pauli P (min-sum form of the
// log-domain scalarisation of Lai and Kuo, the reduction the paper's
// Section I footnote names) is
//   lambda = min over the two Paulis A that anticommute with P of
//            (Gamma^A - own output) - min(0, Gamma^P).
// FP32 rounding is monotone, so the min of the two rounded differences is
// the rounded difference of the min: each variable publishes, per check
// type, the pair (A, W) = (min of the two anticommuting beliefs,
// |min(0, Gamma^P)|) and a check forms lambda = (A - own) + |W| (two
// roundings).  The hard decision of Algorithm 1 is the argmin over
// (I, X, Y, Z) of (0, Gamma^X, Gamma^Y, Gamma^Z), first minimum on ties:
// z_hat = [min(Gamma^Y, Gamma^Z) < min(0, Gamma^X)] and x_hat =
// [min(Gamma^X, Gamma^Y) < 0 and <= Gamma^Z].  An X-type check sees z_hat,
// a Z-type check x_hat (the symplectic product of eq. (resid)), so W carries
// that bit in its sign: the check XORs the sign bits of its W's, exactly as
// the binary decoder XORs posterior signs.  Check update: eq. (ms_cn) scaled
// per eq. (alphaeff) / (sagms_cn) with the gains of the binary decoder, the
// output magnitude saturated at 2^64.  Round order, gains, exit test and
// round count are those of the binary decoder (decode_core.h).
#include "decode_core.h"
#include "schedule.h"

namespace sagms {

constexpr int kJointWavesPerBlock = 4;  // the kernel's bound
// One wave per block at launch: a block's LDS is released only when its last
// wave ends, and with four waves per block the compute units held on
// average half of the wavefronts they could (1.32x faster with one).
constexpr int kJointLaunchWavesPerBlock = 1;
constexpr float kMsCap = 0x1p64f;  // saturation of the check outputs

template <int DC, int DV, int CPL, int VPL>
struct JLay {
    static constexpr int CW = 64 * CPL;
    static constexpr int ZERO = DC * CW;
    static constexpr int PAIRX = ZERO + 64;
    static constexpr int PAIRZ = PAIRX + 128 * VPL;
    static constexpr int PADPAIR = PAIRZ + 128 * VPL;
    static constexpr int GAIN0 = PADPAIR + 128;
    static constexpr int WORDS = GAIN0 + 2 * (CW + 1);
};

// Beliefs of one variable from its two sums, the two (A, W) pairs and the
// hard decision.
struct JointVar {
    float gx, gy, gz;
    float2 px, pz;  // pairs for the X-type and the Z-type checks
    bool xh, zh;
};

__device__ __forceinline__ JointVar joint_var(float l0, float sx, float sz) {
    JointVar v;
    v.gx = l0 + sz;
    v.gz = l0 + sx;
    v.gy = l0 + (sx + sz);
    const float ax = fminf(v.gy, v.gz), bx = fminf(0.0f, v.gx);  // P = X: anticommuting Y, Z
    const float az = fminf(v.gx, v.gy), bz = fminf(0.0f, v.gz);  // P = Z: anticommuting X, Y
    v.zh = ax < bx;
    v.xh = az < 0.0f && az <= v.gz;
    v.px = make_float2(ax, __uint_as_float(bits(fabsf(bx)) | (v.zh ? kSign : 0u)));
    v.pz = make_float2(az, __uint_as_float(bits(fabsf(bz)) | (v.xh ? kSign : 0u)));
    return v;
}

// Syndrome words of frame f (a vector load: the wave-uniform address is
// moved to vector registers, since scalar loads of the syndromes fetched
// twice their bytes from HBM; still a global-memory pointer, so that the
// load is not a flat load, which the LDS waits would also wait for).
template <int CPL>
__device__ __forceinline__ void joint_syndrome(const uint64_t* synd, int wm, int64_t f, uint64_t (&word)[CPL]) {
    using GlobalWord = const __attribute__((address_space(1))) uint64_t;
    GlobalWord* row = (GlobalWord*)(synd + f * wm);  // address-space cast
    asm("" : "+v"(row));
#pragma unroll
    for (int k = 0; k < CPL; ++k) word[k] = k < wm ? row[k] : 0ull;
}

// At most 128 VGPRs: four resident wavefronts per SIMD.
template <int DC, int DV, int CPL, int VPL>
__global__ void __launch_bounds__(64 * kJointWavesPerBlock) __attribute__((amdgpu_waves_per_eu(4)))
joint_kernel(JointArgs a, WaveSchedule ws) {
    using LY = JLay<DC, DV, CPL, VPL>;
    constexpr int DVH = DV / 2;
    extern __shared__ float jlds_all[];
    const int lane = threadIdx.x & 63;
    // wave-uniform: frame index and output addresses are scalar values
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float* lds = jlds_all + wib * LY::WORDS;
    float2* pairx = reinterpret_cast<float2*>(lds + LY::PAIRX);
    float2* pairz = reinterpret_cast<float2*>(lds + LY::PAIRZ);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + wib;
    if (wave >= ws.wave0[ws.levels]) return;
    int lv = 0;
    while (lv + 1 < ws.levels && wave >= ws.wave0[lv + 1]) ++lv;
    const int64_t f_begin = ws.frame0[lv] + (wave - ws.wave0[lv]) * ws.chunk[lv];
    const int64_t f_end = min(f_begin + (int64_t)ws.chunk[lv], ws.frame0[lv + 1]);
    if (f_begin >= f_end) return;

    uint32_t caddr[CPL][DC];
    uint32_t vaddr[VPL][DV];
    float L0[VPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k)
#pragma unroll
        for (int p = 0; p < DC; ++p) caddr[k][p] = a.cn_addr[(k * DC + p) * 64 + lane];
#pragma unroll
    for (int k = 0; k < VPL; ++k)
#pragma unroll
        for (int r = 0; r < DV; ++r) vaddr[k][r] = a.vn_addr[(k * DV + r) * 64 + lane];
#pragma unroll
    for (int k = 0; k < VPL; ++k) {
        const int j = k * 64 + lane;
        L0[k] = j < a.n ? a.llr0[j] + 0.0f : 0.0f;
    }
    write_gains(a.gains, a.m, LY::CW + 1, lds + LY::GAIN0, lane);
    lds[LY::ZERO + lane] = 0.0f;
    reinterpret_cast<float2*>(lds + LY::PADPAIR)[lane] = make_float2(__builtin_inff(), 0.0f);
    // the syndrome words of the wave's next frame are loaded while the
    // current frame decodes
    uint64_t word[CPL];
    joint_syndrome<CPL>(a.synd, a.wm, f_begin, word);
    for (int64_t f = f_begin; f < f_end; ++f) {
        uint32_t sb[CPL];  // original syndrome bits at the sign position
#pragma unroll
        for (int k = 0; k < CPL; ++k)
            sb[k] = (k * 64 + lane < a.m) ? (uint32_t)((word[k] >> lane) & 1ull) << 31 : 0u;
        joint_syndrome<CPL>(a.synd, a.wm, f + 1 < f_end ? f + 1 : f, word);
        // round 0: beliefs are the prior.  Only the decisions of the latest
        // beliefs are kept through the rounds (bit 0: x_hat, bit 1: z_hat)
        uint32_t dec[VPL];
#pragma unroll
        for (int k = 0; k < VPL; ++k) {
            const JointVar v0 = joint_var(L0[k], 0.0f, 0.0f);
            pairx[k * 64 + lane] = v0.px;
            pairz[k * 64 + lane] = v0.pz;
            dec[k] = (v0.xh ? 1u : 0u) | (v0.zh ? 2u : 0u);
        }
        // the check's own previous outputs: written by the first round before
        // any read (the first round's are zero and not subtracted)
        float c2v[CPL][DC];
        wave_lds_sync();

        int it = 0;
        bool conv = false;
        // one round; false once the frame is done.  first: the frame's first
        // round (A - 0 is A bit for bit)
        auto round = [&](auto first) -> bool {
            constexpr bool FIRST = decltype(first)::value;
            // top of the round: scalar messages, residual syndrome
            float v[CPL][DC];
            bool unsat[CPL];
            int w = 0;
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                float2 pw[DC];
#pragma unroll
                for (int p = 0; p < DC; ++p) pw[p] = *reinterpret_cast<const float2*>(lds + caddr[k][p]);
                float wv[DC];
#pragma unroll
                for (int p = 0; p < DC; ++p) {
                    v[k][p] = (FIRST ? pw[p].x : pw[p].x - c2v[k][p]) + fabsf(pw[p].y);
                    wv[p] = pw[p].y;
                }
                // the decision bits ride in the sign bits of the W's
                unsat[k] = (int32_t)xor_signs<DC>(wv, sb[k]) < 0;
                w += __builtin_popcountll(ballot(unsat[k]));
            }
            if (w == 0) {
                conv = true;
                return false;
            }
            if (it == a.lmax) return false;
            ++it;
            const float2 gg = *reinterpret_cast<const float2*>(&lds[LY::GAIN0 + 2 * w]);
            // check update: min1 / min2 / sign parity, saturated magnitudes
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                const uint32_t par = xor_signs<DC>(v[k], sb[k]);
                const float alpha = unsat[k] ? gg.y : gg.x;
                float m1 = fabsf(v[k][0]), m2 = __builtin_inff();
#pragma unroll
                for (int p = 1; p < DC; ++p) {
                    const float x = fabsf(v[k][p]);
                    m2 = __builtin_amdgcn_fmed3f(m1, x, m2);
                    m1 = fminf(m1, x);
                }
                const uint32_t S1 = or_and(bits(fminf(alpha * m1, kMsCap)), par, kSign);
                const uint32_t S2 = or_and(bits(fminf(alpha * m2, kMsCap)), par, kSign);
#pragma unroll
                for (int p = 0; p < DC; ++p) {
                    const uint32_t sel = fabsf(v[k][p]) == m1 ? S2 : S1;
                    c2v[k][p] = __uint_as_float(xor_and(sel, bits(v[k][p]), kSign));
                    lds[p * LY::CW + k * 64 + lane] = c2v[k][p];
                }
            }
            wave_lds_sync();
            // variable update: the two sums in graph order, beliefs, pairs
#pragma unroll
            for (int k = 0; k < VPL; ++k) {
                float sx = lds[vaddr[k][0]];
#pragma unroll
                for (int r = 1; r < DVH; ++r) sx = sx + lds[vaddr[k][r]];
                float sz = lds[vaddr[k][DVH]];
#pragma unroll
                for (int r = DVH + 1; r < DV; ++r) sz = sz + lds[vaddr[k][r]];
                const JointVar vk = joint_var(L0[k], sx, sz);
                pairx[k * 64 + lane] = vk.px;
                pairz[k * 64 + lane] = vk.pz;
                dec[k] = (vk.xh ? 1u : 0u) | (vk.zh ? 2u : 0u);
            }
            wave_lds_sync();
            return true;
        };
        if (round(std::integral_constant<bool, true>{}))
            while (round(std::integral_constant<bool, false>{})) {
            }
        // take the prefetched words before the output stores are issued: a
        // wait placed after them would also wait for the stores
#pragma unroll
        for (int k = 0; k < CPL; ++k) asm volatile("" ::"v"(word[k]));

        // outputs: x_hat words, then z_hat words; rounds; flag; beliefs
        const int wn = a.wn;
        uint64_t mx = 0, mz = 0;
#pragma unroll
        for (int k = 0; k < VPL; ++k) {
            const int j = k * 64 + lane;
            const uint64_t bx = ballot(j < a.n && (dec[k] & 1u)), bz = ballot(j < a.n && (dec[k] & 2u));
            if (lane == k) {
                mx = bx;
                mz = bz;
            }
        }
        if (lane < wn) {
            a.ehat[f * 2 * wn + lane] = mx;
            a.ehat[f * 2 * wn + wn + lane] = mz;
        }
        if (a.gamma) {
            // the final beliefs, recomputed from the last round's check
            // outputs in their LDS slots (the sums of that round's variable
            // update, in the same order; the prior's when no round ran), so
            // that no register holds them through the rounds
#pragma unroll
            for (int k = 0; k < VPL; ++k) {
                float sx = 0.0f, sz = 0.0f;
                if (it > 0) {
                    sx = lds[vaddr[k][0]];
#pragma unroll
                    for (int r = 1; r < DVH; ++r) sx = sx + lds[vaddr[k][r]];
                    sz = lds[vaddr[k][DVH]];
#pragma unroll
                    for (int r = DVH + 1; r < DV; ++r) sz = sz + lds[vaddr[k][r]];
                }
                const JointVar vk = joint_var(L0[k], sx, sz);
                const int j = k * 64 + lane;
                if (j < a.n) {
                    float* g = a.gamma + (f * a.n + j) * 3;
                    g[0] = vk.gx;
                    g[1] = vk.gy;
                    g[2] = vk.gz;
                }
            }
        }
        if (lane == 0) {
            a.iters[f] = it;
            a.conv[f] = conv ? 1 : 0;
        }
        wave_lds_sync();  // the next frame rewrites the pairs
    }
}

constexpr int kJointFramesPerWave = 16;
constexpr int kJointTaperLevels = 2;

template <int DC, int DV, int CPL, int VPL>
static int launch_joint_shape(const JointArgs& a, hipStream_t st) {
    using LY = JLay<DC, DV, CPL, VPL>;
    if (a.L.cw != LY::CW || a.L.zero != LY::ZERO || a.L.pairx != LY::PAIRX || a.L.pairz != LY::PAIRZ ||
        a.L.padpair != LY::PADPAIR || a.L.gain0 != LY::GAIN0 || a.L.words != LY::WORDS)
        return fail(SAGMS_EUNSUPPORTED, "joint layout mismatch (internal)");
    int wpb = (int)(65536 / ((size_t)LY::WORDS * sizeof(float)));
    wpb = wpb < 1 ? 1 : (wpb > kJointLaunchWavesPerBlock ? kJointLaunchWavesPerBlock : wpb);
    const size_t lds = (size_t)wpb * LY::WORDS * sizeof(float);
    if ((size_t)LY::WORDS * sizeof(float) > 65536) return fail(SAGMS_EUNSUPPORTED, "joint graph too large for LDS");
    const void* fn = reinterpret_cast<const void*>(&joint_kernel<DC, DV, CPL, VPL>);
    int64_t resident = 0;
    if (a.frames_per_wave == 0) {
        const int rc = resident_waves(fn, wpb, lds, &resident);
        if (rc) return rc;
    }
    const WaveSchedule ws = make_schedule(a.nframes, a.frames_per_wave, resident * kJointTaperLevels,
                                          kJointFramesPerWave);
    const int64_t blocks = (ws.wave0[ws.levels] + wpb - 1) / wpb;
    if (blocks > 0x7fffffff) return fail(SAGMS_EINVAL, "too many frames for one launch");
    hipLaunchKernelGGL((joint_kernel<DC, DV, CPL, VPL>), dim3((unsigned)blocks), dim3(64 * wpb), lds, st, a, ws);
    SAGMS_HIP(hipGetLastError());
    return SAGMS_OK;
}

int launch_joint(const DecodeShape& s, const JointArgs& a, hipStream_t st) {
#define JSHAPE(I, DC, DV, CPL, VPL) \
    if (s.dc == DC && s.dv == DV && s.cpl == CPL && s.vpl == VPL) return launch_joint_shape<DC, DV, CPL, VPL>(a, st);
    SAGMS_JOINT_SHAPES(JSHAPE)
#undef JSHAPE
    return fail(SAGMS_EUNSUPPORTED, "no joint kernel for shape dc=%d dv=%d cpl=%d vpl=%d", s.dc, s.dv, s.cpl, s.vpl);
}

}  // namespace sagms
