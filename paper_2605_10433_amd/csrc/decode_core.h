#pragma once
// Device code shared by the decode kernels: MS / SMS / SAGMS (one code path,
// gain table) and BP.
//
// Algorithm 1 of the paper on the binary Tanner graph of H, flooding
// schedule, one wavefront per frame:
//   lane l owns checks c = l + 64 k (k < CPL) and variables j = l + 64 k
//   (k < VPL).  A check keeps its DC outgoing c2v messages in VGPRs; the
//   posteriors of all variables and the c2v messages of the current round
//   live in the wave's LDS slice.  One round:
//     top    every check reads the posteriors of its variables from LDS:
//            v2c = posterior - own c2v (eq. (bp4_vn) as "total minus own"),
//            and the XOR of their signs gives (H e_hat)_c; the residual
//            syndrome s_res = s xor H e_hat is balloted, its popcount w is
//            the unsatisfied-check count of eq. (synratio).  w == 0 ends
//            the frame (converged), as does reaching lmax rounds.
//     CN     eq. (ms_cn) with min1 / min2 / sign parity over the row, the
//            sign of (-1)^{s_c} folded into the parity; the output
//            magnitude is gain * (|v2c| == min1 ? min2 : min1), the gain
//            taken from a table indexed by w and by the check's residual
//            bit (eq. (alphaeff); 1 for MS, alpha for SMS).  BP replaces
//            this by eq. (bp4_cn) in tanh form, evaluated in FP64.
//     VN     every variable sums L0 and its incoming c2v messages in the
//            graph's order (ascending check index, or polynomial-term order
//            for a GB code) and stores the posterior (eq. (bp4_vn)).
//   The hard decision is e_hat_j = [posterior_j < 0].
// Posteriors and v2c messages are never -0.0 (L0 is read as L0 + 0.0f and
// every later value is a sum or a difference of finite floats starting from
// it), so sign bits and "< 0" agree and the kernel uses sign bits.
#include <hip/hip_fp16.h>
#include <type_traits>

#include "internal.h"

namespace sagms {

constexpr uint32_t kSign = 0x80000000u;

// LDS traffic of one wave only: the LDS unit executes a wave's requests in
// order, so a wavefront-scope fence (compiler ordering) is all that is needed.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// FP64 exclusive-product BP check update (eq. (bp4_cn) in tanh form):
// out_p = 2 atanh(prod_{q != p} tanh(|v_q| / 2)), product capped at
// 1 - 2^-40 so that the output stays finite.
template <int DC>
__device__ __forceinline__ void bp_magnitudes(const float (&v)[DC], float (&out)[DC]) {
    double t[DC], pre[DC];
    double acc = 1.0;
#pragma unroll
    for (int p = 0; p < DC; ++p) {
        t[p] = tanh(0.5 * (double)fabsf(v[p]));
        pre[p] = acc;
        acc *= t[p];
    }
    double suf = 1.0;
    const double cap = 1.0 - 0x1.0p-40;
#pragma unroll
    for (int p = DC - 1; p >= 0; --p) {
        double x = fmin(pre[p] * suf, cap);
        out[p] = (float)(2.0 * atanh(x));
        suf *= t[p];
    }
}

// Compile-time LDS layout of one wave (32-bit words); must equal make_layout().
template <int DC, int CPL, int VPL>
struct Lay {
    static constexpr int CW = 64 * CPL;
    static constexpr int ZERO = DC * CW;
    static constexpr int POST0 = ZERO + 64;
    static constexpr int PADPOST = POST0 + 64 * VPL;
    static constexpr int GAIN0 = PADPOST + 64;
    static constexpr int WORDS = GAIN0 + 2 * (CW + 1);
};

// Gains of a satisfied and of an unsatisfied check at residual weight w out
// of m checks (eq. (alphaeff)): 1 for MS and BP, alpha for SMS, and for SAGMS
// g = alpha_max - (alpha_max - alpha_min) * (w / m) and g * eta.  Evaluated
// in IEEE double one rounded operation at a time (the library is compiled
// without contraction, and double division is correctly rounded), then
// rounded to float: the values a host evaluates from the same formula.
__device__ __forceinline__ float2 gain_pair(const GainLaw& law, int w, int m) {
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

// Gain pairs of residual weights 0 .. 64, passed by value as a kernel
// argument by the stand-alone decode kernel of one-block codes (m <= 64):
// the round's pair is then one scalar load at a wave-uniform offset.
struct KernelGains {
    float2 g[65];
};

// Writes the gain pairs of residual weights 0 .. entries - 1 to the wave's
// LDS at gain0 (pairs of floats, 8-byte aligned).
__device__ __forceinline__ void write_gains(const GainLaw& law, int m, int entries, float* gain0, int lane) {
    for (int w = lane; w < entries; w += 64) reinterpret_cast<float2*>(gain0)[w] = gain_pair(law, w, m);
}

__device__ __forceinline__ uint32_t bits(float x) { return __float_as_uint(x); }

// gfx950 3-input bit operations (truth table indexed by a*4 + b*2 + c):
// a ^ b ^ c (0x96) and a ^ (b & c) (0x78).  The compiler re-associates XOR
// chains into 2-input steps unless asked for the 3-input form.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t xor_and(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x78);
}

// init XOR the bit patterns of x[0..N-1], two inputs per step: the sign bit
// is the parity of the signs; the other bits are not used.
template <int N>
__device__ __forceinline__ uint32_t xor_signs(const float (&x)[N], uint32_t init) {
    uint32_t acc = init;
#pragma unroll
    for (int p = 0; p + 1 < N; p += 2) acc = xor3(acc, bits(x[p]), bits(x[p + 1]));
    if constexpr (N % 2) acc ^= bits(x[N - 1]);
    return acc;
}

// a | (b & c) in one 3-input bit operation.
__device__ __forceinline__ uint32_t or_and(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xF8);
}

// Message formats: FP32; FP16 (every message saturated to +-65504 and
// rounded to half, posteriors FP32); INT6 (sign + 6-bit magnitude on a grid
// of step 1/4, saturating at +-63 steps; the prior is quantized as well, so
// posterior sums are exact).  Messages are held as FP32 values.
//
// Only the check outputs are rounded.  Both roundings are monotone and keep
// the sign, so the minimum, the second minimum and the sign parity of the
// rounded v2c messages are the rounded minimum, second minimum and parity of
// the unrounded ones: the check output sign * q(gain * q(exclusive min)) is
// the same either way.  (The FP16 prior lies on the 2^-24 grid, so a v2c is
// +0 or at least 2^-24 in magnitude and never rounds to a signed zero; INT6
// v2c messages are exact grid values.)
template <int MT>
__device__ __forceinline__ float quantize(float x) {
    if constexpr (MT == SAGMS_MSG_FP16) {
        return __half2float(__float2half_rn(__builtin_amdgcn_fmed3f(x, -65504.0f, 65504.0f)));
    } else if constexpr (MT == SAGMS_MSG_INT6) {
        return __builtin_amdgcn_fmed3f(rintf(x * 4.0f), -63.0f, 63.0f) * 0.25f;
    } else {
        return x;
    }
}

// FP16 rounding of two values at once, each exactly quantize<FP16>: one
// packed conversion (nearest even), one packed minimum with the largest half
// (a value at or above the largest half converts to it or to +inf, which the
// minimum brings back to it: the saturation of quantize), two widenings.
// For the non-negative magnitudes of a check update.
typedef _Float16 half2_v __attribute__((ext_vector_type(2)));
typedef float float2_v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2_v quantize_fp16_pair(float a, float b) {
    const float2_v x = {a, b};
    const half2_v cap = {(_Float16)65504.0f, (_Float16)65504.0f};
    const half2_v h = __builtin_elementwise_min(__builtin_convertvector(x, half2_v), cap);
    return __builtin_convertvector(h, float2_v);
}

// The prior as the decoder uses it: -0 read as +0; INT6 puts it on the
// message grid, FP16 on the grid of step 2^-24 (magnitudes >= 1 already are).
template <int MT>
__device__ __forceinline__ float prior(float x) {
    x = x + 0.0f;
    if constexpr (MT == SAGMS_MSG_INT6) {
        return quantize<MT>(x) + 0.0f;
    } else if constexpr (MT == SAGMS_MSG_FP16) {
        return (fabsf(x) < 1.0f ? rintf(x * 16777216.0f) * 0x1.0p-24f : x) + 0.0f;
    } else {
        return x;
    }
}

// Check-node update of one check (eq. (ms_cn) scaled per eq. (alphaeff) /
// (sagms_cn), or eq. (bp4_cn) for BP): v = incoming v2c messages, sb = the
// original syndrome bit at the sign position, unsat = the residual bit,
// gs / gu = the gains of a satisfied / unsatisfied check.
template <int DC, bool BP, int MT>
__device__ __forceinline__ void cn_update(const float (&v)[DC], uint32_t sb, bool unsat, float gs, float gu,
                                          float (&c2v)[DC]) {
    const uint32_t par = xor_signs<DC>(v, sb);  // parity in the sign bit only
    if constexpr (BP) {
        float mag[DC];
        bp_magnitudes<DC>(v, mag);
#pragma unroll
        for (int p = 0; p < DC; ++p) c2v[p] = __uint_as_float(bits(mag[p]) | ((bits(v[p]) ^ par) & kSign));
    } else {
        const float alpha = unsat ? gu : gs;
        float m1 = fabsf(v[0]), m2 = __builtin_inff();
#pragma unroll
        for (int p = 1; p < DC; ++p) {
            float x = fabsf(v[p]);
            m2 = __builtin_amdgcn_fmed3f(m1, x, m2);
            m1 = fminf(m1, x);
        }
        // two products per check, both magnitudes pre-signed with the check
        // parity; per edge: compare, select, and one 3-input bit operation
        // applying the edge's own sign.  The empty asm keeps the compiler
        // from folding the select back into one product per edge.
        uint32_t S1, S2;
        if constexpr (MT == SAGMS_MSG_FP32) {
            // the gain carries the parity sign: m1, m2 >= 0 and a product's
            // sign is the xor of its operands' signs while its magnitude
            // rounds the same either way, so these are the bits of alpha m1
            // and alpha m2 with the parity sign attached
            const float sa = __uint_as_float(xor_and(bits(alpha), par, kSign));
            S1 = bits(sa * m1);
            S2 = bits(sa * m2);
        } else if constexpr (MT == SAGMS_MSG_FP16) {
            // the two magnitudes and the two products rounded pairwise
            const float2_v q = quantize_fp16_pair(m1, m2);
            const float2_v o = quantize_fp16_pair(alpha * q.x, alpha * q.y);
            S1 = or_and(bits(o.x), par, kSign);
            S2 = or_and(bits(o.y), par, kSign);
        } else {
            S1 = or_and(bits(quantize<MT>(alpha * quantize<MT>(m1))), par, kSign);
            S2 = or_and(bits(quantize<MT>(alpha * quantize<MT>(m2))), par, kSign);
        }
        asm("" : "+v"(S1), "+v"(S2));
#pragma unroll
        for (int p = 0; p < DC; ++p) {
            const uint32_t sel = fabsf(v[p]) == m1 ? S2 : S1;
            c2v[p] = __uint_as_float(xor_and(sel, bits(v[p]), kSign));
        }
    }
}

// One wave's decoder for one code: graph tables and priors held in
// registers, loaded once (load) and reused for every frame (frame).  The LDS
// slice `lds` belongs to this wave alone.
//
// The round's two gains are indexed by the residual weight w.  KG: from the
// kernel argument table (KernelGains, one-block codes), by a scalar load;
// otherwise from the gain table that load() writes to the wave's LDS slice,
// by one 8-byte read at a wave-uniform address (a broadcast, no bank
// conflict).  Either latency hides behind the running minima.
template <int DC, int DV, int CPL, int VPL, bool BP, int MT, bool KG = false>
struct WaveDecoder {
    static_assert(!KG || CPL == 1, "kernel-argument gains are for one-block codes");
    using LY = Lay<DC, CPL, VPL>;
    uint32_t caddr[CPL][DC];
    uint32_t vaddr[VPL][DV];
    float L0[VPL];

    __device__ __forceinline__ void load(const DecodeArgs& a, float* lds, int lane) {
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
            int j = k * 64 + lane;
            L0[k] = j < a.n ? prior<MT>(a.llr0[j]) : __builtin_inff();
        }
        if constexpr (!KG) write_gains(a.gains, a.m, LY::CW + 1, lds + LY::GAIN0, lane);
        lds[LY::ZERO + lane] = 0.0f;
        lds[LY::PADPOST + lane] = __builtin_inff();
    }

    // Original syndrome bits of frame f for the lane's checks, at the sign
    // position (checks beyond m read as 0; their rows hold only the +inf
    // padding).
    // (a vector load: the address is moved to vector registers, since scalar
    // loads of the syndromes fetched twice their bytes from HBM; it stays a
    // global-memory pointer, so that the load is not a flat load, which the
    // LDS waits would also wait for)
    __device__ __forceinline__ static void load_syndrome(const DecodeArgs& a, int64_t f, uint64_t (&word)[CPL]) {
        using GlobalWord = const __attribute__((address_space(1))) uint64_t;
        GlobalWord* row = (GlobalWord*)(a.synd + f * a.wm);  // address-space cast
        asm("" : "+v"(row));
#pragma unroll
        for (int k = 0; k < CPL; ++k) word[k] = k < a.wm ? row[k] : 0ull;
    }
    __device__ __forceinline__ static void syndrome_bits(const DecodeArgs& a, int lane, const uint64_t (&word)[CPL],
                                                         uint32_t (&sb)[CPL]) {
#pragma unroll
        for (int k = 0; k < CPL; ++k)
            sb[k] = (k * 64 + lane < a.m) ? (uint32_t)((word[k] >> lane) & 1ull) << 31 : 0u;
    }

    // Decodes frame f, whose syndrome bits are sb, and writes its outputs.
    // The syndrome of frame f_next is loaded when the frame starts and left
    // in sb when its rounds are done, so the load latency hides behind them.
    // UR: rounds per iteration of the round loop (1 or 2; each round keeps
    // its own exit tests, so the results do not depend on it).
    template <int UR = 1>
    __device__ __forceinline__ void frame(const DecodeArgs& a, float* lds, int lane, int64_t f, uint32_t (&sb)[CPL],
                                          int64_t f_next, const KernelGains* kg = nullptr) {
        static_assert(UR == 1 || UR == 2, "one or two rounds per loop iteration");
        uint64_t next_word[CPL];
        load_syndrome(a, f_next, next_word);
        // The posteriors are written to the wave's LDS slice every round.
        // With 16 variables per lane (the l = 511 shape) no register holds
        // them through the rounds and the outputs read them back from LDS
        // (11 % faster there); the smaller shapes keep a register copy.
        constexpr bool kPostInLds = VPL >= 16;
        float post[VPL];
#pragma unroll
        for (int k = 0; k < VPL; ++k) {
            if constexpr (!kPostInLds) post[k] = L0[k];
            lds[LY::POST0 + k * 64 + lane] = L0[k];
        }
        // the check's own previous outputs: written by the first round
        // before any read (the first round's are zero and not subtracted)
        float c2v[CPL][DC];
        wave_lds_sync();

        int it = 0;
        bool conv = false;
        // one round; false once the frame is done.  first: the frame's first
        // round, whose v2c messages are the posteriors themselves (its own
        // previous outputs are zero, and x - 0 is x bit for bit)
        auto round = [&](auto first) -> bool {
            constexpr bool FIRST = decltype(first)::value;
            // top of the round: v2c, hard-decision parity, residual syndrome
            float v[CPL][DC];
            bool unsat[CPL];  // residual syndrome bit: s xor (H e_hat) of the check
            int w = 0;
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                float pj[DC];
#pragma unroll
                for (int p = 0; p < DC; ++p) {
                    pj[p] = lds[caddr[k][p]];
                    v[k][p] = FIRST ? pj[p] : pj[p] - c2v[k][p];  // rounded only through the check output
                }
                unsat[k] = (int32_t)xor_signs<DC>(pj, sb[k]) < 0;
                w += __builtin_popcountll(ballot(unsat[k]));
            }
            if (w == 0) {
                conv = true;
                return false;
            }
            if (it == a.lmax) return false;
            ++it;
            // CN update; gains of the residual weight w (eq. (alphaeff))
            float2 gg;
            if constexpr (KG)
                gg = kg->g[w];
            else
                gg = *reinterpret_cast<const float2*>(&lds[LY::GAIN0 + 2 * w]);
            const float gs = gg.x, gu = gg.y;
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                cn_update<DC, BP, MT>(v[k], sb[k], unsat[k], gs, gu, c2v[k]);
#pragma unroll
                for (int p = 0; p < DC; ++p) lds[p * LY::CW + k * 64 + lane] = c2v[k][p];
            }
            wave_lds_sync();
            // VN update: posterior in the graph's summation order
#pragma unroll
            for (int k = 0; k < VPL; ++k) {
                float s = L0[k];
#pragma unroll
                for (int r = 0; r < DV; ++r) s = s + lds[vaddr[k][r]];
                if constexpr (!kPostInLds) post[k] = s;
                lds[LY::POST0 + k * 64 + lane] = s;
            }
            wave_lds_sync();
            return true;
        };
        using First = std::integral_constant<bool, true>;
        using Later = std::integral_constant<bool, false>;
        if (round(First{}))
            while (round(Later{})) {
                if constexpr (UR == 2)
                    if (!round(Later{})) break;
            }

        syndrome_bits(a, lane, next_word, sb);
        // take the prefetched bits before the output stores are issued: a
        // wait placed after them would also wait for the stores
#pragma unroll
        for (int k = 0; k < CPL; ++k) asm volatile("" ::"v"(sb[k]));
        // outputs: hard decisions, round count, convergence flag
        if constexpr (kPostInLds) {
#pragma unroll
            for (int k = 0; k < VPL; ++k) post[k] = lds[LY::POST0 + k * 64 + lane];
        }
        uint64_t mine = 0;
#pragma unroll
        for (int k = 0; k < VPL; ++k) {
            int j = k * 64 + lane;
            uint64_t word = ballot(j < a.n && post[k] < 0.0f);
            if (lane == k) mine = word;
        }
        if (lane < a.wn) a.ehat[f * a.wn + lane] = mine;
        if (a.post) {
#pragma unroll
            for (int k = 0; k < VPL; ++k) {
                int j = k * 64 + lane;
                if (j < a.n) a.post[f * a.n + j] = post[k];
            }
        }
        if (lane == 0) {
            a.iters[f] = it;
            a.conv[f] = conv ? 1 : 0;
        }
    }
};

}  // namespace sagms
