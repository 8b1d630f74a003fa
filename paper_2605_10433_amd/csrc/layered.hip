// Layered-schedule decoder: the check-serial alternative to the flooding
// schedule of Algorithm 1 (the paper defines only flooding; the reading
// implemented here is stated with SAGMS_LAYERED in sagms.h).
//
// The host splits the checks into layers of checks with pairwise disjoint
// supports (first fit in ascending check index) and packs them into passes
// of at most G checks: in (layer, position) order, each check goes to the
// earliest pass after every pass that holds a check sharing a variable with
// it.  Each variable therefore meets its checks in layer order, and every
// check reads the posteriors the layer-by-layer schedule would give it.  A
// wavefront decodes F = 64 / G frames at once, one per group of G lanes.  In
// pass p, lane q of a group updates check pass_check[p][q] of its frame: it
// reads its variables' posteriors and its own previous outputs, forms
// v2c = posterior - c2v_old, computes the check output with the operations
// of the flooding decoder's check update, and writes c2v_new and
// posterior = v2c + c2v_new back.  The checks of one pass touch disjoint
// variables, and one wavefront's LDS operations complete in order, so the
// passes need no barrier.
//
// A check's DC outputs are kept in three words instead of DC: S1 (the
// output magnitude of the non-minimum edges with the parity sign), S1 xor S2
// (S2: that of the minimum edges), and a mask holding, for edge k, bit k =
// "|v2c_k| was the minimum" and bit 16 + k = the sign of v2c_k.  Output k is
// S1 xor (D and minimum-bit-k) xor (sign-bit-k in the sign position), the
// same 32 bits as when it was computed, so the messages stay exact while a
// frame's LDS shrinks from n + m * DC to n + 4 m words and more frames fit
// on a compute unit.  When the schedule has at most kLayeredRegPasses passes
// (PMAX > 0), lane q keeps the three words of its check of every pass in
// registers instead (the pass loop is unrolled, so each pass names its own
// registers) and a frame needs only its posteriors and syndrome bits in LDS.
// The tables of the next passes are read while the current one computes.
// After the last pass every lane recomputes the residual-syndrome bits of the
// checks q, q + G, ... from the hard decisions; the weight gives the next
// round's gains and the exit test.
//
// A frame's first residual is its syndrome xor H [L0 < 0], the latter
// computed once per wavefront.  A wavefront owns a contiguous run of frames.
// A group that has no frame takes the next unclaimed frame of the run and
// loads its syndrome words then, so groups stay busy until the run is used
// up whatever their frames' round counts.  (A group holding a claimed next
// frame while it decoded the current one could leave two long frames for
// the end of the run.)
#include "decode_core.h"

namespace sagms {

struct LayeredArgs {
    DecodeArgs a;
    const int32_t* pass_check;   // [P][G] check of (pass, lane), -1 = idle
    const uint32_t* check_vars;  // [m][DC / 2] variable pairs as byte offsets 4 j (low, high 16 bits)
    int64_t frames_per_wave;
    int P, npad, gwords, tables;  // tables: LDS words in front of the group slices
};

// The float at byte offset `off` of `base` (LDS tables hold byte offsets).
__device__ __forceinline__ float& at(float* base, uint32_t off) {
    return *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + off);
}

template <int G>
__device__ __forceinline__ uint64_t group_segment(uint64_t ballot, int grp) {
    if constexpr (G == 64) {
        return ballot;
    } else {
        return (ballot >> (grp * G)) & ((1ull << G) - 1);
    }
}

// PMAX = 0: check outputs in LDS; PMAX > 0: in registers, at most PMAX passes
// (register budget: 4 wavefronts per SIMD for up to 16 passes of degree 6 or
// 8, else 3: the outputs of more passes, or the wider check update of degree
// 10, do not fit the 128 VGPRs of a fourth).
template <int DC, int G, int PMAX>
__global__ void __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(PMAX > 0 ? (DC >= 10 || PMAX > kLayeredRegPassesShort ? 3 : 4) : 1)))
layered_kernel(LayeredArgs la) {
    constexpr int F = 64 / G;
    static_assert(F * G == 64, "G must divide 64");
    constexpr int NREG = PMAX > 0 ? PMAX : 1;
    extern __shared__ uint32_t lds_u[];
    const DecodeArgs& a = la.a;
    const int lane = threadIdx.x;
    const int grp = lane / G, q = lane % G;
    const int m = a.m, n = a.n, wm = a.wm, wn = a.wn;

    uint32_t* t_pass = lds_u;
    uint32_t* t_vars = t_pass + la.P * G;
    float* t_gain = reinterpret_cast<float*>(t_vars + m * (DC / 2));
    float* t_l0 = t_gain + 2 * (m + 1);
    uint32_t* t_r0 = reinterpret_cast<uint32_t*>(t_l0 + n);  // residual bits of the prior's hard decision
    float* post = reinterpret_cast<float*>(lds_u + la.tables + grp * la.gwords);
    uint4* cmp = reinterpret_cast<uint4*>(post + la.npad);  // PMAX = 0, per check: S1, S1 ^ S2, mask, unused
    uint32_t* sbits = PMAX > 0 ? reinterpret_cast<uint32_t*>(post + la.npad) : reinterpret_cast<uint32_t*>(cmp + m);
    uint32_t* rbits = sbits + 2 * wm;

    for (int t = lane; t < la.P * G; t += 64) t_pass[t] = (uint32_t)la.pass_check[t];
    for (int t = lane; t < m * (DC / 2); t += 64) t_vars[t] = la.check_vars[t];
    write_gains(a.gains, m, m + 1, t_gain, lane);
    for (int t = lane; t < n; t += 64) t_l0[t] = a.llr0[t] + 0.0f;  // -0 reads as +0
    __syncthreads();
    // H [L0 < 0] (mod 2): a frame's first residual is its syndrome xor this
    for (int r = 0; r * 64 < m; ++r) {
        const int c = r * 64 + lane;
        uint32_t par = 0;
        if (c < m)
            for (int k = 0; k < DC / 2; ++k) {
                const uint32_t pv = t_vars[c * (DC / 2) + k];
                par ^= __float_as_uint(at(t_l0, pv & 0xFFFFu)) >> 31;
                par ^= __float_as_uint(at(t_l0, pv >> 16)) >> 31;
            }
        const uint64_t bal = __ballot(par != 0);
        if (lane == 0) {
            t_r0[2 * r] = (uint32_t)bal;
            t_r0[2 * r + 1] = (uint32_t)(bal >> 32);
        }
    }
    __syncthreads();

    const int64_t f_begin = (int64_t)blockIdx.x * la.frames_per_wave;
    const int64_t f_end = min(f_begin + la.frames_per_wave, a.nframes);
    if (f_begin >= f_end) return;

    // group state (equal in the G lanes of a group)
    int64_t f = -1;           // frame being decoded
    int64_t next = f_begin;   // wave-uniform: next unclaimed frame
    // lanes q < wm: word q of a frame's syndrome, its bits at or above m
    // cleared (the caller's padding bits are not syndrome bits)
    const uint64_t keep = q == wm - 1 && (m & 63) ? (1ull << (m & 63)) - 1 : ~0ull;
    int it = 0, w = 0;
    bool active = false, more = true;  // more: the run may still hold a frame for this group
    // PMAX > 0: outputs of the lane's check in pass p (S1, S1 ^ S2, mask)
    uint32_t rs1[NREG], rd[NREG], rmk[NREG];
#pragma unroll
    for (int p = 0; p < NREG; ++p) rs1[p] = rd[p] = rmk[p] = 0u;

    // Residual bits of the group's frame from its posteriors; returns the
    // weight.  Executed by the lanes of the groups in `on`.
    // (the variable pairs of the next row of checks are read one row ahead;
    // lanes past the last check read the last check's row and ignore it)
    auto residual = [&](bool on) -> int {
        int weight = 0;
        uint32_t pv_next[DC / 2];
#pragma unroll
        for (int k = 0; k < DC / 2; ++k) pv_next[k] = t_vars[min(q, m - 1) * (DC / 2) + k];
        for (int r = 0; r * G < m; ++r) {
            const int c = r * G + q;
            uint32_t pv[DC / 2];
#pragma unroll
            for (int k = 0; k < DC / 2; ++k) pv[k] = pv_next[k];
            if ((r + 1) * G < m) {
#pragma unroll
                for (int k = 0; k < DC / 2; ++k) pv_next[k] = t_vars[min(c + G, m - 1) * (DC / 2) + k];
            }
            bool bit = false;
            if (on && c < m) {
                uint32_t par = (sbits[c >> 5] >> (c & 31)) & 1u;
#pragma unroll
                for (int k = 0; k < DC / 2; ++k) {
                    par ^= __float_as_uint(at(post, pv[k] & 0xFFFFu)) >> 31;
                    par ^= __float_as_uint(at(post, pv[k] >> 16)) >> 31;
                }
                bit = par != 0;
            }
            const uint64_t seg = group_segment<G>(__ballot(bit), grp);
            weight += __popcll(seg);
            if (on && q == 0) {
                if constexpr (G == 64) {
                    rbits[2 * r] = (uint32_t)seg;
                    rbits[2 * r + 1] = (uint32_t)(seg >> 32);
                } else if constexpr (G == 32) {
                    rbits[r] = (uint32_t)seg;
                } else if constexpr (G == 16) {
                    // byte stores: they may alias the 32-bit reads of the bits
                    reinterpret_cast<uint8_t*>(rbits)[2 * r] = (uint8_t)seg;
                    reinterpret_cast<uint8_t*>(rbits)[2 * r + 1] = (uint8_t)(seg >> 8);
                } else {
                    static_assert(G == 8, "group sizes 8, 16, 32, 64");
                    reinterpret_cast<uint8_t*>(rbits)[r] = (uint8_t)seg;
                }
            }
        }
        return weight;
    };

    // Outputs of the group's frame (groups in `on`): hard decisions, rounds,
    // flag and, when asked for, the posteriors.
    auto finish = [&](bool on, int rounds, bool conv) {
        if (__ballot(on) == 0) return;
        uint64_t word = 0;
        for (int r = 0; r * G < n; ++r) {
            const int j = r * G + q;
            const bool neg = on && j < n && post[j] < 0.0f;
            const uint64_t seg = group_segment<G>(__ballot(neg), grp);
            const int bit0 = r * G;
            if (q == (bit0 >> 6)) word |= seg << (bit0 & 63);
        }
        if (on) {
            if (q < wn) a.ehat[f * wn + q] = word;
            if (q == 0) {
                a.iters[f] = rounds;
                a.conv[f] = conv ? 1 : 0;
            }
            if (a.post)
                for (int j = q; j < n; j += G) a.post[f * n + j] = post[j];
        }
    };

    while (true) {
        // idle groups take the next frames of the run (in group order) and
        // finish frames that need no round, until every group decodes a
        // frame or the run is used up
        while (true) {
            const bool want = !active && more;
            const uint64_t takers = __ballot(want && q == 0);
            if (takers == 0) break;
            bool start = false;
            if (want) {
                f = next + __popcll(takers & ((1ull << (grp * G)) - 1));
                more = f < f_end;
                start = more;
            }
            next += __popcll(takers);
            if (start) {
                for (int j = q; j < n; j += G) post[j] = t_l0[j];
                if constexpr (PMAX > 0) {
#pragma unroll
                    for (int p = 0; p < PMAX; ++p) rs1[p] = rd[p] = rmk[p] = 0u;
                } else {
                    for (int t = q; t < m; t += G) cmp[t] = make_uint4(0u, 0u, 0u, 0u);
                }
                if (q < wm) {
                    const uint64_t word = a.synd[f * wm + q] & keep;
                    sbits[2 * q] = (uint32_t)word;
                    sbits[2 * q + 1] = (uint32_t)(word >> 32);
                    rbits[2 * q] = (uint32_t)word ^ t_r0[2 * q];
                    rbits[2 * q + 1] = (uint32_t)(word >> 32) ^ t_r0[2 * q + 1];
                }
            }
            int w0 = 0;
            if (start)
                for (int t = 0; t < 2 * wm; ++t) w0 += __popc(rbits[t]);
            if (start) {
                w = w0;
                it = 0;
                active = w0 != 0;
            }
            finish(start && w0 == 0, 0, true);
        }
        if (__ballot(active) == 0) break;

        // one round: every layer of checks, pass by pass
        const float gs = t_gain[2 * w], gu = t_gain[2 * w + 1];
        // Check update of check c (variable pairs pv) in place of its
        // previous outputs (s1, dd, mk): reads its posteriors, writes the
        // new posteriors and returns the new outputs in (s1, dd, mk).
        auto check_update = [&](int c, const uint32_t (&pv)[DC / 2], uint32_t& s1, uint32_t& dd, uint32_t& mk) {
            // byte offsets of the check's posteriors (the 16-bit halves fold
            // into the address adds)
            uint32_t off[DC];
#pragma unroll
            for (int k = 0; k < DC / 2; ++k) {
                off[2 * k] = pv[k] & 0xFFFFu;
                off[2 * k + 1] = pv[k] >> 16;
            }
            // issue every LDS read of the check before the first use, so that
            // their latencies overlap
            float pj[DC];
#pragma unroll
            for (int k = 0; k < DC; ++k) pj[k] = at(post, off[k]);
            const uint32_t sword = sbits[c >> 5], rword = rbits[c >> 5];
            __builtin_amdgcn_sched_barrier(0);
            float v[DC];
#pragma unroll
            for (int k = 0; k < DC; ++k) {
                const uint32_t minbit = (uint32_t)__builtin_amdgcn_sbfe(mk, k, 1);
                const uint32_t prev = xor_and(s1, dd, minbit) ^ ((mk << (15 - k)) & kSign);
                v[k] = pj[k] - __uint_as_float(prev);
            }
            const uint32_t par = xor_signs<DC>(v, ((sword >> (c & 31)) & 1u) << 31);
            const bool unsat = (rword >> (c & 31)) & 1u;
            const float alpha = unsat ? gu : gs;
            float m1 = fabsf(v[0]), m2 = __builtin_inff();
#pragma unroll
            for (int k = 1; k < DC; ++k) {
                const float x = fabsf(v[k]);
                m2 = __builtin_amdgcn_fmed3f(m1, x, m2);
                m1 = fminf(m1, x);
            }
            const uint32_t S1 = or_and(bits(alpha * m1), par, kSign);
            const uint32_t S2 = or_and(bits(alpha * m2), par, kSign);
            uint32_t mask = 0;
#pragma unroll
            for (int k = 0; k < DC; ++k) {
                const bool is_min = fabsf(v[k]) == m1;
                const uint32_t out = xor_and(is_min ? S2 : S1, bits(v[k]), kSign);
                mask |= (is_min ? 1u << k : 0u) | ((bits(v[k]) >> 31) << (16 + k));
                at(post, off[k]) = v[k] + __uint_as_float(out);
            }
            s1 = S1;
            dd = S1 ^ S2;
            mk = mask;
        };
        // The tables are read ahead: during pass p the check of pass p + 2
        // and the variable pairs of pass p + 1's check, so that no table
        // read waits on another.  (Idle lanes, c = -1, read check 0's row and
        // ignore it.)
        int c_next = la.P > 1 ? (int)t_pass[G + q] : -1;
        uint32_t pv_next[DC / 2];
        int c = (int)t_pass[q];
#pragma unroll
        for (int k = 0; k < DC / 2; ++k) pv_next[k] = t_vars[max(c, 0) * (DC / 2) + k];
        auto read_ahead = [&](int p, uint32_t (&pv)[DC / 2]) -> int {
#pragma unroll
            for (int k = 0; k < DC / 2; ++k) pv[k] = pv_next[k];
            int c_after = -1;
            if (p + 1 < la.P) {
#pragma unroll
                for (int k = 0; k < DC / 2; ++k) pv_next[k] = t_vars[max(c_next, 0) * (DC / 2) + k];
                if (p + 2 < la.P) c_after = (int)t_pass[(p + 2) * G + q];
            }
            return c_after;
        };
        if constexpr (PMAX > 0) {
#pragma unroll
            for (int p = 0; p < PMAX; ++p) {
                if (p < la.P) {
                    uint32_t pv[DC / 2];
                    const int c_after = read_ahead(p, pv);
                    if (active && c >= 0) check_update(c, pv, rs1[p], rd[p], rmk[p]);
                    c = c_next;
                    c_next = c_after;
                }
            }
        } else {
            for (int p = 0; p < la.P; ++p) {
                uint32_t pv[DC / 2];
                const int c_after = read_ahead(p, pv);
                if (active && c >= 0) {
                    const uint4 old = cmp[c];
                    uint32_t s1 = old.x, dd = old.y, mk = old.z;
                    check_update(c, pv, s1, dd, mk);
                    cmp[c] = make_uint4(s1, dd, mk, 0u);
                }
                c = c_next;
                c_next = c_after;
            }
        }
        const int w1 = residual(active);
        bool done = false;
        if (active) {
            ++it;
            w = w1;
            done = w1 == 0 || it >= a.lmax;
        }
        finish(done, it, w1 == 0);
        if (done) active = false;
    }
}

namespace {

template <int DC, int G, int PMAX>
int launch_dg(const LayeredArgs& la, size_t lds, int num_cu, hipStream_t st) {
    const void* fn = reinterpret_cast<const void*>(&layered_kernel<DC, G, PMAX>);
    int per_cu = 0;
    SAGMS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, lds));
    if (per_cu < 1) return fail(SAGMS_EUNSUPPORTED, "layered kernel does not fit a compute unit");
    constexpr int F = 64 / G;
    const int64_t groups_needed = (la.a.nframes + F - 1) / F;
    int64_t waves = std::min<int64_t>((int64_t)per_cu * num_cu, groups_needed);
    LayeredArgs x = la;
    x.frames_per_wave = (la.a.nframes + waves - 1) / waves;
    waves = (la.a.nframes + x.frames_per_wave - 1) / x.frames_per_wave;
    hipLaunchKernelGGL((layered_kernel<DC, G, PMAX>), dim3((unsigned)waves), dim3(64), lds, st, x);
    SAGMS_HIP(hipGetLastError());
    return SAGMS_OK;
}

template <int DC, int PMAX>
int launch_dp(int G, const LayeredArgs& la, size_t lds, int num_cu, hipStream_t st) {
    switch (G) {
        case 8: return launch_dg<DC, 8, PMAX>(la, lds, num_cu, st);
        case 16: return launch_dg<DC, 16, PMAX>(la, lds, num_cu, st);
        case 32: return launch_dg<DC, 32, PMAX>(la, lds, num_cu, st);
        case 64: return launch_dg<DC, 64, PMAX>(la, lds, num_cu, st);
        default: return fail(SAGMS_EUNSUPPORTED, "layered group size %d (internal)", G);
    }
}

template <int DC>
int launch_d(int G, bool regs, const LayeredArgs& la, size_t lds, int num_cu, hipStream_t st) {
    if (!regs) return launch_dp<DC, 0>(G, la, lds, num_cu, st);
    // the shorter register form where it holds the schedule: fewer registers
    // to clear when a frame starts, and a fourth wavefront for degrees 6, 8
    if (la.P <= kLayeredRegPassesShort) return launch_dp<DC, kLayeredRegPassesShort>(G, la, lds, num_cu, st);
    return launch_dp<DC, kLayeredRegPasses>(G, la, lds, num_cu, st);
}

}  // namespace

// One lane per frame for the compiled l = 63 code (layered_lane.hip).
int launch_layered_lane(const DecodeArgs& a, hipStream_t st);

int launch_layered(const LayeredPlan& plan, const DecodeArgs& a, hipStream_t st) {
    if (a.nframes <= 0) return SAGMS_OK;
    if (plan.group == 1) return launch_layered_lane(a, st);
    LayeredArgs la{};
    la.a = a;
    la.pass_check = plan.pass_check;
    la.check_vars = plan.check_vars;
    la.P = plan.passes;
    la.npad = plan.npad;
    la.gwords = plan.group_words;
    la.tables = plan.table_words;
    const int F = 64 / plan.group;
    const size_t lds = (size_t)(plan.table_words + F * plan.group_words) * sizeof(uint32_t);
    int dev = 0, num_cu = 0;
    SAGMS_HIP(hipGetDevice(&dev));
    SAGMS_HIP(hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    switch (plan.dc) {
        case 6: return launch_d<6>(plan.group, plan.regs, la, lds, num_cu, st);
        case 8: return launch_d<8>(plan.group, plan.regs, la, lds, num_cu, st);
        case 10: return launch_d<10>(plan.group, plan.regs, la, lds, num_cu, st);
        default: return fail(SAGMS_EUNSUPPORTED, "layered schedule: check degree %d not compiled", plan.dc);
    }
}

}  // namespace sagms
